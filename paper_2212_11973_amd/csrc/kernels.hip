// gfx950 kernels of the one-site tangent-space sweep.
//
//  * k_gemm      : grouped GEMM over charge blocks with gather/scatter index
//                  maps (each operand index is a stride or a table), FP64
//                  MFMA 16x16x4 tiles, one 64x64 output tile per workgroup of
//                  four 64-wide waves.  Used for every dense contraction of the
//                  sweep: L.A, .R, the environment updates, the bond apply
//                  and the absorb step (SM Fig. Lanczos, Fig. optimalB), for
//                  problems large in all three dimensions.
//  * k_wgemm     : the same grouped contractions for small, short-K or
//                  skinny charge blocks (most blocks of a U(1)xU(1) sweep):
//                  one wave per 64x16 / 32x32 / 16x64 output block, operands
//                  straight from global memory, optional four-way K split
//                  inside the workgroup; one launch per contraction.
//  * k_wstage    : the contraction with the Hamiltonian MPO tensor W, which is
//                  sparse (a few nonzero 4x4 operators per bond pair); a
//                  bandwidth-bound weighted sum of strided blocks.
//  * k_qr_*      : Householder QR of the charge blocks with non-negative
//                  diagonal (SM Sec. II.F step 3): in LDS, tall blocks as a
//                  two-level tall-skinny QR; blocks wider than 64 columns in
//                  global memory, one workgroup each.
//  * Lanczos     : deterministic fixed-order reductions, Gram-Schmidt
//                  updates and the small tridiagonal exponential on the device
//                  (SM Sec. II.H), so a local exponential needs no host sync.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace tt {

typedef double double4_t __attribute__((ext_vector_type(4)));

#define HIP_CHECK_LAUNCH()                                                       \
  do {                                                                           \
    ++g_launches;                                                                \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e_));        \
  } while (0)

long long g_launches = 0;   // kernels enqueued by this library since load
long long launch_count() { return g_launches; }

// ------------------------------------------------------------------ profiling
namespace {
// events recorded since the last read; a record spans two of them
struct ProfRec { int a, b; int kind; double flops, bytes; };
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_ev;
std::vector<hipEvent_t> g_pool;
int g_open = -1, g_last = -1;
int record_event(hipStream_t st) {
  hipEvent_t e;
  if (!g_pool.empty()) {
    e = g_pool.back();
    g_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    throw Error(TT_EDEVICE, "hipEventCreate failed");
  }
  g_ev.push_back(e);
  if (hipEventRecord(e, st) != hipSuccess) throw Error(TT_EDEVICE, "hipEventRecord failed");
  return (int)g_ev.size() - 1;
}
}  // namespace

void prof_enable(bool on) { g_prof = on; }
bool prof_enabled() { return g_prof; }
void prof_begin(hipStream_t st) {
  if (!g_prof) return;
  g_open = g_last = record_event(st);
}
void prof_mark(hipStream_t st, int kind, double flops, double bytes) {
  if (!g_prof || g_open < 0) return;
  int e = record_event(st);
  g_recs.push_back({g_last, e, kind, flops, bytes});
  g_last = e;
}
void prof_end(hipStream_t st, int kind, double flops, double bytes) {
  if (!g_prof || g_open < 0) return;
  int e = (g_last != g_open) ? g_last : record_event(st);
  g_recs.push_back({g_open, e, kind, flops, bytes});
  g_open = g_last = -1;
}
void prof_read(double out[PROF_KINDS][4]) {
  for (int k = 0; k < PROF_KINDS; ++k)
    for (int j = 0; j < 4; ++j) out[k][j] = 0.0;
  if (!g_ev.empty() && hipEventSynchronize(g_ev.back()) != hipSuccess)
    throw Error(TT_EDEVICE, "hipEventSynchronize failed");
  for (auto& r : g_recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_ev[r.a], g_ev[r.b]) != hipSuccess)
      throw Error(TT_EDEVICE, "hipEventElapsedTime failed");
    out[r.kind][0] += ms;
    out[r.kind][1] += r.flops;
    out[r.kind][2] += r.bytes;
    out[r.kind][3] += 1;
  }
  g_recs.clear();
  g_pool.insert(g_pool.end(), g_ev.begin(), g_ev.end());
  g_ev.clear();
  g_open = g_last = -1;
}

// ------------------------------------------------------------------ GEMM
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ long long idx_map(const long long* __restrict__ tabs, long long tab, long long stride,
                                             long long i) {
  return tab >= 0 ? tabs[tab + i] : i * stride;
}

// K depth of one LDS tile per precision (the BF16 MFMA consumes 32 K per instruction)
template <int PREC> struct PrecTraits;
template <> struct PrecTraits<TT_FP64> { static constexpr int BK = 16, PARTS = 1; };
template <> struct PrecTraits<TT_FP32> { static constexpr int BK = 16, PARTS = 1; };
template <> struct PrecTraits<TT_BF16X3> { static constexpr int BK = 32, PARTS = 2; };
template <> struct PrecTraits<TT_BF16X6> { static constexpr int BK = 32, PARTS = 3; };
constexpr int kBfPad = 8;   // keeps the 8-element BF16 rows 16-byte aligned

template <int WGM, int WGN, int FM, int FN, bool SPLITK, int PREC>
constexpr int gemm_smem_bytes_t() {
  constexpr int BK = PrecTraits<PREC>::BK, P = PrecTraits<PREC>::PARTS;
  constexpr int BM = WGM * 16 * FM, BN = WGN * 16 * FN;
  constexpr int tiles = (PREC == TT_FP64) ? 8 * (BK * (BM + 1) + BK * (BN + 1))
                        : (PREC == TT_FP32) ? 4 * (BK * (BM + 1) + BK * (BN + 1))
                                            : 2 * P * (BM + BN) * (BK + kBfPad);
  constexpr int tabs = 8 * (2 * BM + BN + 2 * BK);
  constexpr int red = SPLITK ? 8 * 4 * BM * BN : 0;
  return tiles + tabs + red;
}

// split a double into BF16 parts x ~ p0 + p1 (+ p2), each rounded to nearest
template <int P>
__device__ __forceinline__ void bf16_split(double x, __bf16* out) {
  __bf16 h = (__bf16)(float)x;
  out[0] = h;
  double r = x - (double)(float)h;
  __bf16 m = (__bf16)(float)r;
  out[1] = m;
  if (P == 3) out[2] = (__bf16)(float)(r - (double)(float)m);
}

// One BM x BN output tile of one problem.  Four 64-wide waves in a WGM x WGN
// grid, each owning FM x FN MFMA 16x16 blocks; with SPLITK all waves own the
// whole tile and take alternate 4-deep K sub-steps, reduced through LDS.  A
// K-split problem covers only the K slice of this tile and writes a partial
// that k_gemm_reduce adds up in slice order.
// FP64: f64 MFMA.  FP32 / BF16: f32-accumulating MFMA inside each K tile,
// added into FP64 accumulators after every K tile.
// Global loads of the next K tile are issued before the MFMAs of the current
// one (register double buffering), so their latency overlaps the compute.
// With PL (split BF16 only) both operands are BF16 planes (part p of an
// element at plane p, pl.s[slot] elements apart: the element offsets of the
// plan apply to every plane), read without splitting; with pl.c the result is
// written as planes too (each value split into the NP parts).
template <int WGM, int WGN, int FM, int FN, bool SPLITK, int PREC, bool PL = false>
__device__ __forceinline__ void gemm_tile(const GemmProb& P, const GemmTile& T, const long long* __restrict__ tabs,
                                          const Slots& slots, char* smem, double* __restrict__ pws,
                                          const Planes& pl = Planes{}) {
  constexpr int BK = PrecTraits<PREC>::BK, NP = PrecTraits<PREC>::PARTS;
  constexpr int WM = 16 * FM, WN = 16 * FN;
  constexpr int BM = WGM * WM, BN = WGN * WN;
  constexpr bool F64 = (PREC == TT_FP64), F32 = (PREC == TT_FP32);
  constexpr int tile_bytes = F64 ? 8 * (BK * (BM + 1) + BK * (BN + 1))
                             : F32 ? 4 * (BK * (BM + 1) + BK * (BN + 1))
                                   : 2 * NP * (BM + BN) * (BK + kBfPad);
  constexpr int EA = (BM * BK + 255) / 256, EB = (BN * BK + 255) / 256;
  // LDS carve-up
  double(*dA)[BM + 1] = reinterpret_cast<double(*)[BM + 1]>(smem);
  double(*dB)[BN + 1] = reinterpret_cast<double(*)[BN + 1]>(smem + 8 * BK * (BM + 1));
  float(*fA)[BM + 1] = reinterpret_cast<float(*)[BM + 1]>(smem);
  float(*fB)[BN + 1] = reinterpret_cast<float(*)[BN + 1]>(smem + 4 * BK * (BM + 1));
  __bf16* bA = reinterpret_cast<__bf16*>(smem);                          // [NP][BM][BK+pad]
  __bf16* bB = bA + NP * BM * (BK + kBfPad);                              // [NP][BN][BK+pad]
  long long* rA = reinterpret_cast<long long*>(smem + tile_bytes);
  long long* rC = rA + BM;
  long long* cB = rC + BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tm = T.tm, tn = T.tn;
  const int m0 = tm * BM, n0 = tn * BN;
  const double* __restrict__ A = slots.p[P.ia] + P.offA;
  const double* __restrict__ B = slots.p[P.ib] + P.offB;
  double* C = slots.p[P.ic] + P.offC;
  const __bf16* __restrict__ Ap = reinterpret_cast<const __bf16*>(slots.p[P.ia]) + P.offA;
  const __bf16* __restrict__ Bp = reinterpret_cast<const __bf16*>(slots.p[P.ib]) + P.offB;
  __bf16* Cp = reinterpret_cast<__bf16*>(slots.p[P.ic]) + P.offC;
  for (int i = tid; i < BM; i += 256) {
    int m = m0 + i;
    rA[i] = m < P.M ? idx_map(tabs, P.tam, P.sam, m) : 0;
    rC[i] = m < P.M ? idx_map(tabs, P.tcm, P.scm, m) : 0;
  }
  for (int j = tid; j < BN; j += 256) {
    int n = n0 + j;
    cB[j] = n < P.N ? idx_map(tabs, P.tbn, P.sbn, n) : 0;
  }
  const bool a_kfast = (P.tak < 0 && P.sak == 1);
  const bool b_nfast = (P.tbn < 0 && P.sbn == 1);
  const int wm = SPLITK ? 0 : (wave / WGN) * WM, wn = SPLITK ? 0 : (wave % WGN) * WN;
  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  int kbeg = 0, kstop = P.K;
  if (T.nk > 1) {
    const int per = ((P.K + T.nk - 1) / T.nk + BK - 1) / BK * BK;
    kbeg = T.ks * per;
    kstop = kbeg + per < P.K ? kbeg + per : P.K;
  }
  // element e = tid + 256 q of a tile -> (row/col, k) inside the tile
  auto a_ik = [&](int e, int& i, int& kk) {
    if (a_kfast) { i = e / BK; kk = e % BK; } else { i = e % BM; kk = e / BM; }
  };
  auto b_jk = [&](int e, int& j, int& kk) {
    if (b_nfast) { j = e % BN; kk = e / BN; } else { j = e / BK; kk = e % BK; }
  };
  double ra[PL ? 1 : EA], rb[PL ? 1 : EB];
  __bf16 pa[PL ? EA : 1][NP], pb[PL ? EB : 1][NP];
  __syncthreads();   // row / column offsets ready
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int e = tid + q * 256, i, kk;
      a_ik(e, i, kk);
      const int k = k0 + kk;
      const bool ok = (e < BM * BK) && (m0 + i < P.M) && (k < kstop);
      const long long o = ok ? rA[i] + idx_map(tabs, P.tak, P.sak, k) : 0;
      if constexpr (PL) {
#pragma unroll
        for (int p = 0; p < NP; ++p) pa[q][p] = ok ? Ap[p * pl.s[P.ia] + o] : (__bf16)0.0f;
      } else {
        ra[q] = ok ? A[o] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int e = tid + q * 256, j, kk;
      b_jk(e, j, kk);
      const int k = k0 + kk;
      const bool ok = (e < BN * BK) && (n0 + j < P.N) && (k < kstop);
      const long long o = ok ? idx_map(tabs, P.tbk, P.sbk, k) + cB[j] : 0;
      if constexpr (PL) {
#pragma unroll
        for (int p = 0; p < NP; ++p) pb[q][p] = ok ? Bp[p * pl.s[P.ib] + o] : (__bf16)0.0f;
      } else {
        rb[q] = ok ? B[o] : 0.0;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int e = tid + q * 256, i, kk;
      if (e >= BM * BK) break;
      a_ik(e, i, kk);
      if constexpr (PL) {
#pragma unroll
        for (int p = 0; p < NP; ++p) bA[(p * BM + i) * (BK + kBfPad) + kk] = pa[q][p];
      } else if (F64) dA[kk][i] = ra[q];
      else if (F32) fA[kk][i] = (float)ra[q];
      else {
        __bf16 parts[3];
        bf16_split<NP>(ra[q], parts);
#pragma unroll
        for (int p = 0; p < NP; ++p) bA[(p * BM + i) * (BK + kBfPad) + kk] = parts[p];
      }
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int e = tid + q * 256, j, kk;
      if (e >= BN * BK) break;
      b_jk(e, j, kk);
      if constexpr (PL) {
#pragma unroll
        for (int p = 0; p < NP; ++p) bB[(p * BN + j) * (BK + kBfPad) + kk] = pb[q][p];
      } else if (F64) dB[kk][j] = rb[q];
      else if (F32) fB[kk][j] = (float)rb[q];
      else {
        __bf16 parts[3];
        bf16_split<NP>(rb[q], parts);
#pragma unroll
        for (int p = 0; p < NP; ++p) bB[(p * BN + j) * (BK + kBfPad) + kk] = parts[p];
      }
    }
  };
  if (kbeg < kstop) fetch(kbeg);
  for (int k0 = kbeg; k0 < kstop; k0 += BK) {
    __syncthreads();   // the previous K tile is consumed
    stash();
    __syncthreads();
    if (k0 + BK < kstop) fetch(k0 + BK);
    const int kend = (kstop - k0 < BK) ? kstop - k0 : BK;
    if (F64) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        if (kk >= kend) break;
        if (SPLITK && (kk >> 2) != wave) continue;
        const int kr = kk + (lane >> 4), c = lane & 15;
        double a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = dA[kr][wm + i * 16 + c];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = dB[kr][wn + j * 16 + c];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else if (F32) {
      float4_t a32[FM][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) a32[i][j] = (float4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        if (kk >= kend) break;
        if (SPLITK && (kk >> 2) != wave) continue;
        const int kr = kk + (lane >> 4), c = lane & 15;
        float a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = fA[kr][wm + i * 16 + c];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = fB[kr][wn + j * 16 + c];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], a32[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)a32[i][j][v];
    } else {
      // one 32-deep MFMA step per K tile; lane (r, g) reads k = 8g..8g+7 of row r
      const int r = lane & 15, g = lane >> 4;
      bf16x8_t a[NP][FM], b[NP][FN];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
          a[p][i] = *reinterpret_cast<const bf16x8_t*>(bA + (p * BM + wm + i * 16 + r) * (BK + kBfPad) + 8 * g);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          b[p][j] = *reinterpret_cast<const bf16x8_t*>(bB + (p * BN + wn + j * 16 + r) * (BK + kBfPad) + 8 * g);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          float4_t t = (float4_t){0.f, 0.f, 0.f, 0.f};
          if (NP == 3) {
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2 % NP][i], b[0][j], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2 % NP][j], t, 0, 0, 0);
          }
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], t, 0, 0, 0);
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], t, 0, 0, 0);
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], t, 0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)t[v];
        }
    }
  }
  // row of accumulator element v inside a 16x16 block (measured on gfx950):
  // f64 MFMA: lane/16 + 4v; f32-accumulating MFMA: 4*(lane/16) + v
  auto brow = [&](int v) { return F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v; };
  auto store = [&](int row, int col, double v) {
    const int m = m0 + row, n = n0 + col;
    if (m < P.M && n < P.N) {
      if (PL && pl.c) {   // the result as BF16 planes (beta = 0 only)
        __bf16 parts[3];
        bf16_split<NP>(P.alpha * v, parts);
#pragma unroll
        for (int p = 0; p < NP; ++p) Cp[p * pl.s[P.ic] + rC[row] + n] = parts[p];
        return;
      }
      double* cp = C + rC[row] + n;
      double val = P.alpha * v;
      if (P.beta != 0.0) val += P.beta * (*cp);
      *cp = val;
    }
  };
  if (SPLITK) {
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem + tile_bytes + 8 * (2 * BM + BN + 2 * BK));
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row = i * 16 + brow(v), col = j * 16 + (lane & 15);
          red[(wave * BM + row) * BN + col] = acc[i][j][v];
        }
    __syncthreads();
    for (int e = tid; e < BM * BN; e += 256) {
      double v = red[e] + red[BM * BN + e] + red[2 * BM * BN + e] + red[3 * BM * BN + e];
      if (T.nk > 1) pws[T.pw + (long long)T.ks * BM * BN + e] = v;
      else store(e / BN, e % BN, v);
    }
  } else {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row = wm + i * 16 + brow(v);
          int col = wn + j * 16 + (lane & 15);
          if (T.nk > 1) pws[T.pw + (long long)T.ks * BM * BN + row * BN + col] = acc[i][j][v];
          else store(row, col, acc[i][j][v]);
        }
  }
}

// C = alpha * (sum of the K-slice partials in slice order) + beta * C
__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmProb* __restrict__ probs,
                                                     const GemmSplit* __restrict__ splits,
                                                     const long long* __restrict__ tabs, BSlots bs,
                                                     BPtr<double> b_pws) {
  __shared__ long long rC[256];
  const Slots& slots = bs.s[blockIdx.y];
  const double* __restrict__ pws = b_pws.p[blockIdx.y];
  const GemmSplit S = splits[blockIdx.x];
  const GemmProb P = probs[S.prob];
  const int BM = kGemmBM[S.cfg], BN = kGemmBN[S.cfg];
  double* C = slots.p[P.ic] + P.offC;
  const int m0 = S.tm * BM, n0 = S.tn * BN;
  for (int i = threadIdx.x; i < BM; i += blockDim.x) rC[i] = (m0 + i < P.M) ? idx_map(tabs, P.tcm, P.scm, m0 + i) : 0;
  __syncthreads();
  for (int e = threadIdx.x; e < BM * BN; e += blockDim.x) {
    int row = e / BN, col = e % BN;
    int m = m0 + row, n = n0 + col;
    if (m >= P.M || n >= P.N) continue;
    double v = 0.0;
    for (int ks = 0; ks < S.nk; ++ks) v += pws[S.pw + (long long)ks * BM * BN + e];
    double* cp = C + rC[row] + n;
    double val = P.alpha * v;
    if (P.beta != 0.0) val += P.beta * (*cp);
    *cp = val;
  }
}

// ------------------------------------------------------------------ wave GEMM
// Workgroup b of n: consecutive workgroups go round-robin to the eight XCDs, so
// hand each XCD a contiguous range of work items (neighbouring blocks of one
// problem then share that XCD's L2).  A bijection of [0, n).
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, slot = b >> 3;
  return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// k addressing of a wave GEMM problem: index tables or general strides; A
// contiguous in k (B strided); both contiguous in k
constexpr int kKGeneric = 0, kKAContig = 1, kKBothContig = 2;

// Element i of a wave-uniform base.  The byte offset is formed in 32 bits (the
// plans keep element offsets below 2^29), so the load takes the scalar-base
// form with a single 32-bit vector offset.
template <typename T>
__device__ __forceinline__ double ld32(const T* __restrict__ base, unsigned i) {
  return (double)*reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (i * (unsigned)sizeof(T)));
}
// Elements i and i + 1 of a wave-uniform base in one load (8-byte alignment
// suffices: the device runs in unaligned-access mode).
template <typename T>
__device__ __forceinline__ void ld32x2(const T* __restrict__ base, unsigned i, double& x0, double& x1) {
  typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  const v2 v = *reinterpret_cast<const v2*>(reinterpret_cast<const char*>(base) + (i * (unsigned)sizeof(T)));
  x0 = (double)v.x;
  x1 = (double)v.y;
}

// One wave's (16 FM) x (16 FN) output block from global memory, f64 MFMA
// 16x16x4 (in every precision mode: these blocks are bound by memory and
// issue, so FP32 mode only keeps its float intermediates).  In a 16-deep chunk, lane (r, g) = (lane % 16, lane / 16) supplies
// row r / column r at k = 4s + g on MFMA step s = 0..3 (the four lane groups
// read four consecutive k).  The job takes chunks part, part + nparts, ...
// With nparts = 4 the four waves of the workgroup hold the four
// K parts of one block and wave 0 adds them in part order.
// TA / TB are the element types of the two operands (float where the plan
// keeps that operand in single precision).  Loads are unconditional: rows,
// columns and k past the ends are clamped to the last valid index (an
// element of the same problem), so a half chunk issues all of its loads
// before its first wait.
// Multiply of one 16-deep chunk in split BF16: each lane holds four k values
// of its A row and B column (the same four k for both, so their order inside
// the chunk does not matter); every value is split into 2 (bf16x3) or 3
// (bf16x6) BF16 parts (x ~ p0 + p1 (+ p2), each rounded to nearest) and the 3 /
// 6 leading part products are taken with the 16x16x16 BF16 MFMA, smallest
// first.  The chunk's FP32 result is added into the FP64 accumulators, so
// precision is lost only inside one chunk.
template <int MM>
__device__ __forceinline__ float4_t chunk_mul(const double (&a)[4], const double (&b)[4]) {
  float4_t t = (float4_t){0.f, 0.f, 0.f, 0.f};
  {
    constexpr int NP = MM == TT_BF16X3 ? 2 : 3;
    short4_t pa[NP], pb[NP];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __bf16 xa[3], xb[3];
      bf16_split<NP>(a[q], xa);
      bf16_split<NP>(b[q], xb);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        pa[p][q] = __builtin_bit_cast(short, xa[p]);
        pb[p][q] = __builtin_bit_cast(short, xb[p]);
      }
    }
    if constexpr (NP == 3) {
      t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[2], pb[0], t, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[1], pb[1], t, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[0], pb[2], t, 0, 0, 0);
    }
    t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[1], pb[0], t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[0], pb[1], t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[0], pb[0], t, 0, 0, 0);
  }
  return t;
}

template <int FM, int FN, typename TA, typename TB, int KM, int MM>
__device__ __forceinline__ void wave_tile(const GemmProb& P, const GemmJob& J, const long long* __restrict__ tabs,
                                          const Slots& slots, double* red) {
  constexpr bool F64 = MM == TT_FP64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  // operand bases are wave-uniform (scalar registers); element offsets from
  // them fit 32 bits (checked when the plan is built).  Operands flagged in
  // P.dt are float arrays (offsets count floats).
  const bool fc = P.dt & kDtC;
  const TA* __restrict__ A = reinterpret_cast<const TA*>(slots.p[P.ia]) + P.offA;
  const TB* __restrict__ B = reinterpret_cast<const TB*>(slots.p[P.ib]) + P.offB;
  double* C = slots.p[P.ic] + P.offC;
  float* Cf = reinterpret_cast<float*>(slots.p[P.ic]) + P.offC;
  const int m0 = J.tm * 16 * FM, n0 = J.tn * 16 * FN;
  unsigned ra[FM], cb[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) ra[i] = (unsigned)idx_map(tabs, P.tam, P.sam, min(m0 + 16 * i + r16, P.M - 1));
#pragma unroll
  for (int j = 0; j < FN; ++j) cb[j] = (unsigned)idx_map(tabs, P.tbn, P.sbn, min(n0 + 16 * j + r16, P.N - 1));
  // row / column offsets with this lane group's first k of a full chunk
  // (4g for contiguous operands, g * 4 * stride for a strided B)
  unsigned rg[FM], cg[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) rg[i] = ra[i] + 4u * g;
#pragma unroll
  for (int j = 0; j < FN; ++j) cg[j] = cb[j] + (KM == kKBothContig ? 4u * g : 4u * g * (unsigned)P.sbk);
  const int nch = (P.K + 15) >> 4;
  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
  // no register double buffering, and a chunk is loaded in two halves of two
  // MFMA steps: few live registers, and the occupancy that buys hides the
  // load latency better on these short loops.  Steps past the end of K are
  // skipped (most blocks of a sweep have K below 16).
  const int nfull = P.K >> 4;
  for (int c = J.part; c < nfull; c += J.nparts) {
    // full chunk: every k is valid and clamped rows / columns only feed
    // outputs that are never stored, so the loads need no mask
    double a4[F64 ? 1 : FM][4], b4[F64 ? 1 : FN][4];   // the whole chunk (lower precisions)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double a[FM][2], b[FN][2];
      if (KM == kKGeneric) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int k = c * 16 + 4 * (2 * h + q) + g;
          const unsigned ka = (unsigned)idx_map(tabs, P.tak, P.sak, k);
          const unsigned kb = (unsigned)idx_map(tabs, P.tbk, P.sbk, k);
#pragma unroll
          for (int i = 0; i < FM; ++i) a[i][q] = ld32(A, ra[i] + ka);
#pragma unroll
          for (int j = 0; j < FN; ++j) b[j][q] = ld32(B, kb + cb[j]);
        }
      } else {
        // k-contiguous operands: lane group g takes k = 16c + 4g + s on
        // step s, so steps 2h and 2h + 1 are one two-element load per row
        // (the four lane groups together read each row's whole chunk)
        const int k0 = c * 16 + 2 * h;   // wave-uniform part of the k of step 2h
        const TA* As = A + k0;
#pragma unroll
        for (int i = 0; i < FM; ++i) ld32x2(As, rg[i], a[i][0], a[i][1]);
        if (KM == kKBothContig) {
          const TB* Bs = B + k0;
#pragma unroll
          for (int j = 0; j < FN; ++j) ld32x2(Bs, cg[j], b[j][0], b[j][1]);
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const TB* Bs = B + (long long)(k0 + q) * P.sbk;
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j][q] = ld32(Bs, cg[j]);
          }
        }
      }
      if constexpr (F64) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int i = 0; i < FM; ++i) a4[i][2 * h + q] = a[i][q];
#pragma unroll
          for (int j = 0; j < FN; ++j) b4[j][2 * h + q] = b[j][q];
        }
      }
    }
    if constexpr (!F64) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const float4_t t = chunk_mul<MM>(a4[i], b4[j]);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)t[v];
        }
    }
  }
  if (nfull < nch && nfull % J.nparts == J.part) {
    const int c = nfull;
    // the last, partial chunk: k past the end is clamped to K - 1 and its B
    // value replaced by zero (that alone cancels the product)
    const int ns = (P.K - 16 * c + 3) >> 2;   // steps holding a valid k (wave-uniform)
    double a4[F64 ? 1 : FM][4], b4[F64 ? 1 : FN][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (F64 && 2 * h >= ns) break;
      double a[FM][2], b[FN][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = c * 16 + 4 * (2 * h + q) + g;
        const bool ok = k < P.K;
        const int kc = ok ? k : P.K - 1;
        const unsigned ka = KM == kKGeneric ? (unsigned)idx_map(tabs, P.tak, P.sak, kc) : (unsigned)kc;
        const unsigned kb = KM == kKGeneric ? (unsigned)idx_map(tabs, P.tbk, P.sbk, kc)
                            : KM == kKBothContig ? (unsigned)kc : (unsigned)kc * (unsigned)P.sbk;
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i][q] = ld32(A, ra[i] + ka);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          double v = ld32(B, kb + cb[j]);
          // keeps the load unconditional (a select on a loaded value is
          // otherwise turned into a branch around the load and a wait)
          asm volatile("" : "+v"(v));
          b[j][q] = ok ? v : 0.0;
        }
      }
      if constexpr (F64) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (2 * h + q >= ns) break;
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][q], b[j][q], acc[i][j], 0, 0, 0);
        }
      } else {
        // k past the end carries a zero B value: the whole chunk is multiplied
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int i = 0; i < FM; ++i) a4[i][2 * h + q] = a[i][q];
#pragma unroll
          for (int j = 0; j < FN; ++j) b4[j][2 * h + q] = b[j][q];
        }
      }
    }
    if constexpr (!F64) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const float4_t t = chunk_mul<MM>(a4[i], b4[j]);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)t[v];
        }
    }
  }
  if (J.nparts > 1) {   // uniform over the workgroup: its four jobs are the parts of one block
    if (wave > 0) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[(wave - 1) * 1024 + ((i * FN + j) * 4 + v) * 64 + lane] = acc[i][j][v];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = ((i * FN + j) * 4 + v) * 64 + lane;
          acc[i][j][v] = ((acc[i][j][v] + red[e]) + red[1024 + e]) + red[2048 + e];
        }
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // accumulator row inside a 16x16 block: lane/16 + 4v for the f64 MFMA,
      // 4 (lane/16) + v for the f32-accumulating ones
      const int m = m0 + 16 * i + (F64 ? g + 4 * v : 4 * g + v);
      if (m >= P.M) continue;
      const unsigned rowc = (unsigned)idx_map(tabs, P.tcm, P.scm, m);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = n0 + 16 * j + r16;
        if (n >= P.N) continue;
        double val = P.alpha * acc[i][j][v];
        if (fc) {
          if (P.beta != 0.0) val += P.beta * (double)Cf[rowc + n];
          Cf[rowc + n] = (float)val;
        } else {
          if (P.beta != 0.0) val += P.beta * C[rowc + n];
          C[rowc + n] = val;
        }
      }
    }
}

// operand element types and the k addressing are wave-uniform (one problem
// per wave)
template <int FM, int FN, int KM, int MM>
__device__ __forceinline__ void wave_tile_dt(const GemmProb& P, const GemmJob& J, const long long* __restrict__ tabs,
                                             const Slots& slots, double* red) {
  switch (P.dt & (kDtA | kDtB)) {
    case 0: wave_tile<FM, FN, double, double, KM, MM>(P, J, tabs, slots, red); break;
    case kDtA: wave_tile<FM, FN, float, double, KM, MM>(P, J, tabs, slots, red); break;
    case kDtB: wave_tile<FM, FN, double, float, KM, MM>(P, J, tabs, slots, red); break;
    default: wave_tile<FM, FN, float, float, KM, MM>(P, J, tabs, slots, red); break;
  }
}
template <int FM, int FN, int MM>
__device__ __forceinline__ void wave_tile_k(const GemmProb& P, const GemmJob& J, const long long* __restrict__ tabs,
                                            const Slots& slots, double* red) {
  if (P.tak >= 0 || P.tbk >= 0 || P.sak != 1) wave_tile_dt<FM, FN, kKGeneric, MM>(P, J, tabs, slots, red);
  else if (P.sbk == 1) wave_tile_dt<FM, FN, kKBothContig, MM>(P, J, tabs, slots, red);
  else wave_tile_dt<FM, FN, kKAContig, MM>(P, J, tabs, slots, red);
}

// five waves per SIMD: the register budget (96) that keeps a half chunk's
// loads of the next steps in flight without spilling
// MM: the precision of the multiplies (TT_FP64, TT_BF16X3, TT_BF16X6)
// waves per SIMD the wave GEMM is compiled for (4x16 D=2000 sweep: 0.316 s/step at
// 5 and at 6, 0.325 at 4)
#ifndef TT_WGEMM_WPE
#define TT_WGEMM_WPE 5
#endif
template <int MM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TT_WGEMM_WPE))) void k_wgemm(const GemmProb* __restrict__ probs, const GemmJob* __restrict__ jobs,
                                               int nblocks, const long long* __restrict__ tabs, BSlots bs) {
  __shared__ double red[3 * 1024];
  const Slots& slots = bs.s[blockIdx.y];
  const int blk = xcd_block(blockIdx.x, nblocks);
  // the job index is wave-uniform: job and problem descriptors load into scalar registers
  const int jidx = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  const GemmJob J = jobs[jidx];
  if (J.prob < 0) return;   // an unused slot: only in workgroups of unsplit jobs, which never synchronise
  const GemmProb P = probs[J.prob];
  switch (J.shape) {
    case 0: wave_tile_k<4, 1, MM>(P, J, tabs, slots, red); break;
    case 1: wave_tile_k<2, 2, MM>(P, J, tabs, slots, red); break;
    case 2: wave_tile_k<1, 4, MM>(P, J, tabs, slots, red); break;
    default: wave_tile_k<1, 1, MM>(P, J, tabs, slots, red); break;
  }
}

// ------------------------------------------------------------------ fused apply
// One wave's 16 x (16 FN) tile of a fused-apply output block (FzOut).  For
// each of its b blocks and each 16-wide chunk of that block's y range, the
// chunk of T2^T (rows y, columns x') is summed over the terms t as
// x_t^T LW_t^T with the f64 MFMA 16x16x4, then out += T2 R^T takes that chunk
// as its A operand.  Lane (r, g) = (lane % 16, lane / 16) ends the first
// product holding T2[x' = row0 + r][y = y0 + g + 4 v] in register v, which is
// exactly its A operand of the second product's step v (k = y = y0 + 4 v + g):
// the two products chain in registers.  In the first product lane (r, g)
// supplies the input row y = y0 + r and the LW row x' = row0 + r; a full
// 16-deep chunk of x takes k = 16 c + 4 g + s on step s (one 32-byte run of
// an LW row per lane), the partial last chunk k = 16 c + 4 s + g with LW
// zeroed past dl.  Rows x', y and columns y' past the ends are clamped to the
// last valid index (an element of the same block), so every load is
// unconditional and in bounds; the clamped products reach only outputs that
// are never stored, or meet the R value zeroed past dc.
// The descriptors of the b blocks sit one per lane (lane i: block b0 + i)
// and those of a window of 64 consecutive terms likewise; the loop reads them
// with readlane (no memory access), so the only memory round trips of a b
// block are its operand loads, and the R values of a chunk are loaded before
// the product they enter.
__device__ __forceinline__ long long rl64(int lo, int hi, int i) {
  return (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readlane(hi, i) << 32) |
                     (unsigned long long)(unsigned)__builtin_amdgcn_readlane(lo, i));
}

template <int FN>
__device__ __forceinline__ void fz_tile(const FzOut& O, const FzJob& J, const FzB* __restrict__ bs,
                                        const FzT* __restrict__ ts, const Slots& slots, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const double* __restrict__ LW = slots.p[0];
  const double* __restrict__ X = slots.p[1];
  const double* __restrict__ R = slots.p[2] + O.rrow;
  const unsigned xr = (unsigned)min(J.row0 + r16, O.dp - 1);
  unsigned rr[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) rr[j] = (unsigned)min(J.col0 + 16 * j + r16, O.dr - 1) * (unsigned)O.ldr;
  double4_t acc[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) acc[j] = (double4_t){0.0, 0.0, 0.0, 0.0};
  // b block descriptors, lane i: block b0 + i (nb <= 64, checked by the planner)
  int b_rlo = 0, b_rhi = 0, b_dc = 1, b_t0 = 0, b_nt = 0;
  if (lane < O.nb) {
    const FzB B = bs[O.b0 + lane];
    b_rlo = (int)(unsigned)(B.rcol & 0xffffffffLL);
    b_rhi = (int)(B.rcol >> 32);
    b_dc = B.dc;
    b_t0 = B.t0;
    b_nt = B.nt;
  }
  const int t_end = O.nb > 0 ? __builtin_amdgcn_readlane(b_t0, O.nb - 1) + __builtin_amdgcn_readlane(b_nt, O.nb - 1) : 0;
  // a window of term descriptors, lane i: term tw + i
  int tw = -(1 << 30);
  int t_llo = 0, t_lhi = 0, t_alo = 0, t_ahi = 0, t_ldlw = 1, t_lda = 1, t_dl = 1;
  for (int bi = J.part; bi < O.nb; bi += J.nparts) {
    const long long rcol = rl64(b_rlo, b_rhi, bi);
    const int dc = __builtin_amdgcn_readlane(b_dc, bi);
    const int t0 = __builtin_amdgcn_readlane(b_t0, bi), nt = __builtin_amdgcn_readlane(b_nt, bi);
    if (t0 < tw || t0 + nt > tw + 64) {   // uniform: move the window to start at this block's terms
      tw = t0;
      if (tw + lane < t_end) {
        const FzT T = ts[tw + lane];
        t_llo = (int)(unsigned)(T.lw & 0xffffffffLL);
        t_lhi = (int)(T.lw >> 32);
        t_alo = (int)(unsigned)(T.a & 0xffffffffLL);
        t_ahi = (int)(T.a >> 32);
        t_ldlw = T.ldlw;
        t_lda = T.lda;
        t_dl = T.dl;
      }
    }
    const double* __restrict__ Rb = R + rcol;
    for (int y0 = 0; y0 < dc; y0 += 16) {
      // R values of this chunk: step s of the product with R takes y = y0 + 4 s + g
      // (loaded ahead of the first product for up to two column tiles)
      constexpr int FP = FN <= 2 ? FN : 1;
      const int ns = min(4, (dc - y0 + 3) >> 2);
      auto rval = [&](int j, int s) {
        const int y = y0 + 4 * s + g;
        const bool ok = y < dc;
        double v = ld32(Rb, rr[j] + (unsigned)(ok ? y : dc - 1));
        asm volatile("" : "+v"(v));   // keeps the load unconditional
        return ok ? v : 0.0;
      };
      double rv[FP][4];
      if constexpr (FN <= 2) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (s < ns) rv[j][s] = rval(j, s);
      }
      const unsigned yl = (unsigned)min(y0 + r16, dc - 1);
      double4_t t2 = (double4_t){0.0, 0.0, 0.0, 0.0};
      for (int ti = 0; ti < nt; ++ti) {
        const int li = t0 - tw + ti;
        const long long tlw = rl64(t_llo, t_lhi, li), ta = rl64(t_alo, t_ahi, li);
        const int ldlw = __builtin_amdgcn_readlane(t_ldlw, li), lda = __builtin_amdgcn_readlane(t_lda, li);
        const int dl = __builtin_amdgcn_readlane(t_dl, li);
        const double* __restrict__ Lr = LW + tlw + xr * (unsigned)ldlw;
        const double* __restrict__ Xa = X + ta + yl;
        const int nfull = dl >> 4;
#pragma unroll 2
        for (int c = 0; c < nfull; ++c) {
          const unsigned k0 = 16u * c + 4u * g;
          double lv[4], av[4];
          ld32x2(Lr, k0, lv[0], lv[1]);
          ld32x2(Lr, k0 + 2u, lv[2], lv[3]);
#pragma unroll
          for (int s = 0; s < 4; ++s) av[s] = ld32(Xa, (k0 + s) * (unsigned)lda);
#pragma unroll
          for (int s = 0; s < 4; ++s) t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], lv[s], t2, 0, 0, 0);
        }
        if (16 * nfull < dl) {
          const int c = nfull;
          const int nk = (dl - 16 * c + 3) >> 2;   // steps holding a valid k (wave-uniform)
          double lv[4], av[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (s < nk) {
              const int k = 16 * c + 4 * s + g;
              const bool ok = k < dl;
              const unsigned kc = (unsigned)(ok ? k : dl - 1);
              double v = ld32(Lr, kc);
              asm volatile("" : "+v"(v));
              lv[s] = ok ? v : 0.0;
              av[s] = ld32(Xa, kc * (unsigned)lda);
            }
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (s < nk) t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], lv[s], t2, 0, 0, 0);
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < ns)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            double r;
            if constexpr (FN <= 2) r = rv[j][s];
            else r = rval(j, s);
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(t2[s], r, acc[j], 0, 0, 0);
          }
    }
  }
  if (J.nparts > 1) {   // uniform over the workgroup: its four jobs are the parts of one tile
    if (wave > 0) {
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave - 1) * 1024 + (j * 4 + v) * 64 + lane] = acc[j][v];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = (j * 4 + v) * 64 + lane;
        acc[j][v] = ((acc[j][v] + red[e]) + red[1024 + e]) + red[2048 + e];
      }
  }
  double* __restrict__ out = slots.p[3] + O.out;
  const int ncol = min(O.dr, J.col0 + kFzCols);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = J.row0 + g + 4 * v;
    if (m >= O.dp) continue;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = J.col0 + 16 * j + r16;
      if (n < ncol) out[(long long)m * O.ldo + n] = acc[j][v];
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_fused_apply(const FzOut* __restrict__ outs, const FzB* __restrict__ bs,
                                                     const FzT* __restrict__ ts, const FzJob* __restrict__ jobs,
                                                     int nblocks, BSlots bsl) {
  __shared__ double red[3 * 1024];
  const Slots& slots = bsl.s[blockIdx.y];
  const int blk = xcd_block(blockIdx.x, nblocks);
  const int jidx = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  const FzJob J = jobs[jidx];
  if (J.o < 0) return;   // an unused slot: only in workgroups of unsplit jobs, which never synchronise
  const FzOut O = outs[J.o];
  switch ((min(O.dr - J.col0, kFzCols) + 15) >> 4) {
    case 1: fz_tile<1>(O, J, bs, ts, slots, red); break;
    case 2: fz_tile<2>(O, J, bs, ts, slots, red); break;
    case 3: fz_tile<3>(O, J, bs, ts, slots, red); break;
    default: fz_tile<4>(O, J, bs, ts, slots, red); break;
  }
}

void launch_fused(const FzPlan& p, const BSlots& s, int nb, hipStream_t st) {
  if (p.nblocks == 0) return;
  TT_REQUIRE(nb >= 1 && nb <= kMaxBatch, TT_EINVAL, "batch size out of range");
  prof_begin(st);
  hipLaunchKernelGGL(k_fused_apply, dim3(p.nblocks, nb), dim3(256), 0, st, p.d_outs, p.d_bs, p.d_terms, p.d_jobs,
                     p.nblocks, s);
  HIP_CHECK_LAUNCH();
  prof_end(st, PROF_FUSED, nb * p.flops, nb * p.bytes);
}

// tile shapes: 0 64x64, 1 128x32, 2 256x16, 3 32x128, 4 32x32 (split K over the
// waves; with BF16 the four waves take one 16x16 block each instead)
template <int CFG, int PREC> struct CfgT;
template <int PREC> struct CfgT<0, PREC> { static constexpr int WGM = 2, WGN = 2, FM = 2, FN = 2; static constexpr bool SK = false; };
template <int PREC> struct CfgT<1, PREC> { static constexpr int WGM = 4, WGN = 1, FM = 2, FN = 2; static constexpr bool SK = false; };
template <int PREC> struct CfgT<2, PREC> { static constexpr int WGM = 4, WGN = 1, FM = 4, FN = 1; static constexpr bool SK = false; };
template <int PREC> struct CfgT<3, PREC> { static constexpr int WGM = 1, WGN = 4, FM = 2, FN = 2; static constexpr bool SK = false; };
template <int PREC> struct CfgT<4, PREC> {
  static constexpr bool BFP = PREC >= TT_BF16X3;
  static constexpr int WGM = BFP ? 2 : 1, WGN = BFP ? 2 : 1, FM = BFP ? 1 : 2, FN = BFP ? 1 : 2;
  static constexpr bool SK = !BFP;
};

template <int CFG, int PREC>
__global__ __launch_bounds__(256) void k_gemm(const GemmProb* __restrict__ probs, const GemmTile* __restrict__ tiles,
                                              int tile0, const long long* __restrict__ tabs, BSlots bs,
                                              BPtr<double> b_pws) {
  extern __shared__ __attribute__((aligned(16))) char smem_gemm[];
  const Slots& slots = bs.s[blockIdx.y];
  double* __restrict__ pws = b_pws.p[blockIdx.y];
  using C = CfgT<CFG, PREC>;
  const GemmTile t = tiles[tile0 + blockIdx.x];
  const GemmProb P = probs[t.prob];
  gemm_tile<C::WGM, C::WGN, C::FM, C::FN, C::SK, PREC>(P, t, tabs, slots, smem_gemm, pws);
}


template <int CFG, int PREC>
int cfg_smem() {
  using C = CfgT<CFG, PREC>;
  return gemm_smem_bytes_t<C::WGM, C::WGN, C::FM, C::FN, C::SK, PREC>();
}

int gemm_smem_bytes(int cfg) {   // FP64 tiles (the largest LDS of the precisions)
  switch (cfg) {
    case 0: return cfg_smem<0, TT_FP64>();
    case 1: return cfg_smem<1, TT_FP64>();
    case 2: return cfg_smem<2, TT_FP64>();
    case 3: return cfg_smem<3, TT_FP64>();
    default: return cfg_smem<4, TT_FP64>();
  }
}

template <int CFG, int PREC>
void launch_cfg(const GemmPlan& p, const long long* d_tabs, const BSlots& s, int nb, BPtr<double> pws,
                hipStream_t st) {
  const int n = p.cfg_off[CFG + 1] - p.cfg_off[CFG];
  if (n == 0) return;
  static bool attr = false;
  const int smem = cfg_smem<CFG, PREC>();
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_gemm<CFG, PREC>, hipFuncAttributeMaxDynamicSharedMemorySize, smem) !=
        hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the GEMM kernel");
    attr = true;
  }
  hipLaunchKernelGGL((k_gemm<CFG, PREC>), dim3(n, nb), dim3(256), smem, st, p.d_probs, p.d_tiles, p.cfg_off[CFG], d_tabs,
                     s, pws);
  HIP_CHECK_LAUNCH();
  prof_mark(st, PROF_GEMM_CFG0 + CFG, nb * p.cfg_flops[CFG], nb * p.cfg_bytes[CFG]);
}

template <int PREC>
void launch_prec(const GemmPlan& p, const long long* d_tabs, const BSlots& s, int nb, BPtr<double> pws, hipStream_t st) {
  launch_cfg<0, PREC>(p, d_tabs, s, nb, pws, st);
  launch_cfg<1, PREC>(p, d_tabs, s, nb, pws, st);
  launch_cfg<2, PREC>(p, d_tabs, s, nb, pws, st);
  launch_cfg<3, PREC>(p, d_tabs, s, nb, pws, st);
  launch_cfg<4, PREC>(p, d_tabs, s, nb, pws, st);
}

// the same tiles on pre-split BF16 operands (no K slices: the plan has none)
template <int CFG, int PREC>
__global__ __launch_bounds__(256) void k_gemm_planes(const GemmProb* __restrict__ probs,
                                                     const GemmTile* __restrict__ tiles, int tile0,
                                                     const long long* __restrict__ tabs, Slots slots, Planes pl) {
  extern __shared__ __attribute__((aligned(16))) char smem_gemm[];
  using C = CfgT<CFG, PREC>;
  const GemmTile t = tiles[tile0 + blockIdx.x];
  const GemmProb P = probs[t.prob];
  gemm_tile<C::WGM, C::WGN, C::FM, C::FN, C::SK, PREC, true>(P, t, tabs, slots, smem_gemm, nullptr, pl);
}

template <int CFG, int PREC>
void launch_cfg_planes(const GemmPlan& p, const long long* d_tabs, const Slots& s, const Planes& pl, hipStream_t st) {
  const int n = p.cfg_off[CFG + 1] - p.cfg_off[CFG];
  if (n == 0) return;
  static bool attr = false;
  const int smem = cfg_smem<CFG, PREC>();
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_gemm_planes<CFG, PREC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            smem) != hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the GEMM kernel");
    attr = true;
  }
  hipLaunchKernelGGL((k_gemm_planes<CFG, PREC>), dim3(n), dim3(256), smem, st, p.d_probs, p.d_tiles, p.cfg_off[CFG],
                     d_tabs, s, pl);
  HIP_CHECK_LAUNCH();
}

template <int PREC>
void launch_prec_planes(const GemmPlan& p, const long long* d_tabs, const Slots& s, const Planes& pl, hipStream_t st) {
  launch_cfg_planes<0, PREC>(p, d_tabs, s, pl, st);
  launch_cfg_planes<1, PREC>(p, d_tabs, s, pl, st);
  launch_cfg_planes<2, PREC>(p, d_tabs, s, pl, st);
  launch_cfg_planes<3, PREC>(p, d_tabs, s, pl, st);
  launch_cfg_planes<4, PREC>(p, d_tabs, s, pl, st);
}

void launch_gemm_planes(const GemmPlan& p, const long long* d_tabs, const Slots& s, const Planes& pl, int precision,
                        hipStream_t st) {
  if (p.ntiles == 0) return;
  TT_REQUIRE(p.wave_blocks == 0 && p.splits.empty(), TT_EINVAL, "planes: the plan must have LDS tiles only, unsplit");
  prof_begin(st);
  if (precision == TT_BF16X3) launch_prec_planes<TT_BF16X3>(p, d_tabs, s, pl, st);
  else if (precision == TT_BF16X6) launch_prec_planes<TT_BF16X6>(p, d_tabs, s, pl, st);
  else throw Error(TT_EINVAL, "planes: split-BF16 precisions only");
  prof_end(st, p.tag, p.flops, p.bytes);
}

// out[p * pstride + i] = part p of x[i] (x ~ part 0 + part 1 (+ part 2), each
// rounded to nearest BF16)
template <int NP>
__global__ void k_split(const double* __restrict__ x, long long n, __bf16* __restrict__ out, long long pstride) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    __bf16 parts[3];
    bf16_split<NP>(x[i], parts);
#pragma unroll
    for (int p = 0; p < NP; ++p) out[p * pstride + i] = parts[p];
  }
}

void launch_split(const double* x, long long n, void* out, long long pstride, int precision, hipStream_t st) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  if (precision == TT_BF16X3)
    hipLaunchKernelGGL(k_split<2>, dim3((unsigned)blocks), dim3(256), 0, st, x, n, (__bf16*)out, pstride);
  else if (precision == TT_BF16X6)
    hipLaunchKernelGGL(k_split<3>, dim3((unsigned)blocks), dim3(256), 0, st, x, n, (__bf16*)out, pstride);
  else
    throw Error(TT_EINVAL, "split: split-BF16 precisions only");
  HIP_CHECK_LAUNCH();
}

void launch_gemm(const GemmPlan& p, const long long* d_tabs, const BSlots& s, int nb, int precision,
                 BPtr<double> pws, hipStream_t st) {
  if (p.ntiles == 0 && p.wave_blocks == 0) return;
  TT_REQUIRE(nb >= 1 && nb <= kMaxBatch, TT_EINVAL, "batch size out of range");
  prof_begin(st);
  if (p.wave_blocks > 0) {
    // the finer job list when the launch would otherwise hold few waves
    const bool fine = p.wave_blocks_fine > 0 && 4LL * p.wave_blocks * nb < kWaveMinJobs;
    const int nblk = fine ? p.wave_blocks_fine : p.wave_blocks;
    const GemmJob* jobs = fine ? p.d_jobs_fine : p.d_jobs;
    const dim3 grid(nblk, nb), block(256);
    switch (precision) {
      // FP32 mode: the wave GEMM's blocks are bound by memory and latency, so
      // it multiplies in FP64 and the mode's saving is the float storage of the
      // intermediates (P.dt).  Measured on the 4x16 D=2000 sweep, FP32 MFMA here
      // was no faster (0.278 vs 0.271 s/step) and its error after four sweeps
      // was 1.3e-6 in E against 2e-10 with FP64 multiplies.
      case TT_FP64:
      case TT_FP32: hipLaunchKernelGGL(k_wgemm<TT_FP64>, grid, block, 0, st, p.d_probs, jobs, nblk, d_tabs, s); break;
      case TT_BF16X3: hipLaunchKernelGGL(k_wgemm<TT_BF16X3>, grid, block, 0, st, p.d_probs, jobs, nblk, d_tabs, s); break;
      case TT_BF16X6: hipLaunchKernelGGL(k_wgemm<TT_BF16X6>, grid, block, 0, st, p.d_probs, jobs, nblk, d_tabs, s); break;
      default: throw Error(TT_EINVAL, "unknown precision");
    }
    HIP_CHECK_LAUNCH();
    prof_mark(st, PROF_GEMM_WAVE, nb * p.wave_flops, nb * p.wave_bytes);
  }
  switch (precision) {
    case TT_FP64: launch_prec<TT_FP64>(p, d_tabs, s, nb, pws, st); break;
    case TT_FP32: launch_prec<TT_FP32>(p, d_tabs, s, nb, pws, st); break;
    case TT_BF16X3: launch_prec<TT_BF16X3>(p, d_tabs, s, nb, pws, st); break;
    case TT_BF16X6: launch_prec<TT_BF16X6>(p, d_tabs, s, nb, pws, st); break;
    default: throw Error(TT_EINVAL, "unknown precision");
  }
  if (!p.splits.empty()) {
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)p.splits.size(), nb), dim3(256), 0, st, p.d_probs, p.d_splits,
                       d_tabs, s, pws);
    HIP_CHECK_LAUNCH();
    prof_mark(st, PROF_GEMM_REDUCE, 0.0, nb * p.red_bytes);
  }
  prof_end(st, p.tag, nb * p.flops, nb * p.bytes);
}

// ------------------------------------------------------------------ W stage
// One workgroup of TT_WSTAGE_THREADS threads per task; lanes run over the
// task's elements, each summing its terms in order.  The task index is
// uniform (descriptors in scalar registers).  A thread takes up to four
// elements at a time (indices past the end clamped to the last element, the
// result not stored) so that their loads are in flight together.  Offsets
// inside a block are 32-bit unless the plan has a block spanning 2^29
// elements or more (OFF = long long).
#ifndef TT_WSTAGE_THREADS
#define TT_WSTAGE_THREADS 256
#endif
template <typename TV, typename OFF>
__device__ __forceinline__ void wstage_task(const WTask& t, const WTerm* __restrict__ terms,
                                            const TV* __restrict__ in, TV* __restrict__ out) {
  constexpr int U = 4, T = TT_WSTAGE_THREADS;
  const int nj = t.nj, n = t.ni * nj;
  const OFF dsi = (OFF)t.dsi, dsj = (OFF)t.dsj;
  TV* __restrict__ dst = out + t.dst;
  for (int e0 = threadIdx.x; e0 < n; e0 += U * T) {
    int ii[U], jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * T, n - 1);
      ii[u] = e / nj;
      jj[u] = e - ii[u] * nj;
    }
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (int q = 0; q < t.nt; ++q) {
      const WTerm w = terms[t.t0 + q];
      const TV* __restrict__ src = in + w.src;
      const OFF ssi = (OFF)w.ssi, ssj = (OFF)w.ssj;
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const OFF o = (OFF)ii[u] * ssi + (OFF)jj[u] * ssj;
        if constexpr (sizeof(OFF) == 4) v[u] = ld32(src, (unsigned)o);
        else v[u] = (double)src[o];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc[u] += w.w * v[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * T < n) {
        const OFF o = (OFF)ii[u] * dsi + (OFF)jj[u] * dsj;
        if constexpr (sizeof(OFF) == 4) dst[(unsigned)o] = (TV)acc[u];
        else dst[o] = (TV)acc[u];
      }
  }
}

// TV: the stored type of the input and output intermediates (float in FP32 mode)
template <typename TV, typename OFF>
__global__ __launch_bounds__(TT_WSTAGE_THREADS) void k_wstage(const WTask* __restrict__ tasks,
                                                              BPtr<const WTerm> b_terms, BPtr<const double> b_in,
                                                              BPtr<double> b_out) {
  const int ib = blockIdx.y;
  wstage_task<TV, OFF>(tasks[blockIdx.x], b_terms.p[ib], reinterpret_cast<const TV*>(b_in.p[ib]),
                       reinterpret_cast<TV*>(b_out.p[ib]));
}

void launch_wstage(const WPlan& p, BPtr<const WTerm> terms, BPtr<const double> in, BPtr<double> out, int nb,
                   hipStream_t st) {
  if (p.ntasks == 0) return;
  prof_begin(st);
  const dim3 grid(p.ntasks, nb), block(TT_WSTAGE_THREADS);
  if (p.f32) {
    if (p.wide) hipLaunchKernelGGL((k_wstage<float, long long>), grid, block, 0, st, p.d_tasks, terms, in, out);
    else hipLaunchKernelGGL((k_wstage<float, int>), grid, block, 0, st, p.d_tasks, terms, in, out);
  } else {
    if (p.wide) hipLaunchKernelGGL((k_wstage<double, long long>), grid, block, 0, st, p.d_tasks, terms, in, out);
    else hipLaunchKernelGGL((k_wstage<double, int>), grid, block, 0, st, p.d_tasks, terms, in, out);
  }
  HIP_CHECK_LAUNCH();
  prof_end(st, PROF_WSTAGE, nb * p.flops, nb * p.bytes * (p.f32 ? 0.5 : 1.0));
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block-wide sum with a fixed order; result valid in every thread
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ QR
// Householder QR of a block wider than the register kernels take, in global
// memory, blocked in panels of kQrPanel columns (compact WY form, I - V T V^T
// for the product of a panel's reflectors): the panel's columns are factored
// one by one with the reflectors applied inside the panel (one workgroup per
// block), its T factor is formed from the Gram matrix of V, and every later
// column gets the whole panel's product in two passes (the kQrPanel dot
// products, then the update), instead of one pass per reflector.  Q is formed
// explicitly the same way, panels in reverse order.  Same reflectors as the
// column-by-column algorithm; only the order of the sums differs.  The
// updates of the later columns and of Q spread over the GPU: one launch per
// panel step, one column per workgroup.
// Workspace of a task (ws + T.ws, qr_wide_ws doubles): Wm (m x n column-major:
// R above the diagonal, reflectors below), Qm (m x n), the n taus, then the
// T factor of every panel (kQrPanel x kQrPanel, row-major, zero past the panel).
// The launches take blockIdx.x = wide block, blockIdx.z = state of the batch.
constexpr int kQrPanel = 8;
constexpr int kQrApplyCols = 1;   // columns per workgroup of the panel updates
constexpr int kQrRowU = 4;         // rows per thread whose loads the panel's passes issue together
constexpr int kQrSpread = 64;   // workgroups per block of the copy-in and copy-out launches
long long qr_wide_ws(int m, int n) {
  return 2LL * m * n + n + (long long)((n + kQrPanel - 1) / kQrPanel) * kQrPanel * kQrPanel;
}
__device__ __forceinline__ double* qrw_tfac(double* Wm, int m, int n, int j0) {
  return Wm + 2LL * m * n + n + (long long)(j0 / kQrPanel) * kQrPanel * kQrPanel;
}
__device__ __forceinline__ long long qrw_row(const QRTask& T, const long long* tabs, int i) {
  return T.rtab >= 0 ? tabs[T.rtab + i] : (long long)i * T.rs;
}

// Wm, Qm of every wide block of the launch: Wm the block, Qm = [I; 0]
__global__ __launch_bounds__(256) void k_qrw_load(const QRTask* __restrict__ tasks, const int* __restrict__ wide,
                                                  const long long* __restrict__ tabs, BPtr<const double> b_A,
                                                  BPtr<double> b_ws) {
  const double* A = b_A.p[blockIdx.z];
  const QRTask T = tasks[wide[blockIdx.x]];
  const int m = T.m, n = T.n;
  double* Wm = b_ws.p[blockIdx.z] + T.ws;
  double* Qm = Wm + (long long)m * n;
  for (long long e = (long long)blockIdx.y * blockDim.x + threadIdx.x; e < (long long)m * n;
       e += (long long)gridDim.y * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    Wm[e] = A[T.rbase + qrw_row(T, tabs, i) + (long long)j * T.cs];
    Qm[e] = (i == j) ? 1.0 : 0.0;
  }
}

// the panel at j0 of every wide block with more than j0 columns, one
// workgroup each: its columns factored one by one, then its T factor from tau
// and G = V^T V (T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i])
// stored for the later updates.  Every pass over the rows is shared by the
// whole workgroup (rows strided by the 256 threads, kQrRowU rows per thread
// with their loads issued together): one pass per column step (below), and
// one for G with all its pairs.  Sums: per thread, then per wave, then the
// four waves in order.
__global__ __launch_bounds__(256) void k_qrw_panel(const QRTask* __restrict__ tasks, const int* __restrict__ wide,
                                                   BPtr<double> b_ws, int j0) {
  constexpr int kPairs = kQrPanel * (kQrPanel - 1) / 2;
  const QRTask T = tasks[wide[blockIdx.x]];
  const int m = T.m, n = T.n;
  if (j0 >= n) return;
  const int pb = min(kQrPanel, n - j0), tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Wm = b_ws.p[blockIdx.z] + T.ws;
  double* taus = Wm + 2LL * m * n;
  __shared__ double red[4 * kPairs];
  __shared__ double fsh[kQrPanel], sums[kQrPanel], rowj[kQrPanel];
  __shared__ double Tm[kQrPanel][kQrPanel];
  __shared__ double Gm[kQrPanel][kQrPanel];
  // One pass over the rows per column step.  The pass of step j writes the
  // reflector v_j = scal x_j below the diagonal, applies it to the later
  // columns of the panel, and sums, from the updated values, what step j + 1
  // needs: ||x_{j+1}||^2 below row j + 1 and x_{j+1} . col_c for every later
  // column c (so v . col_c = col_c[j+1] + scal D_c).  acc[0] is the norm
  // partial, acc[1 + q] the dot with column (current + 1 + q).
  double acc[kQrPanel];
#pragma unroll
  for (int q = 0; q < kQrPanel; ++q) acc[q] = 0.0;
  {
    const int nc = pb - 1;
    const double* x0 = Wm + (long long)j0 * m;
    const double* yb = nc > 0 ? x0 + m : x0;   // later columns (none: the column itself, unused)
    for (int i0 = j0 + 1 + tid; i0 < m; i0 += kQrRowU * 256) {
      double x[kQrRowU], y[kQrRowU][kQrPanel - 1];
#pragma unroll
      for (int u = 0; u < kQrRowU; ++u) {
        const int i = min(i0 + 256 * u, m - 1);
        x[u] = x0[i];
#pragma unroll
        for (int q = 0; q < kQrPanel - 1; ++q) y[u][q] = yb[i + (long long)min(q, max(nc - 1, 0)) * m];
      }
#pragma unroll
      for (int u = 0; u < kQrRowU; ++u)
        if (i0 + 256 * u < m) {
          acc[0] += x[u] * x[u];
#pragma unroll
          for (int q = 0; q < kQrPanel - 1; ++q)
            if (q < nc) acc[1 + q] += x[u] * y[u][q];
        }
    }
  }
  for (int j = j0; j < j0 + pb; ++j) {
    const int nc = j0 + pb - j - 1;   // later columns of the panel (uniform)
    // the step's sums: per wave, then the four waves in order
#pragma unroll
    for (int q = 0; q < kQrPanel; ++q) {
      if (q > nc) break;
      const double sq = wave_sum(acc[q]);
      if (lane == 0) red[wave * kQrPanel + q] = sq;
    }
    __syncthreads();
    // the step's sums and the row-j entries they combine with, one thread each,
    // then tau and scal in every thread (the same arithmetic on the same values)
    if (tid <= nc) {
      sums[tid] = ((red[tid] + red[kQrPanel + tid]) + red[2 * kQrPanel + tid]) + red[3 * kQrPanel + tid];
      rowj[tid] = Wm[j + (long long)(j + tid) * m];   // tid 0: alpha; else row j of column j + tid
    }
    __syncthreads();
    const double xn2 = sums[0], alpha = rowj[0];
    double tau = 0.0, scal = 1.0, beta = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      if (xn2 > 0.0) Wm[j + (long long)j * m] = beta;
      taus[j] = tau;
    } else if (tid <= nc) {   // row j of v is 1
      const double f = tau * (rowj[tid] + scal * sums[tid]);
      Wm[j + (long long)(j + tid) * m] = rowj[tid] - f;
      fsh[tid - 1] = f;
    }
    __syncthreads();
    double fq[kQrPanel - 1];
#pragma unroll
    for (int q = 0; q < kQrPanel - 1; ++q) fq[q] = q < nc ? fsh[q] : 0.0;
#pragma unroll
    for (int q = 0; q < kQrPanel; ++q) acc[q] = 0.0;
    double* xj = Wm + (long long)j * m;
    double* c1 = xj + m;
    const double* yb = nc > 0 ? c1 : xj;   // later columns (none: the column itself, unused)
    for (int i0 = j + 1 + tid; i0 < m; i0 += kQrRowU * 256) {
      double x[kQrRowU], y[kQrRowU][kQrPanel - 1];
#pragma unroll
      for (int u = 0; u < kQrRowU; ++u) {
        const int i = min(i0 + 256 * u, m - 1);
        x[u] = xj[i];
#pragma unroll
        for (int q = 0; q < kQrPanel - 1; ++q) y[u][q] = yb[i + (long long)min(q, max(nc - 1, 0)) * m];
      }
#pragma unroll
      for (int u = 0; u < kQrRowU; ++u) {
        const int i = i0 + 256 * u;
        if (i < m) {
          const double v = x[u] * scal;
          xj[i] = v;
#pragma unroll
          for (int q = 0; q < kQrPanel - 1; ++q)
            if (q < nc) {
              y[u][q] -= fq[q] * v;
              c1[i + (long long)q * m] = y[u][q];
            }
          if (i > j + 1 && nc > 0) {   // step j + 1: column j + 1 is y[u][0]
            acc[0] += y[u][0] * y[u][0];
#pragma unroll
            for (int q = 1; q < kQrPanel - 1; ++q)
              if (q < nc) acc[q] += y[u][0] * y[u][q];
          }
        }
      }
    }
    __syncthreads();
  }
  // G[r][i] = sum over rows q > j0 + i of v_r[q] v_i[q], plus v_r[j0 + i] (v_i is 1 there);
  // pair (r < i) at index i (i - 1) / 2 + r
  double g[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) g[p] = 0.0;
  for (int q0 = j0 + 1 + tid; q0 < m; q0 += 2 * 256) {
    double vq[2][kQrPanel];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = min(q0 + 256 * u, m - 1);
#pragma unroll
      for (int r = 0; r < kQrPanel; ++r) vq[u][r] = Wm[q + (long long)(j0 + min(r, pb - 1)) * m];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = q0 + 256 * u;
      if (q >= m) break;
#pragma unroll
      for (int i = 1; i < kQrPanel; ++i)
#pragma unroll
        for (int r = 0; r < i; ++r)
          if (i < pb && q > j0 + i) g[i * (i - 1) / 2 + r] += vq[u][r] * vq[u][i];
    }
  }
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    const double sp = wave_sum(g[p]);
    if (lane == 0) red[wave * kPairs + p] = sp;
  }
  __syncthreads();
  if (tid < kPairs) {
    int i = 1;
    while ((i + 1) * i / 2 <= tid) ++i;
    const int r = tid - i * (i - 1) / 2;
    if (i < pb)
      Gm[r][i] = (((red[tid] + red[kPairs + tid]) + red[2 * kPairs + tid]) + red[3 * kPairs + tid]) +
                 Wm[(j0 + i) + (long long)(j0 + r) * m];
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < pb; ++i) {
      const double ti = taus[j0 + i];
      for (int r = 0; r < i; ++r) {
        double t = 0.0;
        for (int q = r; q < i; ++q) t += Tm[r][q] * Gm[q][i];
        Tm[r][i] = -ti * t;
      }
      Tm[i][i] = ti;
      for (int r = i + 1; r < kQrPanel; ++r) Tm[r][i] = 0.0;
    }
    for (int i = pb; i < kQrPanel; ++i)
      for (int r = 0; r < kQrPanel; ++r) Tm[r][i] = 0.0;
  }
  __syncthreads();
  if (tid < kQrPanel * kQrPanel) qrw_tfac(Wm, m, n, j0)[tid] = Tm[tid / kQrPanel][tid % kQrPanel];
}

// the panel at j0 applied to one column per workgroup (blockIdx.y): qmode 0,
// the columns of Wm after the panel, with Q_panel^T = I - V T^T V^T; qmode 1,
// the columns >= j0 of Qm, with I - V T V^T (Q's earlier columns are unit
// vectors that the panel's reflectors leave alone).  w = V^T col over the rows
// >= j0 (rows j0 .. j0 + pb - 1 hold the unit diagonal of V, one thread each;
// below them every v_r is a stored column of Wm), u = T' w, col -= V u; the
// rows strided over the 256 threads, two per thread with their loads issued
// together (rows past the end clamped to the last one, not used); sums per
// thread, per wave, then the four waves in order.
__global__ __launch_bounds__(256) void k_qrw_apply(const QRTask* __restrict__ tasks, const int* __restrict__ wide,
                                                   BPtr<double> b_ws, int j0, int qmode) {
  const QRTask T = tasks[wide[blockIdx.x]];
  const int m = T.m, n = T.n;
  if (j0 >= n) return;
  const int pb = min(kQrPanel, n - j0), tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = (qmode ? j0 : j0 + pb) + (int)blockIdx.y;
  if (c >= n) return;   // uniform over the workgroup
  double* Wm = b_ws.p[blockIdx.z] + T.ws;
  double* col = (qmode ? Wm + (long long)m * n : Wm) + (long long)c * m;
  const double* V = Wm + (long long)j0 * m;
  const bool trans = !qmode;
  __shared__ double Tm[kQrPanel][kQrPanel];
  __shared__ double red[4][kQrPanel];
  __shared__ double wsh[kQrPanel];
  const double* tf = qrw_tfac(Wm, m, n, j0);
  if (tid < kQrPanel * kQrPanel) Tm[tid / kQrPanel][tid % kQrPanel] = tf[tid];
  double w[kQrPanel];
#pragma unroll
  for (int r = 0; r < kQrPanel; ++r) w[r] = 0.0;
  for (int i0 = j0 + pb + tid; i0 < m; i0 += 2 * 256) {
    double x[2], vv[2][kQrPanel];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = min(i0 + 256 * h, m - 1);
      x[h] = col[i];
#pragma unroll
      for (int r = 0; r < kQrPanel; ++r) vv[h][r] = V[i + (long long)min(r, pb - 1) * m];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (i0 + 256 * h < m) {
#pragma unroll
        for (int r = 0; r < kQrPanel; ++r) w[r] += (r < pb ? vv[h][r] : 0.0) * x[h];
      }
  }
  if (tid < pb) {
    const int i = j0 + tid;
    const double x = col[i];
#pragma unroll
    for (int r = 0; r < kQrPanel; ++r)
      w[r] += (r < tid ? V[i + (long long)r * m] : (r == tid ? 1.0 : 0.0)) * x;
  }
#pragma unroll
  for (int r = 0; r < kQrPanel; ++r) {
    const double sr = wave_sum(w[r]);
    if (lane == 0) red[wave][r] = sr;
  }
  __syncthreads();
  if (tid < kQrPanel) wsh[tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  __syncthreads();
  double u[kQrPanel];
#pragma unroll
  for (int r = 0; r < kQrPanel; ++r) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kQrPanel; ++q) t += (trans ? Tm[q][r] : Tm[r][q]) * wsh[q];
    u[r] = t;
  }
  for (int i0 = j0 + pb + tid; i0 < m; i0 += 2 * 256) {
    double x[2], vv[2][kQrPanel];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = min(i0 + 256 * h, m - 1);
      x[h] = col[i];
#pragma unroll
      for (int r = 0; r < kQrPanel; ++r) vv[h][r] = V[i + (long long)min(r, pb - 1) * m];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (i0 + 256 * h < m) {
        double y = x[h];
#pragma unroll
        for (int r = 0; r < kQrPanel; ++r) y -= (r < pb ? vv[h][r] : 0.0) * u[r];
        col[i0 + 256 * h] = y;
      }
  }
  if (tid < pb) {
    const int i = j0 + tid;
    double x = col[i];
#pragma unroll
    for (int r = 0; r < kQrPanel; ++r) x -= (r < tid ? V[i + (long long)r * m] : (r == tid ? 1.0 : 0.0)) * u[r];
    col[i] = x;
  }
}

// non-negative diagonal: column j of Q and row j of R flipped when R_jj < 0;
// Q into the block's place in A, R into S
__global__ __launch_bounds__(256) void k_qrw_out(const QRTask* __restrict__ tasks, const int* __restrict__ wide,
                                                 const long long* __restrict__ tabs, BPtr<double> b_A,
                                                 BPtr<double> b_S, BPtr<const double> b_ws) {
  double* A = b_A.p[blockIdx.z];
  double* S = b_S.p[blockIdx.z];
  const QRTask T = tasks[wide[blockIdx.x]];
  const int m = T.m, n = T.n;
  const double* Wm = b_ws.p[blockIdx.z] + T.ws;
  const double* Qm = Wm + (long long)m * n;
  const long long stride = (long long)gridDim.y * blockDim.x, e0 = (long long)blockIdx.y * blockDim.x + threadIdx.x;
  for (long long e = e0; e < (long long)m * n; e += stride) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double sg = Wm[j + (long long)j * m] < 0.0 ? -1.0 : 1.0;
    A[T.rbase + qrw_row(T, tabs, i) + (long long)j * T.cs] = sg * Qm[e];
  }
  for (long long e = e0; e < (long long)n * n; e += stride) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double sg = Wm[i + (long long)i * m] < 0.0 ? -1.0 : 1.0;
    const double val = (i <= j) ? sg * Wm[i + (long long)j * m] : 0.0;
    S[T.sdst + (T.trans ? (long long)j * n + i : (long long)i * n + j)] = val;
  }
}

__device__ __forceinline__ long long qr_row(const QRTask& T, const long long* tabs, int i) {
  return T.rtab >= 0 ? tabs[T.rtab + i] : (long long)i * T.rs;
}

// ---- register-resident Householder QR of an m x n block (m <= 16 SL,
// n <= kQrLdsMaxN) by one workgroup of kQrWaves waves.  Column c lives in
// DPP row c % 4 (lanes 16 (c % 4) .. 16 (c % 4) + 15) of wave c / 4, lane
// 16 r + l holding rows l, l + 16, ..., l + 16 (SL - 1) (so that the 16 lanes
// of a row read 16 consecutive reflector entries from LDS: no bank conflicts).  A column's dot product is a
// sum over its 16 lanes by DPP row rotations, four columns of a wave at once,
// and a wave whose columns are all finished skips the step.  The reflector of
// the step goes through LDS (two buffers, alternating by step, written in
// full: zero above the diagonal and past m), so every step needs one barrier:
// while applying reflector j, the owner of column j + 1 updates that column
// first and then turns it into reflector j + 1.
constexpr int kQrWaves = 16;
static_assert(kQrWaves * 4 == kQrLdsMaxN, "one column per DPP row");
// SL: rows per lane; the chunk kernel uses kQrChunkRows / 16, the stack
// kernel kQrStackRows / 16
template <int SL> struct QrCol { double x[SL]; };
// a column index is below kQrLdsMaxN = 64, so only a lane's first four slots
// (rows below 64) can lie at or above the diagonal; later slots never do
constexpr int kQrHead = kQrLdsMaxN / 16;

// DPP move of a double within rows of 16 lanes (lanes without a source get 0)
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_shift(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
// sum over the 16 lanes of each DPP row, in every lane of the row (rotations
// by 8, 4, 2, 1; lanes of a row differ only in the order of the additions)
__device__ __forceinline__ double row_allsum(double v) {
  v += dpp_shift<0x128, 0xf>(v);
  v += dpp_shift<0x124, 0xf>(v);
  v += dpp_shift<0x122, 0xf>(v);
  v += dpp_shift<0x121, 0xf>(v);
  return v;
}
// the value of a wave-uniform lane, as a scalar
__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// reflector of column c (held by this wave, c < m): row c := beta, rows
// below := v (v_c = 1, kept for forming Q), rows above untouched; the whole
// v to vout and tau[c].  alpha and |x below c|^2 are read from one lane, so
// every lane uses the same scalars.
template <int SL>
__device__ void qr_reflector(QrCol<SL>& X, int c, int m, double* vout, double* tau) {
  const int lane = threadIdx.x & 63, r = c & 3, l16 = lane & 15;
  double a = 0.0, p[4] = {0.0, 0.0, 0.0, 0.0};   // four partial sums: short dependency chains
#pragma unroll
  for (int t = 0; t < SL; ++t) {   // rows past m hold zero
    const int i = l16 + 16 * t;
    if (t < kQrHead) {
      if (i == c) a = X.x[t];
      if (i > c) p[t & 3] += X.x[t] * X.x[t];
    } else {
      p[t & 3] += X.x[t] * X.x[t];
    }
  }
  const double alpha = lane_value(a, 16 * r + (c & 15));
  const double xn2 = lane_value(row_allsum((p[0] + p[1]) + (p[2] + p[3])), 16 * r);
  double tj = 0.0, beta = alpha, scal = 1.0;
  if (xn2 > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tj = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  if ((lane >> 4) == r) {
#pragma unroll
    for (int t = 0; t < SL; ++t) {
      const int i = l16 + 16 * t;
      if (t < kQrHead) {
        if (i > c) X.x[t] *= scal;   // rows past m hold zero and stay zero
        vout[i] = (i < c) ? 0.0 : (i == c ? 1.0 : X.x[t]);
        if (i == c) X.x[t] = beta;
      } else {
        X.x[t] *= scal;
        vout[i] = X.x[t];
      }
    }
    if (l16 == 0) tau[c] = tj;
  }
}

// x -= tau (v . x) v on every column c of this wave with lo < c < n (v from
// LDS), then the look-ahead reflector of column stop_after if this wave owns it
template <int SL>
__device__ __forceinline__ void qr_apply(QrCol<SL>& X, const double* v, double tj, int lo, int n, int m, int stop_after,
                                         double* vnext, double* tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15;
  const int c0 = 4 * wave, c = c0 + (lane >> 4);
  const double* vl = v + l16;
  // the wave that builds the next reflector is on every step's critical path:
  // it issues first on its SIMD
  const bool owner = stop_after >= 0 && (stop_after >> 2) == wave;
  if (owner) __builtin_amdgcn_s_setprio(3);
  if (tj != 0.0 && c0 + 3 > lo && c0 < n) {   // wave-uniform: some column of the wave is still open
    double d[4] = {0.0, 0.0, 0.0, 0.0};   // four partial sums: short dependency chains
#pragma unroll
    for (int t = 0; t < SL; ++t) d[t & 3] += vl[16 * t] * X.x[t];
    const double f = tj * row_allsum((d[0] + d[1]) + (d[2] + d[3]));
    if (c > lo && c < n) {
#pragma unroll
      for (int t = 0; t < SL; ++t) X.x[t] -= f * vl[16 * t];
    }
  }
  if (owner) {
    qr_reflector(X, stop_after, m, vnext, tau);
    __builtin_amdgcn_s_setprio(0);
  }
}

template <int SL>
__device__ void qr_factor(QrCol<SL>& X, int m, int n, double* vbuf, double* tau) {
  const int wave = threadIdx.x >> 6;
  if (wave == 0) qr_reflector(X, 0, m, vbuf, tau);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    qr_apply(X, vbuf + (j & 1) * 16 * SL, tau[j], j, n, m, j + 1 < n ? j + 1 : -1,
             vbuf + ((j + 1) & 1) * 16 * SL, tau);
    __syncthreads();
  }
}

// signs of the diagonal of R to LDS (the lane holding each diagonal entry),
// then barrier
template <int SL>
__device__ void qr_signs(const QrCol<SL>& X, int n, double* sgn) {
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  const int c = 4 * (threadIdx.x >> 6) + (lane >> 4);
  if (c < n) {
#pragma unroll
    for (int t = 0; t < kQrHead; ++t)
      if (l16 + 16 * t == c) sgn[c] = X.x[t] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
}

// explicit Q (backward accumulation); R must have been written out before
template <int SL>
__device__ void qr_form_q(QrCol<SL>& X, int m, int n, double* vbuf, const double* tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15;
  for (int j = n - 1; j >= 0; --j) {
    double* v = vbuf + (j & 1) * 16 * SL;
    if ((j >> 2) == wave && (lane >> 4) == (j & 3)) {   // publish v_j, then column j := (I - tau_j v v^T) e_j
      const double tj = tau[j];
#pragma unroll
      for (int t = 0; t < SL; ++t) {
        const int i = l16 + 16 * t;
        const double vi = t >= kQrHead ? X.x[t] : ((i < j) ? 0.0 : (i == j ? 1.0 : X.x[t]));
        v[i] = vi;
        X.x[t] = (t < kQrHead && i == j) ? 1.0 - tj : -tj * vi;
      }
    }
    __syncthreads();
    qr_apply(X, v, tau[j], j, n, m, -1, nullptr, nullptr);
  }
  __syncthreads();
}

// kernel 1: QR of one row chunk (at most kQrChunkRows rows).  Single-chunk tasks
// are finished here (sign fix, Q to the matrix, R to S); otherwise Q_c goes to
// ws[qw] and R_c (upper n x n) to the stacked R at ws[rw] (column-major,
// leading dimension nchunks*n).
__global__ __launch_bounds__(kQrWaves * 64) void k_qr_chunk(const QRTask* __restrict__ tasks,
                                                            const QRChunk* __restrict__ chunks,
                                                            const long long* __restrict__ tabs, BPtr<double> b_A,
                                                            BPtr<double> b_S, BPtr<double> b_ws) {
  double* A = b_A.p[blockIdx.y];
  double* S = b_S.p[blockIdx.y];
  double* ws = b_ws.p[blockIdx.y];
  constexpr int SL = kQrChunkRows / 16;
  __shared__ __attribute__((aligned(16))) double vbuf[2 * kQrChunkRows];
  __shared__ double tau[kQrLdsMaxN], sgn[kQrLdsMaxN];
  const QRChunk C = chunks[blockIdx.x];
  const QRTask T = tasks[C.task];
  const int m = C.rows, n = T.n, l16 = threadIdx.x & 15;
  const int c = 4 * (threadIdx.x >> 6) + ((threadIdx.x & 63) >> 4);
  QrCol<SL> X;
#pragma unroll
  for (int t = 0; t < SL; ++t) {
    const int i = l16 + 16 * t;
    X.x[t] = (c < n && i < m) ? A[T.rbase + qr_row(T, tabs, C.row0 + i) + (long long)c * T.cs] : 0.0;
  }
  qr_factor(X, m, n, vbuf, tau);
  const bool last = C.nchunks == 1;
  if (last) qr_signs(X, n, sgn);
  const long long ldr = (long long)C.nchunks * n;
  if (c < n) {
#pragma unroll
    for (int t = 0; t < kQrHead; ++t) {   // R (rows <= c of column c; i < n <= 64)
      const int i = l16 + 16 * t;
      if (i >= n) continue;
      const double r = (i <= c) ? X.x[t] : 0.0;
      if (last) S[T.sdst + (T.trans ? (long long)c * n + i : (long long)i * n + c)] = sgn[i] * r;
      else ws[C.rw + (long long)c * ldr + (long long)C.chunk * n + i] = r;
    }
  }
  qr_form_q(X, m, n, vbuf, tau);
  if (c < n) {
#pragma unroll
    for (int t = 0; t < SL; ++t) {   // Q
      const int i = l16 + 16 * t;
      if (i >= m) continue;
      if (last) A[T.rbase + qr_row(T, tabs, C.row0 + i) + (long long)c * T.cs] = sgn[c] * X.x[t];
      else ws[C.qw + i + (long long)c * m] = X.x[t];
    }
  }
}

// kernel 2: QR of the stacked chunk R factors; final R (non-negative
// diagonal) to S, second-level Q (sign-fixed) back over the stack.
__global__ __launch_bounds__(kQrWaves * 64) void k_qr_stack(const QRTask* __restrict__ tasks,
                                                            const QRStack* __restrict__ stacks, BPtr<double> b_S,
                                                            BPtr<double> b_ws) {
  double* S = b_S.p[blockIdx.y];
  double* ws = b_ws.p[blockIdx.y];
  constexpr int SL = kQrStackRows / 16;
  __shared__ __attribute__((aligned(16))) double vbuf[2 * kQrStackRows];
  __shared__ double tau[kQrLdsMaxN], sgn[kQrLdsMaxN];
  const QRStack K = stacks[blockIdx.x];
  const QRTask T = tasks[K.task];
  const int n = T.n, m = K.nchunks * n, l16 = threadIdx.x & 15;
  const int c = 4 * (threadIdx.x >> 6) + ((threadIdx.x & 63) >> 4);
  QrCol<SL> X;
#pragma unroll
  for (int t = 0; t < SL; ++t) {
    const int i = l16 + 16 * t;
    X.x[t] = (c < n && i < m) ? ws[K.rw + i + (long long)c * m] : 0.0;
  }
  qr_factor(X, m, n, vbuf, tau);
  qr_signs(X, n, sgn);
  if (c < n) {
#pragma unroll
    for (int t = 0; t < kQrHead; ++t) {   // R (i < n <= 64)
      const int i = l16 + 16 * t;
      if (i >= n) continue;
      const double r = (i <= c) ? X.x[t] : 0.0;
      S[T.sdst + (T.trans ? (long long)c * n + i : (long long)i * n + c)] = sgn[i] * r;
    }
  }
  qr_form_q(X, m, n, vbuf, tau);
  if (c < n) {
#pragma unroll
    for (int t = 0; t < SL; ++t) {
      const int i = l16 + 16 * t;
      if (i < m) ws[K.rw + i + (long long)c * m] = sgn[c] * X.x[t];
    }
  }
}

// kernel 3: final Q rows of a chunk = Q_c (rows x n) . Q2_c (n x n)
__global__ __launch_bounds__(256) void k_qr_combine(const QRTask* __restrict__ tasks, const QRChunk* __restrict__ chunks,
                                                    const long long* __restrict__ tabs, BPtr<double> b_A,
                                                    BPtr<double> b_ws) {
  double* A = b_A.p[blockIdx.y];
  const double* __restrict__ ws = b_ws.p[blockIdx.y];
  __shared__ double Q2[kQrLdsMaxN * kQrLdsMaxN];
  const QRChunk C = chunks[blockIdx.x];
  if (C.nchunks == 1) return;
  const QRTask T = tasks[C.task];
  const int m = C.rows, n = T.n, tid = threadIdx.x;
  const long long ldr = (long long)C.nchunks * n;
  for (int e = tid; e < n * n; e += blockDim.x) {
    int k = e % n, j = e / n;
    Q2[k + j * n] = ws[C.rw + (long long)j * ldr + (long long)C.chunk * n + k];
  }
  __syncthreads();
  // a thread forms four outputs of one row (columns j0 .. j0 + 3), so each
  // element of Q_c it loads serves four products; the column group of a
  // lane's neighbours is the same (Q2 entries broadcast from LDS)
  const int ng = (n + 3) >> 2;
  const double* __restrict__ Qc = ws + C.qw;
  for (int e = tid; e < m * ng; e += blockDim.x) {
    const int i = e % m, j0 = 4 * (e / m);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < n; ++k) {
      const double q = Qc[i + (long long)k * m];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += q * Q2[k + min(j0 + u, n - 1) * n];
    }
    const long long row = T.rbase + qr_row(T, tabs, C.row0 + i);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + u < n) A[row + (long long)(j0 + u) * T.cs] = acc[u];
  }
}

void qr_plan_chunks(QRPlan& p) {
  p.chunks.clear();
  p.stacks.clear();
  p.wide.clear();
  long long pos = 0;
  for (int t = 0; t < (int)p.tasks.size(); ++t) {
    const QRTask& T = p.tasks[t];
    const int m = T.m, n = T.n;
    if (n > kQrLdsMaxN) { p.wide.push_back(t); continue; }
    int nc = 1;
    if (m > kQrChunkRows) {
      nc = (m + kQrChunkRows - 1) / kQrChunkRows;
      if ((long long)nc * n > kQrStackRows || m / nc < n) { p.wide.push_back(t); continue; }
    }
    long long rw = pos;
    if (nc > 1) pos += (long long)nc * n * n;
    for (int c = 0; c < nc; ++c) {
      int r0 = (int)((long long)m * c / nc), r1 = (int)((long long)m * (c + 1) / nc);
      QRChunk ch{t, r0, r1 - r0, c, nc, 0, 0, rw};
      if (nc > 1) { ch.qw = pos; pos += (long long)(r1 - r0) * n; }
      p.chunks.push_back(ch);
    }
    if (nc > 1) p.stacks.push_back({t, nc, rw});
  }
  p.lds_ws = pos;
}

void launch_qr(const QRPlan& p, const long long* d_tabs, BPtr<double> A, BPtr<double> S, BPtr<double> ws, int nb,
               hipStream_t st) {
  if (p.ntasks == 0) return;
  prof_begin(st);
  BPtr<double> lws = ws;   // the chunk path's workspace follows the global fallback's
  for (int b = 0; b < nb; ++b) lws.p[b] = ws.p[b] + p.ws_size;
  if (!p.chunks.empty()) {
    hipLaunchKernelGGL(k_qr_chunk, dim3((unsigned)p.chunks.size(), nb), dim3(kQrWaves * 64), 0, st, p.d_tasks,
                       p.d_chunks, d_tabs, A, S, lws);
    HIP_CHECK_LAUNCH();
  }
  if (!p.stacks.empty()) {
    hipLaunchKernelGGL(k_qr_stack, dim3((unsigned)p.stacks.size(), nb), dim3(kQrWaves * 64), 0, st, p.d_tasks,
                       p.d_stacks, S, lws);
    HIP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_qr_combine, dim3((unsigned)p.chunks.size(), nb), dim3(256), 0, st, p.d_tasks, p.d_chunks,
                       d_tabs, A, lws);
    HIP_CHECK_LAUNCH();
  }
  int maxn = 0;
  for (int w : p.wide) {
    const QRTask& t = p.tasks.at(w);
    TT_REQUIRE(t.m >= t.n && t.ws >= 0 && t.ws + qr_wide_ws(t.m, t.n) <= p.ws_size, TT_EINVAL,
               "wide QR: a block outside its workspace");
    maxn = std::max(maxn, t.n);
  }
  if (maxn > 0) {
    const unsigned nw = (unsigned)p.wide.size();
    auto groups = [](int cols) { return (unsigned)((cols + kQrApplyCols - 1) / kQrApplyCols); };
    hipLaunchKernelGGL(k_qrw_load, dim3(nw, kQrSpread, nb), dim3(256), 0, st, p.d_tasks, p.d_wide, d_tabs, cst(A), ws);
    HIP_CHECK_LAUNCH();
    for (int j0 = 0; j0 < maxn; j0 += kQrPanel) {
      hipLaunchKernelGGL(k_qrw_panel, dim3(nw, 1, nb), dim3(256), 0, st, p.d_tasks, p.d_wide, ws, j0);
      HIP_CHECK_LAUNCH();
      if (maxn - j0 - kQrPanel > 0) {
        hipLaunchKernelGGL(k_qrw_apply, dim3(nw, groups(maxn - j0 - kQrPanel), nb), dim3(256), 0, st, p.d_tasks,
                           p.d_wide, ws, j0, 0);
        HIP_CHECK_LAUNCH();
      }
    }
    for (int j0 = ((maxn - 1) / kQrPanel) * kQrPanel; j0 >= 0; j0 -= kQrPanel) {
      hipLaunchKernelGGL(k_qrw_apply, dim3(nw, groups(maxn - j0), nb), dim3(256), 0, st, p.d_tasks, p.d_wide, ws, j0,
                         1);
      HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_qrw_out, dim3(nw, kQrSpread, nb), dim3(256), 0, st, p.d_tasks, p.d_wide, d_tabs, A, S, cst(ws));
    HIP_CHECK_LAUNCH();
  }
  prof_end(st, PROF_QR, nb * p.flops, nb * p.bytes);
}

// ------------------------------------------------------------------ Lanczos
// Sums of the nv per-thread accumulators (then `extra` at index nv when
// with_extra) over the block in a fixed order: wave sums, then the waves in
// order; out[v] written by thread v.  red holds (blockDim / 64) * (MAXV + 1)
// doubles.
template <int MAXV>
__device__ __forceinline__ void block_sums(const double (&acc)[MAXV], int nv, double* red, double* out,
                                           bool with_extra = false, double extra = 0.0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  constexpr int S = MAXV + 1;
#pragma unroll
  for (int v = 0; v < MAXV; ++v) {
    if (v >= nv) break;
    const double s = wave_sum(acc[v]);
    if (lane == 0) red[wave * S + v] = s;
  }
  if (with_extra) {
    const double s = wave_sum(extra);
    if (lane == 0) red[wave * S + nv] = s;
  }
  __syncthreads();
  const int nout = nv + (with_extra ? 1 : 0);
  if ((int)threadIdx.x < nout) {
    const int v = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * S + v];
    out[v] = s;
  }
}

// contiguous chunk of block b (the same in every Lanczos kernel, so each
// partial sum covers the same elements in the same order)
__device__ __forceinline__ void red_chunk(long long n, long long& i0, long long& i1) {
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  i0 = (long long)blockIdx.x * chunk;
  i1 = i0 + chunk < n ? i0 + chunk : n;
}

// part[b*(nv+self) + v] = sum over block b's chunk of Q_v[i] * y[i]; last entry y.y if with_self.
// One pass: y and every Q_v are read once.
template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_mdot(BPtr<const double> b_Q, long long ld, int nv,
                                                      BPtr<const double> b_y, long long n, int with_self,
                                                      BPtr<double> b_part) {
  const double* __restrict__ Q = b_Q.p[blockIdx.y];
  const double* __restrict__ y = b_y.p[blockIdx.y];
  double* __restrict__ part = b_part.p[blockIdx.y];
  __shared__ double red[(kRedThreads / 64) * (MAXV + 1)];
  long long i0, i1;
  red_chunk(n, i0, i1);
  double acc[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) acc[v] = 0.0;
  double self = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double yi = y[i];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      if (v >= nv) break;
      acc[v] += Q[(long long)v * ld + i] * yi;
    }
    self += yi * yi;
  }
  block_sums<MAXV>(acc, nv, red, part + (long long)blockIdx.x * (nv + with_self), with_self != 0, self);
}

__device__ double sum_parts(const double* part, int nparts, int stride, int v) {
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(long long)b * stride + v];
  return s;
}

// c[v] = sum over the kRedBlocks partials part[b*stride + v], v < nv, in a fixed
// order (lane-strided sums, then the wave sum); one wave per value, written to
// LDS by its lane 0.  The caller synchronises before reading c.
__device__ __forceinline__ void gather_parts(const double* __restrict__ part, int stride, int nv, double* c) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int v = wave; v < nv; v += nw) {
    double s = 0.0;
    for (int b = lane; b < kRedBlocks; b += 64) s += part[(long long)b * stride + v];
    s = wave_sum(s);
    if (lane == 0) c[v] = s;
  }
}

// q0 = v / ||v||; scal[0] = ||v||
__global__ void k_lz_start(BPtr<const double> b_v, BPtr<double> b_q0, long long n, BPtr<const double> b_part,
                           BPtr<double> b_scal) {
  const double* __restrict__ v = b_v.p[blockIdx.y];
  double* __restrict__ q0 = b_q0.p[blockIdx.y];
  const double* __restrict__ part = b_part.p[blockIdx.y];
  double* scal = b_scal.p[blockIdx.y];
  __shared__ double s_nv;
  gather_parts(part, 1, 1, &s_nv);
  __syncthreads();
  const double nv = sqrt(s_nv);
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[0] = nv;
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    q0[i] = v[i] * inv;
}

// Fused Gram-Schmidt passes on the same chunks as k_mdot, so every partial
// sum has a fixed order.  k_lz_sub_dot: w -= sum_v c_v Q_v with c from the
// partials of the previous pass (alpha, ||H q|| stored by block 0), and in the
// same pass the partial dots Q_v . w of the updated chunk and its partial w . w
// (part_out stride nv + 1).
template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_lz_sub_dot(BPtr<double> b_w, BPtr<const double> b_Q, long long ld,
                                                            int nv, BPtr<const double> b_part_in, int stride_in,
                                                            long long n, BPtr<double> b_alpha, BPtr<double> b_hn,
                                                            BPtr<double> b_part_out) {
  double* __restrict__ w = b_w.p[blockIdx.y];
  const double* __restrict__ Q = b_Q.p[blockIdx.y];
  const double* __restrict__ part_in = b_part_in.p[blockIdx.y];
  double* alpha_out = b_alpha.p[blockIdx.y];
  double* hn_out = b_hn.p[blockIdx.y];
  double* __restrict__ part_out = b_part_out.p[blockIdx.y];
  __shared__ double c[kMaxKrylov + 1];
  __shared__ double red[(kRedThreads / 64) * (MAXV + 1)];
  gather_parts(part_in, stride_in, stride_in > nv ? nv + 1 : nv, c);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (alpha_out) *alpha_out = c[nv - 1];
    if (hn_out) *hn_out = sqrt(c[nv]);
  }
  double cr[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) cr[v] = v < nv ? c[v] : 0.0;
  long long i0, i1;
  red_chunk(n, i0, i1);
  double acc[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) acc[v] = 0.0;
  double ss = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double q[MAXV];
    double s = w[i];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      q[v] = v < nv ? Q[(long long)v * ld + i] : 0.0;
      s -= cr[v] * q[v];
    }
    w[i] = s;
#pragma unroll
    for (int v = 0; v < MAXV; ++v) acc[v] += q[v] * s;
    ss += s * s;
  }
  block_sums<MAXV>(acc, nv, red, part_out + (long long)blockIdx.x * (nv + 1), true, ss);
}

// Second Gram-Schmidt pass fused with the normalisation: with c' = Q^T w'
// (the dots of the previous pass) the new vector is w'' = w' - Q c', and since
// Q has orthonormal columns ||w''||^2 = ||w'||^2 - ||c'||^2, so beta and
// q_next = w'' / beta come out of one pass.  (Near a lucky breakdown both terms
// are O(eps ||H q||), and so is the computed beta: the test beta <= tol ||H q||
// still holds.)  qn = null: only beta is stored.
template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_lz_sub_next(BPtr<const double> b_w, BPtr<const double> b_Q,
                                                             long long ld, int nv, BPtr<const double> b_part_in,
                                                             long long n, BPtr<double> b_qn, BPtr<double> b_beta,
                                                             BPtr<const double> b_hn, double tol) {
  const double* __restrict__ w = b_w.p[blockIdx.y];
  const double* __restrict__ Q = b_Q.p[blockIdx.y];
  const double* __restrict__ part_in = b_part_in.p[blockIdx.y];
  double* __restrict__ qn = b_qn.p[blockIdx.y];
  double* beta_out = b_beta.p[blockIdx.y];
  const double* hn = b_hn.p[blockIdx.y];
  __shared__ double c[kMaxKrylov + 1];
  __shared__ double s_inv;
  gather_parts(part_in, nv + 1, nv + 1, c);
  __syncthreads();
  if (threadIdx.x == 0) {
    double p = 0.0;
    for (int v = 0; v < nv; ++v) p += c[v] * c[v];
    const double b2 = c[nv] - p;
    const double b = b2 > 0.0 ? sqrt(b2) : 0.0;
    if (blockIdx.x == 0) *beta_out = b;
    const bool brk = !(b > tol * (*hn)) || b == 0.0;
    s_inv = brk ? 0.0 : 1.0 / b;
  }
  __syncthreads();
  if (!qn) return;
  const double inv = s_inv;
  double cr[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) cr[v] = v < nv ? c[v] : 0.0;
  long long i0, i1;
  red_chunk(n, i0, i1);
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double s = w[i];
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      if (v >= nv) break;
      s -= cr[v] * Q[(long long)v * ld + i];
    }
    qn[i] = s * inv;
  }
}

// out = sum_v coeff_v Q_v and the partial out . out of each chunk
__global__ __launch_bounds__(kRedThreads) void k_lz_combine_norm(BPtr<const double> b_Q, long long ld, int K,
                                                                 BPtr<const double> b_coeff, BPtr<double> b_out,
                                                                 long long n, BPtr<double> b_part_out) {
  const double* __restrict__ Q = b_Q.p[blockIdx.y];
  const double* __restrict__ coeff = b_coeff.p[blockIdx.y];
  double* __restrict__ out = b_out.p[blockIdx.y];
  double* __restrict__ part_out = b_part_out.p[blockIdx.y];
  __shared__ double c[kMaxKrylov];
  __shared__ double red[kRedThreads / 64];
  if (threadIdx.x < K) c[threadIdx.x] = coeff[threadIdx.x];
  __syncthreads();
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long i0 = (long long)blockIdx.x * chunk;
  const long long i1 = i0 + chunk < n ? i0 + chunk : n;
  double ss = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double s = 0.0;
    for (int v = 0; v < K; ++v) s += c[v] * Q[(long long)v * ld + i];
    out[i] = s;
    ss += s * s;
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = ss;
}

// coefficients of exp(t T) e_1 * ||v|| for the Krylov tridiagonal T: Taylor
// series of (tT)/2^s with 2^s >= 2 ||tT||_inf, then s squarings; one thread per
// matrix element, everything in LDS.
__global__ __launch_bounds__(64) void k_lz_coeffs(BPtr<const double> b_alpha, BPtr<const double> b_beta,
                                                  BPtr<const double> b_hn, int K, double t, double tol,
                                                  BPtr<const double> b_scal, BPtr<double> b_coeff,
                                                  BPtr<double> b_err) {
  const double* alpha = b_alpha.p[blockIdx.y];
  const double* beta = b_beta.p[blockIdx.y];
  const double* hn = b_hn.p[blockIdx.y];
  const double* scal = b_scal.p[blockIdx.y];
  double* coeff = b_coeff.p[blockIdx.y];
  double* errmax = b_err.p[blockIdx.y];
  __shared__ double A[kMaxKrylov * kMaxKrylov], E[kMaxKrylov * kMaxKrylov], P[kMaxKrylov * kMaxKrylov],
      X[kMaxKrylov * kMaxKrylov];
  __shared__ int s_k, s_sq;
  // one wave (K <= kMaxKrylov <= 64): lane j reads alpha_j, beta_j, ||H q_j||
  const int tid = threadIdx.x;
  const double aj = tid < K ? alpha[tid] : 0.0;
  const double bj = tid < K - 1 ? beta[tid] : 0.0;
  const double hj = tid < K - 1 ? hn[tid] : 0.0;
  // the basis ends at the first j < K - 1 with beta_j <= tol ||H q_j|| (or beta_j = 0): k = j + 1
  const bool brk = tid < K - 1 && (!(bj > tol * hj) || bj == 0.0);
  const unsigned long long mask = __ballot(brk);
  const int kb = mask ? __ffsll((long long)mask) : K;
  // infinity norm of t T_k (row i: |alpha_i| + |beta_{i-1}| + |beta_i| inside the k x k block)
  const double bprev = __shfl(bj, tid > 0 ? tid - 1 : 0, 64);
  double r = 0.0;
  if (tid < kb) r = fabs(t) * (fabs(aj) + (tid > 0 ? fabs(bprev) : 0.0) + (tid + 1 < kb ? fabs(bj) : 0.0));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
  if (tid == 0) {
    double nrm = r;
    int sq = 0;
    while (nrm > 0.5 && sq < 60) { nrm *= 0.5; ++sq; }
    s_k = kb;
    s_sq = sq;
  }
  __syncthreads();
  const int k = s_k, kk = k * k;
  const double sc = ldexp(t, -s_sq);
  for (int e = tid; e < kk; e += blockDim.x) {
    int i = e / k, j = e % k;
    double v = 0.0;
    if (i == j) v = alpha[i];
    else if (j == i + 1) v = beta[i];
    else if (i == j + 1) v = beta[j];
    A[e] = sc * v;
    E[e] = (i == j) ? 1.0 : 0.0;
    P[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // E = sum_{d<=24} A^d / d!  (||A|| <= 1/2: the tail is below 1e-25)
  for (int d = 1; d <= 24; ++d) {
    for (int e = tid; e < kk; e += blockDim.x) {
      int i = e / k, j = e % k;
      double acc = 0.0;
      for (int q = 0; q < k; ++q) acc += P[i * k + q] * A[q * k + j];
      X[e] = acc / d;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += blockDim.x) {
      P[e] = X[e];
      E[e] += X[e];
    }
    __syncthreads();
  }
  for (int r = 0; r < s_sq; ++r) {
    for (int e = tid; e < kk; e += blockDim.x) {
      int i = e / k, j = e % k;
      double acc = 0.0;
      for (int q = 0; q < k; ++q) acc += E[i * k + q] * E[q * k + j];
      X[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += blockDim.x) E[e] = X[e];
    __syncthreads();
  }
  const double nv = scal[0];
  for (int i = tid; i < K; i += blockDim.x) coeff[i] = (i < k) ? nv * E[i * k + 0] : 0.0;
  if (tid == 0 && k == K) {
    double err = beta[K - 1] * fabs(E[(K - 1) * k + 0]);
    if (err > *errmax) *errmax = err;
  }
}

// v /= ||v||; lambda += ln ||v||
__global__ void k_normalize_log(BPtr<double> b_v, long long n, BPtr<const double> b_part, BPtr<double> b_lambda) {
  double* __restrict__ v = b_v.p[blockIdx.y];
  const double* __restrict__ part = b_part.p[blockIdx.y];
  double* lambda = b_lambda.p[blockIdx.y];
  __shared__ double s_n;
  gather_parts(part, 1, 1, &s_n);
  __syncthreads();
  const double nv = sqrt(s_n);
  if (blockIdx.x == 0 && threadIdx.x == 0) *lambda += log(nv);
  const double inv = 1.0 / nv;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    v[i] *= inv;
}

__global__ void k_copy(BPtr<double> b_d, BPtr<const double> b_s, long long n) {
  double* __restrict__ d = b_d.p[blockIdx.y];
  const double* __restrict__ s = b_s.p[blockIdx.y];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void k_fill(double* __restrict__ d, double val, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = val;
}
__global__ void k_dot_final(const double* part, int nparts, int nv, double* out) {
  if (threadIdx.x < nv && blockIdx.x == 0) out[threadIdx.x] = sum_parts(part, nparts, nv, threadIdx.x);
}

static int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

// the Lanczos kernels keep one accumulator per vector in registers: instances
// for up to 9, 17 and kMaxKrylov + 1 vectors
#define TT_BY_MAXV(NV, KERNEL, ...)                                                              \
  do {                                                                                           \
    if ((NV) <= 9) hipLaunchKernelGGL(KERNEL<9>, __VA_ARGS__);                                   \
    else if ((NV) <= 17) hipLaunchKernelGGL(KERNEL<17>, __VA_ARGS__);                            \
    else hipLaunchKernelGGL(KERNEL<kMaxKrylov + 1>, __VA_ARGS__);                                \
  } while (0)

void launch_mdot(BPtr<const double> Q, long long ld, int nv, BPtr<const double> y, long long n, int with_self,
                 BPtr<double> part, int nb, hipStream_t st) {
  TT_BY_MAXV(nv + with_self, k_mdot, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, st, Q, ld, nv, y, n, with_self, part);
  HIP_CHECK_LAUNCH();
}
void launch_lz_start(BPtr<const double> v, BPtr<double> q0, long long n, BPtr<const double> part, BPtr<double> scal,
                     int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_start, dim3(grid_for(n), nb), dim3(256), 0, st, v, q0, n, part, scal);
  HIP_CHECK_LAUNCH();
}
void launch_lz_sub_dot(BPtr<double> w, BPtr<const double> Q, long long ld, int nv, BPtr<const double> part_in,
                       int stride_in, long long n, BPtr<double> alpha_out, BPtr<double> hn_out, BPtr<double> part_out,
                       int nb, hipStream_t st) {
  TT_BY_MAXV(nv, k_lz_sub_dot, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, st, w, Q, ld, nv, part_in, stride_in, n,
             alpha_out, hn_out, part_out);
  HIP_CHECK_LAUNCH();
}
void launch_lz_sub_next(BPtr<const double> w, BPtr<const double> Q, long long ld, int nv, BPtr<const double> part_in,
                        long long n, BPtr<double> qn, BPtr<double> beta_out, BPtr<const double> hn, double tol,
                        int nb, hipStream_t st) {
  TT_BY_MAXV(nv, k_lz_sub_next, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, st, w, Q, ld, nv, part_in, n, qn, beta_out,
             hn, tol);
  HIP_CHECK_LAUNCH();
}
void launch_lz_combine_norm(BPtr<const double> Q, long long ld, int K, BPtr<const double> coeff, BPtr<double> out,
                            long long n, BPtr<double> part_out, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_combine_norm, dim3(kRedBlocks, nb), dim3(kRedThreads), 0, st, Q, ld, K, coeff, out, n,
                     part_out);
  HIP_CHECK_LAUNCH();
}
void launch_lz_coeffs(BPtr<const double> alpha, BPtr<const double> beta, BPtr<const double> hn, int K, double t,
                      double tol, BPtr<const double> scal, BPtr<double> coeff, BPtr<double> errmax, int nb,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_lz_coeffs, dim3(1, nb), dim3(64), 0, st, alpha, beta, hn, K, t, tol, scal, coeff, errmax);
  HIP_CHECK_LAUNCH();
}
void launch_normalize_log(BPtr<double> v, long long n, BPtr<const double> part, BPtr<double> lambda, int nb,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_normalize_log, dim3(grid_for(n), nb), dim3(256), 0, st, v, n, part, lambda);
  HIP_CHECK_LAUNCH();
}
void launch_copy(BPtr<double> dst, BPtr<const double> src, long long n, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n), nb), dim3(256), 0, st, dst, src, n);
  HIP_CHECK_LAUNCH();
}
void launch_fill(double* dst, double val, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, dst, val, n);
  HIP_CHECK_LAUNCH();
}
void launch_dot_final(const double* part, int nparts, int nv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, st, part, nparts, nv, out);
  HIP_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ trace
// v_{k+1}[y] = sum_x v_k[x] sum_sigma A_k[x, (sigma,sigma), y], with a running
// log scale; out2[0] = ln v_N[0] (the final bond has one state).
__global__ __launch_bounds__(256) void k_trace(const TraceEntry* __restrict__ ent, const int* __restrict__ site_start,
                                               int N, double* const* __restrict__ sites, double* vbuf, long long vlen,
                                               double* out2) {
  __shared__ double red[8];
  double* v = vbuf;
  double* w = vbuf + vlen;
  double logscale = 0.0;
  if (threadIdx.x == 0) v[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    for (long long i = threadIdx.x; i < vlen; i += blockDim.x) w[i] = 0.0;
    __syncthreads();
    const double* A = sites[k];
    for (int e = site_start[k]; e < site_start[k + 1]; ++e) {
      const TraceEntry E = ent[e];
      for (long long y = threadIdx.x; y < E.dr; y += blockDim.x) {
        double s = 0.0;
        for (long long x = 0; x < E.dl; ++x) {
          double vx = v[E.xoff + x];
          if (vx == 0.0) continue;
          const double* row = A + E.src + x * E.C;
          double d = 0.0;
          for (int q = 0; q < 4; ++q) d += row[(long long)E.pos[q] * E.dr + y];
          s += vx * d;
        }
        w[E.yoff + y] += s;
      }
      __syncthreads();
    }
    double mx = 0.0;
    for (long long i = threadIdx.x; i < vlen; i += blockDim.x) mx = fmax(mx, fabs(w[i]));
    // max via sum of a one-hot is not needed: use shared reduction of max
    __syncthreads();
    {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
      if (lane == 0) red[wave] = mx;
      __syncthreads();
      mx = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) mx = fmax(mx, red[q]);
      __syncthreads();
    }
    double inv = mx > 0.0 ? 1.0 / mx : 1.0;
    if (mx > 0.0) logscale += log(mx);
    for (long long i = threadIdx.x; i < vlen; i += blockDim.x) v[i] = w[i] * inv;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = log(v[0]) + logscale;
    out2[1] = v[0];
  }
}

void launch_trace(const TraceEntry* d_entries, const int* d_site_start, int N, double* const* d_sites, double* vbuf,
                  long long vlen, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, d_entries, d_site_start, N, d_sites, vbuf, vlen, out2);
  HIP_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- SVD of the 2-TDVP split
// One-sided Jacobi (Hestenes): the columns of X are rotated in pairs until
// every pair is orthogonal to a relative tolerance; then X = U Sigma and the
// product V of the rotations gives X_in = X V^T.  The pairs follow the
// round-robin order (one index fixed, the others rotating), so the n/2
// rotations of a round touch disjoint columns and run on separate waves; sums
// are taken in a fixed order, so the result is deterministic.  Small singular
// values keep their relative accuracy.  One workgroup per task.
//  * X, and V when it fits too, live in LDS for the sweeps (copied back to the
//    work array at the end) when the task is small enough; else in global memory.
//  * The squared column norms are kept in LDS, recomputed exactly at the
//    start of every sweep and updated by each rotation (||u'||^2 = al - t ga,
//    ||v'||^2 = be + t ga), so a pair costs one dot product, not three.
//  * A pair of columns both at the rounding level of the block (squared
//    norms below (m eps ||X||_F)^2) is left alone: their mutual products are
//    rounding noise that no rotation makes orthogonal, and such columns
//    carry singular values far below any kept one.
constexpr int kSvdThreads = 1024;
constexpr int kSvdMaxSweeps = 40;
constexpr int kSvdLdsBytes = 160 * 1024;

__device__ inline double wave_sum64(double v) {
  // butterfly: every lane ends with the same bits (each addition is commutative)
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kSvdThreads) void k_svd_jacobi(const SvdTask* __restrict__ tasks,
                                                           const int* __restrict__ idx,
                                                           const long long* __restrict__ tabs,
                                                           const double* __restrict__ src, double* __restrict__ ws,
                                                           double* __restrict__ sig, int lds_doubles) {
  extern __shared__ __attribute__((aligned(16))) double svd_lds[];
  const SvdTask t = tasks[idx ? idx[blockIdx.x] : blockIdx.x];
  const bool tr = t.R < t.w;
  const int mw = tr ? t.w : t.R, nw = tr ? t.R : t.w;
  double* Xg = ws + t.ws;
  double* Vg = Xg + (long long)mw * nw;
  if (nw > lds_doubles) {   // the norms must fit (the host refuses such tasks): report NaN values
    for (int j = threadIdx.x; j < nw; j += blockDim.x) sig[t.sig + j] = __builtin_nan("");
    return;
  }
  // LDS: the squared norms, then X if it fits, then V if it fits too
  double* nrm = svd_lds;
  const long long need_x = (long long)nw + (long long)mw * nw, need_xv = need_x + (long long)nw * nw;
  const bool x_lds = need_x <= lds_doubles, v_lds = need_xv <= lds_doubles;
  double* X = x_lds ? svd_lds + nw : Xg;
  double* V = v_lds ? svd_lds + need_x : Vg;
  const long long* rt = tabs + t.rtab;
  const long long tot = (long long)t.R * t.w;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const long long i = e / t.w, j = e - i * t.w;
    const double v = src[rt[i] + j];
    if (!tr) X[i + j * mw] = v;
    else X[j + i * mw] = v;
  }
  for (long long e = threadIdx.x; e < (long long)nw * nw; e += blockDim.x) V[e] = (e / nw == e % nw) ? 1.0 : 0.0;
  __shared__ int rotated;
  __shared__ double s_thr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int np = nw + (nw & 1);                 // an idle index when nw is odd
  const double eps = 2.220446049250313e-16;
  const double tol = eps * (double)(mw > 16 ? mw : 16);
  __syncthreads();
  for (int sw = 0; sw < kSvdMaxSweeps && np > 1; ++sw) {
    // exact squared column norms, and the rounding level of the block
    for (int j = wave; j < nw; j += nwaves) {
      const double* xj = X + (long long)j * mw;
      double s2 = 0.0;
      for (int i = lane; i < mw; i += 64) s2 += xj[i] * xj[i];
      s2 = wave_sum64(s2);
      if (lane == 0) nrm[j] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double f = 0.0;
      for (int j = 0; j < nw; ++j) f += nrm[j];
      const double lev = (double)mw * eps;
      s_thr = lev * lev * f;
      rotated = 0;
    }
    __syncthreads();
    const double thr = s_thr;
    for (int rd = 0; rd < np - 1; ++rd) {
      for (int k = wave; k < np / 2; k += nwaves) {
        int a = k == 0 ? 0 : 1 + (k + rd) % (np - 1);
        int b = 1 + ((k == 0 ? 0 : np - 1 - k) + rd) % (np - 1);
        if (a > b) { const int q = a; a = b; b = q; }
        if (b >= nw) continue;
        const double al = nrm[a], be = nrm[b];
        if (al <= thr && be <= thr) continue;
        double* xa = X + (long long)a * mw;
        double* xb = X + (long long)b * mw;
        double ga = 0.0;
        for (int i = lane; i < mw; i += 64) ga += xa[i] * xb[i];
        ga = wave_sum64(ga);
        if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        const double c = 1.0 / sqrt(1.0 + tn * tn), s = c * tn;
        for (int i = lane; i < mw; i += 64) {
          const double u = xa[i], v = xb[i];
          xa[i] = c * u - s * v;
          xb[i] = s * u + c * v;
        }
        double* va = V + (long long)a * nw;
        double* vb = V + (long long)b * nw;
        for (int i = lane; i < nw; i += 64) {
          const double u = va[i], v = vb[i];
          va[i] = c * u - s * v;
          vb[i] = s * u + c * v;
        }
        if (lane == 0) {
          nrm[a] = al - tn * ga;
          nrm[b] = be + tn * ga;
          rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int j = wave; j < nw; j += nwaves) {
    const double* xj = X + (long long)j * mw;
    double s2 = 0.0;
    for (int i = lane; i < mw; i += 64) s2 += xj[i] * xj[i];
    s2 = wave_sum64(s2);
    if (lane == 0) sig[t.sig + j] = sqrt(s2);
  }
  // the emit kernel reads X and V from the work array
  if (x_lds)
    for (long long e = threadIdx.x; e < (long long)mw * nw; e += blockDim.x) Xg[e] = X[e];
  if (v_lds)
    for (long long e = threadIdx.x; e < (long long)nw * nw; e += blockDim.x) Vg[e] = V[e];
}

// The same one-sided Jacobi for blocks too large for one workgroup's LDS, with
// the work of a round spread over the GPU: one launch per round, one wave per
// column pair (all large blocks of the split in the same launch), the squared
// column norms kept in the task's singular-value slots between launches.  The
// pair order, the sums and the rotations are those of k_svd_jacobi, so both
// give the same bits; a block that has had a sweep without rotation takes no
// further part (k_svd_jacobi stops there too).  ctl per large block:
// [0] the rounding-level threshold of the sweep, [1] rotated in this sweep,
// [2] done.
__device__ __forceinline__ void svd_dims(const SvdTask& t, int& mw, int& nw) {
  const bool tr = t.R < t.w;
  mw = tr ? t.w : t.R;
  nw = tr ? t.R : t.w;
}

// X (columns of length mw, transposed when R < w) and V = I into the work array
__global__ __launch_bounds__(256) void k_svd_big_load(const SvdTask* __restrict__ tasks, const int* __restrict__ big,
                                                     const long long* __restrict__ tabs,
                                                     const double* __restrict__ src, double* __restrict__ ws,
                                                     double* __restrict__ ctl) {
  const SvdTask t = tasks[big[blockIdx.y]];
  int mw, nw;
  svd_dims(t, mw, nw);
  const bool tr = t.R < t.w;
  double* X = ws + t.ws;
  double* V = X + (long long)mw * nw;
  const long long* rt = tabs + t.rtab;
  const long long tot = (long long)t.R * t.w, step = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += step) {
    const long long i = e / t.w, j = e - i * t.w;
    const double v = src[rt[i] + j];
    if (!tr) X[i + j * mw] = v;
    else X[j + i * mw] = v;
  }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)nw * nw; e += step)
    V[e] = (e / nw == e % nw) ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl[3 * blockIdx.y + 2] = 0.0;
}

// exact squared column norms (one wave per column) into the singular-value
// slots; fin: their square roots, the singular values
__global__ __launch_bounds__(256) void k_svd_big_norms(const SvdTask* __restrict__ tasks, const int* __restrict__ big,
                                                      const double* __restrict__ ws, double* __restrict__ sig,
                                                      const double* __restrict__ ctl, int fin) {
  const SvdTask t = tasks[big[blockIdx.y]];
  if (!fin && ctl[3 * blockIdx.y + 2] != 0.0) return;
  int mw, nw;
  svd_dims(t, mw, nw);
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nw) return;
  const double* xj = ws + t.ws + (long long)j * mw;
  double s2 = 0.0;
  for (int i = lane; i < mw; i += 64) s2 += xj[i] * xj[i];
  s2 = wave_sum64(s2);
  if (lane == 0) sig[t.sig + j] = fin ? sqrt(s2) : s2;
}

// the sweep's threshold from the norms (summed in column order, one thread) and a cleared rotation flag
__global__ void k_svd_big_thr(const SvdTask* __restrict__ tasks, const int* __restrict__ big,
                              const double* __restrict__ sig, double* __restrict__ ctl) {
  const SvdTask t = tasks[big[blockIdx.x]];
  if (threadIdx.x != 0 || ctl[3 * blockIdx.x + 2] != 0.0) return;
  int mw, nw;
  svd_dims(t, mw, nw);
  double f = 0.0;
  for (int j = 0; j < nw; ++j) f += sig[t.sig + j];
  const double lev = (double)mw * 2.220446049250313e-16;
  ctl[3 * blockIdx.x] = lev * lev * f;
  ctl[3 * blockIdx.x + 1] = 0.0;
}

// one round: wave -> (large block, pair k); pairs[2 q] = index into big, pairs[2 q + 1] = k
__global__ __launch_bounds__(256) void k_svd_big_round(const SvdTask* __restrict__ tasks, const int* __restrict__ big,
                                                      const int* __restrict__ pairs, int npairs, int rd,
                                                      double* __restrict__ ws, double* __restrict__ sig,
                                                      double* __restrict__ ctl) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= npairs) return;
  const int lane = threadIdx.x & 63;
  const int bi = pairs[2 * q], k = pairs[2 * q + 1];
  if (ctl[3 * bi + 2] != 0.0) return;
  const SvdTask t = tasks[big[bi]];
  int mw, nw;
  svd_dims(t, mw, nw);
  const int np = nw + (nw & 1);
  if (rd >= np - 1) return;
  int a = k == 0 ? 0 : 1 + (k + rd) % (np - 1);
  int b = 1 + ((k == 0 ? 0 : np - 1 - k) + rd) % (np - 1);
  if (a > b) { const int x = a; a = b; b = x; }
  if (b >= nw) return;
  double* nrm = sig + t.sig;
  const double al = nrm[a], be = nrm[b], thr = ctl[3 * bi];
  if (al <= thr && be <= thr) return;
  const double tol = 2.220446049250313e-16 * (double)(mw > 16 ? mw : 16);
  double* X = ws + t.ws;
  double* xa = X + (long long)a * mw;
  double* xb = X + (long long)b * mw;
  double ga = 0.0;
  for (int i = lane; i < mw; i += 64) ga += xa[i] * xb[i];
  ga = wave_sum64(ga);
  if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
  const double zeta = (be - al) / (2.0 * ga);
  const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
  const double c = 1.0 / sqrt(1.0 + tn * tn), s = c * tn;
  for (int i = lane; i < mw; i += 64) {
    const double u = xa[i], v = xb[i];
    xa[i] = c * u - s * v;
    xb[i] = s * u + c * v;
  }
  double* V = X + (long long)mw * nw;
  double* va = V + (long long)a * nw;
  double* vb = V + (long long)b * nw;
  for (int i = lane; i < nw; i += 64) {
    const double u = va[i], v = vb[i];
    va[i] = c * u - s * v;
    vb[i] = s * u + c * v;
  }
  if (lane == 0) {
    nrm[a] = al - tn * ga;
    nrm[b] = be + tn * ga;
    ctl[3 * bi + 1] = 1.0;   // every writer stores the same value
  }
}

// after a sweep: a block without a rotation is done
__global__ void k_svd_big_mark(int nbig, double* __restrict__ ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbig && ctl[3 * i + 2] == 0.0 && ctl[3 * i + 1] == 0.0) ctl[3 * i + 2] = 1.0;
}

// M = sum_j s_j u_j v_j^T with unit u_j (R entries) and v_j (w entries), read
// from the Jacobi result: u_j = X_j / s_j, v_j = V_j when R >= w (X = M V);
// u_j = V_j, v_j = X_j / s_j when R < w (X = M^T V).  Written as u to the left
// and s v to the right (left-orthonormal split), or s u and v.
__global__ __launch_bounds__(256) void k_svd_emit(const SvdTask* __restrict__ tasks, const SvdEmit* __restrict__ em,
                                                 const long long* __restrict__ tabs, const double* __restrict__ ws,
                                                 const double* __restrict__ sig, double* __restrict__ Aout,
                                                 double* __restrict__ Bout) {
  const SvdEmit e = em[blockIdx.x];
  const SvdTask t = tasks[e.task];
  const bool tr = t.R < t.w;
  const int mw = tr ? t.w : t.R, nw = tr ? t.R : t.w;
  const double* X = ws + t.ws;
  const double* V = X + (long long)mw * nw;
  for (int mu = 0; mu < e.kappa; ++mu) {
    const int j = (int)tabs[e.sel + mu];
    const double s = sig[t.sig + j];
    const double inv = 1.0 / s;   // only positive singular values are kept
    for (int i = threadIdx.x; i < t.R; i += blockDim.x) {
      const double u = tr ? V[i + (long long)j * nw] : X[i + (long long)j * mw] * inv;
      Aout[tabs[e.atab + i] + mu] = e.left ? u : u * s;
    }
    for (int c = threadIdx.x; c < t.w; c += blockDim.x) {
      const double v = tr ? X[c + (long long)j * mw] * inv : V[c + (long long)j * nw];
      Bout[e.bbase + (long long)mu * e.bstride + c] = e.left ? v * s : v;
    }
  }
}

int svd_lds_doubles() {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    throw Error(TT_EDEVICE, "cannot read the LDS limit");
  return (std::min(lim, kSvdLdsBytes) - 64) / 8;
}

void launch_svd_big(const SvdTask* d_tasks, const int* d_big, int nbig, const int* d_pairs, int npairs, int max_np,
                    const long long* d_tabs, const double* src, double* ws, double* sig, double* ctl,
                    hipStream_t st) {
  if (nbig <= 0) return;
  hipLaunchKernelGGL(k_svd_big_load, dim3(256, nbig), dim3(256), 0, st, d_tasks, d_big, d_tabs, src, ws, ctl);
  HIP_CHECK_LAUNCH();
  // the largest column count among the blocks bounds the norm launch
  const unsigned ncol_blocks = (unsigned)((max_np + 3) / 4);
  std::vector<double> h(3 * (size_t)nbig);
  for (int sw = 0; sw < kSvdMaxSweeps && max_np > 1; ++sw) {
    hipLaunchKernelGGL(k_svd_big_norms, dim3(ncol_blocks, nbig), dim3(256), 0, st, d_tasks, d_big, ws, sig, ctl, 0);
    HIP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_svd_big_thr, dim3(nbig), dim3(64), 0, st, d_tasks, d_big, sig, ctl);
    HIP_CHECK_LAUNCH();
    for (int rd = 0; rd < max_np - 1; ++rd) {
      hipLaunchKernelGGL(k_svd_big_round, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, st, d_tasks, d_big, d_pairs,
                         npairs, rd, ws, sig, ctl);
      HIP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_svd_big_mark, dim3((unsigned)((nbig + 255) / 256)), dim3(256), 0, st, nbig, ctl);
    HIP_CHECK_LAUNCH();
    if (hipMemcpyAsync(h.data(), ctl, 8 * h.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      throw Error(TT_EDEVICE, "SVD: cannot read the sweep flags");
    bool all_done = true;
    for (int i = 0; i < nbig; ++i) all_done = all_done && h[3 * (size_t)i + 2] != 0.0;
    if (all_done) break;
  }
  hipLaunchKernelGGL(k_svd_big_norms, dim3(ncol_blocks, nbig), dim3(256), 0, st, d_tasks, d_big, ws, sig, ctl, 1);
  HIP_CHECK_LAUNCH();
}

void launch_svd(const SvdTask* d_tasks, int ntasks, const int* d_idx, const long long* d_tabs, const double* src,
                double* ws, double* sig, hipStream_t st) {
  if (ntasks <= 0) return;
  // dynamic LDS: the device's per-workgroup limit, at most kSvdLdsBytes, less
  // the kernel's static LDS (two shared scalars)
  static int lds_bytes = -1;
  if (lds_bytes < 0) {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      throw Error(TT_EDEVICE, "cannot read the LDS limit");
    lds_bytes = std::min(lim, kSvdLdsBytes) - 64;
    if (hipFuncSetAttribute((const void*)k_svd_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) !=
        hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the SVD kernel");
  }
  hipLaunchKernelGGL(k_svd_jacobi, dim3(ntasks), dim3(kSvdThreads), lds_bytes, st, d_tasks, d_idx, d_tabs, src, ws,
                     sig, lds_bytes / 8);
  HIP_CHECK_LAUNCH();
}
void launch_svd_emit(const SvdTask* d_tasks, const SvdEmit* d_em, int nem, const long long* d_tabs, const double* ws,
                     const double* sig, double* Aout, double* Bout, hipStream_t st) {
  if (nem <= 0) return;
  hipLaunchKernelGGL(k_svd_emit, dim3(nem), dim3(256), 0, st, d_tasks, d_em, d_tabs, ws, sig, Aout, Bout);
  HIP_CHECK_LAUNCH();
}

}  // namespace tt
