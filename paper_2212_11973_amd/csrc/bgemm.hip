// Large-tile split-BF16 GEMM of the dense effective-Hamiltonian apply
// (SM Fig. optimalB(c): L.A and .R of one site, operands dense).
//
// C(m, n) = sum_k A(m, k) B(n, k), both operands held as NP BF16 planes
// (x ~ part 0 + part 1 (+ part 2), each rounded to nearest) with rows
// contiguous in k and zero-padded to a multiple of 32.  The products of the
// parts that the precision keeps (x3: 00, 01, 10; x6: also 02, 11, 20) are
// taken with the gfx950 BF16 MFMA 16x16x32 into FP32 accumulators, which are
// added into FP64 accumulators every kFold K tiles, so the FP32 sums stay
// short at any K.
//
// One 128 x 128 output tile per workgroup of four waves (2 x 2, 64 x 64 each,
// 4 x 4 MFMA blocks).  K tiles of 32 go global -> LDS directly (one 16-byte
// global_load_lds per lane, no register staging) into a ring of S stages, S - 1
// tiles ahead of the one being multiplied.  An LDS row is 64 bytes (four
// 16-byte chunks); chunk c of row r sits at position c ^ ((r >> 2) & 3), so the
// 16 rows an MFMA operand read touches fall in distinct banks.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace tt {

extern long long g_launches;

namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

#ifndef TT_BG_FOLD
#define TT_BG_FOLD 8
#endif
#ifndef TT_BG_GROUP_M
#define TT_BG_GROUP_M 8
#endif
#ifndef TT_BG_STAGES2
#define TT_BG_STAGES2 2
#endif
#ifndef TT_BG_WPE2
#define TT_BG_WPE2 2
#endif
constexpr int kBM = 128, kBN = 128, kBK = 32;
constexpr int kRowBytes = kBK * 2;             // one LDS row of one plane
constexpr int kFold = TT_BG_FOLD;              // K tiles between FP64 folds
constexpr int kGroupM = TT_BG_GROUP_M;         // tile rows per raster group

#ifndef TT_BG_BM2
#define TT_BG_BM2 128
#endif
template <int NP> struct BgTraits;
// BM: tile rows (BM / 32 waves, 64 x 64 each); S: LDS stages; WPE: waves per SIMD
template <> struct BgTraits<2> { static constexpr int BM = TT_BG_BM2, S = TT_BG_STAGES2, WPE = TT_BG_WPE2; };
template <> struct BgTraits<3> { static constexpr int BM = 128, S = 3, WPE = 1; };
template <int NP> constexpr int bg_waves() { return BgTraits<NP>::BM / 32; }
template <int NP> constexpr int bg_stage_bytes() { return NP * (BgTraits<NP>::BM + kBN) * kRowBytes; }
template <int NP> constexpr int bg_lds_bytes() { return BgTraits<NP>::S * bg_stage_bytes<NP>(); }

// s_waitcnt immediate: vmcnt(n), other counters left alone (gfx9 encoding)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

template <int NP>
__device__ __forceinline__ void bg_split(double x, __bf16* out) {
  const __bf16 h = (__bf16)(float)x;
  out[0] = h;
  const double r = x - (double)(float)h;
  const __bf16 m = (__bf16)(float)r;
  out[1] = m;
  if (NP == 3) out[2] = (__bf16)(float)(r - (double)(float)m);
}

__device__ __forceinline__ int bg_xcd_block(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, slot = b >> 3;
  return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// One K tile (all planes of both operands) into LDS stage `st`.  Wave w loads
// rows 32w .. 32w + 31 of the A and B tiles, 16 rows per instruction: lane l
// takes row 16 j + l / 4 of its group and the logical chunk that lands at
// position l % 4.
template <int NP>
__device__ __forceinline__ void bg_issue(const BgArgs& g, char* lds, int st, int kt, int m0, int n0, int wave,
                                         int lane) {
  constexpr int BM = BgTraits<NP>::BM, BROWS = kBN / bg_waves<NP>();   // B rows per wave
  char* base = lds + st * bg_stage_bytes<NP>();
  const int lc = (lane & 3) ^ (lane >> 4);
  const long long k = (long long)kt * kBK + 8 * lc;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int row = 32 * wave + 16 * j + (lane >> 2);
    const int ma = min(m0 + row, g.M - 1);
    const __bf16* ga = g.A + (long long)ma * g.lda + k;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      char* la = base + (p * BM + 32 * wave + 16 * j) * kRowBytes;
      __builtin_amdgcn_global_load_lds((const void*)(ga + p * g.sa), (lds_void*)la, 16, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < BROWS / 16; ++j) {
    const int row = BROWS * wave + 16 * j + (lane >> 2);
    const int nb = min(n0 + row, g.N - 1);
    const __bf16* gb = g.B + (long long)nb * g.ldb + k;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      char* lb = base + (NP * BM + p * kBN + BROWS * wave + 16 * j) * kRowBytes;
      __builtin_amdgcn_global_load_lds((const void*)(gb + p * g.sb), (lds_void*)lb, 16, 0, 0);
    }
  }
}

typedef float float16_t __attribute__((ext_vector_type(16)));

// Products of one 32-deep K step for one output block: x3 takes 00, 01, 10
// (smallest first), x6 also 02, 11, 20.
template <int NP, typename ACC, typename MF>
__device__ __forceinline__ ACC bg_products(const bf16x8_t (&a)[NP], const bf16x8_t (&b)[NP], ACC t, MF mf) {
  if constexpr (NP == 3) {
    t = mf(a[2], b[0], t);
    t = mf(a[1], b[1], t);
    t = mf(a[0], b[2], t);
  }
  t = mf(a[1], b[0], t);
  t = mf(a[0], b[1], t);
  t = mf(a[0], b[0], t);
  return t;
}

// The 64 x 64 output of a wave as 2 x 2 blocks of the 32x32x16 MFMA: per
// 16-deep step lane l supplies row (l % 32) of an A block and column (l % 32)
// of a B block at k = 8 (l / 32) .. + 7; accumulator element v of a block sits
// at row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
template <int NP>
__global__ __launch_bounds__(64 * bg_waves<NP>()) __attribute__((amdgpu_waves_per_eu(BgTraits<NP>::WPE, BgTraits<NP>::WPE))) void k_bgemm(BgArgs g) {
  extern __shared__ __attribute__((aligned(16))) char bg_lds[];
  constexpr int S = BgTraits<NP>::S, BM = BgTraits<NP>::BM;
  constexpr int LPS = NP * (2 + kBN / bg_waves<NP>() / 16);   // global_load_lds per wave per stage
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;

  // XCD-contiguous block ranges, then a grouped raster (kGroupM tile rows)
  const int ntiles = g.tiles_m * g.tiles_n;
  const int blk = bg_xcd_block(blockIdx.x, ntiles);
  const int per_group = kGroupM * g.tiles_n;
  const int grp = blk / per_group, first = grp * kGroupM;
  const int gsz = min(g.tiles_m - first, kGroupM);
  const int in = blk - grp * per_group;
  const int tm = first + in % gsz, tn = in / gsz;
  const int m0 = tm * BM, n0 = tn * kBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  double acc[2][2][16];
  float16_t part[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0;
      part[i][j] = (float16_t){};
    }

  const int nk = g.K / kBK;
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < nk) bg_issue<NP>(g, bg_lds, s, s, m0, n0, wave, lane);

  // read positions of this lane's chunk (2 s + h) of row r in the two 16-deep steps
  const int rpos0 = r * kRowBytes + 16 * ((0 + h) ^ ((r >> 2) & 3));
  const int rpos1 = r * kRowBytes + 16 * ((2 + h) ^ ((r >> 2) & 3));
  auto mf = [](bf16x8_t x, bf16x8_t y, float16_t t) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, t, 0, 0, 0); };
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's loads of tile kt are done once at most the later issued
    // stages are outstanding
    if (kt + S - 2 < nk) __builtin_amdgcn_s_waitcnt(vmcnt_imm((S - 2) * LPS));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    // every wave's loads of tile kt landed and stage (kt - 1) % S is read:
    // a bare barrier (a fenced one would also wait for the later stages'
    // loads), with the compiler kept from moving memory accesses across it
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kt + S - 1 < nk) bg_issue<NP>(g, bg_lds, (kt + S - 1) % S, kt + S - 1, m0, n0, wave, lane);
    const char* base = bg_lds + (kt % S) * bg_stage_bytes<NP>();
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int rp = st ? rpos1 : rpos0;
      bf16x8_t a[2][NP], b[2][NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i][p] = *reinterpret_cast<const bf16x8_t*>(base + (p * BM + wm + 32 * i) * kRowBytes + rp);
          b[i][p] = *reinterpret_cast<const bf16x8_t*>(base + (NP * BM + p * kBN + wn + 32 * i) * kRowBytes + rp);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) part[i][j] = bg_products<NP>(a[i], b[j], part[i][j], mf);
    }
    if ((kt + 1) % kFold == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[i][j][v] += (double)part[i][j][v];
          part[i][j] = (float16_t){};
        }
    }
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
      if (m >= g.M) continue;
      const long long row = (long long)(m / g.cdiv) * g.ldc1 + (long long)(m % g.cdiv) * g.ldc0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn + 32 * j + r;
        if (n >= g.N) continue;
        const double val = acc[i][j][v];
        if (g.cplanes) {
          __bf16 parts[3];
          bg_split<NP>(val, parts);
          __bf16* c = reinterpret_cast<__bf16*>(g.C) + row + n;
#pragma unroll
          for (int p = 0; p < NP; ++p) c[p * g.sc] = parts[p];
        } else {
          reinterpret_cast<double*>(g.C)[row + n] = val;
        }
      }
    }
}

// bf16x3 with wider waves: each wave's 64 x 128 output as 2 x 4 blocks of the
// 32x32x16 MFMA with FP32 accumulation over the whole K (the three part
// products of a 16-deep step added smallest first), eight waves on a
// 256 x 256 tile, two LDS stages of 64 KB.  Against the 64 x 64 waves with
// FP64 folding it reads a quarter less LDS and half the global data per flop.
#ifndef TT_BG_WIDE2
#define TT_BG_WIDE2 1
#endif
constexpr int kWBM = 256, kWBN = 256, kWStage = 2 * (kWBM + kWBN) * kRowBytes;

__device__ __forceinline__ void bgw_issue(const BgArgs& g, char* lds, int st, int kt, int m0, int n0, int wave,
                                          int lane) {
  char* base = lds + st * kWStage;
  const int lc = (lane & 3) ^ (lane >> 4);
  const long long k = (long long)kt * kBK + 8 * lc;
#pragma unroll
  for (int j = 0; j < 2; ++j) {   // 32 rows of A and of B per wave, 16 per instruction
    const int row = 32 * wave + 16 * j + (lane >> 2);
    const int ma = min(m0 + row, g.M - 1), nb = min(n0 + row, g.N - 1);
    const __bf16* ga = g.A + (long long)ma * g.lda + k;
    const __bf16* gb = g.B + (long long)nb * g.ldb + k;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      char* la = base + (p * kWBM + 32 * wave + 16 * j) * kRowBytes;
      char* lb = base + (2 * kWBM + p * kWBN + 32 * wave + 16 * j) * kRowBytes;
      __builtin_amdgcn_global_load_lds((const void*)(ga + p * g.sa), (lds_void*)la, 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(gb + p * g.sb), (lds_void*)lb, 16, 0, 0);
    }
  }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_bgemm_wide(BgArgs g) {
  extern __shared__ __attribute__((aligned(16))) char bgw_lds[];
  constexpr int LPS = 8;   // global_load_lds per wave per stage
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int ntiles = g.tiles_m * g.tiles_n;
  const int blk = bg_xcd_block(blockIdx.x, ntiles);
  const int per_group = kGroupM * g.tiles_n;
  const int grp = blk / per_group, first = grp * kGroupM;
  const int gsz = min(g.tiles_m - first, kGroupM);
  const int in = blk - grp * per_group;
  const int tm = first + in % gsz, tn = in / gsz;
  const int m0 = tm * kWBM, n0 = tn * kWBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;

  float16_t part[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) part[i][j] = (float16_t){};

  const int nk = g.K / kBK;
  if (nk > 0) bgw_issue(g, bgw_lds, 0, 0, m0, n0, wave, lane);
  const int rpos0 = r * kRowBytes + 16 * ((0 + h) ^ ((r >> 2) & 3));
  const int rpos1 = r * kRowBytes + 16 * ((2 + h) ^ ((r >> 2) & 3));
  auto mf = [](bf16x8_t x, bf16x8_t y, float16_t t) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, t, 0, 0, 0); };
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // this wave's loads of tile kt
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kt + 1 < nk) bgw_issue(g, bgw_lds, (kt + 1) & 1, kt + 1, m0, n0, wave, lane);
    const char* base = bgw_lds + (kt & 1) * kWStage;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int rp = st ? rpos1 : rpos0;
      bf16x8_t a[2][2], b[4][2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          a[i][p] = *reinterpret_cast<const bf16x8_t*>(base + (p * kWBM + wm + 32 * i) * kRowBytes + rp);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[j][p] = *reinterpret_cast<const bf16x8_t*>(base + (2 * kWBM + p * kWBN + wn + 32 * j) * kRowBytes + rp);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[i][j] = bg_products<2>(a[i], b[j], part[i][j], mf);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
      if (m >= g.M) continue;
      const long long row = (long long)(m / g.cdiv) * g.ldc1 + (long long)(m % g.cdiv) * g.ldc0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn + 32 * j + r;
        if (n >= g.N) continue;
        const double val = part[i][j][v];
        if (g.cplanes) {
          __bf16 parts[3];
          bg_split<2>(val, parts);
          __bf16* c = reinterpret_cast<__bf16*>(g.C) + row + n;
          c[0] = parts[0];
          c[g.sc] = parts[1];
        } else {
          reinterpret_cast<double*>(g.C)[row + n] = val;
        }
      }
    }
}

// out[p][r * ldo + k] = part p of x[r * ldx + k] for k < K, zero for K <= k < ldo
template <int NP>
__global__ __launch_bounds__(256) void k_split_rows(const double* __restrict__ x, long long rows, int K, long long ldx,
                                                   __bf16* __restrict__ out, long long ldo, long long plane) {
  const long long n = rows * ldo;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long rr = e / ldo, k = e - rr * ldo;
    __bf16 parts[3] = {(__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
    if (k < K) bg_split<NP>(x[rr * ldx + k], parts);
#pragma unroll
    for (int p = 0; p < NP; ++p) out[p * plane + e] = parts[p];
  }
}

// transposed: out[p][c * ldo + k] = part p of x[k * C + c] for k < K, zero for
// K <= k < ldo; 32 x 32 tiles through LDS
template <int NP>
__global__ __launch_bounds__(256) void k_split_t(const double* __restrict__ x, int K, int C, __bf16* __restrict__ out,
                                                long long ldo, long long plane) {
  __shared__ double t[32][33];
  const int k0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = k0 + ty + 8 * i, c = c0 + tx;
    t[ty + 8 * i][tx] = (k < K && c < C) ? x[(long long)k * C + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = c0 + ty + 8 * i, k = k0 + tx;
    if (c < C && k < ldo) {
      __bf16 parts[3];
      bg_split<NP>(t[tx][ty + 8 * i], parts);
#pragma unroll
      for (int p = 0; p < NP; ++p) out[p * plane + (long long)c * ldo + k] = parts[p];
    }
  }
}

constexpr int kWsMaxO = 80;   // 4 DH at most

// ------------------------------------------------------------------ FP64
// The same tiling for FP64 operands (the FP64 dense apply): K tiles of 16
// doubles, an LDS row of 128 bytes (eight 16-byte chunks) with chunk c of row r
// at position c ^ ((r >> 1) & 7), which keeps the 16 rows x 4 k of an f64 MFMA
// operand read conflict-free; each wave 4 x 4 blocks of the f64 MFMA 16x16x4
// (lane (r, g) supplies row r at k = g; accumulator element v at row g + 4 v,
// column r).  Two stages of 32 KB: two workgroups per CU.
constexpr int kDBK = 16, kDRowBytes = kDBK * 8, kDS = 2;
constexpr int kDStage = (kBM + kBN) * kDRowBytes;

__device__ __forceinline__ void dg_issue(const DgArgs& g, char* lds, int st, int kt, int m0, int n0, int wave,
                                         int lane) {
  char* base = lds + st * kDStage;
#pragma unroll
  for (int j = 0; j < 4; ++j) {   // 8 rows x 8 chunks per instruction: lane l -> row l / 8, position l % 8
    const int row = 32 * wave + 8 * j + (lane >> 3);
    const int lc = (lane & 7) ^ ((row >> 1) & 7);
    const long long k = (long long)kt * kDBK + 2 * lc;
    const int ma = min(m0 + row, g.M - 1), nb = min(n0 + row, g.N - 1);
    char* la = base + (32 * wave + 8 * j) * kDRowBytes;
    char* lb = base + (kBM + 32 * wave + 8 * j) * kDRowBytes;
    __builtin_amdgcn_global_load_lds((const void*)(g.A + (long long)ma * g.lda + k), (lds_void*)la, 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(g.B + (long long)nb * g.ldb + k), (lds_void*)lb, 16, 0, 0);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_dgemm(DgArgs g) {
  extern __shared__ __attribute__((aligned(16))) char dg_lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int ntiles = g.tiles_m * g.tiles_n;
  const int blk = bg_xcd_block(blockIdx.x, ntiles);
  const int per_group = kGroupM * g.tiles_n;
  const int grp = blk / per_group, first = grp * kGroupM;
  const int gsz = min(g.tiles_m - first, kGroupM);
  const int in = blk - grp * per_group;
  const int tm = first + in % gsz, tn = in / gsz;
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  double4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  const int nk = g.K / kDBK;
  if (nk > 0) dg_issue(g, dg_lds, 0, 0, m0, n0, wave, lane);
  // this lane's operand element of step t (k = 4 t + q): chunk 2 t + q / 2, half q % 2
  const int rsw = (r >> 1) & 7;
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // this wave's loads of tile kt
    // every wave's loads of tile kt landed and the other stage is read (a bare
    // barrier: a fenced one waits the same way; memory accesses kept on their side)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kt + 1 < nk) dg_issue(g, dg_lds, (kt + 1) & 1, kt + 1, m0, n0, wave, lane);
    const char* base = dg_lds + (kt & 1) * kDStage;
#pragma unroll
    for (int t = 0; t < kDBK / 4; ++t) {
      const int off = r * kDRowBytes + 16 * ((2 * t + (q >> 1)) ^ rsw) + 8 * (q & 1);
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = *reinterpret_cast<const double*>(base + (wm + 16 * i) * kDRowBytes + off);
        b[i] = *reinterpret_cast<const double*>(base + (kBM + wn + 16 * i) * kDRowBytes + off);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm + 16 * i + q + 4 * v;
      if (m >= g.M) continue;
      const long long row = (long long)(m / g.cdiv) * g.ldc1 + (long long)(m % g.cdiv) * g.ldc0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn + 16 * j + r;
        if (n < g.N) g.C[row + n] = acc[i][j][v];
      }
    }
}

// FP32 operands (the FP32 dense apply): the same tiles with K tiles of 32
// floats (128-byte LDS rows, the same chunk positions).  Each wave's 64 x 64 as
// 2 x 2 blocks of the f32 MFMA 32x32x2 (lane l supplies row l % 32 at
// k = l / 32 of each step; accumulator element v at row 8 (v / 4) + 4 (l / 32)
// + v % 4, column l % 32); on step 4 c + s lane half h takes k = 8 c + 4 h + s,
// so each lane reads one 16-byte chunk per operand block and 8 k, and both
// operands pair the same k.  The FP32 partials are added into FP64
// accumulators every kFold K tiles.
constexpr int kSBK = 32;

__device__ __forceinline__ void sg_issue(const SgArgs& g, char* lds, int st, int kt, int m0, int n0, int wave,
                                         int lane) {
  char* base = lds + st * kDStage;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = 32 * wave + 8 * j + (lane >> 3);
    const int lc = (lane & 7) ^ ((row >> 1) & 7);
    const long long k = (long long)kt * kSBK + 4 * lc;
    const int ma = min(m0 + row, g.M - 1), nb = min(n0 + row, g.N - 1);
    char* la = base + (32 * wave + 8 * j) * kDRowBytes;
    char* lb = base + (kBM + 32 * wave + 8 * j) * kDRowBytes;
    __builtin_amdgcn_global_load_lds((const void*)(g.A + (long long)ma * g.lda + k), (lds_void*)la, 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(g.B + (long long)nb * g.ldb + k), (lds_void*)lb, 16, 0, 0);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sgemm(SgArgs g) {
  extern __shared__ __attribute__((aligned(16))) char sg_lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int ntiles = g.tiles_m * g.tiles_n;
  const int blk = bg_xcd_block(blockIdx.x, ntiles);
  const int per_group = kGroupM * g.tiles_n;
  const int grp = blk / per_group, first = grp * kGroupM;
  const int gsz = min(g.tiles_m - first, kGroupM);
  const int in = blk - grp * per_group;
  const int tm = first + in % gsz, tn = in / gsz;
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  double acc[2][2][16];
  float16_t part[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0;
      part[i][j] = (float16_t){};
    }

  const int nk = g.K / kSBK;
  if (nk > 0) sg_issue(g, sg_lds, 0, 0, m0, n0, wave, lane);
  const int rsw = (r >> 1) & 7;
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // this wave's loads of tile kt
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kt + 1 < nk) sg_issue(g, sg_lds, (kt + 1) & 1, kt + 1, m0, n0, wave, lane);
    const char* base = sg_lds + (kt & 1) * kDStage;
#pragma unroll 2
    for (int c = 0; c < 4; ++c) {
      const int off = r * kDRowBytes + 16 * ((2 * c + h) ^ rsw);
      float4_t a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const float4_t*>(base + (wm + 32 * i) * kDRowBytes + off);
        b[i] = *reinterpret_cast<const float4_t*>(base + (kBM + wn + 32 * i) * kDRowBytes + off);
      }
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            part[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][st], b[j][st], part[i][j], 0, 0, 0);
    }
    if ((kt + 1) % kFold == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[i][j][v] += (double)part[i][j][v];
          part[i][j] = (float16_t){};
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
      if (m >= g.M) continue;
      const long long row = (long long)(m / g.cdiv) * g.ldc1 + (long long)(m % g.cdiv) * g.ldc0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn + 32 * j + r;
        if (n >= g.N) continue;
        if (g.cfloat) reinterpret_cast<float*>(g.C)[row + n] = (float)acc[i][j][v];
        else reinterpret_cast<double*>(g.C)[row + n] = acc[i][j][v];
      }
    }
}

// out[r * ldo + k] = x[r * ldx + k] for k < K, zero for K <= k < ldo (TO: double, or float rounded to nearest)
template <typename TO>
__global__ __launch_bounds__(256) void k_pad_rows(const double* __restrict__ x, long long rows, int K, long long ldx,
                                                 TO* __restrict__ out, long long ldo) {
  const long long n = rows * ldo;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long rr = e / ldo, k = e - rr * ldo;
    out[e] = k < K ? (TO)x[rr * ldx + k] : (TO)0;
  }
}

// out[c * ldo + k] = x[k * C + c] for k < K, zero for K <= k < ldo (32 x 32 tiles through LDS)
template <typename TO>
__global__ __launch_bounds__(256) void k_pad_t(const double* __restrict__ x, int K, int C, TO* __restrict__ out,
                                              long long ldo) {
  __shared__ double t[32][33];
  const int k0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = k0 + ty + 8 * i, c = c0 + tx;
    t[ty + 8 * i][tx] = (k < K && c < C) ? x[(long long)k * C + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = c0 + ty + 8 * i, k = k0 + tx;
    if (c < C && k < ldo) out[(long long)c * ldo + k] = (TO)t[tx][ty + 8 * i];
  }
}

// The dense apply's W stage on the matrix cores: for each (x', sp) the product
// T2[(o = DH so + b)][y] = sum_(k = 4 a + si) W^T[o][k] T1[k][y] with W^T as
// the A operand (from LDS: rows o padded to kWsMaxO with zeros) and T1 as the
// B operand straight from memory (lane (r, g) takes k = 4 t + g, i.e. a = t,
// si = g, at y = y0 + r: 128-byte rows), so the result rows o come out as
// 128-byte runs of y.  NP = 0: FP64 T1 and T2 (f64 MFMA 16x16x4); NP = 1: FP32
// T1 and T2; NP = 2, 3: BF16 planes; NP >= 1 multiply in FP32 (f32 MFMA
// 16x16x4, W rounded to FP32, the parts of a T1 element summed smallest first).  T2's K padding is written as
// zeros.  One workgroup per (x', sp); a wave takes kWsYB adjacent blocks of
// 16 y at a time (their loads in flight together, each W operand read once
// for all of them), the four waves every fourth such group.  Measured at
// D = 2000: FP64 5.7 ms with two blocks (7.3 with one, 8.7 with four, where
// the accumulators leave one wave per SIMD), planes 4.3 ms with four (4.8 with one).
template <int NP>
__global__ __launch_bounds__(256) void k_wstage_mfma(const void* __restrict__ T1v, long long sT1,
                                                     const double* __restrict__ W, int DH, int Dl, int Dr,
                                                     void* __restrict__ T2v, long long sT2, long long kp3) {
  constexpr int kWsYB = NP == 0 ? 2 : 4;
  using E = typename std::conditional<NP == 0, double, float>::type;
  using E4 = typename std::conditional<NP == 0, double4_t, float4_t>::type;
  constexpr int OB = kWsMaxO / 16;
  __shared__ E wl[kWsMaxO * kWsMaxO];   // wl[k][o]
  const int KO = 4 * DH;
  for (int e = threadIdx.x; e < kWsMaxO * kWsMaxO; e += 256) {
    const int k = e / kWsMaxO, o = e - k * kWsMaxO;
    E v = 0;
    if (k < KO && o < KO) {
      const int a = k >> 2, si = k & 3, so = o / DH, b = o - so * DH;
      v = (E)W[((a * 4 + so) * 4 + si) * DH + b];
    }
    wl[e] = v;
  }
  const int x = blockIdx.x >> 2, sp = blockIdx.x & 3;
  const long long used = (long long)DH * Dr;
  for (int y = threadIdx.x; y < kp3 - used; y += 256)   // the K padding of this (x', sp)'s four T2 rows
#pragma unroll
    for (int so = 0; so < 4; ++so) {
      const long long e = (long long)(16 * x + 4 * so + sp) * kp3 + used + y;
      if constexpr (NP == 0) reinterpret_cast<double*>(T2v)[e] = 0.0;
      else if constexpr (NP == 1) reinterpret_cast<float*>(T2v)[e] = 0.f;
      else
#pragma unroll
        for (int p = 0; p < NP; ++p) reinterpret_cast<__bf16*>(T2v)[p * sT2 + e] = (__bf16)0.f;
    }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  const int nob = (KO + 15) / 16;
  const long long N1 = 16LL * Dr;
  // this lane's B element for a = t: T1[t][x'][g][sp][y]
  const long long base = (long long)x * N1 + (long long)g * 4 * Dr + (long long)sp * Dr;
  const long long astep = (long long)Dl * N1;
  for (int yb0 = kWsYB * wave; 16 * yb0 < Dr; yb0 += 4 * kWsYB) {
    E4 acc[kWsYB][OB];
#pragma unroll
    for (int s = 0; s < kWsYB; ++s)
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) acc[s][ob] = (E4){0, 0, 0, 0};
#pragma unroll 2
    for (int t = 0; t < DH; ++t) {
      E bv[kWsYB];
#pragma unroll
      for (int s = 0; s < kWsYB; ++s) {
        const long long e = base + t * astep + min(16 * (yb0 + s) + r, Dr - 1);
        if constexpr (NP == 0) {
          bv[s] = reinterpret_cast<const double*>(T1v)[e];
        } else if constexpr (NP == 1) {
          bv[s] = reinterpret_cast<const float*>(T1v)[e];
        } else {
          const __bf16* t1 = reinterpret_cast<const __bf16*>(T1v);
          float f = 0.f;
#pragma unroll
          for (int p = NP - 1; p >= 0; --p) f += (float)t1[p * sT1 + e];
          bv[s] = f;
        }
      }
      const E* wr = wl + (4 * t + g) * kWsMaxO + r;
#pragma unroll
      for (int ob = 0; ob < OB; ++ob)
        if (ob < nob) {
          const E wv = wr[16 * ob];
#pragma unroll
          for (int s = 0; s < kWsYB; ++s) {
            if constexpr (NP == 0) acc[s][ob] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv, bv[s], acc[s][ob], 0, 0, 0);
            else acc[s][ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv, bv[s], acc[s][ob], 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int s = 0; s < kWsYB; ++s) {
      const int y = 16 * (yb0 + s) + r;
      if (y >= Dr) continue;
#pragma unroll
      for (int ob = 0; ob < OB; ++ob)
        if (ob < nob)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // accumulator row: g + 4 v (f64 MFMA), 4 g + v (f32 MFMA)
            const int o = 16 * ob + (NP == 0 ? g + 4 * v : 4 * g + v);
            if (o >= KO) continue;
            const int so = o / DH, b = o - so * DH;
            const long long e = (long long)(16 * x + 4 * so + sp) * kp3 + (long long)b * Dr + y;
            if constexpr (NP == 0) {
              reinterpret_cast<double*>(T2v)[e] = acc[s][ob][v];
            } else if constexpr (NP == 1) {
              reinterpret_cast<float*>(T2v)[e] = acc[s][ob][v];
            } else {
              __bf16 parts[3];
              bg_split<NP>((double)acc[s][ob][v], parts);
#pragma unroll
              for (int p = 0; p < NP; ++p) reinterpret_cast<__bf16*>(T2v)[p * sT2 + e] = parts[p];
            }
          }
    }
  }
}

template <int NP>
void bgemm_np(BgArgs a, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_bgemm<NP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            bg_lds_bytes<NP>()) != hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the split-BF16 GEMM");
    attr = true;
  }
  a.tiles_m = (a.M + BgTraits<NP>::BM - 1) / BgTraits<NP>::BM;
  a.tiles_n = (a.N + kBN - 1) / kBN;
  TT_REQUIRE((long long)a.tiles_m * a.tiles_n < (1LL << 31), TT_EINVAL, "bgemm: too many tiles");
  hipLaunchKernelGGL(k_bgemm<NP>, dim3(a.tiles_m * a.tiles_n), dim3(64 * bg_waves<NP>()), bg_lds_bytes<NP>(), st, a);
}

}  // namespace

int bgemm_kpad(long long K) { return (int)((K + kBK - 1) / kBK * kBK); }

void launch_bgemm(BgArgs a, int precision, hipStream_t st) {
  TT_REQUIRE(precision == TT_BF16X3 || precision == TT_BF16X6, TT_EINVAL, "bgemm: split-BF16 precisions only");
  TT_REQUIRE(a.M >= 1 && a.N >= 1 && a.K >= kBK && a.K % kBK == 0, TT_EINVAL, "bgemm: K must be a positive multiple of 32");
  TT_REQUIRE(a.lda >= a.K && a.ldb >= a.K && a.lda % 8 == 0 && a.ldb % 8 == 0 && a.sa % 8 == 0 && a.sb % 8 == 0,
             TT_EINVAL, "bgemm: operand rows must hold K and start 16-byte aligned");
  TT_REQUIRE(a.cdiv >= 1, TT_EINVAL, "bgemm: bad row map");
  TT_REQUIRE(((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0, TT_EINVAL, "bgemm: operands not 16-byte aligned");
  // the 256 x 256 tiles only when they give every CU one: below that the
  // 128 x 128 form's four times as many workgroups win
  const long long wide_tiles = (long long)((a.M + kWBM - 1) / kWBM) * ((a.N + kWBN - 1) / kWBN);
  if (precision == TT_BF16X3 && TT_BG_WIDE2 && wide_tiles >= 256) {
    static bool attr = false;
    if (!attr) {
      if (hipFuncSetAttribute((const void*)k_bgemm_wide, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kWStage) !=
          hipSuccess)
        throw Error(TT_EDEVICE, "cannot set the LDS limit of the split-BF16 GEMM");
      attr = true;
    }
    a.tiles_m = (a.M + kWBM - 1) / kWBM;
    a.tiles_n = (a.N + kWBN - 1) / kWBN;
    TT_REQUIRE((long long)a.tiles_m * a.tiles_n < (1LL << 31), TT_EINVAL, "bgemm: too many tiles");
    hipLaunchKernelGGL(k_bgemm_wide, dim3(a.tiles_m * a.tiles_n), dim3(512), 2 * kWStage, st, a);
  } else if (precision == TT_BF16X3) {
    bgemm_np<2>(a, st);
  } else {
    bgemm_np<3>(a, st);
  }
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

int wstage_planes_max_dh() { return kWsMaxO / 4; }

void launch_wstage_planes(const void* T1, long long sT1, const double* W, int DH, int Dl, int Dr, void* T2, long long sT2,
                          long long kp3, int precision, hipStream_t st) {
  TT_REQUIRE(precision == TT_BF16X3 || precision == TT_BF16X6, TT_EINVAL, "W stage: split-BF16 precisions only");
  TT_REQUIRE(DH >= 1 && 4 * DH <= kWsMaxO && Dl >= 1 && Dr >= 1 && 4LL * Dl < 65536 && kp3 >= (long long)DH * Dr &&
                 kp3 - (long long)DH * Dr <= 256,
             TT_EINVAL, "W stage: shape out of range");
  const dim3 grid((unsigned)(4 * Dl));
  if (precision == TT_BF16X3)
    hipLaunchKernelGGL(k_wstage_mfma<2>, grid, dim3(256), 0, st, T1, sT1, W, DH, Dl, Dr, T2, sT2, kp3);
  else
    hipLaunchKernelGGL(k_wstage_mfma<3>, grid, dim3(256), 0, st, T1, sT1, W, DH, Dl, Dr, T2, sT2, kp3);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

int dgemm_kpad(long long K) { return (int)((K + kDBK - 1) / kDBK * kDBK); }

void launch_dgemm(DgArgs a, hipStream_t st) {
  TT_REQUIRE(a.M >= 1 && a.N >= 1 && a.K >= kDBK && a.K % kDBK == 0, TT_EINVAL,
             "dgemm: K must be a positive multiple of 16");
  TT_REQUIRE(a.lda >= a.K && a.ldb >= a.K && a.lda % 2 == 0 && a.ldb % 2 == 0 && a.cdiv >= 1, TT_EINVAL,
             "dgemm: operand rows must hold K and start 16-byte aligned");
  TT_REQUIRE(((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0, TT_EINVAL, "dgemm: operands not 16-byte aligned");
  a.tiles_m = (a.M + kBM - 1) / kBM;
  a.tiles_n = (a.N + kBN - 1) / kBN;
  TT_REQUIRE((long long)a.tiles_m * a.tiles_n < (1LL << 31), TT_EINVAL, "dgemm: too many tiles");
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_dgemm, hipFuncAttributeMaxDynamicSharedMemorySize, kDS * kDStage) !=
        hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the FP64 GEMM");
    attr = true;
  }
  hipLaunchKernelGGL(k_dgemm, dim3(a.tiles_m * a.tiles_n), dim3(256), kDS * kDStage, st, a);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

int sgemm_kpad(long long K) { return (int)((K + kSBK - 1) / kSBK * kSBK); }

void launch_sgemm(SgArgs a, hipStream_t st) {
  TT_REQUIRE(a.M >= 1 && a.N >= 1 && a.K >= kSBK && a.K % kSBK == 0, TT_EINVAL,
             "sgemm: K must be a positive multiple of 32");
  TT_REQUIRE(a.lda >= a.K && a.ldb >= a.K && a.lda % 4 == 0 && a.ldb % 4 == 0 && a.cdiv >= 1, TT_EINVAL,
             "sgemm: operand rows must hold K and start 16-byte aligned");
  TT_REQUIRE(((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0, TT_EINVAL, "sgemm: operands not 16-byte aligned");
  a.tiles_m = (a.M + kBM - 1) / kBM;
  a.tiles_n = (a.N + kBN - 1) / kBN;
  TT_REQUIRE((long long)a.tiles_m * a.tiles_n < (1LL << 31), TT_EINVAL, "sgemm: too many tiles");
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_sgemm, hipFuncAttributeMaxDynamicSharedMemorySize, kDS * kDStage) !=
        hipSuccess)
      throw Error(TT_EDEVICE, "cannot set the LDS limit of the FP32 GEMM");
    attr = true;
  }
  hipLaunchKernelGGL(k_sgemm, dim3(a.tiles_m * a.tiles_n), dim3(256), kDS * kDStage, st, a);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

template <typename TO>
void pad_rows_t(const double* x, long long rows, int K, long long ldx, TO* out, long long ldo, hipStream_t st) {
  TT_REQUIRE(ldo >= K && ldx >= K, TT_EINVAL, "pad: rows shorter than K");
  const long long n = rows * ldo;
  if (n <= 0) return;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_pad_rows<TO>, dim3(blocks), dim3(256), 0, st, x, rows, K, ldx, out, ldo);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}
template <typename TO>
void pad_t_t(const double* x, int K, int C, TO* out, long long ldo, hipStream_t st) {
  TT_REQUIRE(ldo >= K && K >= 1 && C >= 1, TT_EINVAL, "pad: bad shape");
  const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((ldo + 31) / 32));
  hipLaunchKernelGGL(k_pad_t<TO>, grid, dim3(256), 0, st, x, K, C, out, ldo);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}
void launch_pad_rows(const double* x, long long rows, int K, long long ldx, float* out, long long ldo, hipStream_t st) {
  pad_rows_t(x, rows, K, ldx, out, ldo, st);
}
void launch_pad_t(const double* x, int K, int C, float* out, long long ldo, hipStream_t st) {
  pad_t_t(x, K, C, out, ldo, st);
}
void launch_wstage_f32(const float* T1, const double* W, int DH, int Dl, int Dr, float* T2, long long kp3,
                       hipStream_t st) {
  TT_REQUIRE(DH >= 1 && 4 * DH <= kWsMaxO && Dl >= 1 && Dr >= 1 && kp3 >= (long long)DH * Dr, TT_EINVAL,
             "W stage: shape out of range");
  hipLaunchKernelGGL(k_wstage_mfma<1>, dim3((unsigned)(4 * Dl)), dim3(256), 0, st, (const void*)T1, 0LL, W, DH, Dl, Dr,
                     (void*)T2, 0LL, kp3);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

void launch_pad_rows(const double* x, long long rows, int K, long long ldx, double* out, long long ldo, hipStream_t st) {
  pad_rows_t(x, rows, K, ldx, out, ldo, st);
}
void launch_pad_t(const double* x, int K, int C, double* out, long long ldo, hipStream_t st) {
  pad_t_t(x, K, C, out, ldo, st);
}

void launch_wstage_f64(const double* T1, const double* W, int DH, int Dl, int Dr, double* T2, long long kp3,
                       hipStream_t st) {
  TT_REQUIRE(DH >= 1 && 4 * DH <= kWsMaxO && Dl >= 1 && Dr >= 1 && 4LL * Dl < 65536 && kp3 >= (long long)DH * Dr &&
                 kp3 - (long long)DH * Dr <= 256,
             TT_EINVAL, "W stage: shape out of range");
  const dim3 grid((unsigned)(4 * Dl));
  hipLaunchKernelGGL(k_wstage_mfma<0>, grid, dim3(256), 0, st, (const void*)T1, 0LL, W, DH, Dl, Dr, (void*)T2, 0LL, kp3);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

void launch_split_rows(const double* x, long long rows, int K, long long ldx, void* out, long long ldo,
                       long long plane, int precision, hipStream_t st) {
  TT_REQUIRE(precision == TT_BF16X3 || precision == TT_BF16X6, TT_EINVAL, "split: split-BF16 precisions only");
  TT_REQUIRE(ldo >= K && ldx >= K, TT_EINVAL, "split: rows shorter than K");
  const long long n = rows * ldo;
  if (n <= 0) return;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 16384);
  if (precision == TT_BF16X3)
    hipLaunchKernelGGL(k_split_rows<2>, dim3(blocks), dim3(256), 0, st, x, rows, K, ldx, (__bf16*)out, ldo, plane);
  else
    hipLaunchKernelGGL(k_split_rows<3>, dim3(blocks), dim3(256), 0, st, x, rows, K, ldx, (__bf16*)out, ldo, plane);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

void launch_split_t(const double* x, int K, int C, void* out, long long ldo, long long plane, int precision,
                    hipStream_t st) {
  TT_REQUIRE(precision == TT_BF16X3 || precision == TT_BF16X6, TT_EINVAL, "split: split-BF16 precisions only");
  TT_REQUIRE(ldo >= K && K >= 1 && C >= 1, TT_EINVAL, "split: bad shape");
  const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((ldo + 31) / 32));
  if (precision == TT_BF16X3)
    hipLaunchKernelGGL(k_split_t<2>, grid, dim3(256), 0, st, x, K, C, (__bf16*)out, ldo, plane);
  else
    hipLaunchKernelGGL(k_split_t<3>, grid, dim3(256), 0, st, x, K, C, (__bf16*)out, ldo, plane);
  ++g_launches;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e));
}

}  // namespace tt
