// gfx950 kernels of the one-site tangent-space sweep.
//
//  * k_gemm      : grouped GEMM over charge blocks with gather/scatter index
//                  maps (each operand index is a stride or a table), FP64
//                  MFMA 16x16x4 tiles, one 64x64 output tile per workgroup of
//                  four 64-wide waves.  Used for every dense contraction of the
//                  sweep: L.A, .R, the environment updates, the bond apply
//                  and the absorb step (SM Fig. Lanczos, Fig. optimalB).
//  * k_wstage    : the contraction with the Hamiltonian MPO tensor W, which is
//                  sparse (a few nonzero 4x4 operators per bond pair); a
//                  bandwidth-bound weighted sum of strided blocks.
//  * k_qr        : Householder QR of one charge block per workgroup with
//                  non-negative diagonal (SM Sec. II.F step 3).
//  * Lanczos     : deterministic fixed-order reductions, Gram-Schmidt
//                  updates and the small tridiagonal exponential on the device
//                  (SM Sec. II.H), so a local exponential needs no host sync.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace tt {

typedef double double4_t __attribute__((ext_vector_type(4)));

#define HIP_CHECK_LAUNCH()                                                       \
  do {                                                                           \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) throw Error(TT_EDEVICE, hipGetErrorString(e_));        \
  } while (0)

// ------------------------------------------------------------------ GEMM
constexpr int BM = 64, BN = 64, BK = 16;

__device__ __forceinline__ long long idx_map(const long long* __restrict__ tabs, long long tab, long long stride,
                                             long long i) {
  return tab >= 0 ? tabs[tab + i] : i * stride;
}

__global__ __launch_bounds__(256) void k_gemm_f64(const GemmProb* __restrict__ probs,
                                                  const GemmTile* __restrict__ tiles,
                                                  const long long* __restrict__ tabs, Slots slots) {
  __shared__ double sA[BK][BM + 1];
  __shared__ double sB[BK][BN + 1];
  __shared__ long long rA[BM], cB[BN], rC[BM], kA[BK], kB[BK];
  const GemmTile t = tiles[blockIdx.x];
  const GemmProb P = probs[t.prob];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const double* __restrict__ A = slots.p[P.ia] + P.offA;
  const double* __restrict__ B = slots.p[P.ib] + P.offB;
  double* C = slots.p[P.ic] + P.offC;
  if (tid < BM) {
    int m = m0 + tid;
    rA[tid] = m < P.M ? idx_map(tabs, P.tam, P.sam, m) : 0;
    rC[tid] = m < P.M ? idx_map(tabs, P.tcm, P.scm, m) : 0;
  } else if (tid < BM + BN) {
    int n = n0 + tid - BM;
    cB[tid - BM] = n < P.N ? idx_map(tabs, P.tbn, P.sbn, n) : 0;
  }
  const bool a_kfast = (P.tak < 0 && P.sak == 1);
  const bool b_nfast = (P.tbn < 0 && P.sbn == 1);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < P.K; k0 += BK) {
    __syncthreads();
    if (tid < BK) {
      int k = k0 + tid;
      kA[tid] = k < P.K ? idx_map(tabs, P.tak, P.sak, k) : 0;
    } else if (tid >= 64 && tid < 64 + BK) {
      int k = k0 + tid - 64;
      kB[tid - 64] = k < P.K ? idx_map(tabs, P.tbk, P.sbk, k) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int e0 = 0; e0 < (BM * BK) / 256; ++e0) {
      int e = tid + e0 * 256;
      int i, kk;
      if (a_kfast) { i = e / BK; kk = e % BK; } else { i = e % BM; kk = e / BM; }
      bool ok = (m0 + i < P.M) && (k0 + kk < P.K);
      sA[kk][i] = ok ? A[rA[i] + kA[kk]] : 0.0;
    }
#pragma unroll
    for (int e0 = 0; e0 < (BN * BK) / 256; ++e0) {
      int e = tid + e0 * 256;
      int j, kk;
      if (b_nfast) { j = e % BN; kk = e / BN; } else { j = e / BK; kk = e % BK; }
      bool ok = (n0 + j < P.N) && (k0 + kk < P.K);
      sB[kk][j] = ok ? B[kB[kk] + cB[j]] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      double a0 = sA[kr][wm + c], a1 = sA[kr][wm + 16 + c];
      double b0 = sB[kr][wn + c], b1 = sB[kr][wn + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // D[i][j] of a 16x16 f64 MFMA block sits in lane j + 16*(i%4), element i/4
  // (measured on gfx950; A[i][k] in lane i + 16k, B[k][j] in lane j + 16k)
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = wm + bi * 16 + (lane >> 4) + 4 * v;
        int col = wn + bj * 16 + (lane & 15);
        int m = m0 + row, n = n0 + col;
        if (m < P.M && n < P.N) {
          double* cp = C + rC[row] + n;
          double val = P.alpha * acc[bi][bj][v];
          if (P.beta != 0.0) val += P.beta * (*cp);
          *cp = val;
        }
      }
}

void launch_gemm(const GemmPlan& p, const long long* d_tabs, Slots s, int precision, hipStream_t st) {
  (void)precision;
  if (p.ntiles == 0) return;
  hipLaunchKernelGGL(k_gemm_f64, dim3(p.ntiles), dim3(256), 0, st, p.d_probs, p.d_tiles, d_tabs, s);
  HIP_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ W stage
__global__ __launch_bounds__(256) void k_wstage(const WTask* __restrict__ tasks, const WTerm* __restrict__ terms,
                                                const double* __restrict__ in, double* __restrict__ out) {
  const WTask t = tasks[blockIdx.x];
  const int n = t.ni * t.nj;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int i = e / t.nj, j = e - i * t.nj;
    double acc = 0.0;
    for (int q = 0; q < t.nt; ++q) {
      const WTerm w = terms[t.t0 + q];
      acc += w.w * in[w.src + i * w.ssi + j * w.ssj];
    }
    out[t.dst + i * t.dsi + j * t.dsj] = acc;
  }
}

void launch_wstage(const WPlan& p, const double* in, double* out, hipStream_t st) {
  if (p.ntasks == 0) return;
  hipLaunchKernelGGL(k_wstage, dim3(p.ntasks), dim3(256), 0, st, p.d_tasks, p.d_terms, in, out);
  HIP_CHECK_LAUNCH();
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
__global__ __launch_bounds__(256) void k_qr(const QRTask* __restrict__ tasks, const long long* __restrict__ tabs,
                                            double* A, double* S, double* ws) {
  __shared__ double red[8];
  __shared__ double s_tau[1];
  const QRTask T = tasks[blockIdx.x];
  const int m = T.m, n = T.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Wm = ws + T.ws;                 // m x n column-major
  double* Qm = Wm + (long long)m * n;     // m x n column-major
  double* taus = Qm + (long long)m * n;   // n
  auto row = [&](int i) -> long long { return T.rtab >= 0 ? tabs[T.rtab + i] : (long long)i * T.rs; };
  for (long long e = tid; e < (long long)m * n; e += blockDim.x) {
    int i = (int)(e % m), j = (int)(e / m);
    Wm[e] = A[T.rbase + row(i) + (long long)j * T.cs];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) {
      double x = Wm[i + (long long)j * m];
      part += x * x;
    }
    double xn2 = block_sum(part, red);
    double alpha = Wm[j + (long long)j * m];
    double tau = 0.0;
    if (xn2 > 0.0) {
      double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      double scal = 1.0 / (alpha - beta);
      for (int i = j + 1 + tid; i < m; i += blockDim.x) Wm[i + (long long)j * m] *= scal;
      __syncthreads();
      if (tid == 0) Wm[j + (long long)j * m] = beta;
    }
    if (tid == 0) { taus[j] = tau; s_tau[0] = tau; }
    __syncthreads();
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += 4) {
        double* col = Wm + (long long)c * m;
        const double* v = Wm + (long long)j * m;
        double d = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) d += v[i] * col[i];
        d = wave_sum(d);
        d = __shfl(d, 0, 64) + col[j];
        double f = tau * d;
        if (lane == 0) col[j] -= f;
        for (int i = j + 1 + lane; i < m; i += 64) col[i] -= f * v[i];
      }
    }
    __syncthreads();
  }
  // explicit Q = H_0 ... H_{n-1} [I; 0]
  for (long long e = tid; e < (long long)m * n; e += blockDim.x) {
    int i = (int)(e % m), j = (int)(e / m);
    Qm[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    double tau = taus[j];
    if (tau != 0.0) {
      const double* v = Wm + (long long)j * m;
      for (int c = j + wave; c < n; c += 4) {
        double* col = Qm + (long long)c * m;
        double d = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) d += v[i] * col[i];
        d = wave_sum(d);
        d = __shfl(d, 0, 64) + col[j];
        double f = tau * d;
        if (lane == 0) col[j] -= f;
        for (int i = j + 1 + lane; i < m; i += 64) col[i] -= f * v[i];
      }
    }
    __syncthreads();
  }
  // non-negative diagonal: flip column j of Q and row j of R when R_jj < 0
  for (long long e = tid; e < (long long)m * n; e += blockDim.x) {
    int i = (int)(e % m), j = (int)(e / m);
    double sg = Wm[j + (long long)j * m] < 0.0 ? -1.0 : 1.0;
    A[T.rbase + row(i) + (long long)j * T.cs] = sg * Qm[e];
  }
  for (int e = tid; e < n * n; e += blockDim.x) {
    int i = e / n, j = e % n;
    double sg = Wm[i + (long long)i * m] < 0.0 ? -1.0 : 1.0;
    double val = (i <= j) ? sg * Wm[i + (long long)j * m] : 0.0;
    S[T.sdst + (T.trans ? (long long)j * n + i : (long long)i * n + j)] = val;
  }
}

void launch_qr(const QRPlan& p, const long long* d_tabs, double* A, double* S, double* ws, hipStream_t st) {
  if (p.ntasks == 0) return;
  hipLaunchKernelGGL(k_qr, dim3(p.ntasks), dim3(256), 0, st, p.d_tasks, d_tabs, A, S, ws);
  HIP_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ Lanczos
// part[b*(nv+self) + v] = sum over block b's chunk of Q_v[i] * y[i]; last entry y.y if with_self
__global__ __launch_bounds__(256) void k_mdot(const double* __restrict__ Q, long long ld, int nv,
                                              const double* __restrict__ y, long long n, int with_self,
                                              double* __restrict__ part) {
  __shared__ double red[8];
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long i0 = (long long)blockIdx.x * chunk;
  const long long i1 = i0 + chunk < n ? i0 + chunk : n;
  const int nout = nv + with_self;
  for (int v = 0; v < nout; ++v) {
    const double* x = (v < nv) ? Q + (long long)v * ld : y;
    double s = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) s += x[i] * y[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * nout + v] = s;
  }
}

__device__ double sum_parts(const double* part, int nparts, int stride, int v) {
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(long long)b * stride + v];
  return s;
}

// q0 = v / ||v||; scal[0] = ||v||
__global__ void k_lz_start(const double* __restrict__ v, double* __restrict__ q0, long long n,
                           const double* __restrict__ part, double* scal) {
  __shared__ double s_nv;
  if (threadIdx.x == 0) s_nv = sqrt(sum_parts(part, kRedBlocks, 1, 0));
  __syncthreads();
  const double nv = s_nv;
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[0] = nv;
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    q0[i] = v[i] * inv;
}

// w -= sum_v c_v Q_v with c_v = sum of partials; optionally store alpha = c_{nv-1}, hn = sqrt(self)
__global__ void k_lz_sub(double* __restrict__ w, const double* __restrict__ Q, long long ld, int nv,
                         const double* __restrict__ part, int stride, long long n, double* alpha_out,
                         double* hn_out) {
  __shared__ double c[kMaxKrylov + 1];
  if (threadIdx.x < nv) c[threadIdx.x] = sum_parts(part, kRedBlocks, stride, threadIdx.x);
  if (threadIdx.x == 0 && stride > nv) c[nv] = sum_parts(part, kRedBlocks, stride, nv);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (alpha_out) *alpha_out = c[nv - 1];
    if (hn_out) *hn_out = sqrt(c[nv]);
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = w[i];
    for (int v = 0; v < nv; ++v) s -= c[v] * Q[(long long)v * ld + i];
    w[i] = s;
  }
}

// beta = ||w||; qn = w / beta unless beta <= tol * ||H q|| (lucky breakdown: qn = 0)
__global__ void k_lz_next(const double* __restrict__ w, double* __restrict__ qn, long long n,
                          const double* __restrict__ part, double* beta_out, const double* hn, double tol) {
  __shared__ double s_b;
  if (threadIdx.x == 0) s_b = sqrt(sum_parts(part, kRedBlocks, 1, 0));
  __syncthreads();
  const double b = s_b;
  if (blockIdx.x == 0 && threadIdx.x == 0) *beta_out = b;
  if (!qn) return;
  const bool brk = !(b > tol * (*hn)) || b == 0.0;
  const double inv = brk ? 0.0 : 1.0 / b;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    qn[i] = w[i] * inv;
}

// coefficients of exp(t T) e_1 * ||v|| for the Krylov tridiagonal T (cyclic Jacobi eigensolver)
__global__ void k_lz_coeffs(const double* alpha, const double* beta, const double* hn, int K, double t,
                            double tol, const double* scal, double* coeff, double* errmax) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a[kMaxKrylov][kMaxKrylov], V[kMaxKrylov][kMaxKrylov];
  int k = K;
  for (int j = 0; j < K - 1; ++j)
    if (!(beta[j] > tol * hn[j]) || beta[j] == 0.0) { k = j + 1; break; }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      a[i][j] = 0.0;
      V[i][j] = (i == j) ? 1.0 : 0.0;
    }
  for (int i = 0; i < k; ++i) a[i][i] = alpha[i];
  for (int i = 0; i + 1 < k; ++i) a[i][i + 1] = a[i + 1][i] = beta[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < k; ++i) {
      dia += a[i][i] * a[i][i];
      for (int j = i + 1; j < k; ++j) off += a[i][j] * a[i][j];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        if (a[p][q] == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int r = 0; r < k; ++r) {
          double arp = a[r][p], arq = a[r][q];
          a[r][p] = c * arp - s * arq;
          a[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          double apr = a[p][r], aqr = a[q][r];
          a[p][r] = c * apr - s * aqr;
          a[q][r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          double vrp = V[r][p], vrq = V[r][q];
          V[r][p] = c * vrp - s * vrq;
          V[r][q] = s * vrp + c * vrq;
        }
      }
  }
  const double nv = scal[0];
  for (int i = 0; i < K; ++i) coeff[i] = 0.0;
  for (int i = 0; i < k; ++i) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[i][j] * exp(t * a[j][j]) * V[0][j];
    coeff[i] = nv * s;
  }
  if (k == K) {
    double err = beta[K - 1] * fabs(coeff[K - 1]) / (nv > 0 ? nv : 1.0);
    if (err > *errmax) *errmax = err;
  }
}

__global__ void k_lz_combine(const double* __restrict__ Q, long long ld, int K, const double* __restrict__ coeff,
                             double* __restrict__ out, long long n) {
  __shared__ double c[kMaxKrylov];
  if (threadIdx.x < K) c[threadIdx.x] = coeff[threadIdx.x];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int v = 0; v < K; ++v) s += c[v] * Q[(long long)v * ld + i];
    out[i] = s;
  }
}

// v /= ||v||; lambda += ln ||v||
__global__ void k_normalize_log(double* __restrict__ v, long long n, const double* __restrict__ part, double* lambda) {
  __shared__ double s_n;
  if (threadIdx.x == 0) s_n = sqrt(sum_parts(part, kRedBlocks, 1, 0));
  __syncthreads();
  const double nv = s_n;
  if (blockIdx.x == 0 && threadIdx.x == 0) *lambda += log(nv);
  const double inv = 1.0 / nv;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    v[i] *= inv;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, long long n) {
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

void launch_mdot(const double* Q, long long ld, int nv, const double* y, long long n, int with_self, double* part,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_mdot, dim3(kRedBlocks), dim3(256), 0, st, Q, ld, nv, y, n, with_self, part);
  HIP_CHECK_LAUNCH();
}
void launch_lz_start(const double* v, double* q0, long long n, const double* part, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_start, dim3(grid_for(n)), dim3(256), 0, st, v, q0, n, part, scal);
  HIP_CHECK_LAUNCH();
}
void launch_lz_sub(double* w, const double* Q, long long ld, int nv, const double* part, int nparts, long long n,
                   double* alpha_out, double* hn_out, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_sub, dim3(grid_for(n)), dim3(256), 0, st, w, Q, ld, nv, part, nparts, n, alpha_out, hn_out);
  HIP_CHECK_LAUNCH();
}
void launch_lz_next(const double* w, double* qn, long long n, const double* part, double* beta_out, const double* hn,
                    double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_next, dim3(grid_for(n)), dim3(256), 0, st, w, qn, n, part, beta_out, hn, tol);
  HIP_CHECK_LAUNCH();
}
void launch_lz_coeffs(const double* alpha, const double* beta, const double* hn, int K, double t, double tol,
                      const double* scal, double* coeff, double* errmax, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_coeffs, dim3(1), dim3(64), 0, st, alpha, beta, hn, K, t, tol, scal, coeff, errmax);
  HIP_CHECK_LAUNCH();
}
void launch_lz_combine(const double* Q, long long ld, int K, const double* coeff, double* out, long long n,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_lz_combine, dim3(grid_for(n)), dim3(256), 0, st, Q, ld, K, coeff, out, n);
  HIP_CHECK_LAUNCH();
}
void launch_normalize_log(double* v, long long n, const double* part, double* lambda, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize_log, dim3(grid_for(n)), dim3(256), 0, st, v, n, part, lambda);
  HIP_CHECK_LAUNCH();
}
void launch_copy(double* dst, const double* src, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, st, dst, src, n);
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
          for (int q = 0; q < 4; ++q) d += row[(long long)q * E.diag_stride * E.dr + y];
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

}  // namespace tt
