// Launch wrappers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace tt {

// reduction geometry: fixed block count so that every sum has a fixed order
constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 1024;   // threads per block of the reducing kernels
constexpr int kMaxKrylov = 32;

// Optional timing of the grouped kernels: HIP events on the launch stream.
// kinds 0..TAG_COUNT-1 are the grouped GEMM contractions by tag, then the W
// stage and the QR, then the individual GEMM kernels (one kind per tile shape,
// then the K-slice reduce, then the wave GEMM), each timed per dispatch, and
// the fused apply (one dispatch per apply).
enum ProfKind {
  PROF_WSTAGE = TAG_COUNT, PROF_QR = TAG_COUNT + 1, PROF_GEMM_CFG0 = TAG_COUNT + 2,
  PROF_GEMM_REDUCE = PROF_GEMM_CFG0 + kGemmCfgs, PROF_GEMM_WAVE = PROF_GEMM_REDUCE + 1,
  PROF_FUSED = PROF_GEMM_WAVE + 1, PROF_KINDS = PROF_FUSED + 1
};
// kernels enqueued by the library since it was loaded (every launch wrapper counts)
long long launch_count();

void prof_enable(bool on);
bool prof_enabled();
// begin an operation; prof_mark closes the dispatch launched since the previous
// event (kind = a single kernel); prof_end closes the whole operation
void prof_begin(hipStream_t st);
void prof_mark(hipStream_t st, int kind, double flops, double bytes);
void prof_end(hipStream_t st, int kind, double flops, double bytes);
// (ms, flops, bytes, launches) per kind since the last read; synchronises the events
void prof_read(double out[PROF_KINDS][4]);

// Batched launches: every kernel of the sweep runs a batch of nb <= kMaxBatch
// independent states with identical plans in one launch (blockIdx.y = state);
// the plan descriptors and index tables are shared, data pointers are per
// state.  A single state is a batch of one.
constexpr int kMaxBatch = 16;
template <typename T> struct BPtr { T* p[kMaxBatch]; };
struct BSlots { Slots s[kMaxBatch]; };
template <typename T> BPtr<const T> cst(BPtr<T> x) {
  BPtr<const T> r;
  for (int i = 0; i < kMaxBatch; ++i) r.p[i] = x.p[i];
  return r;
}
template <typename T> BPtr<T> one(T* x) {
  BPtr<T> r{};
  r.p[0] = x;
  return r;
}
inline BSlots one(Slots s) {
  BSlots r{};
  r.s[0] = s;
  return r;
}

// pws: partial-tile workspace of at least p.pws_size doubles (split problems)
void launch_gemm(const GemmPlan& p, const long long* d_tabs, const BSlots& s, int nb, int precision,
                 BPtr<double> pws, hipStream_t st);
// Pre-split BF16 operands: part p of an element lives p * s[slot] elements
// after its first part; c: the result is written as planes too.
struct Planes { long long s[kSlots] = {0, 0, 0, 0}; int c = 0; };
// the LDS-tile GEMM on pre-split operands (split-BF16 precisions; plan with
// LDS tiles only and no K slices)
void launch_gemm_planes(const GemmPlan& p, const long long* d_tabs, const Slots& s, const Planes& pl, int precision,
                        hipStream_t st);
// the BF16 parts of n doubles into planes pstride elements apart
void launch_split(const double* x, long long n, void* out, long long pstride, int precision, hipStream_t st);

// Large-tile split-BF16 GEMM of dense operands (the dense apply's L.A and .R):
// C(m, n) = sum_k A(m, k) B(n, k) with A(m, k) = A[p sa + m lda + k] and
// B(n, k) = B[p sb + n ldb + k] for the BF16 planes p, K a multiple of 32
// (rows zero-padded), results at C + (m / cdiv) ldc1 + (m % cdiv) ldc0 + n,
// as FP64 or (cplanes) as BF16 planes sc elements apart.
struct BgArgs {
  const __bf16* A; long long lda, sa;
  const __bf16* B; long long ldb, sb;
  int M, N, K;
  void* C; long long ldc0, ldc1, sc; int cdiv, cplanes;
  int tiles_m, tiles_n;   // set by the launcher
};
int bgemm_kpad(long long K);   // K rounded up to the GEMM's K tile
void launch_bgemm(BgArgs a, int precision, hipStream_t st);
// the dense apply's W stage on BF16 planes (layouts of tt_heff_apply's split-BF16
// path: T1[a][x'][s][y], T2 rows (x', s) kp3 apart, their K padding written as
// zeros); DH at most wstage_planes_max_dh()
int wstage_planes_max_dh();
void launch_wstage_planes(const void* T1, long long sT1, const double* W, int DH, int Dl, int Dr, void* T2, long long sT2,
                          long long kp3, int precision, hipStream_t st);
// The FP64 large-tile GEMM of the dense apply: C(m, n) = sum_k A[m lda + k]
// B[n ldb + k], K a multiple of 16 (rows zero-padded), results at
// C + (m / cdiv) ldc1 + (m % cdiv) ldc0 + n.
struct DgArgs {
  const double* A; long long lda;
  const double* B; long long ldb;
  int M, N, K;
  double* C; long long ldc0, ldc1; int cdiv;
  int tiles_m, tiles_n;   // set by the launcher
};
int dgemm_kpad(long long K);   // K rounded up to the FP64 GEMM's K tile
void launch_dgemm(DgArgs a, hipStream_t st);
// The FP32 version (the FP32 dense apply): float operands, K a multiple of 32,
// FP32 MFMA with the partials added in FP64; results as double or (cfloat) float.
struct SgArgs {
  const float* A; long long lda;
  const float* B; long long ldb;
  int M, N, K;
  void* C; long long ldc0, ldc1; int cdiv, cfloat;
  int tiles_m, tiles_n;   // set by the launcher
};
int sgemm_kpad(long long K);   // K rounded up to the FP32 GEMM's K tile
void launch_sgemm(SgArgs a, hipStream_t st);
// out[r ldo + k] = x[r ldx + k] (k < K), zero up to ldo (float: rounded to nearest)
void launch_pad_rows(const double* x, long long rows, int K, long long ldx, double* out, long long ldo, hipStream_t st);
void launch_pad_rows(const double* x, long long rows, int K, long long ldx, float* out, long long ldo, hipStream_t st);
// out[c ldo + k] = x[k C + c] (k < K), zero up to ldo
void launch_pad_t(const double* x, int K, int C, double* out, long long ldo, hipStream_t st);
void launch_pad_t(const double* x, int K, int C, float* out, long long ldo, hipStream_t st);
// the W stage with float T1 and T2 (FP32 multiplies)
void launch_wstage_f32(const float* T1, const double* W, int DH, int Dl, int Dr, float* T2, long long kp3,
                       hipStream_t st);
// the dense apply's W stage in FP64 (T1[a][x'][s][y] -> T2 rows (x', s) kp3 apart)
void launch_wstage_f64(const double* T1, const double* W, int DH, int Dl, int Dr, double* T2, long long kp3,
                       hipStream_t st);
// out[p plane + r ldo + k] = part p of x[r ldx + k] (k < K), zero up to ldo
void launch_split_rows(const double* x, long long rows, int K, long long ldx, void* out, long long ldo,
                       long long plane, int precision, hipStream_t st);
// out[p plane + c ldo + k] = part p of x[k C + c] (k < K), zero up to ldo
void launch_split_t(const double* x, int K, int C, void* out, long long ldo, long long plane, int precision,
                    hipStream_t st);
// the fused one-site apply LW . x . R of every state of the batch (slots:
// 0 = LW, 1 = input site vector, 2 = R env, 3 = output site vector)
void launch_fused(const FzPlan& p, const BSlots& s, int nb, hipStream_t st);
// terms: each state's copy of the plan's terms (the weights may differ)
void launch_wstage(const WPlan& p, BPtr<const WTerm> terms, BPtr<const double> in, BPtr<double> out, int nb,
                   hipStream_t st);
// QR of every task of the plan: LDS chunk/stack/combine kernels for n <= 64,
// the global-memory kernel for wider tasks.  ws holds p.ws_size + p.lds_ws doubles.
void launch_qr(const QRPlan& p, const long long* d_tabs, BPtr<double> A, BPtr<double> S, BPtr<double> ws, int nb,
               hipStream_t st);
// split the tasks of a plan into LDS chunks and stacks (host)
void qr_plan_chunks(QRPlan& p);
// workspace doubles of a block that the global-memory (wide) QR factors
long long qr_wide_ws(int m, int n);

// Lanczos pieces (see engine for the sequence)
void launch_mdot(BPtr<const double> Q, long long ld, int nv, BPtr<const double> y, long long n, int with_self,
                 BPtr<double> part, int nb, hipStream_t st);
void launch_lz_start(BPtr<const double> v, BPtr<double> q0, long long n, BPtr<const double> part, BPtr<double> scal,
                     int nb, hipStream_t st);
void launch_lz_sub_dot(BPtr<double> w, BPtr<const double> Q, long long ld, int nv, BPtr<const double> part_in,
                       int stride_in, long long n, BPtr<double> alpha_out, BPtr<double> hn_out, BPtr<double> part_out,
                       int nb, hipStream_t st);
// second pass and normalisation in one: qn = (w - Q c') / beta, beta from
// ||w||^2 - ||c'||^2 (part_in: stride nv + 1 partials of k_lz_sub_dot); qn null: beta only
void launch_lz_sub_next(BPtr<const double> w, BPtr<const double> Q, long long ld, int nv, BPtr<const double> part_in,
                        long long n, BPtr<double> qn, BPtr<double> beta_out, BPtr<const double> hn, double tol,
                        int nb, hipStream_t st);
void launch_lz_combine_norm(BPtr<const double> Q, long long ld, int K, BPtr<const double> coeff, BPtr<double> out,
                            long long n, BPtr<double> part_out, int nb, hipStream_t st);
void launch_lz_coeffs(BPtr<const double> alpha, BPtr<const double> beta, BPtr<const double> hn, int K, double t,
                      double tol, BPtr<const double> scal, BPtr<double> coeff, BPtr<double> errmax, int nb,
                      hipStream_t st);
void launch_normalize_log(BPtr<double> v, long long n, BPtr<const double> part, BPtr<double> lambda, int nb,
                          hipStream_t st);
void launch_copy(BPtr<double> dst, BPtr<const double> src, long long n, int nb, hipStream_t st);
void launch_fill(double* dst, double val, long long n, hipStream_t st);
void launch_dot_final(const double* part, int nparts, int nv, double* out, hipStream_t st);

// the smaller dimension of an SVD task is at most this (its column norms live in LDS)
constexpr int kSvdMaxMinDim = 16384;
// SVD of every task (one-sided Jacobi, one workgroup per task; ws holds the
// plan's svd_ws doubles, sig its svd_nsig singular values), then the kept
// vectors of every emit entry into the two site tensors
void launch_svd(const SvdTask* d_tasks, int ntasks, const int* d_idx, const long long* d_tabs, const double* src,
                double* ws, double* sig, hipStream_t st);
// doubles of LDS a workgroup of the SVD kernel can hold (blocks whose X needs
// more run as launch_svd_big)
int svd_lds_doubles();
// The same Jacobi for the large blocks d_big[0..nbig) of d_tasks, one launch
// per round spread over the GPU (d_pairs: (index into d_big, pair k) for every
// pair of every large block; max_np: the largest column count rounded up to
// even); ctl: 3 doubles per large block.  Synchronises once per sweep.
void launch_svd_big(const SvdTask* d_tasks, const int* d_big, int nbig, const int* d_pairs, int npairs, int max_np,
                    const long long* d_tabs, const double* src, double* ws, double* sig, double* ctl,
                    hipStream_t st);
void launch_svd_emit(const SvdTask* d_tasks, const SvdEmit* d_em, int nem, const long long* d_tabs, const double* ws,
                     const double* sig, double* Aout, double* Bout, hipStream_t st);

// pos[q]: position of the diagonal super index s = 5q (sigma = sigma' = q) in its charge group
struct TraceEntry { long long src, C, xoff, dl, yoff, dr; int site, pos[4]; };
void launch_trace(const TraceEntry* d_entries, const int* d_site_start, int N, double* const* d_sites,
                  double* vbuf, long long vlen, double* out2, hipStream_t st);

}  // namespace tt
