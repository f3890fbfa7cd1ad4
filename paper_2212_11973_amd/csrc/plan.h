// Device-visible descriptors of the grouped contractions and the host-side
// plans that hold them.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

#include "tt_internal.h"

namespace tt {

constexpr int kSlots = 4;
struct Slots { double* p[kSlots]; };

// One GEMM of a grouped launch: C = alpha * A B + beta * C with
//   A(m,k) = slot[ia][offA + am(m) + ak(k)]
//   B(k,n) = slot[ib][offB + bk(k) + bn(n)]
//   C(m,n) = slot[ic][offC + cm(m) + n]
// where each index map is either i * stride (table < 0) or tables[table + i].
// dt: operands stored as float instead of double (bit 0 A, bit 1 B, bit 2 C;
// offsets then count floats); only the wave GEMM takes such problems.
constexpr int kDtA = 1, kDtB = 2, kDtC = 4;
struct GemmProb {
  int M, N, K;
  int ia, ib, ic, dt;
  long long offA, offB, offC;
  long long sam, sak, sbk, sbn, scm;
  long long tam, tak, tbk, tbn, tcm;
  double alpha, beta;
};
// tile shapes of the grouped GEMM, chosen per problem from its M and N:
//   0: 64x64   1: 128x32   2: 256x16   3: 32x128   4: 32x32 with the K sub-steps split over the four waves
// A problem with a long K is split into nk K-slices over separate workgroups:
// each writes its partial BM x BN tile to the plan's partial buffer at
// pw + ks*BM*BN, and a reduce pass adds the slices in order (deterministic).
struct GemmTile { int prob, tm, tn, cfg, ks, nk, sidx, pad; long long pw; };
struct GemmSplit { int prob, tm, tn, cfg, nk, pad; long long pw; };
#ifndef TT_KSLICE
#define TT_KSLICE 128
#endif
#ifndef TT_MAX_KSPLIT
#define TT_MAX_KSPLIT 8
#endif
#ifndef TT_SPLIT_BELOW_TILES
#define TT_SPLIT_BELOW_TILES 2048
#endif
constexpr int kKSlice = TT_KSLICE;          // K per slice when a problem is split
constexpr int kMaxKSplit = TT_MAX_KSPLIT;
constexpr long long kSplitBelowTiles = TT_SPLIT_BELOW_TILES;   // split only launches with fewer tiles
constexpr int kGemmCfgs = 5;
constexpr int kGemmBM[kGemmCfgs] = {64, 128, 256, 32, 32};
constexpr int kGemmBN[kGemmCfgs] = {64, 32, 16, 128, 32};

// Wave GEMM for small, short-K or skinny problems: one 64-wide wave computes a
// 64x16, 32x32, 16x64 or 16x16 output block (shape 0, 1, 2, 3) straight from
// global memory.  A job is one wave's share: a whole block (nparts = 1), or
// part `part` of the nparts = 4 interleaved K parts of a block, whose partial
// sums the four waves of one workgroup add in LDS.  Jobs are grouped four per
// workgroup; the four jobs of a split block fill one workgroup, and unused
// slots of a workgroup have prob = -1.  A plan whose blocks give fewer than
// kWaveMinJobs jobs also holds a finer job list (16x16 blocks, K split from
// four 16-deep chunks on); a launch takes it when the plan's jobs times the
// batch's states stay below kWaveMinJobs, so that more waves share the latency.
struct GemmJob { int prob, tm, tn, shape, part, nparts; };
constexpr int kWaveShapes = 4;
constexpr int kWaveBM[kWaveShapes] = {64, 32, 16, 16};
constexpr int kWaveBN[kWaveShapes] = {16, 32, 64, 16};
#ifndef TT_WAVE_MIN_JOBS
#define TT_WAVE_MIN_JOBS 4096
#endif
constexpr int kWaveMinJobs = TT_WAVE_MIN_JOBS;
// problems at least this large in M, N and K use the LDS-staged tile kernel.
// Below K = 128 the wave kernel (one pass over each operand row, paired
// loads) is faster: that covers every block of a block-sparse sweep, whose K
// is at most the sector cap; the dense apply (K = D) stays on LDS tiles.
#ifndef TT_LDS_MIN_MN
#define TT_LDS_MIN_MN 128
#endif
#ifndef TT_LDS_MIN_K
#define TT_LDS_MIN_K 128
#endif
constexpr int kLdsMinMN = TT_LDS_MIN_MN;
constexpr int kLdsMinK = TT_LDS_MIN_K;

// W stage: dst(i,j) = sum_t w_t src_t(i,j) for i < ni, j < nj, with
// dst(i,j) = out[dst + i*dsi + j*dsj] and src_t(i,j) = in[src + i*ssi + j*ssj].
struct WTask { long long dst, dsi, dsj; int ni, nj, t0, nt; };
struct WTerm { long long src, ssi, ssj; double w; };

// Householder QR of an m x n (m >= n) matrix M(i,j) = buf[rbase + row(i) + j*cs]
// (row(i) = rtab[i] if rtab >= 0 else i*rs).  Q overwrites M; R (n x n) goes
// to S[sdst + i*n + j] (upper) or, if trans, to S[sdst + j*n + i] (lower: L = R^T).
struct QRTask { int m, n, trans, pad; long long rbase, rs, cs, rtab, sdst, ws; };

// Register-resident QR (n <= kQrLdsMaxN): a task is split into row chunks of
// at most kQrChunkRows rows; chunk QRs, then one QR of the stacked chunk R
// factors (at most kQrStackRows rows), then the product of the two Q levels
// (tall-skinny QR in two levels).  A task with one chunk is finished by the
// chunk kernel; wider or taller tasks use the global-memory kernel.
constexpr int kQrLdsMaxN = 64;
constexpr int kQrChunkRows = 256;
constexpr int kQrStackRows = 256;   // 16 rows per lane, as the chunks (larger stacks spill)
struct QRChunk { int task, row0, rows, chunk, nchunks, pad; long long qw, rw; };
struct QRStack { int task, nchunks; long long rw; };

// Fused one-site apply with the MPO folded into L (SM Fig. Lanczos; W summed
// into L once per environment).  Output block o = (p, so, sp) of H^(1) x has
// the rows x' of bra sector p and the columns y' of the right sector r' it
// reaches:
//   out[x', y'] = sum_b sum_{y in c(b)} T2_b[x', y] R_r'[y', (b, y)],
//   T2_b[x', y] = sum_t sum_{x < dl_t} LW_t[x', x] x_t[x, y],
// with T2 formed in registers 16 x 16 at a time, so neither the L.A
// intermediate nor T2 goes to memory.  Element offsets: out at
// out + x' ldo + y' (the output site vector), R at rrow + y' ldr + rcol + y,
// LW at lw + x' ldlw + x, the input site vector at a + x lda + y.
struct FzOut { long long out, rrow; int ldo, ldr, dp, dr, b0, nb; };
struct FzB { long long rcol; int dc, t0, nt, pad; };
struct FzT { long long lw, a; int ldlw, lda, dl, pad; };
// One wave's share: rows row0 .. row0 + 15 and columns col0 .. col0 + 63 of
// block o, over the b blocks part, part + nparts, ...; with nparts = 4 the
// four waves of a workgroup hold the four parts and add them in part order.
// Split jobs come first, whole workgroups each; unused slots have o = -1.
struct FzJob { int o, row0, col0, part, nparts, pad; };
constexpr int kFzCols = 64;   // output columns per job
constexpr int kFzMaxB = 64;   // b blocks per output block and terms per b block (one per lane)
struct FzPlan {
  std::vector<FzOut> outs;
  std::vector<FzB> bs;
  std::vector<FzT> terms;
  std::vector<FzJob> jobs;
  FzOut* d_outs = nullptr;
  FzB* d_bs = nullptr;
  FzT* d_terms = nullptr;
  FzJob* d_jobs = nullptr;
  int nblocks = 0;          // workgroups (four jobs each)
  double flops = 0;         // algorithmic: 2 dp dc dl per term and 2 dp dc dr per b block
  double bytes = 0;         // minimum: LW rows, input, R rows read once, output written once
};

// A plan: descriptors uploaded once, launched many times with varying slots.
// profiler tags of the grouped GEMMs (which contraction a launch belongs to)
enum GemmTag { TAG_LA = 0, TAG_R = 1, TAG_ENVL = 2, TAG_ENVR1 = 3, TAG_ENVR3 = 4, TAG_BOND = 5, TAG_ABSORB = 6,
               TAG_WGEMM = 7, TAG_COUNT = 8 };
struct GemmPlan {
  int tag = TAG_LA;
  std::vector<GemmProb> probs;
  std::vector<GemmTile> tiles;
  double flops = 0;
  double bytes = 0;        // algorithmic: every operand element read once, C written once
  GemmProb* d_probs = nullptr;
  GemmTile* d_tiles = nullptr;
  int ntiles = 0;
  std::vector<GemmSplit> splits;
  GemmSplit* d_splits = nullptr;
  int cfg_off[kGemmCfgs + 1] = {0, 0, 0, 0, 0, 0};   // tiles are sorted by shape
  long long pws_size = 0;   // doubles of partial tiles
  int smem_bytes = 0;       // LDS of the largest tile shape in the plan
  // per tile shape: algorithmic flops and bytes of the problems given that shape
  double cfg_flops[kGemmCfgs] = {0, 0, 0, 0, 0};
  double cfg_bytes[kGemmCfgs] = {0, 0, 0, 0, 0};
  double red_bytes = 0;     // the K-slice reduce: partials read once, C written once
  // wave-GEMM jobs (only when wave_ok: FP64 / FP32 launches)
  bool wave_ok = false;
  // slots that hold float data (FP32 mode keeps the contraction intermediates in float)
  bool slot_f32[kSlots] = {false, false, false, false};
  std::vector<GemmJob> jobs;
  GemmJob* d_jobs = nullptr;
  int wave_blocks = 0;
  std::vector<GemmJob> jobs_fine;   // empty unless it has more jobs than `jobs`
  GemmJob* d_jobs_fine = nullptr;
  int wave_blocks_fine = 0;
  double wave_flops = 0, wave_bytes = 0;
  bool no_split = false;    // never split K (tiles whose result is written as BF16 planes)
};
struct WPlan {
  bool f32 = false;    // input and output stored as float
  bool wide = false;   // some block spans 2^29 elements or more (64-bit offsets)
  std::vector<WTask> tasks;
  std::vector<WTerm> terms;
  std::vector<long long> widx;   // per term: the flat index of its weight in the site's MPO tensor
  WTask* d_tasks = nullptr;
  WTerm* d_terms = nullptr;
  int ntasks = 0;
  double flops = 0;
  double bytes = 0;        // algorithmic: every source block read once, every output written once
};
struct QRPlan {
  std::vector<QRTask> tasks;
  QRTask* d_tasks = nullptr;
  int ntasks = 0;
  // LDS path: chunks of every task (n <= kQrLdsMaxN), stacks of multi-chunk tasks,
  // and the global-memory fallback for wider tasks (indices into tasks)
  std::vector<QRChunk> chunks;
  std::vector<QRStack> stacks;
  std::vector<int> wide;
  QRChunk* d_chunks = nullptr;
  QRStack* d_stacks = nullptr;
  int* d_wide = nullptr;
  long long lds_ws = 0;     // doubles: chunk Q factors and stacked R / Q2
  long long ws_size = 0;    // doubles of workspace (2 m n per task)
  double flops = 0;         // Householder QR + explicit Q: 4 m n^2 - 4/3 n^3 per task
  double bytes = 0;         // matrix read and written once, R written once
};

// bookkeeping of one site tensor: row block per left sector l, columns
// (group g, s in g, y in the right sector l + delta_g)
struct SiteLayout {
  int nl = 0;
  std::vector<int> dl, C;
  std::vector<long long> base;
  std::vector<std::array<int, 9>> rsec, colb;
  long long size = 0;
};
// environment on a bond: row block per bra sector p, columns (a, ket x in p - qH(a))
struct EnvLayout {
  int np = 0;
  std::vector<int> dp, K;
  std::vector<long long> base;
  std::vector<std::vector<int>> csec, colb;
  long long size = 0;
};
// packed block-diagonal bond matrix S: one d x d block per sector
struct BondMatLayout {
  std::vector<long long> off;
  long long size = 0;
};

SiteLayout make_site_layout(const Bond& left, const Bond& right, const Groups& G);
EnvLayout make_env_layout(const Bond& bond, const std::vector<Q>& qH);
BondMatLayout make_bondmat_layout(const Bond& bond);

// All descriptors of one site k (left bond k, right bond k+1).
struct SitePlan {
  // sizes of intermediates (doubles)
  long long t1_size = 0, t2_size = 0, y_size = 0, z_size = 0;
  // heff1 / env-left: stage 1 (L.A), W stage, stage 3 (.R), env-left final
  GemmPlan s1, s3, el;
  WPlan w2;
  // env-right: stage 1' (R.A), W stage, final
  GemmPlan r1, r3;
  WPlan wr;
  // gauge moves
  QRPlan qr, lq;
  // absorb from the left (S_k . A, S on the left bond) and from the right (A . S_{k+1})
  GemmPlan absL, absR;
  // bond effective Hamiltonian on the left bond k (H^(0) with L_k, R_k); fzb:
  // the same as one fused launch (slots: 0 = L env, 1 = S, 2 = R env, 3 = output)
  GemmPlan b1, b2;
  FzPlan fzb;
  long long u_size = 0;
  // transfer-matrix trace: per left sector l with a (0,0) group, (row block, col base, d)
  std::vector<std::array<long long, 4>> tr;
  // The MPO folded into the left environment (ket-only MPOs): lw builds
  // LW^{b,so,si}[x', x] = sum_a W[a,so,si,b] L^a[x', x] (one block per bra
  // sector and group (b, so, si) with an entry), then T2 = LW . A runs as the
  // grouped GEMMs s1w[0..n_s1w): pass j adds the j-th si of every output block
  // (b, so, sp) of T2 (beta 0 in pass 0), written straight into stage 3's T2
  // layout; t2zero clears the T2 blocks no term reaches.
  static constexpr int kMaxLwPasses = 4;
  WPlan lw, t2zero;
  GemmPlan s1w[kMaxLwPasses];
  int n_s1w = 0;
  long long lw_size = 0;
  // the whole apply LW . x . R in one launch (slots: 0 = LW, 1 = input site
  // vector, 2 = R env, 3 = output site vector)
  FzPlan fz;
};

// slot conventions (kernel argument order)
//   s1 : 0 = L env, 1 = site vector, 2 = T1
//   w2 : in = T1, out = T2
//   lw : in = L env, out = LW
//   s1w: 0 = LW, 1 = site vector, 2 = T2 (t2zero: out = T2)
//   s3 : 0 = T2, 1 = R env, 2 = output site vector
//   el : 0 = site tensor (A^L), 1 = T2, 2 = new L env
//   r1 : 0 = R env, 1 = site tensor, 2 = Y
//   wr : in = Y, out = Z
//   r3 : 0 = site tensor, 1 = Z, 2 = new R env
//   absL: 0 = S (left bond), 1 = site tensor, 2 = output
//   absR: 0 = site tensor, 1 = S (right bond), 2 = output
//   b1 : 0 = L env (bond k), 1 = S (bond k), 2 = U
//   b2 : 0 = U, 1 = R env (bond k), 2 = output S
// Tables of all plans of a site live in one device array; offsets are into it.
struct SiteTables {
  std::vector<long long> host;
  long long* dev = nullptr;
  long long add(const std::vector<long long>& t) {
    long long o = (long long)host.size();
    host.insert(host.end(), t.begin(), t.end());
    return o;
  }
};

SitePlan build_site_plan(int k, const Bond& bl, const Bond& br, const Groups& G,
                         const std::vector<Q>& qHl, const std::vector<Q>& qHr,
                         const std::vector<double>& W,    // DHl*16*DHr (super_op: DHl*256*DHr)
                         const std::vector<double>& Wp,   // pattern: entries kept when nonzero in W or Wp
                         SiteTables& tabs,
                         bool super_op = false,           // W acts on the super index s = 4 sigma + sigma'
                         bool with_lw = true);            // also plan the MPO folded into L (lw, s1w, t2zero)

// ---------------------------------------------------------------- 2-TDVP
// Two-site tensor Theta = A_k A_{k+1} on the bonds (k, k+2) (SM Sec. "2-TDVP in
// the initial stage", Eq. S-2TDVP): row block per left sector l (row-major),
// columns (group g1, s1 in g1, then the columns of the middle charge
// m = l + Delta(g1): group g2, s2 in g2, y in the right sector m + Delta(g2)).
// Every middle charge that reaches the right bond is present, whether or not
// the current middle bond holds it: the two-site update can grow new sectors.
// Within a middle charge the columns are ordered as the row block of A_{k+1}.
struct MidBlock { int g2, r; long long off; };
struct PairLayout {
  int nl = 0;
  std::vector<int> dl;
  std::vector<long long> C, base;
  std::vector<std::array<long long, 9>> colg;   // per (l, g1): first column, or -1
  std::map<Q, std::vector<MidBlock>> mid;       // middle charge -> its column blocks
  std::map<Q, long long> width;                 // middle charge -> its column count
  long long size = 0;
  long long w(const Q& m) const { auto it = width.find(m); return it == width.end() ? 0 : it->second; }
};
// SVD of the split: the matrix M of one middle charge, rows (l, s1, x) of
// Theta (M(i, j) = theta[tabs[rtab + i] + j], i < R, j < w).  The work array
// holds X = M (R >= w) or M^T (R < w) column-major, then the accumulated
// rotations V; the singular values go to sig.
struct SvdTask { int R, w; long long rtab, ws, sig; };
// Output of one task: kappa kept vectors (tabs[sel + mu] = column of X) into
// the left site tensor (row i of M at tabs[atab + i], plus mu) and the right
// one (bbase + mu * bstride + j); left: U to the left site (left-orthonormal
// split), else U S to the left and V^+ to the right.
struct SvdEmit { int task, kappa, left, pad; long long atab, bbase, bstride, sel; };
struct PairPlan {
  PairLayout L;
  // join: 0 = A_k, 1 = A_{k+1}, 2 = Theta (blocks whose middle charge the
  // current middle bond lacks stay as cleared beforehand)
  GemmPlan join;
  // H^(2): s1 (0 = L env, 1 = Theta, 2 = T1), w1 (T1 -> T2: the MPO of site
  // k), w2 (T2 -> T3: the MPO of site k+1, rows grouped by the right bra
  // sector), s4 (0 = T3, 1 = R env, 2 = output)
  GemmPlan s1, s4;
  WPlan w1, w2;
  long long t1_size = 0, t2_size = 0, t3_size = 0;
  // split: one SVD task per middle charge (rows in (l, g1, s1, x) order)
  std::vector<Q> mq;
  std::vector<std::vector<std::array<int, 3>>> rowgroups;   // per task: (l, g1, position of s1), dl rows each
  std::vector<SvdTask> svd;
  long long svd_ws = 0, svd_nsig = 0;
};
PairPlan build_pair_plan(const Bond& bl, const Bond& bm, const Bond& br, const Groups& G,
                         const std::vector<Q>& qHl, const std::vector<Q>& qHm, const std::vector<Q>& qHr,
                         const std::vector<double>& W1, const std::vector<double>& W2,   // ket-only DH x 4 x 4 x DH
                         const SiteLayout& SA, const SiteLayout& SB, SiteTables& tabs);

// tile the problems of a plan (shape per problem)
int gemm_cfg_for(int M, int N);
int gemm_smem_bytes(int cfg);     // LDS bytes of one tile of shape cfg
void tile_plan(GemmPlan& p, const std::vector<long long>* tabs);   // tabs: host copy of the index tables

}  // namespace tt
