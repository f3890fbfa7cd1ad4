/*
 * tantrg.h - C ABI of the one-site tangent-space imaginary-time sweep of the
 * density-operator MPO rho(beta) for the Hubbard model (tanTRG,
 * arXiv:2212.11973), on AMD MI355X (gfx950).
 *
 * The state is the super-MPS |rho>> of the Choi map (SM Sec. II.A): site k
 * holds A_k[x, s, y] with s = 4*sigma + sigma' (sigma the ket index, on which
 * H acts; sigma' the ancilla), bond dimensions D_k, k = 0..N.  The library
 * keeps rho = e^Lambda * (normalised mixed-canonical MPS), Lambda = ln||rho||_F.
 *
 * Conventions for every entry point:
 *   - returns 0 (TT_OK) on success, a negative TT_E* code on failure; the
 *     failing call leaves a message for tt_last_error() (thread-local);
 *     no C++ exception crosses the ABI;
 *   - pointers named host_* are host memory owned by the caller; pointers
 *     named dev_* are device memory owned by the caller; tt_state handles and
 *     all device memory behind them are owned by the library and released by
 *     tt_state_free();
 *   - all device work is enqueued on the stream set by tt_set_stream()
 *     (default: the null stream); calls that return values to the host
 *     synchronise that stream before returning;
 *   - a tt_state is not thread-safe; distinct states may be used from
 *     distinct threads.
 */
#ifndef TANTRG_H
#define TANTRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque state handle. */
typedef struct tt_state tt_state;

/* error codes */
#define TT_OK 0
#define TT_EINVAL -1    /* bad argument (sizes, enums, null pointers, unsupported option) */
#define TT_ENOMEM -2    /* device or host allocation failed */
#define TT_EDEVICE -3   /* a HIP call failed or no gfx950 device is usable */
#define TT_ENUMERIC -4  /* NaN/Inf met, or a sector QR with more columns than rows */
#define TT_EIO -5       /* file I/O failed or the file is not a saved state */

/* lattice geometry: main text, Hubbard-model paragraph (cylinders CL WxL,
 * periodic across W, open along L; open squares OS) and Fig. 1a (snake) */
#define TT_CHAIN 0
#define TT_CYLINDER 1
#define TT_OPEN_SQUARE 2

/* precision of the bulk contractions (FP64 is always kept for the Lanczos
 * scalars and reorthogonalisation, the QR gauge moves and Lambda) */
#define TT_FP64 0
#define TT_FP32 1    /* the contraction intermediates (T1, T2 and those of the environment updates)
                        stored in float; the small blocks of a block-sparse sweep multiply in FP64,
                        dense tiles (M, N, K >= 128) with FP32 MFMA (FP32 inside a K tile, FP64 across) */
#define TT_BF16X3 2  /* split-BF16: hi*hi + hi*lo + lo*hi per 16- or 32-deep chunk, FP32 MFMA
                        accumulation inside a chunk, FP64 across chunks */
#define TT_BF16X6 3  /* split-BF16 with three parts, six products */

/* Eq. (3): H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum n_iu n_id - mu sum n_i,
 * with the next-nearest hopping of SM Eq. S1, -tp sum_<<ij>>,s (c+_is c_js +
 * h.c.), over diagonal neighbours (squared lattice distance 2, a cylinder's
 * width taken the short way for W >= 3; a chain has none).  tp = 0 gives the
 * MPO of Eq. (3) unchanged; tp != 0 adds the diagonal partners to its
 * channels (larger D_H).  hp != 0 adds the d-wave pairing field of the main
 * text's pairing paragraph, -hp sum_<ij> s_ij (Delta_ij + Delta_ij^+)/2 with
 * Delta_ij = (c_i,dn c_j,up - c_i,up c_j,dn)/sqrt 2 and s_ij = +1 (-1) for a
 * bond along the length (across the width); it breaks the particle numbers,
 * so it needs symmetry = 0 or 2 (TT_EINVAL otherwise). */
typedef struct {
  int W, L;          /* width and length; chain: W = 1 */
  int geometry;      /* TT_CHAIN, TT_CYLINDER (wrap across W only for W >= 3), TT_OPEN_SQUARE */
  double t, tp, U, mu;
  double hp;         /* pairing field (0: none) */
} tt_model;

typedef struct {
  int D;               /* target bond dimension (bonds never exceed the maximal one) */
  int symmetry;        /* 0 dense, 1 U(1)charge x U(1)spin block-sparse, 2 block-sparse
                          in q_up - q_dn alone (the charge a pairing field keeps;
                          sectors reported as (sz, 0)) */
  double beta0;        /* rho0 = 1 - beta0 H (main text: high-temperature start) */
  int taylor_order;    /* 1: rho0 = 1 - beta0 H; 2..4: the SETTN start
                          sum_{n <= order} (-beta0 H)^n / n! (SM I.E), the
                          product MPO of H reduced exactly to independent bond
                          states (ordered Gram-Schmidt); TT_EINVAL if the
                          product is too large or a reduction decision would
                          rest on rounding */
  int krylov_dim;      /* Lanczos dimension K (SM Sec. II.H), 1..32 */
  double krylov_tol;   /* lucky breakdown when beta_j <= tol*||H q_j|| (default 1e-13) */
  int precision;       /* TT_FP64 / TT_FP32 / TT_BF16X3 / TT_BF16X6 */
  double pad_eps;      /* amplitude of the seeded padding noise (0: zero padding) */
  uint64_t seed;       /* SplitMix64 seed of the padding noise */
  int env_on_host;     /* must be 0 (not supported) */
  int sector_cap;      /* largest sector of a padded block-sparse bond (0: no cap) */
} tt_options;

typedef struct {
  double beta;         /* MPO parameter: |rho>> approximates exp(-beta H) (1 - beta0 H) */
  double beta_phys;    /* 2*beta: inverse temperature of the bilayer values */
  double lnZ;          /* ln ||rho(beta)||_F^2 = ln Z(beta_phys) (bilayer, SM Sec. II.A) */
  double f;            /* -lnZ / (N beta_phys) */
  double E;            /* <<rho|H (x) 1|rho>> / <<rho|rho>> */
  double e;            /* E / N */
  double lnZ_single;   /* ln Tr rho(beta) (single layer) */
  double lambda;       /* Lambda = ln ||rho||_F */
  int n_sites;
  double herm_defect;  /* ||rho - rho^T||_F / ||rho||_F = sqrt(2 - 2 <<rho|P|rho>>/<<rho|rho>>), P the
                          exchange sigma <-> sigma' on every site (rho real, so rho^T = rho^dagger); zero
                          for the exact state, and a measure of the one-sided flow's projection error
                          (resolution about 1e-8: the square root of rounding in the overlap) */
} tt_observables;

typedef struct {
  double seconds;          /* wall time of the call (host clock, stream synchronised) */
  double flops_alg;        /* algorithmic flops of all contractions (sum of 2mnk per GEMM) */
  double flops_heff;       /* of which in effective-Hamiltonian applies (site and bond) */
  int n_applies;           /* site + bond effective-Hamiltonian applies */
  int n_exps;              /* local exponentials */
  double max_krylov_err;   /* max a-posteriori Lanczos estimate beta_K |[exp(tT)]_{K,1}| */
  double bytes_min;        /* minimum HBM bytes of the applies: 8 (|L| + |R| + 2 |x|) per apply (each operand
                              read once, the result written once; x the site tensor or bond matrix) */
  /* device milliseconds per phase, from HIP events around every occurrence
     (zeros unless tt_phase_timing is on): site applies (the MPO folded into the
     left environment included), bond applies, the Lanczos vector work of the
     local exponentials (their time minus their applies), QR/LQ, environment
     updates, absorbs */
  double t_heff, t_bond, t_lanczos, t_qr, t_env, t_absorb;
  long long n_launches;    /* kernels enqueued (a replayed sweep graph counts the launches it holds) */
  double discarded;        /* tdvp_sweep2: the largest discarded weight of a split, sum of the dropped
                              squared singular values over the sum of all of them; 0 otherwise */
} tt_sweep_stats;

/* Default options: D=64, symmetry=1, beta0=1e-2, taylor_order=1, K=8,
 * tol=1e-13, FP64, pad_eps=0, seed=1, env_on_host=0, sector_cap=64. */
int tt_options_default(tt_options* opts);

/* Build rho0 = 1 - beta0*H (main text, noninteracting-benchmark paragraph)
 * as a super-MPS from the finite-state-machine MPO of Eq. (3), pad every
 * bond to opts->D (U(1)xU(1) sectors sized by the rule documented with the
 * library), add pad_eps seeded noise on padding entries, right-canonicalise
 * by LQ (diag >= 0) and build the right environments.  beta = beta0.
 * *out receives a new state owned by the caller (free with tt_state_free). */
int mpo_init_highT(const tt_model* model, const tt_options* opts, tt_state** out);

/* One symmetric 1-TDVP step beta -> beta + dbeta (SM Sec. II.F steps 1-7,
 * SM Sec. II.E splitting): left-to-right with tau = dbeta/2 (site
 * exp(-tau H^(1)), QR, left environment, bond exp(+tau H^(0)), absorb), the
 * two last-site exponentials merged into one with 2*tau, then right-to-left
 * with LQ.  Every local exponential is a Lanczos exponential (SM Sec. II.H)
 * and is followed by normalisation into Lambda.  stats may be NULL.
 * Enqueued asynchronously unless stats is non-NULL. */
int tdvp_sweep(tt_state* state, double dbeta, tt_sweep_stats* stats);

/* The same step for n independent states (e.g. a chemical-potential scan).
 * Consecutive states with identical plans (same lattice, options and bond
 * sectors; the couplings may differ) advance together, up to 16 per kernel
 * launch; others run in their own groups.  Results equal those of separate
 * tdvp_sweep calls bit for bit.  A state may appear only once (TT_EINVAL).
 * stats (may be NULL) are summed. */
int tdvp_sweep_batch(tt_state** states, int n, double dbeta, tt_sweep_stats* stats);

/* One symmetric 2-TDVP step beta -> beta + dbeta (SM Sec. "2-TDVP in the
 * initial stage", Eq. S-2TDVP), which grows the bonds: left to right over the
 * pairs (k, k+1), the two-site tensor Theta = A_k A_{k+1} <- exp(-tau
 * H^(2)) Theta (Lanczos, normalised into Lambda), split by an SVD in every
 * charge sector of the middle bond with a left-orthonormal A_k, the left
 * environment, then the backward step A_{k+1} <- exp(+tau H^(1)) A_{k+1};
 * the two exponentials of the last pair merged into one with 2 tau; right to
 * left mirrored (A_k = U S, A_{k+1} = V^+, the right environment, then
 * A_k <- exp(+tau H^(1)) A_k for k > 0).  Each split keeps the largest
 * singular values over all sectors: at most D_max, each above cutoff times
 * the largest (cutoff 0: no relative threshold), exact zeros never, at least
 * one.  A sector may appear or vanish at every split; the bond sectors of the
 * state change accordingly and every plan is rebuilt for them before the
 * call returns (cached observable plans and a captured sweep are dropped).
 * Typical use: start at the bare rho0 (opts.D = 1, pad_eps = 0), run a few
 * tdvp_sweep2 steps until the bonds reach the wanted size, then tdvp_sweep.
 * FP64 states only (TT_EINVAL otherwise).  TT_ENUMERIC if a later
 * truncation left a bond sector with more states than the one-site gauge
 * moves can hold (the bond's neighbours reach fewer states): then only
 * tdvp_sweep2 and the observables run on the state until a further
 * tdvp_sweep2 repairs it.  Synchronises; stats may be NULL. */
int tdvp_sweep2(tt_state* state, double dbeta, int D_max, double cutoff, tt_sweep_stats* stats);

/* How each site applies H^(1) (SM Fig. optimalB(c)), and its left bond
 * H^(0) (SM Fig. optimalB(d)); the result is the same up to rounding.  Site
 * form 0 is the contraction order of SM Fig. Lanczos: T1 = L.A, the sparse MPO
 * stage into T2, then .R.  Form 1 folds the MPO into the left environment
 * once per environment (LW^{b,so,si} = sum_a W[a,so,si,b] L^a) and applies
 * T2 = LW.A, then .R: no T1 and no per-apply MPO stage, but grouped GEMMs one
 * charge sector wide.  Form 2 (FP64 states only) uses the same fold and runs
 * LW.A.R as one kernel per apply: each output block sums (LW.A)_b R_b^T over
 * the MPO index b with the T2 block held in registers, so neither T1 nor T2
 * is written.  The bond apply is L.S into an intermediate then .R (bond form
 * 0), or (bond form 1, FP64 states) the same kernel with one term L^a S per
 * MPO index a.  host_forms[k] = f + 4 b holds site k's form f and its left
 * bond's form b.  mode 0 or 1 sets site form 0 or 1 and bond form 0
 * everywhere, mode 4 sets site form 2 and bond form 1 everywhere; mode 2
 * times every form of every site's apply and of its bond apply on the device
 * (the fold's build spread over the 2K + 1 uses it serves per sweep) and
 * keeps the fastest; mode 3 sets the forms from host_forms (N entries; e.g.
 * one instance's tuned choice for a whole batch).  The state starts in forms
 * 0.  For modes 0-2 and 4, host_forms (may be NULL) receives the N chosen
 * values.  States advance together in tdvp_sweep_batch only with equal forms.
 * TT_EINVAL for the fused forms on a state that is not FP64.  Synchronises. */
int tt_tune_apply(tt_state* state, int mode, int* host_forms);

/* Bilayer observables of SM Sec. II.A at beta_phys = 2*beta: lnZ = 2 Lambda,
 * E from one H^(1) apply at the canonical centre, the single-layer
 * ln Tr rho(beta) and the hermiticity defect by transfer matrices.  Valid for
 * a state as left by mpo_init_highT or tdvp_sweep (centre at site 0).
 * Synchronises. */
int thermo_observables(tt_state* state, tt_observables* out);

/* Local observables per site at beta_phys = 2 beta (same bilayer meaning as
 * thermo_observables): host_out2[0] = particle density n = <N>/N_sites,
 * host_out2[1] = double occupancy D_n = <sum_i n_up,i n_dn,i>/N_sites (the
 * quantity of main text Fig. 2), each <<rho|O (x) 1|rho>> / <<rho|rho>> for a
 * sum of on-site operators O (SM Sec. II.A, bilayer).  Evaluated with the
 * two-channel MPO of O through right environments to the centre (site 0):
 * valid for a state as left by mpo_init_highT or tdvp_sweep.  The first call
 * on a state builds the needed plans; FP64 in every precision mode.
 * Synchronises.  TT_ENUMERIC for non-finite results. */
int thermo_local_observables(tt_state* s, double* host_out2);

/* Spin correlation F(d) = (1/N_d) sum over the N_d pairs (i, j) at squared
 * lattice distance d2 of <S_i . S_j> (main text, Fig. 2(c)), S_i . S_j =
 * Sz_i Sz_j + (S+_i S-_j + S-_i S+_j)/2, as the bilayer value at beta_phys =
 * 2 beta (<<rho|O (x) 1|rho>> / <<rho|rho>>, SM Sec. II.A).  The distance is
 * dx^2 + dy^2 on the lattice, dy the short way round a cylinder's width;
 * *host_npairs (may be NULL) receives N_d.  Evaluated with a finite-state-
 * machine MPO of the pair sum through right environments to the centre
 * (site 0): valid for a state as left by mpo_init_highT or tdvp_sweep.  The
 * first call for a d2 builds its plans; FP64 in every precision mode.
 * Synchronises.  TT_EINVAL if no pair lies at that distance. */
int thermo_spin_correlation(tt_state* s, int d2, double* host_F, int* host_npairs);

/* Single-particle Matsubara Green's function at half the imaginary time
 * (main text, Fermi-surface paragraph): *host_G = G(k, beta_phys/2) =
 * sum_s <exp(beta_phys H/2) c+_ks exp(-beta_phys H/2) c_ks> at beta_phys = 2 beta,
 * c_ks = N^-1/2 sum_r exp(-i k.r) c_rs, i.e. Tr[rho c+_k rho c_k] / Tr[rho rho]
 * for the state's rho(beta): the bilayer expectation of a super-operator MPO
 * that acts on both the ket and the ancilla index (Choi map, SM Sec. II.A).
 * r = (x, y) lattice coordinates, x = 0..L-1 along the length, y = 0..W-1
 * across the width; k = (kx, ky) in radians per lattice spacing.  The first
 * call builds the plans (FP64 in every precision mode); a later call with
 * another k rewrites their weights only.  Synchronises.  TT_EINVAL for a
 * non-finite k. */
int thermo_green_function(tt_state* s, double kx, double ky, double* host_G);

/* d-wave pairing order per bond (main text, pairing paragraph):
 * *host_delta = <Delta_tot> / N_p at beta_phys = 2 beta (bilayer), Delta_tot
 * as in tt_model with N_p nearest-neighbour bonds (*host_nbonds, may be NULL);
 * the susceptibility is chi_SC = Delta_p / hp.  Needs a state with
 * symmetry = 0 or 2 (TT_EINVAL otherwise: with both U(1) charges the value is
 * 0 by symmetry).  The first call builds the plans; FP64.  Synchronises. */
int thermo_pairing_order(tt_state* s, double* host_delta, int* host_nbonds);

/* Entropy and specific heat per site from n >= 3 bilayer observables taken
 * along a sweep (host arrays of length n, beta = beta_phys strictly
 * increasing, e and f per site as in tt_observables): s_out[i] = beta (e - f)
 * and c_out[i] = C_e = -beta de/dln(beta) (main text, Fig. 2(b); SM Fig.
 * S1(c)), the slope from the quadratic through three neighbouring points
 * (centred, one-sided at the ends).  Host arithmetic only; TT_EINVAL for
 * n < 3, null pointers, non-finite or non-increasing input. */
int tt_thermo_derived(int n, const double* beta, const double* e, const double* f, double* c_out, double* s_out);

void tt_state_free(tt_state* state);
const char* tt_last_error(void);

/* n_sites and the N+1 bond dimensions (host_dims may be NULL). */
int tt_state_info(const tt_state* state, int* n_sites, int* host_dims);
/* Sectors of bond k: counts into *nsec; if the arrays are non-NULL they must
 * hold *nsec entries on input (query with NULL first). */
int tt_state_bond_sectors(const tt_state* state, int k, int* nsec,
                          int* host_qup, int* host_qdn, int* host_dim);
/* Site tensor k as a dense host array [D_k][16][D_{k+1}] (bond index order:
 * sectors by (q_up, q_dn), then the index inside the sector).  Export writes
 * zeros outside the charge-allowed blocks; import ignores them.  Synchronises. */
int tt_state_export_site(const tt_state* state, int k, double* host_dense);
int tt_state_import_site(tt_state* state, int k, const double* host_dense);
/* Save / load the whole state (tensors, sectors, beta, Lambda, sweep count)
 * to a binary file; load rebuilds the environments. */
int tt_state_save(const tt_state* state, const char* path);
int tt_state_load(const char* path, tt_state** out);

/* One dense effective-Hamiltonian apply (SM Fig. optimalB(c), contraction
 * order of SM Fig. Lanczos):
 *   out[x,so,sp,y] = sum L[x,a,al] A[al,si,sp,be] W[a,so,si,b] R[y,b,be]
 * with dev_L [Dl][DH][Dl], dev_W [DH][4][4][DH], dev_A and dev_out
 * [Dl][4][4][Dr], dev_R [Dr][DH][Dr], all FP64 row-major device arrays owned
 * by the caller; stream is a hipStream_t (NULL: the library stream).
 * L.A and .R run as large-tile MFMA GEMMs on copies of the operands whose
 * rows run along the contracted index, zero-padded to the GEMM's K tile (A
 * transposed): FP64 copies (TT_FP64), copies rounded to FP32 (TT_FP32, FP32
 * multiplies, partial sums added in FP64), or BF16 planes (the split-BF16
 * precisions: each element split once into 2 or 3 BF16 parts, 3 or 6 part
 * products; bf16x6 adds its partial sums in FP64, bf16x3 accumulates in FP32
 * on launches large enough for its 256 x 256 tiles).  The W stage runs on the
 * matrix cores between them.  T1 and T2
 * are kept in the precision's storage (FP64, FP32 or planes).  For DH > 20
 * the FP64 and FP32 modes use the grouped-GEMM path of the sweep instead.
 * Workspace of about 8*(Dl*DH*16*Dr)*2 bytes plus the padded copies is kept
 * by the library between calls.  Returns after enqueueing. */
int tt_heff_apply(int Dl, int Dr, int DH, const double* dev_L, const double* dev_W,
                  const double* dev_A, const double* dev_R, double* dev_out, int precision,
                  void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the apply of
 * tt_heff_apply, same arguments, layouts and result (the same kernels and
 * launch plans, so in FP64 and FP32 the output is bit for bit that of
 * tt_heff_apply; in the split-BF16 modes it runs the sweep's grouped GEMMs,
 * which split every element inside the tiles and keep T1 and T2 in FP64,
 * where tt_heff_apply works on operands and intermediates pre-split into BF16
 * planes), with
 * every byte of device memory it needs beyond the caller's inputs and output
 * (the intermediates T1 = L.A and T2, the padded operand copies, the K-slice
 * partial tiles and the launch descriptors) taken from a static device array
 * of 192 MiB that each GPU the library runs on holds until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine.  TT_EINVAL for sizes whose
 * intermediates do not fit (16*Dl*DH*16*Dr bytes for T1 and T2 alone; e.g.
 * Dl = Dr = 128 at DH = 18 fits), for non-positive sizes, null pointers, an
 * unknown precision, or kernel profiling switched on.  Every call on one GPU
 * shares that GPU's array and leaves its contents (descriptors of the last
 * sizes are reused when the sizes repeat; nothing needs to start at zero):
 * calls that overlap on one GPU (other streams, other threads) race and must
 * be serialised by the caller.  Enqueued on `stream` (NULL: the library's
 * stream), no synchronisation. */
int tt_heff_apply_noalloc(int Dl, int Dr, int DH, const double* dev_L, const double* dev_W,
                          const double* dev_A, const double* dev_R, double* dev_out, int precision,
                          void* stream);

/* The two-site generator of 2-TDVP (SM Sec. "2-TDVP in the initial stage",
 * Eq. S-2TDVP) on dense operands, for measurement and tests:
 * out[x][s1][s2][y] = sum L[x][a][x'] C[x'][s1'][s2'][y'] W1[a][so1][si1][b]
 * W2[b][so2][si2][c] R[y][c][y'], the MPO tensors acting on the ket index
 * sigma of s = 4 sigma + sigma'.  Device pointers, row-major FP64:
 * L[Dl][DH][Dl], W1 and W2 [DH][4][4][DH], C and out [Dl][16][16][Dr],
 * R[Dr][DH][Dr]; out must not alias an input.  Four grouped GEMMs in the
 * order L.C, W1, W2, .R (the ancilla indices ride along), in the given
 * precision (TT_FP64 ...).  Enqueued on `stream` (NULL: the library's stream),
 * no synchronisation.  TT_EINVAL for non-positive sizes, null pointers or an
 * intermediate above 4e9 elements. */
int tt_heff2_apply(int Dl, int Dr, int DH, const double* L, const double* W1, const double* W2,
                   const double* C, const double* R, double* out, int precision, void* stream);

/* Stream for all later work (a hipStream_t; NULL for the null stream). */
int tt_set_stream(void* stream);
/* Device allocator used for all later allocations (both NULL: hipMalloc/hipFree). */
typedef void* (*tt_alloc_fn)(size_t bytes, void* ctx);
typedef void (*tt_free_fn)(void* ptr, void* ctx);
int tt_set_allocator(tt_alloc_fn alloc, tt_free_fn free_fn, void* ctx);

/* Device time (ms) of the last tt_heff_apply per stage, measured with HIP
 * events on the stream it ran on: [0] L.A, [1] W stage, [2] .R, [3] total.
 * Synchronises. */
int tt_heff_last_timing(double* host_ms4);

/* The 2-TDVP split's SVD (SM Sec. "2-TDVP in the initial stage"): a
 * middle-charge block whose matrix X (and its column norms) fits max_doubles
 * doubles of one workgroup's LDS is orthogonalised by one workgroup; larger
 * blocks run the same one-sided Jacobi with each round spread over the GPU
 * (one launch per round, one wave per column pair; one host synchronisation
 * per sweep).  0 (the default): the device's LDS.  A smaller limit sends more
 * blocks to the spread form; both forms take the same pairs in the same
 * order with the same arithmetic.  Takes effect for the splits planned after
 * the call.  TT_EINVAL for a negative size. */
int tt_svd_lds_limit(long long max_doubles);

/* Sweeps as replayed hipGraphs (default off).  When on, the first
 * tdvp_sweep of a state with a step dbeta captures the sweep's launches
 * into a graph (on a private stream; the call's results are those of the
 * graph's first launch), and later tdvp_sweep calls with the same dbeta
 * launch that graph on the registered stream; a different dbeta captures
 * anew.  Results equal those of uncaptured sweeps bit for bit.  Not used
 * while profiling is enabled, nor by tdvp_sweep_batch. */
int tt_sweep_graphs(int on);

/* Per-phase device timing of sweeps that return stats (default off): every
 * phase occurrence of tdvp_sweep / tdvp_sweep_batch is bracketed by HIP events
 * on the library stream and summed into the t_* fields of tt_sweep_stats
 * (sweep graphs are not used meanwhile).  The events cost host time per phase,
 * so timed runs leave it off. */
int tt_phase_timing(int on);

/* Opt-in kernel timing: when on, every launch of the grouped GEMM, the MPO
 * (W) stage and the QR kernels is bracketed by HIP events on its stream, and
 * inside a grouped GEMM every kernel dispatch is timed on its own.
 * tt_profile_read synchronises those events and fills host_out72 with
 * {ms, flops, bytes, launches} for eighteen kinds accumulated since the
 * previous read, then resets:
 *   0-7   the grouped GEMM by contraction (all its dispatches together):
 *         L.A, .R, left environment, right environment (R.A), right
 *         environment (A.Z), bond apply, absorb, dense W stage;
 *   8, 9  the sparse W stage and the QR;
 *   10-14 the GEMM kernel of each tile shape (64x64, 128x32, 256x16, 32x128,
 *         32x32), one record per dispatch;
 *   15    the K-slice reduce kernel, one record per dispatch;
 *   16    the wave GEMM kernel (small and skinny problems), one record per
 *         dispatch;
 *   17    the fused one-site apply (L with the MPO folded in, times the site
 *         tensor, times R, in one kernel), one record per dispatch.
 * Flops and bytes are algorithmic (sum of 2mnk; every operand element read
 * once, every output written once); for the reduce, the partial tiles read
 * and the outputs written. */
int tt_profile_enable(int on);
int tt_profile_read(double* host_out72);

/* Host-only: the sectors bond k would get for this model and options (same
 * calling convention as tt_state_bond_sectors).  No GPU needed. */
int tt_model_bond_sectors(const tt_model* model, const tt_options* opts, int k, int* nsec,
                          int* host_qup, int* host_qdn, int* host_dim);

/* Host-only consistency check (no GPU needed): builds every descriptor the
 * kernels of a state with this model and options would use and counts index
 * ranges that fall outside the buffers they address (*violations; details
 * via tt_last_error()).  *work_doubles (may be NULL) receives the doubles held
 * by the site tensors and environments. */
int tt_check_plans(const tt_model* model, const tt_options* opts, long long* violations,
                   long long* work_doubles);

#ifdef __cplusplus
}
#endif
#endif
