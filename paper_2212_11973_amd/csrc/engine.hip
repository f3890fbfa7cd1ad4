// State, sweep driver and C ABI of the tanTRG library.
//
// The sweep follows SM Sec. II.F steps 1-7 with the splitting of SM Sec. II.E:
// left-to-right (site exp(-tau H1), QR, left environment, bond exp(+tau H0),
// absorb), the two last-site exponentials merged into one with 2 tau, then
// right-to-left with LQ.  Every local exponential is a Lanczos exponential
// (SM Sec. II.H) followed by normalisation, whose log-norm is accumulated into
// Lambda = ln ||rho||_F on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>

#include "kernels.h"

using namespace tt;

namespace {

thread_local std::string g_err;
hipStream_t g_stream = nullptr;
bool g_graphs = false;   // sweeps captured into hipGraphs and replayed (tt_sweep_graphs)
bool g_phase = false;    // per-phase device timing of sweeps with stats (tt_phase_timing)
tt_alloc_fn g_alloc = nullptr;
tt_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;

#define HIPX(call)                                                              \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) throw Error(TT_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// Allocations made through a registered allocator, with the free function
// and context that must release them (the registration may change meanwhile).
std::mutex g_alloc_mu;
std::unordered_map<void*, std::pair<tt_free_fn, void*>> g_custom;

void* dalloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (g_alloc) {
    p = g_alloc(bytes, g_alloc_ctx);
    if (!p) throw Error(TT_ENOMEM, "device allocation failed (custom allocator)");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_custom[p] = {g_free, g_alloc_ctx};
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Error(TT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return p;
}
void dfree(void* p) {
  if (!p) return;
  std::pair<tt_free_fn, void*> f{nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_custom.find(p);
    if (it != g_custom.end()) {
      f = it->second;
      g_custom.erase(it);
    }
  }
  if (f.first) f.first(p, f.second);
  else (void)hipFree(p);
}
template <class T>
T* upload(const std::vector<T>& v, hipStream_t st) {
  T* d = (T*)dalloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) HIPX(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  return d;
}

void check_device() {
  int n = 0;
  HIPX(hipGetDeviceCount(&n));
  if (n < 1) throw Error(TT_EDEVICE, "no HIP device");
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPX(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    throw Error(TT_EDEVICE, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
}

void upload_plan(GemmPlan& p, const std::vector<long long>* tabs, hipStream_t st) {
  tile_plan(p, tabs);
  p.d_probs = upload(p.probs, st);
  p.d_tiles = upload(p.tiles, st);
  p.d_splits = upload(p.splits, st);
  p.d_jobs = upload(p.jobs, st);
  p.d_jobs_fine = upload(p.jobs_fine, st);
}
void upload_plan(WPlan& p, hipStream_t st) {
  p.ntasks = (int)p.tasks.size();
  p.d_tasks = upload(p.tasks, st);
  p.d_terms = upload(p.terms, st);
}
// assign workspace (global fallback area first, then the LDS path's chunk
// factors) and upload every descriptor of a QR plan
void upload_plan(QRPlan& p, hipStream_t st) {
  p.ntasks = (int)p.tasks.size();
  long long pos = 0;
  for (auto& t : p.tasks) {
    TT_REQUIRE(t.m >= t.n, TT_ENUMERIC, "QR of a charge block with more columns than rows");
    t.ws = pos;
    pos += qr_wide_ws(t.m, t.n);
  }
  p.ws_size = pos;
  qr_plan_chunks(p);
  p.d_tasks = upload(p.tasks, st);
  p.d_chunks = upload(p.chunks, st);
  p.d_stacks = upload(p.stacks, st);
  p.d_wide = upload(p.wide, st);
}
void free_plan(GemmPlan& p) {
  dfree(p.d_probs); dfree(p.d_tiles); dfree(p.d_splits); dfree(p.d_jobs); dfree(p.d_jobs_fine);
  p.d_probs = nullptr; p.d_tiles = nullptr; p.d_splits = nullptr; p.d_jobs = nullptr; p.d_jobs_fine = nullptr;
}
void free_plan(WPlan& p) { dfree(p.d_tasks); dfree(p.d_terms); p.d_tasks = nullptr; p.d_terms = nullptr; }
void upload_plan(FzPlan& p, hipStream_t st) {
  p.d_outs = upload(p.outs, st);
  p.d_bs = upload(p.bs, st);
  p.d_terms = upload(p.terms, st);
  p.d_jobs = upload(p.jobs, st);
}
void free_plan(FzPlan& p) {
  dfree(p.d_outs); dfree(p.d_bs); dfree(p.d_terms); dfree(p.d_jobs);
  p.d_outs = nullptr; p.d_bs = nullptr; p.d_terms = nullptr; p.d_jobs = nullptr;
}
void free_plan(QRPlan& p) {
  dfree(p.d_tasks); dfree(p.d_chunks); dfree(p.d_stacks); dfree(p.d_wide);
  p.d_tasks = nullptr; p.d_chunks = nullptr; p.d_stacks = nullptr; p.d_wide = nullptr;
}

}  // namespace

// ====================================================================== state
struct tt_state {
  tt_model model{};
  tt_options opts{};
  int N = 0;
  Lattice lat;
  Mpo mpo;
  Rho0 rho0;                                // the start (cleared once the site tensors are filled)
  Groups G;
  std::vector<Bond> bonds;                  // 0..N
  std::vector<std::vector<Q>> qH;           // environment MPO charges per bond
  std::vector<std::vector<double>> Wenv;    // environment MPO tensors per site
  std::vector<std::vector<double>> Wpat;    // the same for generic couplings (nonzero pattern of the lattice)
  std::vector<SiteLayout> site;
  std::vector<EnvLayout> env;
  std::vector<BondMatLayout> bmat;
  std::vector<SitePlan> plans;
  SiteTables tabs;
  // device memory
  std::vector<double*> A, Lenv, Renv;
  // the swap overlap <<rho|P|rho>> (hermiticity defect): per site the plans
  // X = E_k A^{P(s)} and E_{k+1} = sum (A^s)^T X, transfer matrices E on (q, -q) blocks
  std::vector<GemmPlan> swp1, swp2;
  long long swp_e = 1, swp_x = 1;
  double *Ea = nullptr, *Eb = nullptr, *Xs = nullptr;
  double *T1 = nullptr, *T2 = nullptr, *Y = nullptr, *Z = nullptr, *U = nullptr;
  double *Sbuf = nullptr, *tmp = nullptr, *kry = nullptr, *wv = nullptr, *qrws = nullptr;
  double* pws = nullptr;                   // partial tiles of K-split GEMMs
  // capacities (doubles) of the scratch buffers above; the 2-TDVP steps grow them
  long long cap_T1 = 0, cap_T2 = 0, cap_Y = 0, cap_Z = 0, cap_U = 0, cap_pws = 0, cap_tmp = 0, cap_Sbuf = 0,
            cap_kry = 0, cap_wv = 0;
  // 2-TDVP: the two-site tensor, the H^(2) intermediates, the SVD work array
  // and singular values (allocated by the first two-site sweep)
  double *th = nullptr, *P1 = nullptr, *P2 = nullptr, *P3 = nullptr, *svw = nullptr, *svs = nullptr;
  long long cap_th = 0, cap_P1 = 0, cap_P2 = 0, cap_P3 = 0, cap_svw = 0, cap_svs = 0;
  bool one_site_ok = true;                 // every QR/LQ block has at least as many rows as columns
  double* LW = nullptr;                    // the MPO folded into the left environment of site lw_site
  int lw_site = -1;                        // -1: LW holds no current fold
  std::vector<char> fold;                  // per site: 1 = apply with the MPO folded into L, 0 = L.A, W, .R
  std::vector<char> bfz;                   // per site: 1 = its left bond's H^(0) apply as one fused launch
  double *part = nullptr, *lz = nullptr;   // lz: alpha[K] beta[K] hn[K] coeff[K] scal[4] lambda errmax scratch[4]
  double** d_sites = nullptr;
  TraceEntry* d_trace = nullptr;
  int* d_trace_start = nullptr;
  double* vtr = nullptr;
  long long max_site = 0, max_bond = 0, max_bmat = 0, max_env = 0;
  double beta = 0.0;
  long long sweeps = 0;
  // statistics of the current call
  double flops = 0.0, flops_heff = 0.0, bytes_min = 0.0;
  int n_applies = 0, n_exps = 0;

  // observables given as MPOs (sums of on-site operators, sums of spin
  // pairs), keyed by kind: plans and buffers built on the first request
  struct ObsMpo {
    SiteTables tabs;
    std::vector<SitePlan> plans;
    double kx = 0.0, ky = 0.0;   // the momentum whose weights the plans hold (Green's function)
    double *ea = nullptr, *eb = nullptr, *unit = nullptr, *pws = nullptr;
    double *T1 = nullptr, *T2 = nullptr, *Y = nullptr, *Z = nullptr;
  };
  std::map<int, ObsMpo> obs;

  // a captured sweep (hipGraph) for one step dbeta, replayed by later sweeps
  // with the same step; the host counters of one sweep are kept with it
  struct SweepGraph {
    hipGraphExec_t exec = nullptr;
    double dbeta = 0.0, flops = 0.0, flops_heff = 0.0, bytes_min = 0.0;
    int n_applies = 0, n_exps = 0;
    long long n_launches = 0;
  } sg;

  double* lam_ptr() { return lz + 4 * kMaxKrylov + 4; }
  double* err_ptr() { return lz + 4 * kMaxKrylov + 5; }
  double* obs_ptr() { return lz + 4 * kMaxKrylov + 6; }   // 4 scratch values
  ~tt_state();
};

// release every plan descriptor, table and scratch buffer sized by the plans
// (everything the bonds determine apart from the site tensors, environments,
// Lambda and the 2-TDVP buffers); cached observable plans and a captured sweep too
void free_scratch(tt_state& s) {
  auto free_site = [](SitePlan& p) {
    free_plan(p.s1); free_plan(p.s3); free_plan(p.el); free_plan(p.r1); free_plan(p.r3);
    free_plan(p.absL); free_plan(p.absR); free_plan(p.b1); free_plan(p.b2);
    free_plan(p.w2); free_plan(p.wr); free_plan(p.qr); free_plan(p.lq);
    free_plan(p.lw); free_plan(p.t2zero); free_plan(p.fz); free_plan(p.fzb);
    for (auto& g : p.s1w) free_plan(g);
  };
  for (auto& p : s.plans) free_site(p);
  for (double** p : {&s.T1, &s.T2, &s.Y, &s.Z, &s.U, &s.Sbuf, &s.tmp, &s.kry, &s.wv, &s.qrws, &s.vtr, &s.pws, &s.LW,
                     &s.Ea, &s.Eb, &s.Xs}) {
    dfree(*p);
    *p = nullptr;
  }
  s.cap_T1 = s.cap_T2 = s.cap_Y = s.cap_Z = s.cap_U = s.cap_pws = s.cap_tmp = s.cap_Sbuf = s.cap_kry = s.cap_wv = 0;
  dfree(s.d_sites); dfree(s.d_trace); dfree(s.d_trace_start); dfree(s.tabs.dev);
  s.d_sites = nullptr; s.d_trace = nullptr; s.d_trace_start = nullptr;
  s.tabs = SiteTables();
  for (auto& g : s.swp1) free_plan(g);
  for (auto& g : s.swp2) free_plan(g);
  if (s.sg.exec) (void)hipGraphExecDestroy(s.sg.exec);
  s.sg = tt_state::SweepGraph();
  for (auto& kv : s.obs) {
    tt_state::ObsMpo& O = kv.second;
    for (auto& p : O.plans) {
      free_plan(p.s1); free_plan(p.s3); free_plan(p.r1); free_plan(p.r3); free_plan(p.w2); free_plan(p.wr);
    }
    for (double* p : {O.ea, O.eb, O.unit, O.pws, O.T1, O.T2, O.Y, O.Z}) dfree(p);
    dfree(O.tabs.dev);
  }
  s.obs.clear();
}

tt_state::~tt_state() {
  // work enqueued on this state's buffers (a construction that failed part way
  // included) must finish before they go back to the allocator
  (void)hipStreamSynchronize(g_stream);
  free_scratch(*this);
  for (auto p : A) dfree(p);
  for (auto p : Lenv) dfree(p);
  for (auto p : Renv) dfree(p);
  for (double* p : {part, lz, th, P1, P2, P3, svw, svs}) dfree(p);
}

namespace {

hipStream_t ST() { return g_stream; }

// -------------------------------------------------------------- batches
// A batch: up to kMaxBatch states with identical plans (same lattice, bond
// sectors and options; the couplings may differ), advanced by the same
// launches.  Plan descriptors and tables come from the lead state; every
// data pointer is per state.  A single state is a batch of one.
struct Batch {
  int n = 0;
  tt_state* s[kMaxBatch] = {};
  tt_state& lead() const { return *s[0]; }
};
Batch batch_of(tt_state& st) {
  Batch b;
  b.n = 1;
  b.s[0] = &st;
  return b;
}
template <typename F> BPtr<double> per_state(const Batch& b, F f) {
  BPtr<double> r{};
  for (int i = 0; i < b.n; ++i) r.p[i] = f(*b.s[i]);
  return r;
}
BPtr<double> offset(BPtr<double> x, const Batch& b, long long off) {
  for (int i = 0; i < b.n; ++i) x.p[i] = x.p[i] ? x.p[i] + off : nullptr;
  return x;
}
BPtr<double> pws_of(const Batch& b) { return per_state(b, [](tt_state& s) { return s.pws; }); }
// Slots of every state: slot j = f_j(state, index in batch)
template <typename F> BSlots slots_of(const Batch& b, F f) {
  BSlots r{};
  for (int i = 0; i < b.n; ++i) r.s[i] = f(*b.s[i], i);
  return r;
}
template <typename F> BPtr<const WTerm> terms_of(const Batch& b, F f) {
  BPtr<const WTerm> r{};
  for (int i = 0; i < b.n; ++i) r.p[i] = f(*b.s[i]).d_terms;
  return r;
}
void add_flops(const Batch& b, double f, bool heff) {
  for (int i = 0; i < b.n; ++i) {
    b.s[i]->flops += f;
    if (heff) {
      b.s[i]->flops_heff += f;
      b.s[i]->n_applies++;
    }
  }
}

// -------------------------------------------------------------- phase clock
// With tt_phase_timing on, a sweep that returns stats brackets every phase
// occurrence with HIP events on the library stream: site applies (the MPO
// fold included), bond applies, whole local exponentials, QR/LQ, environment
// updates and absorbs.  The Lanczos vector work is an exponential's time
// minus its applies.
enum Phase { PH_HEFF = 0, PH_BOND, PH_EXP, PH_QR, PH_ENV, PH_ABSORB, PH_COUNT };
bool g_phase_on = false;   // set for the duration of a sweep whose stats are wanted
struct PhaseRec { hipEvent_t a, b; int ph; };
std::vector<PhaseRec> g_phase_recs;
std::vector<hipEvent_t> g_phase_pool;
hipEvent_t phase_event() {
  hipEvent_t e;
  if (!g_phase_pool.empty()) {
    e = g_phase_pool.back();
    g_phase_pool.pop_back();
    return e;
  }
  HIPX(hipEventCreate(&e));
  return e;
}
struct PhaseScope {
  int ph;
  hipEvent_t a = nullptr;
  explicit PhaseScope(int p) : ph(p) {
    if (!g_phase_on) return;
    a = phase_event();
    HIPX(hipEventRecord(a, ST()));
  }
  ~PhaseScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!g_phase_pool.empty()) {
      b = g_phase_pool.back();
      g_phase_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      g_phase_pool.push_back(a);
      return;
    }
    if (hipEventRecord(b, ST()) != hipSuccess) {
      g_phase_pool.push_back(a);
      g_phase_pool.push_back(b);
      return;
    }
    g_phase_recs.push_back({a, b, ph});
  }
};
// device ms per phase since the last read (synchronises the events)
void phase_read(double out[PH_COUNT]) {
  for (int i = 0; i < PH_COUNT; ++i) out[i] = 0.0;
  if (!g_phase_recs.empty()) HIPX(hipEventSynchronize(g_phase_recs.back().b));
  for (auto& r : g_phase_recs) {
    float ms = 0.f;
    HIPX(hipEventElapsedTime(&ms, r.a, r.b));
    out[r.ph] += ms;
    g_phase_pool.push_back(r.a);
    g_phase_pool.push_back(r.b);
  }
  g_phase_recs.clear();
}

// -------------------------------------------------------------- contractions
// LW <- the MPO of site k folded into L_k (once per environment; every apply
// and the left-environment update of site k read it)
void build_lw(const Batch& b, int k) {
  if (b.lead().lw_site == k) return;
  launch_wstage(b.lead().plans[k].lw, terms_of(b, [&](tt_state& s) -> WPlan& { return s.plans[k].lw; }),
                cst(per_state(b, [&](tt_state& s) { return s.Lenv[k]; })),
                per_state(b, [](tt_state& s) { return s.LW; }), b.n, ST());
  for (int i = 0; i < b.n; ++i) b.s[i]->lw_site = k;
  add_flops(b, b.lead().plans[k].lw.flops, false);
}

// T2 = LW . x in stage 3's layout: the pass-0 GEMMs, the cleared blocks, then
// the passes that add the further terms of an output block
void lw_times(const Batch& b, int k, BPtr<double> x) {
  SitePlan& P = b.lead().plans[k];
  const int prec = b.lead().opts.precision;
  const long long* tabs = b.lead().tabs.dev;
  for (int j = 0; j < P.n_s1w; ++j) {
    launch_gemm(P.s1w[j], tabs, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.LW, x.p[i], s.T2, nullptr}}; }),
                b.n, prec, pws_of(b), ST());
    if (j == 0)
      launch_wstage(P.t2zero, BPtr<const WTerm>{}, BPtr<const double>{}, per_state(b, [](tt_state& s) { return s.T2; }),
                    b.n, ST());
  }
  double f = 0.0;
  for (int j = 0; j < P.n_s1w; ++j) f += P.s1w[j].flops;
  add_flops(b, f, false);
}

// H^(1) x at site k in the site's form: the paper's order (T1 = L.x, the W
// stage into T2, then .R) or, with the MPO folded into L, T2 = LW.x then .R
void apply_heff1(const Batch& b, int k, BPtr<double> x, BPtr<double> out) {
  PhaseScope ps(PH_HEFF);
  SitePlan& P = b.lead().plans[k];
  const int prec = b.lead().opts.precision;
  const long long* tabs = b.lead().tabs.dev;
  double f1 = 0.0;
  if (b.lead().fold[k] == 2) {   // LW . x . R in one launch
    TT_REQUIRE(!P.fz.outs.empty(), TT_EINVAL, "fused apply: the site has no fused plan");
    build_lw(b, k);
    launch_fused(P.fz, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.LW, x.p[i], s.Renv[k + 1], out.p[i]}}; }),
                 b.n, ST());
    add_flops(b, P.fz.flops, true);
    const tt_state& L0 = b.lead();
    const double bm = 8.0 * (L0.env[k].size + L0.env[k + 1].size + 2.0 * L0.site[k].size);
    for (int i = 0; i < b.n; ++i) b.s[i]->bytes_min += bm;
    return;
  }
  if (b.lead().fold[k]) {
    build_lw(b, k);
    lw_times(b, k, x);
    for (int j = 0; j < P.n_s1w; ++j) f1 += P.s1w[j].flops;
    add_flops(b, -f1, false);   // lw_times counted them as other work: they belong to the apply
  } else {
    launch_gemm(P.s1, tabs, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.Lenv[k], x.p[i], s.T1, nullptr}}; }),
                b.n, prec, pws_of(b), ST());
    launch_wstage(P.w2, terms_of(b, [&](tt_state& s) -> WPlan& { return s.plans[k].w2; }),
                  cst(per_state(b, [](tt_state& s) { return s.T1; })), per_state(b, [](tt_state& s) { return s.T2; }),
                  b.n, ST());
    f1 = P.s1.flops + P.w2.flops;
  }
  launch_gemm(P.s3, tabs, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.T2, s.Renv[k + 1], out.p[i], nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  add_flops(b, f1 + P.s3.flops, true);
  const tt_state& L = b.lead();
  const double bmin = 8.0 * (L.env[k].size + L.env[k + 1].size + 2.0 * L.site[k].size);
  for (int i = 0; i < b.n; ++i) b.s[i]->bytes_min += bmin;
}

void apply_heff0(const Batch& b, int k, BPtr<double> x, BPtr<double> out) {
  PhaseScope ps(PH_BOND);
  SitePlan& P = b.lead().plans[k];
  const int prec = b.lead().opts.precision;
  const long long* tabs = b.lead().tabs.dev;
  if (b.lead().bfz[k]) {   // sum_a (L^a S) (R^a)^T in one launch
    TT_REQUIRE(!P.fzb.outs.empty(), TT_EINVAL, "fused bond apply: the bond has no fused plan");
    launch_fused(P.fzb, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.Lenv[k], x.p[i], s.Renv[k], out.p[i]}}; }),
                 b.n, ST());
    add_flops(b, P.fzb.flops, true);
    const double bm = 8.0 * (2.0 * b.lead().env[k].size + 2.0 * b.lead().bmat[k].size);
    for (int i = 0; i < b.n; ++i) b.s[i]->bytes_min += bm;
    return;
  }
  launch_gemm(P.b1, tabs, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.Lenv[k], x.p[i], s.U, nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  launch_gemm(P.b2, tabs, slots_of(b, [&](tt_state& s, int i) { return Slots{{s.U, s.Renv[k], out.p[i], nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  add_flops(b, P.b1.flops + P.b2.flops, true);
  const double bmin = 8.0 * (2.0 * b.lead().env[k].size + 2.0 * b.lead().bmat[k].size);
  for (int i = 0; i < b.n; ++i) b.s[i]->bytes_min += bmin;
}

void env_left(const Batch& b, int k) {   // Lenv[k+1] from Lenv[k], A_k (left-canonical), W_k, in the site's form
  PhaseScope ps(PH_ENV);
  SitePlan& P = b.lead().plans[k];
  const int prec = b.lead().opts.precision;
  const long long* tabs = b.lead().tabs.dev;
  if (b.lead().fold[k]) {
    build_lw(b, k);
    lw_times(b, k, per_state(b, [&](tt_state& s) { return s.A[k]; }));
  } else {
    launch_gemm(P.s1, tabs, slots_of(b, [&](tt_state& s, int) { return Slots{{s.Lenv[k], s.A[k], s.T1, nullptr}}; }),
                b.n, prec, pws_of(b), ST());
    launch_wstage(P.w2, terms_of(b, [&](tt_state& s) -> WPlan& { return s.plans[k].w2; }),
                  cst(per_state(b, [](tt_state& s) { return s.T1; })), per_state(b, [](tt_state& s) { return s.T2; }),
                  b.n, ST());
    add_flops(b, P.s1.flops + P.w2.flops, false);
  }
  launch_gemm(P.el, tabs, slots_of(b, [&](tt_state& s, int) { return Slots{{s.A[k], s.T2, s.Lenv[k + 1], nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  for (int i = 0; i < b.n; ++i)
    if (b.s[i]->lw_site == k + 1) b.s[i]->lw_site = -1;
  add_flops(b, P.el.flops, false);
}

void env_right(const Batch& b, int k) {  // Renv[k] from Renv[k+1], A_k (right-canonical), W_k
  PhaseScope ps(PH_ENV);
  SitePlan& P = b.lead().plans[k];
  const int prec = b.lead().opts.precision;
  const long long* tabs = b.lead().tabs.dev;
  launch_gemm(P.r1, tabs, slots_of(b, [&](tt_state& s, int) { return Slots{{s.Renv[k + 1], s.A[k], s.Y, nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  launch_wstage(P.wr, terms_of(b, [&](tt_state& s) -> WPlan& { return s.plans[k].wr; }),
                cst(per_state(b, [](tt_state& s) { return s.Y; })), per_state(b, [](tt_state& s) { return s.Z; }),
                b.n, ST());
  launch_gemm(P.r3, tabs, slots_of(b, [&](tt_state& s, int) { return Slots{{s.A[k], s.Z, s.Renv[k], nullptr}}; }),
              b.n, prec, pws_of(b), ST());
  add_flops(b, P.r1.flops + P.wr.flops + P.r3.flops, false);
}

// -------------------------------------------------------------- Lanczos exp
// v <- exp(t H) v / ||exp(t H) v||, Lambda += ln ||exp(t H) v||, for every state of the batch
void lanczos_exp(const Batch& b, double t, BPtr<double> v, long long n,
                 const std::function<void(BPtr<double>, BPtr<double>)>& H) {
  PhaseScope ps(PH_EXP);
  const tt_state& L = b.lead();
  const int K = L.opts.krylov_dim;
  const double tol = L.opts.krylov_tol;
  const int nb = b.n;
  BPtr<double> lz = per_state(b, [](tt_state& s) { return s.lz; });
  BPtr<double> alpha = lz, beta = offset(lz, b, kMaxKrylov), hn = offset(lz, b, 2 * kMaxKrylov);
  BPtr<double> coeff = offset(lz, b, 3 * kMaxKrylov), scal = offset(lz, b, 4 * kMaxKrylov);
  BPtr<double> err = per_state(b, [](tt_state& s) { return s.err_ptr(); });
  BPtr<double> lam = per_state(b, [](tt_state& s) { return s.lam_ptr(); });
  BPtr<double> Qb = per_state(b, [](tt_state& s) { return s.kry; });
  BPtr<double> wv = per_state(b, [](tt_state& s) { return s.wv; });
  BPtr<double> p1 = per_state(b, [](tt_state& s) { return s.part; });
  BPtr<double> p2 = offset(p1, b, (long long)kRedBlocks * (kMaxKrylov + 2));
  BPtr<double> none{};
  launch_mdot(cst(none), 0, 0, cst(v), n, 1, p1, nb, ST());
  launch_lz_start(cst(v), Qb, n, cst(p1), scal, nb, ST());
  for (int j = 0; j < K; ++j) {
    H(offset(Qb, b, (long long)j * n), wv);
    // pass 1: c = Q^T w (and ||w||), w -= Q c, dots and norm of the result;
    // pass 2: q_{j+1} = (w - Q c') / beta
    launch_mdot(cst(Qb), n, j + 1, cst(wv), n, 1, p1, nb, ST());
    launch_lz_sub_dot(wv, cst(Qb), n, j + 1, cst(p1), j + 2, n, offset(alpha, b, j), offset(hn, b, j), p2, nb, ST());
    launch_lz_sub_next(cst(wv), cst(Qb), n, j + 1, cst(p2), n, j + 1 < K ? offset(Qb, b, (long long)(j + 1) * n) : none,
                       offset(beta, b, j), cst(offset(hn, b, j)), tol, nb, ST());
  }
  launch_lz_coeffs(cst(alpha), cst(beta), cst(hn), K, t, tol, cst(scal), coeff, err, nb, ST());
  launch_lz_combine_norm(cst(Qb), n, K, cst(coeff), v, n, p1, nb, ST());
  launch_normalize_log(v, n, cst(p1), lam, nb, ST());
  for (int i = 0; i < nb; ++i) b.s[i]->n_exps++;
}

void site_exp(const Batch& b, int k, double t) {
  lanczos_exp(b, t, per_state(b, [&](tt_state& s) { return s.A[k]; }), b.lead().site[k].size,
              [&](BPtr<double> x, BPtr<double> y) { apply_heff1(b, k, x, y); });
}
void bond_exp(const Batch& b, int k, double t) {
  lanczos_exp(b, t, per_state(b, [](tt_state& s) { return s.Sbuf; }), b.lead().bmat[k].size,
              [&](BPtr<double> x, BPtr<double> y) { apply_heff0(b, k, x, y); });
}

void qr_site(const Batch& b, int k) {
  PhaseScope ps(PH_QR);
  launch_qr(b.lead().plans[k].qr, b.lead().tabs.dev, per_state(b, [&](tt_state& s) { return s.A[k]; }),
            per_state(b, [](tt_state& s) { return s.Sbuf; }), per_state(b, [](tt_state& s) { return s.qrws; }), b.n,
            ST());
}
void lq_site(const Batch& b, int k) {
  PhaseScope ps(PH_QR);
  launch_qr(b.lead().plans[k].lq, b.lead().tabs.dev, per_state(b, [&](tt_state& s) { return s.A[k]; }),
            per_state(b, [](tt_state& s) { return s.Sbuf; }), per_state(b, [](tt_state& s) { return s.qrws; }), b.n,
            ST());
}
void absorb_left(const Batch& b, int k) {   // A_k <- S_k A_k (S on the left bond k)
  PhaseScope ps(PH_ABSORB);
  SitePlan& P = b.lead().plans[k];
  launch_gemm(P.absL, b.lead().tabs.dev,
              slots_of(b, [&](tt_state& s, int) { return Slots{{s.Sbuf, s.A[k], s.tmp, nullptr}}; }), b.n, TT_FP64,
              pws_of(b), ST());
  launch_copy(per_state(b, [&](tt_state& s) { return s.A[k]; }), cst(per_state(b, [](tt_state& s) { return s.tmp; })),
              b.lead().site[k].size, b.n, ST());
  add_flops(b, P.absL.flops, false);
}
void absorb_right(const Batch& b, int k) {  // A_k <- A_k S_{k+1}
  PhaseScope ps(PH_ABSORB);
  SitePlan& P = b.lead().plans[k];
  launch_gemm(P.absR, b.lead().tabs.dev,
              slots_of(b, [&](tt_state& s, int) { return Slots{{s.A[k], s.Sbuf, s.tmp, nullptr}}; }), b.n, TT_FP64,
              pws_of(b), ST());
  launch_copy(per_state(b, [&](tt_state& s) { return s.A[k]; }), cst(per_state(b, [](tt_state& s) { return s.tmp; })),
              b.lead().site[k].size, b.n, ST());
  add_flops(b, P.absR.flops, false);
}

void normalize_site(const Batch& b, int k) {
  BPtr<double> A = per_state(b, [&](tt_state& s) { return s.A[k]; });
  BPtr<double> part = per_state(b, [](tt_state& s) { return s.part; });
  BPtr<const double> none{};
  launch_mdot(none, 0, 0, cst(A), b.lead().site[k].size, 1, part, b.n, ST());
  launch_normalize_log(A, b.lead().site[k].size, cst(part), per_state(b, [](tt_state& s) { return s.lam_ptr(); }), b.n,
                       ST());
}

void sweep_once(const Batch& b, double dbeta) {
  const int N = b.lead().N;
  const double tau = 0.5 * dbeta;
  for (int i = 0; i < b.n; ++i) b.s[i]->lw_site = -1;   // the first apply folds L_0 again
  for (int k = 0; k < N - 1; ++k) {
    site_exp(b, k, -tau);
    qr_site(b, k);
    env_left(b, k);
    bond_exp(b, k + 1, +tau);
    absorb_left(b, k + 1);
  }
  site_exp(b, N - 1, -2.0 * tau);
  for (int k = N - 1; k >= 1; --k) {
    lq_site(b, k);
    env_right(b, k);
    bond_exp(b, k, +tau);
    absorb_right(b, k - 1);
    site_exp(b, k - 1, -tau);
  }
  for (int i = 0; i < b.n; ++i) {
    b.s[i]->beta += dbeta;
    b.s[i]->sweeps++;
  }
}

// -------------------------------------------------------------- construction
long long pow16_cap(int e, long long cap) {
  long long v = 1;
  for (int i = 0; i < e; ++i) {
    v *= 16;
    if (v > cap) return cap + 1;
  }
  return v;
}

// Plans of the swap overlap <<rho|P|rho>>, P exchanging sigma and sigma' on
// every site (P|rho>> = |rho^T>>, Choi map of SM Sec. II.A).  P maps s =
// 4 sigma + sigma' to 4 sigma' + sigma and negates its charge, so the transfer
// matrix of bond k pairs sector q with -q: E_k[q] is d(q) x d(-q), laid out
// sector by sector (sectors whose -q is absent hold no block).  Site k:
//   X^{s,q} = E_k[q] A^{P(s)}[-q]              (one GEMM per (s, q))
//   E_{k+1}[q'] = sum_{(s,q): q + Delta(s) = q'} (A^s[q])^T X^{s,q}
// the second as one GEMM per q' with its K running over the rows of every
// (s, q) in order.  E_0 = 1 and the value is E_N.
static Q negq(Q q) { return {-q.first, -q.second}; }
void build_swap_plans(tt_state& s) {
  const int N = s.N;
  std::vector<std::vector<long long>> eoff(N + 1);
  s.swp_e = 1;
  for (int k = 0; k <= N; ++k) {
    const Bond& b = s.bonds[k];
    long long pos = 0;
    eoff[k].assign(b.secs.size(), -1);
    for (size_t i = 0; i < b.secs.size(); ++i) {
      const int j = b.find(negq(b.secs[i].q));
      if (j < 0) continue;
      eoff[k][i] = pos;
      pos += (long long)b.secs[i].dim * b.secs[j].dim;
    }
    s.swp_e = std::max(s.swp_e, pos);
  }
  s.swp1.assign(N, GemmPlan());
  s.swp2.assign(N, GemmPlan());
  s.swp_x = 1;
  auto gp0 = [](int M, int Nn, int K) {
    GemmProb g{};
    g.M = M; g.N = Nn; g.K = K;
    g.ia = 0; g.ib = 1; g.ic = 2;
    g.tam = g.tak = g.tbk = g.tbn = g.tcm = -1;
    g.alpha = 1.0; g.beta = 0.0;
    return g;
  };
  for (int k = 0; k < N; ++k) {
    const Bond &bl = s.bonds[k], &br = s.bonds[k + 1];
    const SiteLayout& S = s.site[k];
    GemmPlan &h1 = s.swp1[k], &h2 = s.swp2[k];
    h1.wave_ok = h2.wave_ok = true;
    long long xpos = 0;
    std::map<int, std::vector<std::pair<long long, std::pair<int, int>>>> into;   // q' -> (X offset, (s, l))
    for (int l = 0; l < (int)bl.secs.size(); ++l) {
      if (eoff[k][l] < 0) continue;
      const int ln = bl.find(negq(bl.secs[l].q));
      for (int sg = 0; sg < 16; ++sg) {
        const int ps = 4 * (sg & 3) + (sg >> 2);
        const int g = s.G.group_of[sg], gp = s.G.group_of[ps];
        const int r = S.rsec[l][g], rn = S.rsec[ln][gp];
        if (r < 0 || rn < 0) continue;
        if (br.find(negq(br.secs[r].q)) != rn || eoff[k + 1][r] < 0) continue;
        const int dq = bl.secs[l].dim, dn = bl.secs[ln].dim, dyn = br.secs[rn].dim;
        GemmProb g1 = gp0(dq, dyn, dn);
        g1.offA = eoff[k][l]; g1.sam = dn; g1.sak = 1;
        g1.offB = S.base[ln] + S.colb[ln][gp] + (long long)s.G.pos_of[ps] * dyn; g1.sbk = S.C[ln]; g1.sbn = 1;
        g1.offC = xpos; g1.scm = dyn;
        h1.probs.push_back(g1);
        h1.flops += 2.0 * dq * (double)dyn * dn;
        into[r].push_back({xpos, {sg, l}});
        xpos += (long long)dq * dyn;
      }
    }
    s.swp_x = std::max(s.swp_x, xpos);
    for (auto& kv : into) {
      const int r = kv.first, rn = br.find(negq(br.secs[r].q));
      const int dy = br.secs[r].dim, dyn = br.secs[rn].dim;
      std::vector<long long> ak, bk;
      for (auto& e : kv.second) {
        const int sg = e.second.first, l = e.second.second;
        const int g = s.G.group_of[sg];
        for (int x = 0; x < bl.secs[l].dim; ++x) {
          ak.push_back(S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)s.G.pos_of[sg] * dy);
          bk.push_back(e.first + (long long)x * dyn);
        }
      }
      GemmProb g2 = gp0(dy, dyn, (int)ak.size());
      g2.sam = 1; g2.tak = s.tabs.add(ak);
      g2.tbk = s.tabs.add(bk); g2.sbn = 1;
      g2.offC = eoff[k + 1][r]; g2.scm = dyn;
      h2.probs.push_back(g2);
      h2.flops += 2.0 * dy * (double)dyn * ak.size();
    }
  }
}

// every contraction block of a sweep goes to the wave GEMM, which multiplies
// in the state's precision; the absorb step always runs in FP64
void configure_plan(const tt_options& o, SitePlan& P) {
  for (GemmPlan* g : {&P.s1, &P.s3, &P.el, &P.r1, &P.r3, &P.b1, &P.b2}) g->wave_ok = true;
  for (GemmPlan& g : P.s1w) g.wave_ok = true;
  P.absL.wave_ok = P.absR.wave_ok = true;
  if (o.precision == TT_FP32) {
    // FP32 mode keeps the intermediates of H_eff and of the environment
    // updates (T1, T2, Y, Z) in float: half the memory traffic of those stages
    P.s1.slot_f32[2] = P.r1.slot_f32[2] = true;   // T1, Y written
    P.s3.slot_f32[0] = true;                      // T2 read
    P.el.slot_f32[1] = P.r3.slot_f32[1] = true;   // T2, Z read
    P.w2.f32 = P.wr.f32 = true;
    for (GemmPlan& g : P.s1w) g.slot_f32[2] = true;   // T2 written (and read back by the later passes)
    P.t2zero.f32 = true;
  }
}

void build_layouts(tt_state& s, const std::vector<std::map<Q, int>>& dims) {
  const int N = s.N;
  s.bonds.assign(N + 1, Bond());
  for (int k = 0; k <= N; ++k)
    for (auto& kv : dims[k]) s.bonds[k].add(kv.first, kv.second);
  // environment MPO: bond 0 [start], bond N [done]; W_{N-1} contracted with the done selector
  s.qH.assign(N + 1, {});
  for (int k = 0; k < N; ++k)
    for (int a = 0; a < s.mpo.DH[k]; ++a) s.qH[k].push_back(project_charge(s.mpo.charge(k, a), s.opts.symmetry));
  s.qH[N] = {Q{0, 0}};
  // W_{N-1} contracted with the done selector
  auto env_tensors = [&](const Mpo& mpo) {
    std::vector<std::vector<double>> W = mpo.W;
    int DL = mpo.DH[N - 1], DR = mpo.DH[N];   // DR = 2: start, done
    std::vector<double> w((size_t)DL * 16, 0.0);
    for (int a = 0; a < DL; ++a)
      for (int q = 0; q < 16; ++q) w[(size_t)a * 16 + q] = mpo.W[N - 1][((size_t)a * 16 + q) * DR + 1];
    W[N - 1] = w;
    return W;
  };
  s.Wenv = env_tensors(s.mpo);
  // the plans keep every MPO entry that is nonzero for generic couplings, so
  // states that differ only in t, U, mu (an exact zero such as U - 2 mu at
  // half filling included) get identical plans and can share launches
  s.Wpat = env_tensors(make_hubbard_mpo(s.lat, 1.0, s.model.tp != 0.0 ? 0.7 : 0.0, 1.0, 0.3,
                                        s.model.hp != 0.0 ? 0.45 : 0.0));
  s.site.clear(); s.env.clear(); s.bmat.clear();
  for (int k = 0; k < N; ++k) s.site.push_back(make_site_layout(s.bonds[k], s.bonds[k + 1], s.G));
  for (int k = 0; k <= N; ++k) {
    s.env.push_back(make_env_layout(s.bonds[k], s.qH[k]));
    s.bmat.push_back(make_bondmat_layout(s.bonds[k]));
  }
  s.plans.clear();
  for (int k = 0; k < N; ++k)
    s.plans.push_back(
        build_site_plan(k, s.bonds[k], s.bonds[k + 1], s.G, s.qH[k], s.qH[k + 1], s.Wenv[k], s.Wpat[k], s.tabs));
  for (auto& P : s.plans) configure_plan(s.opts, P);
  build_swap_plans(s);
}

bool qr_fits(const QRPlan& p) {
  for (const QRTask& t : p.tasks)
    if (t.m < t.n) return false;
  return true;
}

// plan descriptors, tables and the scratch buffers the plans size, for the
// current bonds (the site tensors must exist: the trace kernel takes their
// addresses).  A state marked !one_site_ok keeps no QR/LQ descriptors for
// blocks with fewer rows than columns.
void alloc_scratch(tt_state& s) {
  const int N = s.N;
  hipStream_t st = ST();
  s.tabs.dev = upload(s.tabs.host, st);
  long long t1 = 0, lw = 0, t2 = 0, y = 0, z = 0, u = 0, qw = 0;
  for (auto& P : s.plans) {
    const std::vector<long long>* T = &s.tabs.host;
    upload_plan(P.s1, T, st); upload_plan(P.s3, T, st); upload_plan(P.el, T, st);
    upload_plan(P.r1, T, st); upload_plan(P.r3, T, st); upload_plan(P.absL, T, st); upload_plan(P.absR, T, st);
    upload_plan(P.b1, T, st); upload_plan(P.b2, T, st);
    for (int j = 0; j < P.n_s1w; ++j) upload_plan(P.s1w[j], T, st);
    upload_plan(P.w2, st); upload_plan(P.lw, st); upload_plan(P.t2zero, st); upload_plan(P.wr, st);
    upload_plan(P.fz, st); upload_plan(P.fzb, st);
    if (s.one_site_ok || qr_fits(P.qr)) upload_plan(P.qr, st);
    if (s.one_site_ok || qr_fits(P.lq)) upload_plan(P.lq, st);
    t1 = std::max(t1, P.t1_size); lw = std::max(lw, P.lw_size); t2 = std::max(t2, P.t2_size);
    y = std::max(y, P.y_size); z = std::max(z, P.z_size); u = std::max(u, P.u_size);
    qw = std::max(qw, std::max(P.qr.ws_size + P.qr.lds_ws, P.lq.ws_size + P.lq.lds_ws));
  }
  long long pw = 1;
  for (auto& P : s.plans)
  {
    for (GemmPlan* g : {&P.s1, &P.s3, &P.el, &P.r1, &P.r3, &P.absL, &P.absR, &P.b1, &P.b2})
      pw = std::max(pw, g->pws_size);
    for (int j = 0; j < P.n_s1w; ++j) pw = std::max(pw, P.s1w[j].pws_size);
  }
  s.pws = (double*)dalloc(8 * pw);
  s.cap_pws = pw;
  s.max_site = 0;
  for (auto& l : s.site) s.max_site = std::max(s.max_site, l.size);
  s.max_bmat = 0;
  s.max_bond = 0;
  s.max_env = 0;
  for (int k = 0; k <= N; ++k) {
    s.max_bmat = std::max(s.max_bmat, s.bmat[k].size);
    s.max_bond = std::max(s.max_bond, s.bonds[k].total);
    s.max_env = std::max(s.max_env, s.env[k].size);
  }
  long long nvec = std::max(s.max_site, s.max_bmat);
  auto buf = [](double*& p, long long& cap, long long n) {
    cap = std::max(n, 1LL);
    p = (double*)dalloc(8 * cap);
  };
  buf(s.T1, s.cap_T1, t1);
  long long cap_lw = 0;
  buf(s.LW, cap_lw, lw);
  s.lw_site = -1;
  s.fold.assign(N, 0);
  s.bfz.assign(N, 0);
  buf(s.T2, s.cap_T2, t2);
  buf(s.Y, s.cap_Y, y);
  buf(s.Z, s.cap_Z, z);
  buf(s.U, s.cap_U, u);
  buf(s.Sbuf, s.cap_Sbuf, s.max_bmat);
  buf(s.tmp, s.cap_tmp, s.max_site);
  buf(s.kry, s.cap_kry, nvec * (long long)s.opts.krylov_dim);
  buf(s.wv, s.cap_wv, nvec);
  s.qrws = (double*)dalloc(8 * std::max(qw, 1LL));
  s.vtr = (double*)dalloc(8 * 2 * s.max_bond);
  for (auto& g : s.swp1) upload_plan(g, &s.tabs.host, st);
  for (auto& g : s.swp2) upload_plan(g, &s.tabs.host, st);
  s.Ea = (double*)dalloc(8 * s.swp_e);
  s.Eb = (double*)dalloc(8 * s.swp_e);
  s.Xs = (double*)dalloc(8 * s.swp_x);
  // trace entries
  std::vector<TraceEntry> te;
  std::vector<int> start{0};
  for (int k = 0; k < N; ++k) {
    for (auto& e : s.plans[k].tr) {
      int l = (int)e[2], r = (int)e[3];
      TraceEntry t;
      t.src = e[0]; t.C = e[1];
      t.xoff = s.bonds[k].secs[l].off; t.dl = s.bonds[k].secs[l].dim;
      t.yoff = s.bonds[k + 1].secs[r].off; t.dr = s.bonds[k + 1].secs[r].dim;
      t.site = k;
      for (int q = 0; q < 4; ++q) t.pos[q] = s.G.pos_of[5 * q];
      te.push_back(t);
    }
    start.push_back((int)te.size());
  }
  s.d_trace = upload(te, st);
  s.d_trace_start = upload(start, st);
  s.d_sites = upload(s.A, st);
}

void alloc_state(tt_state& s) {
  const int N = s.N;
  hipStream_t st = ST();
  s.A.resize(N);
  for (int k = 0; k < N; ++k) s.A[k] = (double*)dalloc(8 * s.site[k].size);
  s.Lenv.assign(N + 1, nullptr);
  s.Renv.assign(N + 1, nullptr);
  for (int k = 0; k <= N; ++k) {
    s.Lenv[k] = (double*)dalloc(8 * s.env[k].size);
    s.Renv[k] = (double*)dalloc(8 * s.env[k].size);
    launch_fill(s.Lenv[k], 0.0, s.env[k].size, st);   // defined contents before the first sweep builds them
  }
  s.part = (double*)dalloc(8 * 2 * (long long)kRedBlocks * (kMaxKrylov + 2));
  s.lz = (double*)dalloc(8 * (4 * kMaxKrylov + 16));
  launch_fill(s.lz, 0.0, 4 * kMaxKrylov + 16, st);
  alloc_scratch(s);
}

// rho0 tensors embedded in the padded block-sparse layout, plus the noise
void fill_initial_tensors(tt_state& s, std::vector<std::vector<double>>& host) {
  const int N = s.N;
  const Rho0& r0 = s.rho0;
  TT_REQUIRE((int)r0.A.size() == N, TT_EINVAL, "rho0 tensors are not available");
  // embedding of rho0 bond states: (sector, local index)
  std::vector<std::vector<std::pair<int, int>>> emb(N + 1);
  std::vector<std::vector<int>> n0(N + 1);
  for (int k = 0; k <= N; ++k) {
    n0[k].assign(s.bonds[k].secs.size(), 0);
    int nst = (int)r0.q[k].size();
    for (int a = 0; a < nst; ++a) {
      Q q = k == N ? Q{0, 0} : project_charge(r0.q[k][a], s.opts.symmetry);
      int sec = s.bonds[k].find(q);
      TT_REQUIRE(sec >= 0 && n0[k][sec] < s.bonds[k].secs[sec].dim, TT_EINVAL, "rho0 does not fit the bond sectors");
      emb[k].push_back({sec, n0[k][sec]});
      n0[k][sec]++;
    }
  }
  host.assign(N, {});
  for (int k = 0; k < N; ++k) {
    const SiteLayout& S = s.site[k];
    std::vector<double>& h = host[k];
    h.assign(S.size, 0.0);
    const int DL = (int)r0.q[k].size(), DRo = (int)r0.q[k + 1].size();
    const Bond& br = s.bonds[k + 1];
    for (int a = 0; a < DL; ++a)
      for (int q = 0; q < 16; ++q)
        for (int b = 0; b < DRo; ++b) {
          const double v = r0.A[k][((size_t)a * 16 + q) * DRo + b];
          if (v == 0.0) continue;
          int l = emb[k][a].first, x = emb[k][a].second;
          int r = emb[k + 1][b].first, y = emb[k + 1][b].second;
          int g = s.G.group_of[q];
          TT_REQUIRE(S.rsec[l][g] == r, TT_EINVAL, "rho0 breaks charge conservation");
          h[S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)s.G.pos_of[q] * br.secs[r].dim + y] = v;
        }
    if (s.opts.pad_eps != 0.0) {
      const Bond& bl = s.bonds[k];
      const long long Dr = br.total;
      for (int l = 0; l < S.nl; ++l)
        for (int g = 0; g < s.G.ng; ++g) {
          int r = S.rsec[l][g];
          if (r < 0) continue;
          int ns = (int)s.G.s[g].size();
          for (int x = 0; x < S.dl[l]; ++x)
            for (int si = 0; si < ns; ++si)
              for (int y = 0; y < br.secs[r].dim; ++y) {
                bool pad = (x >= n0[k][l]) || (y >= n0[k + 1][r]);
                if (!pad) continue;
                long long xg = bl.secs[l].off + x, yg = br.secs[r].off + y;
                int sidx = s.G.s[g][si];
                uint64_t flat = (uint64_t)((xg * 16 + sidx) * Dr + yg);
                h[S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)si * br.secs[r].dim + y] =
                    s.opts.pad_eps * noise_uniform(s.opts.seed, k, flat);
              }
        }
    }
  }
}

void set_unit_env(double* e, hipStream_t st) { launch_fill(e, 1.0, 1, st); }

void canonicalise_and_envs(tt_state& s) {
  const int N = s.N;
  const Batch b = batch_of(s);
  for (int k = N - 1; k >= 1; --k) {
    lq_site(b, k);
    absorb_right(b, k - 1);
  }
  launch_fill(s.lam_ptr(), 0.0, 1, ST());
  s.lw_site = -1;
  normalize_site(b, 0);
  set_unit_env(s.Lenv[0], ST());
  set_unit_env(s.Renv[N], ST());
  for (int k = N - 1; k >= 1; --k) env_right(b, k);
}

std::vector<std::map<Q, int>> bond_dims(const tt_state& s) {
  const int N = s.N;
  std::vector<std::map<Q, int>> n0(N + 1);
  for (int k = 0; k <= N; ++k)
    for (const Q& q : s.rho0.q[k]) n0[k][project_charge(q, s.opts.symmetry)]++;
  if (s.opts.symmetry) return allocate_sectors(N, s.opts.D, n0, s.opts.sector_cap, s.opts.symmetry);
  std::vector<std::map<Q, int>> d(N + 1);
  for (int k = 0; k <= N; ++k) {
    int n = (int)s.rho0.q[k].size();
    long long mx = pow16_cap(std::min(k, N - k), 1LL << 40);
    long long v = std::max<long long>(std::min<long long>(s.opts.D, mx), n);
    d[k][{0, 0}] = (int)v;
  }
  return d;
}

void validate(const tt_model& m, const tt_options& o) {
  TT_REQUIRE(o.D >= 1, TT_EINVAL, "D must be positive");
  TT_REQUIRE(o.symmetry >= 0 && o.symmetry <= 2, TT_EINVAL, "symmetry must be 0, 1 or 2");
  TT_REQUIRE(o.taylor_order >= 1 && o.taylor_order <= 4, TT_EINVAL, "taylor_order must be in 1..4");
  TT_REQUIRE(o.krylov_dim >= 1 && o.krylov_dim <= kMaxKrylov, TT_EINVAL, "krylov_dim must be in 1..32");
  TT_REQUIRE(o.krylov_tol >= 0.0, TT_EINVAL, "krylov_tol must be >= 0");
  TT_REQUIRE(o.precision >= TT_FP64 && o.precision <= TT_BF16X6, TT_EINVAL, "unknown precision");
  TT_REQUIRE(o.env_on_host == 0, TT_EINVAL, "host-resident environments are not supported");
  TT_REQUIRE(o.sector_cap >= 0, TT_EINVAL, "sector_cap must be >= 0");
  TT_REQUIRE(std::isfinite(o.beta0) && std::isfinite(o.pad_eps), TT_EINVAL, "beta0 and pad_eps must be finite");
  TT_REQUIRE(std::isfinite(m.t) && std::isfinite(m.tp) && std::isfinite(m.U) && std::isfinite(m.mu) &&
                 std::isfinite(m.hp), TT_EINVAL, "model parameters must be finite");
  TT_REQUIRE(m.hp == 0.0 || o.symmetry != 1, TT_EINVAL,
             "the pairing field breaks the U(1) charges: it needs symmetry = 0 or 2");
}

std::unique_ptr<tt_state> make_host_state(const tt_model& m, const tt_options& o, bool with_plans = true) {
  validate(m, o);
  auto s = std::make_unique<tt_state>();
  s->model = m;
  s->opts = o;
  s->lat = make_lattice(m.W, m.L, m.geometry);
  s->N = s->lat.N;
  s->mpo = make_hubbard_mpo(s->lat, m.t, m.tp, m.U, m.mu, m.hp);
  s->rho0 = make_rho0(s->mpo, o.beta0, o.taylor_order);
  s->G = make_groups(o.symmetry);
  auto dims = bond_dims(*s);
  if (with_plans) {
    build_layouts(*s, dims);
  } else {
    s->bonds.assign(s->N + 1, Bond());
    for (int k = 0; k <= s->N; ++k)
      for (auto& kv : dims[k]) s->bonds[k].add(kv.first, kv.second);
  }
  return s;
}

void require_sweep_plans(tt_state& s);

std::unique_ptr<tt_state> make_state(const tt_model& m, const tt_options& o) {
  auto s = make_host_state(m, o);
  require_sweep_plans(*s);
  check_device();
  alloc_state(*s);
  return s;
}

// ---------------------------------------------------------------- plan bounds check
// Every index a kernel will form, checked on the host against the buffer it addresses.
struct Range { long long lo = 0, hi = -1; void add(long long v) { if (hi < lo) { lo = hi = v; } else { lo = std::min(lo, v); hi = std::max(hi, v); } } };

Range map_range(const std::vector<long long>& tabs, long long tab, long long stride, int n) {
  Range r;
  if (n <= 0) return r;
  if (tab >= 0) {
    for (int i = 0; i < n; ++i) r.add(tabs.at(tab + i));
  } else {
    r.add(0);
    r.add((long long)(n - 1) * stride);
  }
  return r;
}

long long check_gemm(const GemmPlan& p, const std::vector<long long>& tabs, const long long size[kSlots],
                     const char* name, std::string& rep) {
  long long bad = 0;
  for (size_t i = 0; i < p.probs.size(); ++i) {
    const GemmProb& g = p.probs[i];
    Range am = map_range(tabs, g.tam, g.sam, g.M), ak = map_range(tabs, g.tak, g.sak, g.K);
    Range bk = map_range(tabs, g.tbk, g.sbk, g.K), bn = map_range(tabs, g.tbn, g.sbn, g.N);
    Range cm = map_range(tabs, g.tcm, g.scm, g.M);
    auto chk = [&](int slot, long long off, Range a, Range b, long long extra_hi, const char* op) {
      if (g.K == 0 && op[0] != 'C') return;
      long long lo = off + a.lo + b.lo, hi = off + a.hi + b.hi + extra_hi;
      if (slot < 0 || slot >= kSlots || lo < 0 || hi >= size[slot]) {
        ++bad;
        if (rep.size() < 2000)
          rep += std::string(name) + " prob " + std::to_string(i) + " operand " + op + " [" + std::to_string(lo) +
                 "," + std::to_string(hi) + "] size " + std::to_string(slot >= 0 && slot < kSlots ? size[slot] : -1) + "\n";
      }
    };
    chk(g.ia, g.offA, am, ak, 0, "A");
    chk(g.ib, g.offB, bk, bn, 0, "B");
    chk(g.ic, g.offC, cm, Range{0, 0}, g.N - 1, "C");
  }
  for (auto& t : p.tiles) {
    if (t.prob < 0 || t.prob >= (int)p.probs.size() || t.cfg < 0 || t.cfg >= kGemmCfgs) { ++bad; continue; }
    const GemmProb& g = p.probs[t.prob];
    if (t.tm < 0 || t.tn < 0 || t.tm * kGemmBM[t.cfg] >= g.M || t.tn * kGemmBN[t.cfg] >= g.N) ++bad;
    if (t.nk < 1 || t.ks < 0 || t.ks >= t.nk) ++bad;
    if (t.nk > 1 && (t.sidx < 0 || t.sidx >= (int)p.splits.size())) ++bad;
    if (t.nk > 1 && (t.pw < 0 || t.pw + (long long)t.nk * kGemmBM[t.cfg] * kGemmBN[t.cfg] > p.pws_size)) ++bad;
  }
  for (auto& sp : p.splits)
    if (sp.prob < 0 || sp.prob >= (int)p.probs.size() || sp.pw < 0 ||
        sp.pw + (long long)sp.nk * kGemmBM[sp.cfg] * kGemmBN[sp.cfg] > p.pws_size) ++bad;
  // wave jobs: four per workgroup; a split block fills its workgroup with parts 0..3
  auto check_jobs = [&](const std::vector<GemmJob>& jobs, int wave_blocks) {
    if (jobs.size() % 4 != 0 || (long long)jobs.size() != 4LL * wave_blocks) ++bad;
    for (size_t w = 0; w + 3 < jobs.size(); w += 4) {
      const GemmJob& j0 = jobs[w];
      for (int q = 0; q < 4; ++q) {
        const GemmJob& j = jobs[w + q];
        if (j.nparts != j0.nparts) ++bad;
        if (j.prob < 0) { if (j.nparts != 1) ++bad; continue; }
        if (j.prob >= (int)p.probs.size() || j.shape < 0 || j.shape >= kWaveShapes) { ++bad; continue; }
        const GemmProb& g = p.probs[j.prob];
        if (j.tm < 0 || j.tn < 0 || j.tm * kWaveBM[j.shape] >= g.M || j.tn * kWaveBN[j.shape] >= g.N) ++bad;
        if (j.nparts == 4) {
          if (j.part != q || j.prob != j0.prob || j.tm != j0.tm || j.tn != j0.tn || j.shape != j0.shape) ++bad;
        } else if (j.nparts != 1 || j.part != 0) {
          ++bad;
        }
      }
    }
  };
  check_jobs(p.jobs, p.wave_blocks);
  check_jobs(p.jobs_fine, p.wave_blocks_fine);
  return bad;
}

// the fused apply's descriptors against LW (lw_size), the input and output
// site vectors (in_size, out_size) and the R environment (r_size); the kernel
// forms in-block offsets in 32 bits (below 2^29 elements) and clamps rows and
// columns to each block, so these ranges bound every access
long long check_fz(const FzPlan& p, long long lw_size, long long in_size, long long out_size, long long r_size,
                   std::string& rep) {
  long long bad = 0;
  const long long lim = 1LL << 29;
  auto fail = [&](const char* what, size_t i) {
    ++bad;
    if (rep.size() < 2000) rep += std::string("fz ") + what + " " + std::to_string(i) + "\n";
  };
  for (size_t i = 0; i < p.outs.size(); ++i) {
    const FzOut& o = p.outs[i];
    if (o.dp < 1 || o.dr < 1 || o.ldo < o.dr || o.ldr < 1) { fail("out shape", i); continue; }
    const long long oh = (long long)(o.dp - 1) * o.ldo + o.dr - 1;
    if (o.out < 0 || o.out + oh >= out_size || oh >= lim) fail("out range", i);
    if (o.b0 < 0 || o.nb < 0 || o.nb > kFzMaxB || (long long)o.b0 + o.nb > (long long)p.bs.size()) {
      fail("out b range", i);
      continue;
    }
    for (int bi = 0; bi < o.nb; ++bi) {
      const FzB& b = p.bs[o.b0 + bi];
      const long long rh = (long long)(o.dr - 1) * o.ldr + b.rcol + b.dc - 1;
      if (b.dc < 1 || b.rcol < 0 || o.rrow < 0 || o.rrow + rh >= r_size || rh >= lim) fail("R range", i);
      if (b.nt < 1 || b.nt > kFzMaxB || b.t0 < 0 || (long long)b.t0 + b.nt > (long long)p.terms.size()) {
        fail("b terms", i);
        continue;
      }
      if (bi > 0 && b.t0 != p.bs[o.b0 + bi - 1].t0 + p.bs[o.b0 + bi - 1].nt) fail("b terms not consecutive", i);
      for (int ti = 0; ti < b.nt; ++ti) {
        const FzT& t = p.terms[b.t0 + ti];
        if (t.dl < 1 || t.ldlw < t.dl || t.lda < b.dc) { fail("term shape", i); continue; }
        const long long lh = (long long)(o.dp - 1) * t.ldlw + t.dl - 1;
        const long long ah = (long long)(t.dl - 1) * t.lda + b.dc - 1;
        if (t.lw < 0 || t.lw + lh >= lw_size || lh >= lim) fail("LW range", i);
        if (t.a < 0 || t.a + ah >= in_size || ah >= lim) fail("input range", i);
      }
    }
  }
  if (p.jobs.size() % 4 != 0 || (long long)p.jobs.size() != 4LL * p.nblocks) fail("job count", 0);
  for (size_t w = 0; w + 3 < p.jobs.size(); w += 4) {
    const FzJob& j0 = p.jobs[w];
    for (int q = 0; q < 4; ++q) {
      const FzJob& j = p.jobs[w + q];
      if (j.nparts != j0.nparts) fail("job parts", w);
      if (j.o < 0) { if (j.nparts != 1) fail("empty split job", w); continue; }
      if (j.o >= (int)p.outs.size()) { fail("job block", w); continue; }
      const FzOut& o = p.outs[j.o];
      if (j.row0 < 0 || j.row0 >= o.dp || j.row0 % 16 || j.col0 < 0 || j.col0 >= o.dr || j.col0 % kFzCols)
        fail("job tile", w);
      if (j.nparts == 4) {
        if (j.part != q || j.o != j0.o || j.row0 != j0.row0 || j.col0 != j0.col0) fail("split job", w);
      } else if (j.nparts != 1 || j.part != 0) {
        fail("job part", w);
      }
    }
  }
  return bad;
}

long long check_w(const WPlan& p, long long in_size, long long out_size, const char* name, std::string& rep) {
  long long bad = 0;
  for (size_t i = 0; i < p.tasks.size(); ++i) {
    const WTask& t = p.tasks[i];
    if (t.ni <= 0 || t.nj <= 0) continue;
    long long hi = t.dst + (long long)(t.ni - 1) * t.dsi + (long long)(t.nj - 1) * t.dsj;
    if (t.dst < 0 || hi >= out_size) ++bad;
    if (t.t0 < 0 || t.t0 + t.nt > (int)p.terms.size()) { ++bad; continue; }
    for (int q = t.t0; q < t.t0 + t.nt; ++q) {
      const WTerm& w = p.terms[q];
      long long h2 = w.src + (long long)(t.ni - 1) * w.ssi + (long long)(t.nj - 1) * w.ssj;
      if (w.src < 0 || h2 >= in_size) {
        ++bad;
        if (rep.size() < 2000) rep += std::string(name) + " task " + std::to_string(i) + " term out of range\n";
      }
    }
  }
  return bad;
}

long long check_qr(const QRPlan& p, const std::vector<long long>& tabs, long long a_size, long long s_size,
                   const char* name, std::string& rep) {
  long long bad = 0;
  long long ws = 0;
  for (size_t i = 0; i < p.tasks.size(); ++i) {
    const QRTask& t = p.tasks[i];
    if (t.m < t.n) { ++bad; rep += std::string(name) + " task with m < n\n"; continue; }
    Range r = map_range(tabs, t.rtab, t.rs, t.m);
    long long lo = t.rbase + r.lo, hi = t.rbase + r.hi + (long long)(t.n - 1) * t.cs;
    if (lo < 0 || hi >= a_size) ++bad;
    if (t.sdst < 0 || t.sdst + (long long)t.n * t.n > s_size) ++bad;
    ws += qr_wide_ws(t.m, t.n);
  }
  (void)ws;
  QRPlan q = p;
  qr_plan_chunks(q);
  std::vector<int> covered(q.tasks.size(), 0);
  for (auto& c : q.chunks) {
    const QRTask& t = q.tasks.at(c.task);
    if (c.row0 < 0 || c.rows < t.n || c.row0 + c.rows > t.m) ++bad;
    if (c.rows > kQrChunkRows || t.n > kQrLdsMaxN) ++bad;
    if (c.nchunks > 1) {
      if (c.qw < 0 || c.qw + (long long)c.rows * t.n > q.lds_ws) ++bad;
      if (c.rw < 0 || c.rw + (long long)c.nchunks * t.n * t.n > q.lds_ws) ++bad;
      if ((long long)c.nchunks * t.n > kQrStackRows) ++bad;
    }
    covered[c.task] += c.rows;
  }
  for (int w : q.wide) covered.at(w) += q.tasks[w].m;
  for (size_t i = 0; i < q.tasks.size(); ++i)
    if (covered[i] != q.tasks[i].m) { ++bad; rep += std::string(name) + " QR rows not covered exactly once\n"; }
  return bad;
}

std::vector<SitePlan> make_obs_plans(const tt_state& s, const Mpo& m, const Mpo& pat, SiteTables& tabs);
long long check_obs_plans(const tt_state& s, const Mpo& m, std::vector<SitePlan>& plans, const SiteTables& tabs,
                          std::string& rep);

// every descriptor of the sweep's launches (contractions, W stages, QR/LQ,
// trace) against the buffers alloc_state sizes from the same plans
long long check_sweep_plans(tt_state& s, std::string& rep) {
  long long bad = 0;
  const int N = s.N;
  long long t1 = 0, lw = 0, t2 = 0, y = 0, z = 0, u = 0, msite = 0, mb = 0;
  for (auto& P : s.plans) {
    t1 = std::max(t1, P.t1_size); lw = std::max(lw, P.lw_size); t2 = std::max(t2, P.t2_size); y = std::max(y, P.y_size);
    z = std::max(z, P.z_size); u = std::max(u, P.u_size);
  }
  for (auto& l : s.site) msite = std::max(msite, l.size);
  for (auto& b : s.bmat) mb = std::max(mb, b.size);
  const auto& T = s.tabs.host;
  for (int k = 0; k < N; ++k) {
    SitePlan& P = s.plans[k];
    for (GemmPlan* g : {&P.s1, &P.s3, &P.el, &P.r1, &P.r3, &P.absL, &P.absR, &P.b1, &P.b2}) tile_plan(*g, &T);
    for (int j = 0; j < P.n_s1w; ++j) tile_plan(P.s1w[j], &T);
    long long ns = s.site[k].size, el = s.env[k].size, er = s.env[k + 1].size;
    long long s1w[kSlots] = {lw, ns, t2, 0}, s1[kSlots] = {el, ns, t1, 0};
    long long s3[kSlots] = {t2, er, ns, 0}, se[kSlots] = {ns, t2, er, 0};
    long long r1[kSlots] = {er, ns, y, 0}, r3[kSlots] = {ns, z, el, 0};
    long long aL[kSlots] = {s.bmat[k].size, ns, msite, 0}, aR[kSlots] = {ns, s.bmat[k + 1].size, msite, 0};
    long long b1[kSlots] = {el, s.bmat[k].size, u, 0}, b2[kSlots] = {u, el, s.bmat[k].size, 0};
    bad += check_gemm(P.s1, T, s1, "s1", rep);
    bad += check_w(P.w2, P.t1_size, P.t2_size, "w2", rep);
    for (int j = 0; j < P.n_s1w; ++j) bad += check_gemm(P.s1w[j], T, s1w, "s1w", rep);
    bad += check_w(P.lw, el, P.lw_size, "lw", rep);
    bad += check_w(P.t2zero, 0, t2, "t2zero", rep);
    bad += check_fz(P.fz, lw, ns, ns, er, rep);
    bad += check_fz(P.fzb, el, s.bmat[k].size, s.bmat[k].size, el, rep);
    bad += check_gemm(P.s3, T, s3, "s3", rep);
    bad += check_gemm(P.el, T, se, "el", rep);
    bad += check_gemm(P.r1, T, r1, "r1", rep);
    bad += check_gemm(P.r3, T, r3, "r3", rep);
    bad += check_gemm(P.absL, T, aL, "absL", rep);
    bad += check_gemm(P.absR, T, aR, "absR", rep);
    bad += check_gemm(P.b1, T, b1, "b1", rep);
    bad += check_gemm(P.b2, T, b2, "b2", rep);
    bad += check_w(P.wr, P.y_size, P.z_size, "wr", rep);
    if (s.one_site_ok || qr_fits(P.qr)) bad += check_qr(P.qr, T, ns, s.bmat[k + 1].size, "qr", rep);
    if (s.one_site_ok || qr_fits(P.lq)) bad += check_qr(P.lq, T, ns, s.bmat[k].size, "lq", rep);
    if (k < (int)s.swp1.size()) {
      tile_plan(s.swp1[k], &T);
      tile_plan(s.swp2[k], &T);
      long long h1[kSlots] = {s.swp_e, ns, s.swp_x, 0}, h2[kSlots] = {ns, s.swp_x, s.swp_e, 0};
      bad += check_gemm(s.swp1[k], T, h1, "swap1", rep);
      bad += check_gemm(s.swp2[k], T, h2, "swap2", rep);
    }
    int pmax = 0;
    for (int q = 0; q < 4; ++q) pmax = std::max(pmax, s.G.pos_of[5 * q]);
    for (auto& e : P.tr) {
      int l = (int)e[2], r = (int)e[3];
      long long dl = s.bonds[k].secs[l].dim, dr = s.bonds[k + 1].secs[r].dim;
      long long hi = e[0] + (dl - 1) * e[1] + (long long)pmax * dr + dr - 1;
      if (hi >= ns) ++bad;
      for (int q = 0; q < 4; ++q)
        if (s.G.group_of[5 * q] != s.G.group_of[0]) ++bad;
    }
  }
  return bad;
}

long long check_all_plans(tt_state& s, std::string& rep) {
  long long bad = 0;
  {   // the Green's-function observable (super-operator W stage), all momenta
    const Mpo pat = make_green_mpo(s.lat, 0.0, 0.0, true);
    SiteTables gt;
    std::vector<SitePlan> gp = make_obs_plans(s, pat, pat, gt);
    bad += check_obs_plans(s, pat, gp, gt, rep);
  }
  return bad + check_sweep_plans(s, rep);
}

// refuse a state whose descriptors address anything outside their buffers,
// before the first launch (a bad descriptor would be a GPU memory fault)
void require_sweep_plans(tt_state& s) {
  std::string rep;
  const long long bad = check_sweep_plans(s, rep);
  TT_REQUIRE(bad == 0, TT_EINVAL, "plans out of bounds (" + std::to_string(bad) + "): " + rep);
}

// ------------------------------------------------------------ 2-TDVP
// SM Sec. "2-TDVP in the initial stage" (Eq. S-2TDVP): the two-site flow
// grows (or truncates) every bond by an SVD of the evolved two-site tensor.
// Bond sectors change at every split, so the descriptors of the two sites a
// step touches are rebuilt there (the other sites' plans and tables are not
// launched until the sweep ends) and every plan is rebuilt for the final
// bonds afterwards.

void grow(double*& p, long long& cap, long long n) {
  n = std::max(n, 1LL);
  if (p && n <= cap) return;
  if (p) HIPX(hipStreamSynchronize(ST()));
  dfree(p);
  p = nullptr;
  p = (double*)dalloc(8 * n);
  cap = n;
}

void free_site_plan(SitePlan& p) {
  free_plan(p.s1); free_plan(p.s3); free_plan(p.el); free_plan(p.r1); free_plan(p.r3);
  free_plan(p.absL); free_plan(p.absR); free_plan(p.b1); free_plan(p.b2);
  free_plan(p.w2); free_plan(p.wr); free_plan(p.qr); free_plan(p.lq);
  free_plan(p.lw); free_plan(p.t2zero); free_plan(p.fz); free_plan(p.fzb);
  for (auto& g : p.s1w) free_plan(g);
}

// device copies of the two-site plan of one step
// Largest X (plus its column norms), in doubles, of an SVD block that one
// workgroup takes in LDS; 0: the device's LDS (tt_svd_lds_limit).
long long g_svd_lds_limit = 0;

struct PairDev {
  PairPlan P;
  SiteTables tabs;
  SvdTask* d_svd = nullptr;
  // the blocks one workgroup takes (small) and those whose rounds spread over the GPU (big)
  int n_small = 0, n_big = 0, n_pairs = 0, max_np = 0;
  std::vector<int> small, big, pairs;   // host copies of the lists below
  int *d_small = nullptr, *d_big = nullptr, *d_pairs = nullptr;
  double* d_ctl = nullptr;
  PairDev() = default;
  PairDev(const PairDev&) = delete;
  PairDev& operator=(const PairDev&) = delete;
  ~PairDev() {
    free_plan(P.join); free_plan(P.s1); free_plan(P.s4); free_plan(P.w1); free_plan(P.w2);
    dfree(d_svd);
    dfree(d_small);
    dfree(d_big);
    dfree(d_pairs);
    dfree(d_ctl);
    dfree(tabs.dev);
  }
};

long long check_pair(const tt_state& s, int k, const PairPlan& P, const std::vector<long long>& T, std::string& rep) {
  long long bad = 0;
  const long long th = P.L.size, el = s.env[k].size, er = s.env[k + 2].size;
  const long long j[kSlots] = {s.site[k].size, s.site[k + 1].size, th, 0};
  const long long a1[kSlots] = {el, th, P.t1_size, 0}, a4[kSlots] = {P.t3_size, er, th, 0};
  bad += check_gemm(P.join, T, j, "join", rep);
  bad += check_gemm(P.s1, T, a1, "pair s1", rep);
  bad += check_w(P.w1, P.t1_size, P.t2_size, "pair w1", rep);
  bad += check_w(P.w2, P.t2_size, P.t3_size, "pair w2", rep);
  bad += check_gemm(P.s4, T, a4, "pair s4", rep);
  for (const SvdTask& t : P.svd) {
    const Range r = map_range(T, t.rtab, 0, t.R);
    const long long mn = std::min(t.R, t.w), mx = std::max(t.R, t.w);
    if (t.R <= 0 || t.w <= 0 || mn > kSvdMaxMinDim || r.lo < 0 || r.hi + t.w - 1 >= th || t.ws < 0 ||
        t.ws + mx * mn + mn * mn > P.svd_ws || t.sig < 0 || t.sig + mn > P.svd_nsig) {
      ++bad;
      if (rep.size() < 2000) rep += "svd task out of range\n";
    }
  }
  return bad;
}

std::unique_ptr<PairDev> make_pair(tt_state& s, int k) {
  auto d = std::make_unique<PairDev>();
  PairPlan& P = d->P;
  P = build_pair_plan(s.bonds[k], s.bonds[k + 1], s.bonds[k + 2], s.G, s.qH[k], s.qH[k + 1], s.qH[k + 2],
                      s.Wenv[k], s.Wenv[k + 1], s.site[k], s.site[k + 1], d->tabs);
  const std::vector<long long>& T = d->tabs.host;
  for (GemmPlan* g : {&P.join, &P.s1, &P.s4}) tile_plan(*g, &T);
  std::string rep;
  const long long bad = check_pair(s, k, P, T, rep);
  TT_REQUIRE(bad == 0, TT_EINVAL, "two-site plans out of bounds (" + std::to_string(bad) + "): " + rep);
  hipStream_t st = ST();
  d->tabs.dev = upload(d->tabs.host, st);
  for (GemmPlan* g : {&P.join, &P.s1, &P.s4}) upload_plan(*g, &T, st);
  upload_plan(P.w1, st);
  upload_plan(P.w2, st);
  d->d_svd = upload(P.svd, st);
  {   // blocks whose X fits one workgroup's LDS, and the rest with their column pairs
    const long long dev_lim = svd_lds_doubles();
    const long long lim = g_svd_lds_limit > 0 ? std::min(g_svd_lds_limit, dev_lim) : dev_lim;
    std::vector<int>& small = d->small;
    std::vector<int>& big = d->big;
    std::vector<int>& pairs = d->pairs;
    for (int t = 0; t < (int)P.svd.size(); ++t) {
      const long long mw = std::max(P.svd[t].R, P.svd[t].w), nw = std::min(P.svd[t].R, P.svd[t].w);
      if (nw + mw * nw <= lim) {
        small.push_back(t);
        continue;
      }
      const int np = (int)(nw + (nw & 1));
      for (int k = 0; k < np / 2; ++k) {
        pairs.push_back((int)big.size());
        pairs.push_back(k);
      }
      d->max_np = std::max(d->max_np, np);
      big.push_back(t);
    }
    d->n_small = (int)small.size();
    d->n_big = (int)big.size();
    d->n_pairs = (int)pairs.size() / 2;
    d->d_small = upload(small, st);
    d->d_big = upload(big, st);
    d->d_pairs = upload(pairs, st);
    if (!big.empty()) d->d_ctl = (double*)dalloc(8 * 3 * big.size());
  }
  const long long n = P.L.size;
  grow(s.th, s.cap_th, n);
  grow(s.P1, s.cap_P1, P.t1_size);
  grow(s.P2, s.cap_P2, P.t2_size);
  grow(s.P3, s.cap_P3, P.t3_size);
  grow(s.svw, s.cap_svw, P.svd_ws);
  grow(s.svs, s.cap_svs, P.svd_nsig);
  grow(s.kry, s.cap_kry, n * (long long)s.opts.krylov_dim);
  grow(s.wv, s.cap_wv, n);
  return d;
}

// H^(2) x (SM Eq. S-2TDVP): L.x, the MPO of site k, the MPO of site k+1, .R
void apply_heff2(tt_state& s, int k, const PairDev& d, BPtr<double> x, BPtr<double> y) {
  PhaseScope ps(PH_HEFF);
  const PairPlan& P = d.P;
  const long long* tb = d.tabs.dev;
  launch_gemm(P.s1, tb, one(Slots{{s.Lenv[k], x.p[0], s.P1, nullptr}}), 1, TT_FP64, one(s.pws), ST());
  launch_wstage(P.w1, one<const WTerm>(P.w1.d_terms), one<const double>(s.P1), one(s.P2), 1, ST());
  launch_wstage(P.w2, one<const WTerm>(P.w2.d_terms), one<const double>(s.P2), one(s.P3), 1, ST());
  launch_gemm(P.s4, tb, one(Slots{{s.P3, s.Renv[k + 2], y.p[0], nullptr}}), 1, TT_FP64, one(s.pws), ST());
  add_flops(batch_of(s), P.s1.flops + P.w1.flops + P.w2.flops + P.s4.flops, true);
  s.bytes_min += 8.0 * (s.env[k].size + s.env[k + 2].size + 2.0 * P.L.size);
}

// Theta = A_k A_{k+1}, then Theta <- exp(t H^(2)) Theta / ||.|| (log-norm into Lambda)
void pair_exp(tt_state& s, int k, const PairDev& d, double t) {
  const Batch b = batch_of(s);
  launch_fill(s.th, 0.0, d.P.L.size, ST());
  launch_gemm(d.P.join, d.tabs.dev, one(Slots{{s.A[k], s.A[k + 1], s.th, nullptr}}), 1, TT_FP64, one(s.pws), ST());
  add_flops(b, d.P.join.flops, false);
  lanczos_exp(b, t, one(s.th), d.P.L.size, [&](BPtr<double> x, BPtr<double> y) { apply_heff2(s, k, d, x, y); });
}

// SVD of every middle-charge block of Theta, the kept values chosen over all
// blocks, the new middle bond, and the two site tensors written in its
// layouts: A_k = U (left) or U S, A_{k+1} = S V^+ or V^+.  Returns the
// discarded weight (dropped squared singular values over all of them).
double split_pair(tt_state& s, int k, const PairDev& d, bool left, int Dmax, double cutoff) {
  PhaseScope ps(PH_QR);
  const PairPlan& P = d.P;
  const int nt = (int)P.svd.size();
  TT_REQUIRE(nt > 0, TT_ENUMERIC, "2-TDVP: the two-site tensor has no block");
  launch_svd(d.d_svd, d.n_small, d.d_small, d.tabs.dev, s.th, s.svw, s.svs, ST());
  launch_svd_big(d.d_svd, d.d_big, d.n_big, d.d_pairs, d.n_pairs, d.max_np, d.tabs.dev, s.th, s.svw, s.svs, d.d_ctl,
                 ST());
  std::vector<double> sig((size_t)P.svd_nsig);
  HIPX(hipMemcpyAsync(sig.data(), s.svs, 8 * (size_t)P.svd_nsig, hipMemcpyDeviceToHost, ST()));
  HIPX(hipStreamSynchronize(ST()));
  struct SV { double v; int task, j; };
  std::vector<SV> all;
  for (int t = 0; t < nt; ++t) {
    const int mn = std::min(P.svd[t].R, P.svd[t].w);
    for (int j = 0; j < mn; ++j) all.push_back({sig[(size_t)(P.svd[t].sig + j)], t, j});
  }
  // largest first; equal values keep the (block, index) order
  std::stable_sort(all.begin(), all.end(), [](const SV& a, const SV& b) { return a.v > b.v; });
  const double smax = all.empty() ? 0.0 : all[0].v;
  TT_REQUIRE(smax > 0.0 && std::isfinite(smax), TT_ENUMERIC, "2-TDVP: the two-site tensor vanished or overflowed");
  size_t keep = 0;
  while (keep < all.size() && keep < (size_t)Dmax && all[keep].v > 0.0 && (cutoff <= 0.0 || all[keep].v > cutoff * smax))
    ++keep;
  keep = std::max<size_t>(keep, 1);
  double tot = 0.0, kept = 0.0;
  for (size_t i = 0; i < all.size(); ++i) {
    tot += all[i].v * all[i].v;
    if (i < keep) kept += all[i].v * all[i].v;
  }
  std::vector<std::vector<int>> sel(nt);
  for (size_t i = 0; i < keep; ++i) sel[all[i].task].push_back(all[i].j);
  std::map<Q, int> dims;
  for (int t = 0; t < nt; ++t)
    if (!sel[t].empty()) dims[P.mq[t]] = (int)sel[t].size();
  Bond nb;
  for (auto& kv : dims) nb.add(kv.first, kv.second);
  const SiteLayout SA = make_site_layout(s.bonds[k], nb, s.G), SB = make_site_layout(nb, s.bonds[k + 2], s.G);
  std::vector<SvdEmit> em;
  std::vector<long long> et;
  long long bad = 0;
  for (int t = 0; t < nt; ++t) {
    if (sel[t].empty()) continue;
    const int mi = nb.find(P.mq[t]);
    const int kap = (int)sel[t].size();
    SvdEmit e{};
    e.task = t;
    e.kappa = kap;
    e.left = left ? 1 : 0;
    e.atab = (long long)et.size();
    for (const auto& rg : P.rowgroups[t]) {
      const int l = rg[0], g1 = rg[1], p1 = rg[2];
      if (SA.rsec[l][g1] != mi) { ++bad; continue; }
      for (int x = 0; x < SA.dl[l]; ++x) {
        const long long o = SA.base[l] + (long long)x * SA.C[l] + SA.colb[l][g1] + (long long)p1 * kap;
        if (o < 0 || o + kap > SA.size) ++bad;
        et.push_back(o);
      }
    }
    if ((long long)et.size() - e.atab != P.svd[t].R) ++bad;
    e.bbase = SB.base[mi];
    e.bstride = SB.C[mi];
    if (SB.C[mi] != P.svd[t].w || e.bbase + (long long)(kap - 1) * e.bstride + P.svd[t].w > SB.size) ++bad;
    e.sel = (long long)et.size();
    for (int j : sel[t]) et.push_back(j);
    em.push_back(e);
  }
  TT_REQUIRE(bad == 0, TT_EINVAL, "2-TDVP: split descriptors out of bounds (" + std::to_string(bad) + ")");
  double* An = (double*)dalloc(8 * std::max(SA.size, 1LL));
  double* Bn = nullptr;
  try {
    Bn = (double*)dalloc(8 * std::max(SB.size, 1LL));
  } catch (...) {
    dfree(An);
    throw;
  }
  long long* dt = upload(et, ST());
  SvdEmit* de = upload(em, ST());
  launch_svd_emit(d.d_svd, de, (int)em.size(), dt, s.svw, s.svs, An, Bn, ST());
  HIPX(hipStreamSynchronize(ST()));
  dfree(dt);
  dfree(de);
  dfree(s.A[k]);
  dfree(s.A[k + 1]);
  s.A[k] = An;
  s.A[k + 1] = Bn;
  s.bonds[k + 1] = nb;
  return tot > 0.0 ? std::max(0.0, tot - kept) / tot : 0.0;
}

// layouts, environments' buffers and the one-site descriptors of sites k and
// k+1 for the current bonds; the tables of every other site are dropped
void install_sites(tt_state& s, int k) {
  HIPX(hipStreamSynchronize(ST()));
  free_site_plan(s.plans[k]);
  free_site_plan(s.plans[k + 1]);
  dfree(s.tabs.dev);
  s.tabs = SiteTables();
  s.env[k + 1] = make_env_layout(s.bonds[k + 1], s.qH[k + 1]);
  s.bmat[k + 1] = make_bondmat_layout(s.bonds[k + 1]);
  for (int j = k; j <= k + 1; ++j) {
    s.site[j] = make_site_layout(s.bonds[j], s.bonds[j + 1], s.G);
    s.plans[j] = build_site_plan(j, s.bonds[j], s.bonds[j + 1], s.G, s.qH[j], s.qH[j + 1], s.Wenv[j], s.Wpat[j],
                                 s.tabs, false, false);
    configure_plan(s.opts, s.plans[j]);
  }
  const auto& T = s.tabs.host;
  std::string rep;
  long long bad = 0;
  for (int j = k; j <= k + 1; ++j) {
    SitePlan& P = s.plans[j];
    for (GemmPlan* g : {&P.s1, &P.s3, &P.el, &P.r1, &P.r3}) tile_plan(*g, &T);
    const long long ns = s.site[j].size, el = s.env[j].size, er = s.env[j + 1].size;
    const long long s1[kSlots] = {el, ns, P.t1_size, 0}, s3[kSlots] = {P.t2_size, er, ns, 0};
    const long long se[kSlots] = {ns, P.t2_size, er, 0}, r1[kSlots] = {er, ns, P.y_size, 0};
    const long long r3[kSlots] = {ns, P.z_size, el, 0};
    bad += check_gemm(P.s1, T, s1, "s1", rep);
    bad += check_w(P.w2, P.t1_size, P.t2_size, "w2", rep);
    bad += check_gemm(P.s3, T, s3, "s3", rep);
    bad += check_gemm(P.el, T, se, "el", rep);
    bad += check_gemm(P.r1, T, r1, "r1", rep);
    bad += check_w(P.wr, P.y_size, P.z_size, "wr", rep);
    bad += check_gemm(P.r3, T, r3, "r3", rep);
  }
  TT_REQUIRE(bad == 0, TT_EINVAL, "2-TDVP: site plans out of bounds (" + std::to_string(bad) + "): " + rep);
  hipStream_t st = ST();
  s.tabs.dev = upload(s.tabs.host, st);
  long long pw = 1;
  for (int j = k; j <= k + 1; ++j) {
    SitePlan& P = s.plans[j];
    for (GemmPlan* g : {&P.s1, &P.s3, &P.el, &P.r1, &P.r3}) {
      upload_plan(*g, &T, st);
      pw = std::max(pw, g->pws_size);
    }
    upload_plan(P.w2, st);
    upload_plan(P.wr, st);
    grow(s.T1, s.cap_T1, P.t1_size);
    grow(s.T2, s.cap_T2, P.t2_size);
    grow(s.Y, s.cap_Y, P.y_size);
    grow(s.Z, s.cap_Z, P.z_size);
    grow(s.kry, s.cap_kry, s.site[j].size * (long long)s.opts.krylov_dim);
    grow(s.wv, s.cap_wv, s.site[j].size);
  }
  grow(s.pws, s.cap_pws, pw);
  for (double** e : {&s.Lenv[k + 1], &s.Renv[k + 1]}) {
    dfree(*e);
    *e = nullptr;
    *e = (double*)dalloc(8 * std::max(s.env[k + 1].size, 1LL));
  }
  s.fold[k] = s.fold[k + 1] = 0;
  s.bfz[k] = s.bfz[k + 1] = 0;
  s.lw_site = -1;
}

// one symmetric 2-TDVP step; returns the largest discarded weight of its splits
double tdvp2_once(tt_state& s, double dbeta, int Dmax, double cutoff) {
  const int N = s.N;
  const Batch b = batch_of(s);
  const double tau = 0.5 * dbeta;
  double disc = 0.0;
  std::fill(s.fold.begin(), s.fold.end(), (char)0);
  std::fill(s.bfz.begin(), s.bfz.end(), (char)0);
  s.lw_site = -1;
  for (int k = 0; k + 2 < N; ++k) {   // left to right
    {
      auto d = make_pair(s, k);
      pair_exp(s, k, *d, -tau);
      disc = std::max(disc, split_pair(s, k, *d, true, Dmax, cutoff));
    }
    install_sites(s, k);
    env_left(b, k);
    site_exp(b, k + 1, +tau);
  }
  for (int k = N - 2; k >= 0; --k) {  // right to left; the last pair's two exponentials merged
    {
      auto d = make_pair(s, k);
      pair_exp(s, k, *d, k == N - 2 ? -2.0 * tau : -tau);
      disc = std::max(disc, split_pair(s, k, *d, false, Dmax, cutoff));
    }
    install_sites(s, k);
    env_right(b, k + 1);
    if (k > 0) site_exp(b, k, +tau);
  }
  s.beta += dbeta;
  s.sweeps++;
  return disc;
}

// every plan, table and scratch buffer for the bonds the two-site sweep left
// (right environments are current; left ones are rebuilt by the next sweep)
void rebuild_plans(tt_state& s) {
  HIPX(hipStreamSynchronize(ST()));
  const int N = s.N;
  std::vector<std::map<Q, int>> dims(N + 1);
  for (int k = 0; k <= N; ++k)
    for (const Sector& sc : s.bonds[k].secs) dims[k][sc.q] = sc.dim;
  free_scratch(s);
  build_layouts(s, dims);
  s.one_site_ok = true;
  for (const SitePlan& P : s.plans)
    if (!qr_fits(P.qr) || !qr_fits(P.lq)) s.one_site_ok = false;
  require_sweep_plans(s);
  for (int k = 0; k < N; ++k)
    if (k > 0) {
      dfree(s.Lenv[k]);
      s.Lenv[k] = nullptr;
      s.Lenv[k] = (double*)dalloc(8 * std::max(s.env[k].size, 1LL));
      launch_fill(s.Lenv[k], 0.0, s.env[k].size, ST());
    }
  alloc_scratch(s);
}

int fail(const Error& e) { g_err = e.what(); return e.code; }

// ------------------------------------------------------------ MPO observables
// <<rho| O (x) 1 |rho>> / <<rho|rho>> for an operator O given as an MPO
// (bilayer value at beta_phys = 2 beta, as for the energy): right
// environments of the MPO of O from the right end to bond 1, then one
// effective-operator apply at the centre (site 0).  Always FP64.
const double kLocalOps[2][4] = {{0.0, 1.0, 1.0, 2.0},    // n = n_up + n_dn
                                {0.0, 0.0, 0.0, 1.0}};   // n_up n_dn
constexpr int kObsSpinPairs = 1000;                      // + d2: spin pairs at squared distance d2

template <typename T> bool same_bytes(const std::vector<T>& x, const std::vector<T>& y) {
  return x.size() == y.size() && (x.empty() || std::memcmp(x.data(), y.data(), sizeof(T) * x.size()) == 0);
}
constexpr int kObsGreen = 2000;                          // the Green's function G(k, beta/2)
constexpr int kObsPairing = 3000;                        // the d-wave pairing sum Delta_tot

// MPO charges per bond of an observable MPO (bond 0: start; bond N: done)
std::vector<std::vector<Q>> obs_charges(const tt_state& s, const Mpo& m) {
  std::vector<std::vector<Q>> qH(s.N + 1);
  for (int k = 0; k < s.N; ++k)
    for (int a = 0; a < m.DH[k]; ++a) qH[k].push_back(project_charge(m.charge(k, a), s.opts.symmetry));
  qH[s.N] = {Q{0, 0}};
  return qH;
}
// site tensors with the last one contracted with the done selector (the last
// state of bond N)
std::vector<std::vector<double>> obs_tensors(const Mpo& m) {
  const int N = m.N, LL = m.ld * m.ld, DRN = m.DH[N];
  std::vector<std::vector<double>> W = m.W;
  std::vector<double> w((size_t)m.DH[N - 1] * LL, 0.0);
  for (int a = 0; a < m.DH[N - 1]; ++a)
    for (int q = 0; q < LL; ++q) w[(size_t)a * LL + q] = m.W[N - 1][((size_t)a * LL + q) * DRN + (DRN - 1)];
  W[N - 1] = w;
  return W;
}
// host plans of an observable MPO m; pat gives the nonzero pattern kept in
// the W stage (so that MPOs differing only in weights share descriptors)
std::vector<SitePlan> make_obs_plans(const tt_state& s, const Mpo& m, const Mpo& pat, SiteTables& tabs) {
  const auto qH = obs_charges(s, m);
  const auto W = obs_tensors(m), Wp = obs_tensors(pat);
  std::vector<SitePlan> plans;
  for (int k = 0; k < s.N; ++k) {
    SitePlan P = build_site_plan(k, s.bonds[k], s.bonds[k + 1], s.G, qH[k], qH[k + 1], W[k], Wp[k], tabs, m.ld == 16,
                                 false);
    for (GemmPlan* g : {&P.s1, &P.s3, &P.r1, &P.r3}) g->wave_ok = true;
    plans.push_back(std::move(P));
  }
  return plans;
}
// descriptor bounds of the launches of obs_expectation: centre apply at site
// 0 (unit, A_0 -> T1 -> T2 -> with R_1 into a site-sized vector) and the
// right environments of sites N-1 .. 1 (R_{k+1}, A_k -> Y -> Z -> R_k)
long long check_obs_plans(const tt_state& s, const Mpo& m, std::vector<SitePlan>& plans, const SiteTables& tabs,
                          std::string& rep) {
  const auto qH = obs_charges(s, m);
  const auto& T = tabs.host;
  long long bad = 0;
  for (int k = 0; k < s.N; ++k) {
    SitePlan& P = plans[k];
    const long long ns = s.site[k].size, el = make_env_layout(s.bonds[k], qH[k]).size,
                    er = make_env_layout(s.bonds[k + 1], qH[k + 1]).size;
    if (k == 0) {
      for (GemmPlan* g : {&P.s1, &P.s3}) tile_plan(*g, &T);
      long long s1[kSlots] = {el, ns, P.t1_size, 0}, s3[kSlots] = {P.t2_size, er, ns, 0};
      bad += check_gemm(P.s1, T, s1, "obs s1", rep);
      bad += check_w(P.w2, P.t1_size, P.t2_size, "obs w2", rep);
      bad += check_gemm(P.s3, T, s3, "obs s3", rep);
    } else {
      for (GemmPlan* g : {&P.r1, &P.r3}) tile_plan(*g, &T);
      long long r1[kSlots] = {er, ns, P.y_size, 0}, r3[kSlots] = {ns, P.z_size, el, 0};
      bad += check_gemm(P.r1, T, r1, "obs r1", rep);
      bad += check_w(P.wr, P.y_size, P.z_size, "obs wr", rep);
      bad += check_gemm(P.r3, T, r3, "obs r3", rep);
    }
  }
  return bad;
}

// plans and buffers of one observable MPO (bond 0: start; bond N: its last
// state, done)
tt_state::ObsMpo& build_obs_mpo(tt_state& s, int key, const Mpo& m, const Mpo* pat = nullptr) {
  const int N = s.N;
  hipStream_t st = ST();
  SiteTables tabs;
  std::vector<SitePlan> plans = make_obs_plans(s, m, pat ? *pat : m, tabs);
  std::string rep;
  TT_REQUIRE(check_obs_plans(s, m, plans, tabs, rep) == 0, TT_EINVAL, "observable plans out of bounds: " + rep);
  auto& O = s.obs[key];
  O.tabs = std::move(tabs);
  O.plans = std::move(plans);
  const auto qH = obs_charges(s, m);
  long long t1 = 1, t2 = 1, y = 1, z = 1, env = 1, pw = 1;
  for (int k = 0; k <= N; ++k) env = std::max(env, make_env_layout(s.bonds[k], qH[k]).size);
  O.tabs.dev = upload(O.tabs.host, st);
  const std::vector<long long>* T = &O.tabs.host;
  for (int k = 0; k < N; ++k) {
    SitePlan& P = O.plans[k];
    if (k == 0) {
      upload_plan(P.s1, T, st); upload_plan(P.w2, st); upload_plan(P.s3, T, st);
      t1 = std::max(t1, P.t1_size); t2 = std::max(t2, P.t2_size);
      pw = std::max(pw, std::max(P.s1.pws_size, P.s3.pws_size));
    } else {
      upload_plan(P.r1, T, st); upload_plan(P.wr, st); upload_plan(P.r3, T, st);
      y = std::max(y, P.y_size); z = std::max(z, P.z_size);
      pw = std::max(pw, std::max(P.r1.pws_size, P.r3.pws_size));
    }
  }
  O.ea = (double*)dalloc(8 * env); O.eb = (double*)dalloc(8 * env); O.unit = (double*)dalloc(8);
  O.pws = (double*)dalloc(8 * pw);
  O.T1 = (double*)dalloc(8 * t1); O.T2 = (double*)dalloc(8 * t2);
  O.Y = (double*)dalloc(8 * y); O.Z = (double*)dalloc(8 * z);
  return O;
}

double obs_expectation(tt_state& s, tt_state::ObsMpo& O) {
  const int N = s.N;
  hipStream_t st = ST();
  double* Rin = O.ea;
  double* Rout = O.eb;
  launch_fill(Rin, 1.0, 1, st);      // bond N: the done channel
  for (int k = N - 1; k >= 1; --k) {
    SitePlan& P = O.plans[k];
    launch_gemm(P.r1, O.tabs.dev, one(Slots{{Rin, s.A[k], O.Y, nullptr}}), 1, TT_FP64, one(O.pws), st);
    launch_wstage(P.wr, one<const WTerm>(P.wr.d_terms), one<const double>(O.Y), one(O.Z), 1, st);
    launch_gemm(P.r3, O.tabs.dev, one(Slots{{s.A[k], O.Z, Rout, nullptr}}), 1, TT_FP64, one(O.pws), st);
    std::swap(Rin, Rout);
  }
  SitePlan& P = O.plans[0];
  launch_fill(O.unit, 1.0, 1, st);   // bond 0: the start channel
  launch_gemm(P.s1, O.tabs.dev, one(Slots{{O.unit, s.A[0], O.T1, nullptr}}), 1, TT_FP64, one(O.pws), st);
  launch_wstage(P.w2, one<const WTerm>(P.w2.d_terms), one<const double>(O.T1), one(O.T2), 1, st);
  launch_gemm(P.s3, O.tabs.dev, one(Slots{{O.T2, Rin, s.wv, nullptr}}), 1, TT_FP64, one(O.pws), st);
  const long long n = s.site[0].size;
  double* ob = s.obs_ptr();
  launch_mdot(one<const double>(s.A[0]), n, 1, one<const double>(s.wv), n, 0, one(s.part), 1, st);
  launch_dot_final(s.part, kRedBlocks, 1, ob, st);
  launch_mdot(BPtr<const double>{}, 0, 0, one<const double>(s.A[0]), n, 1, one(s.part), 1, st);
  launch_dot_final(s.part, kRedBlocks, 1, ob + 1, st);
  double h[2];
  HIPX(hipMemcpyAsync(h, ob, 16, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  return h[0] / h[1];
}

// G(k, beta_phys/2) of the bilayer state: <<rho|X(k)|rho>> / (N <<rho|rho>>).
// The plans keep the nonzero pattern of every momentum, so a new k only
// rewrites the W-stage weights of the cached plans.
double green_expectation(tt_state& s, double kx, double ky) {
  auto it = s.obs.find(kObsGreen);
  const Mpo m = make_green_mpo(s.lat, kx, ky, false);
  if (it == s.obs.end()) {
    const Mpo pat = make_green_mpo(s.lat, kx, ky, true);
    tt_state::ObsMpo& O = build_obs_mpo(s, kObsGreen, m, &pat);
    O.kx = kx; O.ky = ky;
    return obs_expectation(s, O) / s.N;
  }
  tt_state::ObsMpo& O = it->second;
  if (O.kx != kx || O.ky != ky) {
    const auto W = obs_tensors(m);
    hipStream_t st = ST();
    for (int k = 0; k < s.N; ++k) {
      WPlan& P = k == 0 ? O.plans[k].w2 : O.plans[k].wr;
      TT_REQUIRE(P.widx.size() == P.terms.size(), TT_EINVAL, "green function: plan without weight indices");
      for (size_t i = 0; i < P.terms.size(); ++i) P.terms[i].w = W[k].at((size_t)P.widx[i]);
      if (!P.terms.empty())
        HIPX(hipMemcpyAsync(P.d_terms, P.terms.data(), P.terms.size() * sizeof(WTerm), hipMemcpyHostToDevice, st));
    }
    HIPX(hipStreamSynchronize(st));
    O.kx = kx; O.ky = ky;
  }
  return obs_expectation(s, O) / s.N;
}

double local_expectation(tt_state& s, int kind) {
  auto it = s.obs.find(kind);
  tt_state::ObsMpo& O = it != s.obs.end() ? it->second : build_obs_mpo(s, kind, make_local_sum_mpo(s.N, kLocalOps[kind]));
  return obs_expectation(s, O);
}

#define ABI_BEGIN try {
#define ABI_END                                                   \
  }                                                               \
  catch (const Error& e) { return fail(e); }                      \
  catch (const std::bad_alloc&) { g_err = "host allocation failed"; return TT_ENOMEM; } \
  catch (const std::exception& e) { g_err = e.what(); return TT_EINVAL; }             \
  return TT_OK;

void fill_stats(tt_state& s, tt_sweep_stats* st, double secs) {
  double err = 0.0;
  HIPX(hipMemcpyAsync(&err, s.err_ptr(), 8, hipMemcpyDeviceToHost, ST()));
  HIPX(hipStreamSynchronize(ST()));
  st->seconds += secs;
  st->flops_alg += s.flops;
  st->flops_heff += s.flops_heff;
  st->bytes_min += s.bytes_min;
  st->n_applies += s.n_applies;
  st->n_exps += s.n_exps;
  st->max_krylov_err = std::max(st->max_krylov_err, err);
}
// per-phase device time of the call (zeros unless phase timing was on)
void fill_phases(tt_sweep_stats* st) {
  double ph[PH_COUNT];
  phase_read(ph);
  st->t_heff = ph[PH_HEFF];
  st->t_bond = ph[PH_BOND];
  st->t_lanczos = std::max(0.0, ph[PH_EXP] - ph[PH_HEFF] - ph[PH_BOND]);
  st->t_qr = ph[PH_QR];
  st->t_env = ph[PH_ENV];
  st->t_absorb = ph[PH_ABSORB];
}
void reset_counters(tt_state& s) { s.flops = s.flops_heff = s.bytes_min = 0.0; s.n_applies = s.n_exps = 0; }

bool same_gemm(const GemmPlan& x, const GemmPlan& y) {
  return same_bytes(x.probs, y.probs) && same_bytes(x.tiles, y.tiles) && same_bytes(x.jobs, y.jobs) &&
         same_bytes(x.jobs_fine, y.jobs_fine) && same_bytes(x.splits, y.splits) && x.pws_size == y.pws_size &&
         x.wave_blocks == y.wave_blocks && x.wave_blocks_fine == y.wave_blocks_fine;
}
bool same_w(const WPlan& x, const WPlan& y) {   // the weights may differ
  if (!same_bytes(x.tasks, y.tasks) || x.terms.size() != y.terms.size()) return false;
  for (size_t i = 0; i < x.terms.size(); ++i)
    if (x.terms[i].src != y.terms[i].src || x.terms[i].ssi != y.terms[i].ssi || x.terms[i].ssj != y.terms[i].ssj)
      return false;
  return true;
}
bool same_qr(const QRPlan& x, const QRPlan& y) {
  return same_bytes(x.tasks, y.tasks) && same_bytes(x.chunks, y.chunks) && same_bytes(x.stacks, y.stacks) &&
         same_bytes(x.wide, y.wide) && x.ws_size == y.ws_size && x.lds_ws == y.lds_ws;
}
// two states can share launches: same lattice size, options, bond sectors,
// index tables and plans (only MPO weights, i.e. the couplings, may differ)
bool same_plans(const tt_state& a, const tt_state& b) {
  const tt_options &x = a.opts, &y = b.opts;
  if (a.N != b.N || x.D != y.D || x.symmetry != y.symmetry || x.precision != y.precision ||
      x.krylov_dim != y.krylov_dim || x.krylov_tol != y.krylov_tol || x.sector_cap != y.sector_cap)
    return false;
  if (!same_bytes(a.tabs.host, b.tabs.host)) return false;
  for (int k = 0; k <= a.N; ++k) {
    if (a.bonds[k].secs.size() != b.bonds[k].secs.size() || a.qH[k] != b.qH[k]) return false;
    for (size_t i = 0; i < a.bonds[k].secs.size(); ++i)
      if (!(a.bonds[k].secs[i].q == b.bonds[k].secs[i].q) || a.bonds[k].secs[i].dim != b.bonds[k].secs[i].dim)
        return false;
  }
  for (int k = 0; k < a.N; ++k) {
    const SitePlan &P = a.plans[k], &Q = b.plans[k];
    if (a.site[k].size != b.site[k].size || a.bmat[k].size != b.bmat[k].size) return false;
    for (auto pr : {std::make_pair(&P.s1, &Q.s1), std::make_pair(&P.s3, &Q.s3), std::make_pair(&P.el, &Q.el),
                    std::make_pair(&P.r1, &Q.r1), std::make_pair(&P.r3, &Q.r3), std::make_pair(&P.absL, &Q.absL),
                    std::make_pair(&P.absR, &Q.absR), std::make_pair(&P.b1, &Q.b1), std::make_pair(&P.b2, &Q.b2)})
      if (!same_gemm(*pr.first, *pr.second)) return false;
    if (!same_w(P.lw, Q.lw) || !same_w(P.t2zero, Q.t2zero) || !same_w(P.wr, Q.wr) || !same_qr(P.qr, Q.qr) ||
        !same_qr(P.lq, Q.lq) || P.n_s1w != Q.n_s1w)
      return false;
    for (int j = 0; j < P.n_s1w; ++j)
      if (!same_gemm(P.s1w[j], Q.s1w[j])) return false;
    if (!same_gemm(P.s1, Q.s1) || !same_w(P.w2, Q.w2) || a.fold[k] != b.fold[k] || a.bfz[k] != b.bfz[k]) return false;
  }
  return true;
}

// -------------------------------------------------------------- dense microbenchmark
// Host side of the dense apply: the plans of its three launches (L.A, the W
// stage as grouped GEMMs reading W from device memory, .R), tiled, with their
// index tables and the sizes of the intermediates they address.
struct HeffPlans {
  SitePlan plan;
  SiteTables tabs;
  GemmPlan wg;
  long long t1 = 0, t2 = 0, pw = 1;
};

GemmPlan heff_wstage_plan(int Dl, int Dr, int DH, long long t2row, SiteTables& tabs);

HeffPlans heff_plans(int Dl, int Dr, int DH) {
  HeffPlans h;
  Bond bl, br;
  bl.add({0, 0}, Dl);
  br.add({0, 0}, Dr);
  Groups G = make_groups(0);
  std::vector<Q> qh(DH, Q{0, 0});
  // the plan's W stage is replaced by a grouped GEMM reading W from device memory;
  // an all-zero W keeps the sparse W-stage plan empty
  std::vector<double> Wz((size_t)DH * 16 * DH, 0.0);
  h.plan = build_site_plan(0, bl, br, G, qh, qh, Wz, Wz, h.tabs, false, false);
  h.wg = heff_wstage_plan(Dl, Dr, DH, (long long)DH * Dr, h.tabs);
  for (GemmPlan* g : {&h.plan.s1, &h.plan.s3, &h.wg}) tile_plan(*g, &h.tabs.host);
  h.t1 = h.plan.t1_size;
  h.t2 = h.plan.t2_size;
  h.pw = std::max(std::max(h.plan.s1.pws_size, h.plan.s3.pws_size), std::max(h.wg.pws_size, 1LL));
  return h;
}

// The W stage of the dense apply as grouped GEMMs, one per (x', sigma'):
// T2[(x', so, sp)][(b, y)] = sum_(a, si) W[a, so, si, b] T1[a][x'][si][sp][y],
// rows of T2 t2row elements apart (its index tables go into tabs)
GemmPlan heff_wstage_plan(int Dl, int Dr, int DH, long long t2row, SiteTables& tabs) {
  GemmPlan wg;
  std::vector<long long> am, ak, bk, cm;
  for (int so = 0; so < 4; ++so)
    for (int b = 0; b < DH; ++b) am.push_back((long long)so * 4 * DH + b);
  for (int a = 0; a < DH; ++a)
    for (int si = 0; si < 4; ++si) {
      ak.push_back((long long)a * 16 * DH + (long long)si * DH);
      bk.push_back((long long)a * Dl * 16 * Dr + (long long)si * 4 * Dr);
    }
  for (int so = 0; so < 4; ++so)
    for (int b = 0; b < DH; ++b) cm.push_back((long long)4 * so * t2row + (long long)b * Dr);
  long long tam = tabs.add(am), tak = tabs.add(ak), tbk = tabs.add(bk), tcm = tabs.add(cm);
  wg.tag = TAG_WGEMM;
  for (int x = 0; x < Dl; ++x)
    for (int sp = 0; sp < 4; ++sp) {
      GemmProb g{};
      g.M = 4 * DH; g.N = Dr; g.K = 4 * DH;
      g.ia = 0; g.ib = 1; g.ic = 2;
      g.tam = tam; g.tak = tak; g.tbk = tbk; g.tbn = -1; g.tcm = tcm;
      g.sbn = 1;
      g.offB = (long long)x * 16 * Dr + (long long)sp * Dr;
      g.offC = ((long long)x * 16 + sp) * t2row;
      g.alpha = 1.0; g.beta = 0.0;
      wg.probs.push_back(g);
      wg.flops += 2.0 * g.M * (double)g.N * g.K;
    }
  return wg;
}

// The FP64 dense apply on the large-tile kernels: L and A copied into rows of
// the contracted index zero-padded to the GEMM's K tile (A transposed), L.A
// into T1[a][x'][s][y], the W stage on the vector units into T2 rows (x', s)
// padded the same way (their padding written as zeros by it), R padded, .R.
struct DenseF64Sizes {
  int kq1 = 0, kq3 = 0;
  long long lq = 0, aq = 0, rq = 0, t1 = 0, t2q = 0;
};
DenseF64Sizes dense_f64_sizes(int Dl, int Dr, int DH) {
  DenseF64Sizes z;
  z.kq1 = dgemm_kpad(Dl);
  z.kq3 = dgemm_kpad((long long)DH * Dr);
  z.lq = (long long)Dl * DH * z.kq1;
  z.aq = 16LL * Dr * z.kq1;
  z.rq = (long long)Dr * z.kq3;
  z.t1 = (long long)Dl * DH * 16 * Dr;
  z.t2q = 16LL * Dl * z.kq3;
  return z;
}
bool dense_f64_applies(int DH) { return DH <= wstage_planes_max_dh(); }
struct DenseF64Bufs { double *Lq, *Aq, *Rq, *T1, *T2q; };
void dense_apply_f64(int Dl, int Dr, int DH, const double* L, const double* W, const double* A, const double* R,
                     double* out, const DenseF64Bufs& b, const DenseF64Sizes& z, const hipEvent_t* ev, hipStream_t st) {
  const long long M1 = (long long)Dl * DH, N1 = 16LL * Dr;
  if (ev) HIPX(hipEventRecord(ev[0], st));
  launch_pad_rows(L, M1, Dl, Dl, b.Lq, z.kq1, st);
  launch_pad_t(A, Dl, (int)N1, b.Aq, z.kq1, st);
  DgArgs g1{};
  g1.A = b.Lq; g1.lda = z.kq1; g1.B = b.Aq; g1.ldb = z.kq1;
  g1.M = (int)M1; g1.N = (int)N1; g1.K = z.kq1;
  g1.C = b.T1; g1.cdiv = DH; g1.ldc0 = (long long)Dl * N1; g1.ldc1 = N1;
  launch_dgemm(g1, st);
  if (ev) HIPX(hipEventRecord(ev[1], st));
  launch_wstage_f64(b.T1, W, DH, Dl, Dr, b.T2q, z.kq3, st);
  if (ev) HIPX(hipEventRecord(ev[2], st));
  launch_pad_rows(R, Dr, (int)((long long)DH * Dr), (long long)DH * Dr, b.Rq, z.kq3, st);
  DgArgs g3{};
  g3.A = b.T2q; g3.lda = z.kq3; g3.B = b.Rq; g3.ldb = z.kq3;
  g3.M = 16 * Dl; g3.N = Dr; g3.K = z.kq3;
  g3.C = out; g3.cdiv = 16 * Dl; g3.ldc0 = Dr; g3.ldc1 = 0;
  launch_dgemm(g3, st);
  if (ev) HIPX(hipEventRecord(ev[3], st));
}

// The FP32 dense apply on the same plan: float copies of L, A, R (K padded to
// the FP32 GEMM's tile), float T1 and T2, FP32 multiplies with the GEMMs'
// partials added in FP64, the result in FP64.  Its buffers fit in the FP64
// path's (every float piece is at most as many bytes as its FP64 counterpart).
struct DenseF32Bufs { float *Lf, *Af, *Rf, *T1f, *T2f; };
void dense_apply_f32(int Dl, int Dr, int DH, const double* L, const double* W, const double* A, const double* R,
                     double* out, const DenseF32Bufs& b, const hipEvent_t* ev, hipStream_t st) {
  const long long M1 = (long long)Dl * DH, N1 = 16LL * Dr, K3 = (long long)DH * Dr;
  const int kp1 = sgemm_kpad(Dl), kp3 = sgemm_kpad(K3);
  if (ev) HIPX(hipEventRecord(ev[0], st));
  launch_pad_rows(L, M1, Dl, Dl, b.Lf, kp1, st);
  launch_pad_t(A, Dl, (int)N1, b.Af, kp1, st);
  SgArgs g1{};
  g1.A = b.Lf; g1.lda = kp1; g1.B = b.Af; g1.ldb = kp1;
  g1.M = (int)M1; g1.N = (int)N1; g1.K = kp1;
  g1.C = b.T1f; g1.cdiv = DH; g1.ldc0 = (long long)Dl * N1; g1.ldc1 = N1; g1.cfloat = 1;
  launch_sgemm(g1, st);
  if (ev) HIPX(hipEventRecord(ev[1], st));
  launch_wstage_f32(b.T1f, W, DH, Dl, Dr, b.T2f, kp3, st);
  if (ev) HIPX(hipEventRecord(ev[2], st));
  launch_pad_rows(R, Dr, (int)K3, K3, b.Rf, kp3, st);
  SgArgs g3{};
  g3.A = b.T2f; g3.lda = kp3; g3.B = b.Rf; g3.ldb = kp3;
  g3.M = 16 * Dl; g3.N = Dr; g3.K = kp3;
  g3.C = out; g3.cdiv = 16 * Dl; g3.ldc0 = Dr; g3.ldc1 = 0; g3.cfloat = 0;
  launch_sgemm(g3, st);
  if (ev) HIPX(hipEventRecord(ev[3], st));
}

struct HeffCache {
  int Dl = -1, Dr = -1, DH = -1;
  SitePlan plan;
  SiteTables tabs;
  GemmPlan wg;
  double *T1 = nullptr, *T2 = nullptr, *pws = nullptr;
  long long t1 = 0, t2 = 0, pw = 0;
  // split-BF16 modes: L.A and .R by the large-tile BF16 GEMM on operands
  // split (and padded in K) into BF16 planes, the W stage (wgq: T2 rows padded
  // to kp3) by the grouped GEMM on planes; every intermediate as planes
  GemmPlan wgq;
  int kp1 = 0, kp3 = 0;
  void* planes = nullptr;
  long long plane_bytes = 0;
  // FP64: padded copies of L, A, R and the padded T2 (T1 is the buffer above)
  double* f64 = nullptr;
  long long f64_doubles = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
};
HeffCache g_heff;

void build_heff_cache(int Dl, int Dr, int DH) {
  HeffCache& c = g_heff;
  free_plan(c.plan.s1); free_plan(c.plan.s3); free_plan(c.wg);
  dfree(c.tabs.dev); c.tabs = SiteTables();
  HeffPlans h = heff_plans(Dl, Dr, DH);
  c.plan = std::move(h.plan);
  c.tabs = std::move(h.tabs);
  c.wg = std::move(h.wg);
  hipStream_t st = ST();
  c.tabs.dev = upload(c.tabs.host, st);
  upload_plan(c.plan.s1, &c.tabs.host, st);
  upload_plan(c.plan.s3, &c.tabs.host, st);
  upload_plan(c.wg, &c.tabs.host, st);
  free_plan(c.wgq);
  c.kp1 = bgemm_kpad(Dl);
  c.kp3 = bgemm_kpad((long long)DH * Dr);
  c.wgq = heff_wstage_plan(Dl, Dr, DH, c.kp3, c.tabs);
  c.wgq.no_split = true;
  dfree(c.tabs.dev);
  c.tabs.dev = upload(c.tabs.host, st);
  upload_plan(c.wgq, &c.tabs.host, st);
  if (h.t1 > c.t1) { dfree(c.T1); c.T1 = (double*)dalloc(8 * h.t1); c.t1 = h.t1; }
  if (h.t2 > c.t2) { dfree(c.T2); c.T2 = (double*)dalloc(8 * h.t2); c.t2 = h.t2; }
  if (h.pw > c.pw) { dfree(c.pws); c.pws = (double*)dalloc(8 * h.pw); c.pw = h.pw; }
  for (int i = 0; i < 4; ++i)
    if (!c.ev[i]) HIPX(hipEventCreate(&c.ev[i]));
  c.Dl = Dl; c.Dr = Dr; c.DH = DH;
}

}  // namespace

// ---------------------------------------------------------- allocation-free dense apply
// The device memory of tt_heff_apply_noalloc: the intermediates T1 and T2, the
// K-slice partial tiles and every descriptor table of its three launches.  One
// copy per GPU, held until the process ends.  Host code must not pass the
// array's name to a kernel or a copy (in host code it is a host-side stand-in):
// it uses the address hipGetSymbolAddress returns on each device.
constexpr long long kScratchBytes = 192LL << 20;
static __device__ __align__(256) double scratch[kScratchBytes / 8];

namespace {

constexpr int kMaxDevices = 64;
struct NoAllocDev {
  char* base = nullptr;            // this GPU's copy of the scratch array
  int Dl = -1, Dr = -1, DH = -1;   // the sizes whose descriptors the scratch holds
  HeffPlans host;                  // their host copy
  GemmPlan s1, s3, wg;             // the same plans with device pointers into the scratch
  long long* tabs = nullptr;
  double *T1 = nullptr, *T2 = nullptr, *pws = nullptr;
  double *Lq = nullptr, *Aq = nullptr, *Rq = nullptr;   // the FP64 path's padded copies
  int Dl_pending = 0, Dr_pending = 0, DH_pending = 0;   // the sizes being laid out
};
NoAllocDev g_noalloc[kMaxDevices];

// Lay the apply's buffers out in the scratch (256-byte aligned pieces); with
// copy, also upload the descriptors.  Returns the bytes used.
long long noalloc_layout(NoAllocDev& d, bool copy, hipStream_t st) {
  long long used = 0;
  auto carve = [&](long long bytes) -> char* {
    used = (used + 255) & ~255LL;
    char* p = d.base + used;
    used += std::max(bytes, 8LL);
    return p;
  };
  auto put = [&](auto*& dst, const auto& v) {
    using T = typename std::decay<decltype(v)>::type::value_type;
    dst = reinterpret_cast<T*>(carve((long long)(sizeof(T) * v.size())));
    if (copy && !v.empty() && used <= kScratchBytes)
      HIPX(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  };
  HeffPlans& h = d.host;
  const DenseF64Sizes z = dense_f64_sizes(d.Dl_pending, d.Dr_pending, d.DH_pending);
  d.T1 = reinterpret_cast<double*>(carve(8 * h.t1));
  d.T2 = reinterpret_cast<double*>(carve(8 * std::max(h.t2, z.t2q)));   // T2, or the FP64 path's padded T2
  d.Lq = reinterpret_cast<double*>(carve(8 * z.lq));
  d.Aq = reinterpret_cast<double*>(carve(8 * z.aq));
  d.Rq = reinterpret_cast<double*>(carve(8 * z.rq));
  d.pws = reinterpret_cast<double*>(carve(8 * h.pw));
  put(d.tabs, h.tabs.host);
  GemmPlan* dev[3] = {&d.s1, &d.wg, &d.s3};
  const GemmPlan* src[3] = {&h.plan.s1, &h.wg, &h.plan.s3};
  for (int i = 0; i < 3; ++i) {
    *dev[i] = *src[i];
    put(dev[i]->d_probs, src[i]->probs);
    put(dev[i]->d_tiles, src[i]->tiles);
    put(dev[i]->d_splits, src[i]->splits);
    put(dev[i]->d_jobs, src[i]->jobs);
    put(dev[i]->d_jobs_fine, src[i]->jobs_fine);
  }
  return used;
}

// The two-site generator H^(2) C of 2-TDVP on dense operands, in the order
// L.C, then W1, then W2, then R, as four grouped GEMMs.  The ancilla index of
// each site (sigma' in s = 4 sigma + sigma') rides along in the column index of
// the W stages, so no stage multiplies by the identity on it.  Layouts:
//   T1[(x', a)][(s1, s2, y)]                       = L . C
//   T2[x'][so1][b][(a1, s2, y)]                    = W1 stage, one GEMM per x'
//   T3[x'][so1][a1][so2][c][(a2, y)] (T1's buffer) = W2 stage, one GEMM per (x', so1, a1)
//   out[x'][4 so1 + a1][4 so2 + a2][y2]            = T3 . R
struct Heff2Cache {
  int Dl = -1, Dr = -1, DH = -1;
  SiteTables tabs;
  GemmPlan st[4];
  double *T1 = nullptr, *T2 = nullptr, *pws = nullptr;
  long long t = 0, pw = 0;
};
Heff2Cache g_heff2;

void build_heff2_cache(int Dl, int Dr, int DH) {
  Heff2Cache& c = g_heff2;
  for (auto& p : c.st) free_plan(p);
  dfree(c.tabs.dev);
  c.tabs = SiteTables();
  const long long D64 = 64LL * Dr, D256 = 256LL * Dr, D4 = 4LL * Dr;
  const long long tsize = (long long)Dl * DH * D256;
  // W[(so, b)][(a, si)] = W[a][so][si][b]: row and depth tables
  std::vector<long long> wr, wk;
  for (int so = 0; so < 4; ++so)
    for (int b = 0; b < DH; ++b) wr.push_back((long long)so * 4 * DH + b);
  for (int a = 0; a < DH; ++a)
    for (int si = 0; si < 4; ++si) wk.push_back((long long)a * 16 * DH + (long long)si * DH);
  std::vector<long long> t1k, t2k, t3k, t3r, outr;
  for (int a = 0; a < DH; ++a)
    for (int si = 0; si < 4; ++si) t1k.push_back(a * D256 + si * D64);
  for (int b = 0; b < DH; ++b)
    for (int si = 0; si < 4; ++si) t2k.push_back(b * D64 + si * D4);
  for (int cc = 0; cc < DH; ++cc)
    for (int y = 0; y < Dr; ++y) t3k.push_back(cc * D4 + y);
  for (int x = 0; x < Dl; ++x)
    for (int so1 = 0; so1 < 4; ++so1)
      for (int a1 = 0; a1 < 4; ++a1)
        for (int so2 = 0; so2 < 4; ++so2)
          for (int a2 = 0; a2 < 4; ++a2) {
            t3r.push_back((((long long)x * 4 + so1) * 4 + a1) * 16 * DH * Dr + (long long)so2 * DH * D4 + (long long)a2 * Dr);
            outr.push_back((((long long)x * 16 + 4 * so1 + a1) * 16 + 4 * so2 + a2) * Dr);
          }
  const long long twr = c.tabs.add(wr), twk = c.tabs.add(wk), tt1k = c.tabs.add(t1k), tt2k = c.tabs.add(t2k),
                  tt3k = c.tabs.add(t3k), tt3r = c.tabs.add(t3r), tout = c.tabs.add(outr);
  auto prob = [](int M, int N, int K) {
    GemmProb g{};
    g.M = M; g.N = N; g.K = K;
    g.ia = 0; g.ib = 1; g.ic = 2;
    g.tam = g.tak = g.tbk = g.tbn = g.tcm = -1;
    g.alpha = 1.0; g.beta = 0.0;
    return g;
  };
  for (auto& p : c.st) { p = GemmPlan(); p.tag = TAG_WGEMM; p.wave_ok = true; }
  {  // L . C
    GemmProb g = prob(Dl * DH, (int)D256, Dl);
    g.sam = Dl; g.sak = 1; g.sbk = D256; g.sbn = 1; g.scm = D256;
    c.st[0].probs.push_back(g);
  }
  for (int x = 0; x < Dl; ++x) {  // W1 stage
    GemmProb g = prob(4 * DH, (int)D64, 4 * DH);
    g.tam = twr; g.tak = twk;
    g.offB = (long long)x * DH * D256; g.tbk = tt1k; g.sbn = 1;
    g.offC = (long long)x * 4 * DH * D64; g.scm = D64;
    c.st[1].probs.push_back(g);
  }
  for (int x = 0; x < Dl; ++x)  // W2 stage
    for (int so1 = 0; so1 < 4; ++so1)
      for (int a1 = 0; a1 < 4; ++a1) {
        GemmProb g = prob(4 * DH, (int)D4, 4 * DH);
        g.tam = twr; g.tak = twk;
        g.offB = ((long long)x * 4 + so1) * DH * D64 + a1 * 16LL * Dr; g.tbk = tt2k; g.sbn = 1;
        g.offC = (((long long)x * 4 + so1) * 4 + a1) * 4 * DH * D4; g.scm = D4;
        c.st[2].probs.push_back(g);
      }
  {  // . R
    GemmProb g = prob(256 * Dl, Dr, DH * Dr);
    g.tam = tt3r; g.tak = tt3k; g.sbk = 1; g.sbn = (long long)DH * Dr; g.tcm = tout;
    c.st[3].probs.push_back(g);
  }
  for (auto& p : c.st)
    for (auto& g : p.probs) p.flops += 2.0 * g.M * (double)g.N * g.K;
  const long long sizes[4][kSlots] = {{(long long)Dl * DH * Dl, (long long)Dl * D256, tsize, 0},
                                      {(long long)DH * 16 * DH, tsize, tsize, 0},
                                      {(long long)DH * 16 * DH, tsize, tsize, 0},
                                      {tsize, (long long)Dr * DH * Dr, (long long)Dl * D256, 0}};
  std::string rep;
  long long bad = 0, pw = 1;
  for (int i = 0; i < 4; ++i) {
    tile_plan(c.st[i], &c.tabs.host);
    bad += check_gemm(c.st[i], c.tabs.host, sizes[i], "heff2", rep);
    pw = std::max(pw, c.st[i].pws_size);
  }
  TT_REQUIRE(bad == 0, TT_EINVAL, "heff2 plan out of bounds: " + rep);
  hipStream_t st = ST();
  c.tabs.dev = upload(c.tabs.host, st);
  for (auto& p : c.st) upload_plan(p, &c.tabs.host, st);
  if (tsize > c.t) {
    dfree(c.T1); dfree(c.T2);
    c.T1 = (double*)dalloc(8 * tsize); c.T2 = (double*)dalloc(8 * tsize); c.t = tsize;
  }
  if (pw > c.pw) { dfree(c.pws); c.pws = (double*)dalloc(8 * pw); c.pw = pw; }
  c.Dl = Dl; c.Dr = Dr; c.DH = DH;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* tt_last_error(void) { return g_err.c_str(); }

int tt_options_default(tt_options* o) {
  if (!o) { g_err = "null options"; return TT_EINVAL; }
  o->D = 64; o->symmetry = 1; o->beta0 = 1e-2; o->taylor_order = 1;
  o->krylov_dim = 8; o->krylov_tol = 1e-13; o->precision = TT_FP64;
  o->pad_eps = 0.0; o->seed = 1; o->env_on_host = 0; o->sector_cap = 64;
  return TT_OK;
}

int tt_set_stream(void* stream) {
  g_stream = (hipStream_t)stream;
  return TT_OK;
}

int tt_set_allocator(tt_alloc_fn alloc, tt_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) { g_err = "give both allocator functions or neither"; return TT_EINVAL; }
  g_alloc = alloc; g_free = free_fn; g_alloc_ctx = ctx;
  return TT_OK;
}

int mpo_init_highT(const tt_model* model, const tt_options* opts, tt_state** out) {
  ABI_BEGIN
  TT_REQUIRE(model && opts && out, TT_EINVAL, "null argument");
  *out = nullptr;
  auto s = make_state(*model, *opts);
  std::vector<std::vector<double>> host;
  fill_initial_tensors(*s, host);
  s->rho0 = Rho0();
  for (int k = 0; k < s->N; ++k)
    HIPX(hipMemcpyAsync(s->A[k], host[k].data(), 8 * host[k].size(), hipMemcpyHostToDevice, ST()));
  canonicalise_and_envs(*s);
  s->beta = opts->beta0;
  HIPX(hipStreamSynchronize(ST()));
  *out = s.release();
  ABI_END
}

// One sweep through a captured graph: the first sweep with a step dbeta is
// captured on a private stream (the caller's stream may be the null stream,
// which cannot be captured) and instantiated; every sweep launches the graph on
// the caller's stream.  Kernel arguments are fixed by the state's buffers and
// dbeta, and a sweep has no host round trip, so a replay repeats it exactly.
void sweep_graph(tt_state& s, double dbeta) {
  static hipStream_t cap = nullptr;
  if (!cap) HIPX(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  auto& G = s.sg;
  if (!G.exec || G.dbeta != dbeta) {
    if (G.exec) { HIPX(hipGraphExecDestroy(G.exec)); G.exec = nullptr; }
    hipStream_t saved = g_stream;
    g_stream = cap;
    hipGraph_t graph = nullptr;
    HIPX(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
      sweep_once(batch_of(s), dbeta);   // records the launches; advances beta on the host
    } catch (...) {
      (void)hipStreamEndCapture(cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      g_stream = saved;
      throw;
    }
    g_stream = saved;
    HIPX(hipStreamEndCapture(cap, &graph));
    const hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      G.exec = nullptr;
      throw Error(TT_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    G.dbeta = dbeta;
    G.flops = s.flops; G.flops_heff = s.flops_heff; G.bytes_min = s.bytes_min; G.n_applies = s.n_applies;
    G.n_exps = s.n_exps;
  } else {
    s.beta += dbeta;
    s.sweeps++;
    s.flops = G.flops; s.flops_heff = G.flops_heff; s.bytes_min = G.bytes_min; s.n_applies = G.n_applies;
    s.n_exps = G.n_exps;
  }
  HIPX(hipGraphLaunch(G.exec, g_stream));
}

int tdvp_sweep(tt_state* s, double dbeta, tt_sweep_stats* stats) {
  ABI_BEGIN
  TT_REQUIRE(s, TT_EINVAL, "null state");
  TT_REQUIRE(std::isfinite(dbeta), TT_EINVAL, "dbeta must be finite");
  TT_REQUIRE(s->one_site_ok, TT_EINVAL, "a bond sector exceeds what its neighbours reach: run tdvp_sweep2 first");
  reset_counters(*s);
  g_phase_on = g_phase && stats;
  struct PhaseOff { ~PhaseOff() { g_phase_on = false; } } phase_off;
  const long long l0 = launch_count();
  long long launches = 0;
  auto t0 = std::chrono::steady_clock::now();
  if (g_graphs && !prof_enabled() && !g_phase_on) {
    const bool replay = s->sg.exec && s->sg.dbeta == dbeta;
    sweep_graph(*s, dbeta);
    launches = replay ? s->sg.n_launches : launch_count() - l0;
    if (!replay) s->sg.n_launches = launches;
  } else {
    sweep_once(batch_of(*s), dbeta);
    launches = launch_count() - l0;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    HIPX(hipStreamSynchronize(ST()));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(*s, stats, secs);
    fill_phases(stats);
    stats->n_launches = launches;
  }
  ABI_END
}

int tdvp_sweep_batch(tt_state** states, int n, double dbeta, tt_sweep_stats* stats) {
  ABI_BEGIN
  TT_REQUIRE(states && n >= 1, TT_EINVAL, "need at least one state");
  for (int i = 0; i < n; ++i) TT_REQUIRE(states[i], TT_EINVAL, "null state in batch");
  for (int i = 0; i < n; ++i)
    TT_REQUIRE(states[i]->one_site_ok, TT_EINVAL, "a bond sector exceeds what its neighbours reach: run tdvp_sweep2 first");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) TT_REQUIRE(states[i] != states[j], TT_EINVAL, "a state appears twice in the batch");
  g_phase_on = g_phase && stats;
  struct PhaseOff { ~PhaseOff() { g_phase_on = false; } } phase_off;
  const long long l0 = launch_count();
  auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < n; ++i) reset_counters(*states[i]);
  // consecutive states with identical plans run together, up to kMaxBatch per launch
  int i = 0;
  while (i < n) {
    Batch b = batch_of(*states[i]);
    int j = i + 1;
    while (j < n && b.n < kMaxBatch && same_plans(*states[i], *states[j])) b.s[b.n++] = states[j++];
    sweep_once(b, dbeta);
    i = j;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    HIPX(hipStreamSynchronize(ST()));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n; ++i) fill_stats(*states[i], stats, i == 0 ? secs : 0.0);
    fill_phases(stats);
    stats->n_launches = launch_count() - l0;
  }
  ABI_END
}

int tdvp_sweep2(tt_state* s, double dbeta, int D_max, double cutoff, tt_sweep_stats* stats) {
  ABI_BEGIN
  TT_REQUIRE(s, TT_EINVAL, "null state");
  TT_REQUIRE(std::isfinite(dbeta), TT_EINVAL, "dbeta must be finite");
  TT_REQUIRE(D_max >= 1, TT_EINVAL, "D_max must be positive");
  TT_REQUIRE(std::isfinite(cutoff) && cutoff >= 0.0, TT_EINVAL, "cutoff must be finite and >= 0");
  TT_REQUIRE(s->opts.precision == TT_FP64, TT_EINVAL, "tdvp_sweep2 runs on FP64 states only");
  TT_REQUIRE(s->N >= 2, TT_EINVAL, "tdvp_sweep2 needs at least two sites");
  reset_counters(*s);
  g_phase_on = g_phase && stats;
  struct PhaseOff { ~PhaseOff() { g_phase_on = false; } } phase_off;
  const long long l0 = launch_count();
  auto t0 = std::chrono::steady_clock::now();
  const double disc = tdvp2_once(*s, dbeta, D_max, cutoff);
  rebuild_plans(*s);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    HIPX(hipStreamSynchronize(ST()));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(*s, stats, secs);
    fill_phases(stats);
    stats->n_launches = launch_count() - l0;
    stats->discarded = disc;
  }
  TT_REQUIRE(s->one_site_ok, TT_ENUMERIC,
             "tdvp_sweep2: a truncated bond sector exceeds what its neighbours reach; tdvp_sweep refuses this "
             "state until a further tdvp_sweep2");
  ABI_END
}

int tt_tune_apply(tt_state* s, int mode, int* host_forms) {
  ABI_BEGIN
  TT_REQUIRE(s, TT_EINVAL, "null state");
  TT_REQUIRE(mode >= 0 && mode <= 4, TT_EINVAL, "tt_tune_apply: mode must be 0, 1, 2, 3 or 4");
  const int N = s->N;
  const bool fz_ok = s->opts.precision == TT_FP64;   // the fused kernel multiplies and stores in FP64
  TT_REQUIRE(mode != 4 || fz_ok, TT_EINVAL, "tt_tune_apply: the fused applies need an FP64 state");
  if (mode < 2 || mode == 4) {
    s->fold.assign(N, (char)(mode == 4 ? 2 : mode));
    s->bfz.assign(N, (char)(mode == 4 ? 1 : 0));
    s->lw_site = -1;
  } else if (mode == 3) {
    TT_REQUIRE(host_forms, TT_EINVAL, "tt_tune_apply: mode 3 needs the forms");
    for (int k = 0; k < N; ++k) {
      const int f = host_forms[k] & 3, bf = host_forms[k] >> 2;
      TT_REQUIRE(host_forms[k] >= 0 && f <= 2 && bf <= 1 && (fz_ok || (f < 2 && bf == 0)), TT_EINVAL,
                 "tt_tune_apply: forms must be f + 4 b with f in 0..2 and b in 0..1 (f = 2, b = 1: FP64 states)");
    }
    for (int k = 0; k < N; ++k) {
      s->fold[k] = (char)(host_forms[k] & 3);
      s->bfz[k] = (char)(host_forms[k] >> 2);
    }
    s->lw_site = -1;
  } else {
    // time every form of each site's apply on the device (the site tensor as
    // input, the scratch vector as output; the state is not changed); the
    // fold's one-off build (forms 1 and 2) is spread over the 2K + 1 uses it
    // has per sweep.  Then both forms of the left bond's H^(0) apply (the
    // bond scratch matrix as input).
    const int reps = 3;
    const Batch b = batch_of(*s);
    hipEvent_t ev[11];
    for (auto& e : ev) HIPX(hipEventCreate(&e));
    struct Ev { hipEvent_t* e; ~Ev() { for (int i = 0; i < 11; ++i) (void)hipEventDestroy(e[i]); } } guard{ev};
    const double uses = 2.0 * s->opts.krylov_dim + 1.0;
    const double f0 = s->flops, fh0 = s->flops_heff, bm0 = s->bytes_min;
    const int na0 = s->n_applies;
    for (int k = 0; k < N; ++k) {
      BPtr<double> x = one(s->A[k]), y = one(s->wv);
      s->fold[k] = 0;
      apply_heff1(b, k, x, y);   // warm
      HIPX(hipEventRecord(ev[0], ST()));
      for (int r = 0; r < reps; ++r) apply_heff1(b, k, x, y);
      HIPX(hipEventRecord(ev[1], ST()));
      s->fold[k] = 1;
      s->lw_site = -1;
      build_lw(b, k);
      HIPX(hipEventRecord(ev[2], ST()));
      apply_heff1(b, k, x, y);   // warm
      HIPX(hipEventRecord(ev[3], ST()));
      for (int r = 0; r < reps; ++r) apply_heff1(b, k, x, y);
      HIPX(hipEventRecord(ev[4], ST()));
      BPtr<double> sx = one(s->Sbuf);
      if (fz_ok) {
        s->fold[k] = 2;
        apply_heff1(b, k, x, y);   // warm
        HIPX(hipEventRecord(ev[5], ST()));
        for (int r = 0; r < reps; ++r) apply_heff1(b, k, x, y);
        HIPX(hipEventRecord(ev[6], ST()));
        s->bfz[k] = 0;
        apply_heff0(b, k, sx, y);   // warm
        HIPX(hipEventRecord(ev[7], ST()));
        for (int r = 0; r < reps; ++r) apply_heff0(b, k, sx, y);
        HIPX(hipEventRecord(ev[8], ST()));
        s->bfz[k] = 1;
        apply_heff0(b, k, sx, y);   // warm
        HIPX(hipEventRecord(ev[9], ST()));
        for (int r = 0; r < reps; ++r) apply_heff0(b, k, sx, y);
      }
      HIPX(hipEventRecord(ev[10], ST()));
      HIPX(hipEventSynchronize(ev[10]));
      float t0 = 0.f, tb = 0.f, t1 = 0.f, t2 = 0.f, tg = 0.f, tz = 0.f;
      HIPX(hipEventElapsedTime(&t0, ev[0], ev[1]));
      HIPX(hipEventElapsedTime(&tb, ev[1], ev[2]));
      HIPX(hipEventElapsedTime(&t1, ev[3], ev[4]));
      if (fz_ok) {
        HIPX(hipEventElapsedTime(&t2, ev[5], ev[6]));
        HIPX(hipEventElapsedTime(&tg, ev[7], ev[8]));
        HIPX(hipEventElapsedTime(&tz, ev[9], ev[10]));
      }
      const double c0 = t0 / reps, c1 = t1 / reps + tb / uses, c2 = fz_ok ? t2 / reps + tb / uses : 1e30;
      s->fold[k] = (c2 <= c1 && c2 <= c0) ? 2 : (c1 < c0 ? 1 : 0);
      s->bfz[k] = (fz_ok && tz < tg) ? 1 : 0;
    }
    s->lw_site = -1;
    s->flops = f0; s->flops_heff = fh0; s->bytes_min = bm0; s->n_applies = na0;
  }
  if (s->sg.exec) {   // a captured sweep holds the old forms
    HIPX(hipGraphExecDestroy(s->sg.exec));
    s->sg.exec = nullptr;
  }
  if (host_forms && mode != 3)
    for (int k = 0; k < N; ++k) host_forms[k] = s->fold[k] + 4 * s->bfz[k];
  ABI_END
}

int thermo_observables(tt_state* s, tt_observables* o) {
  ABI_BEGIN
  TT_REQUIRE(s && o, TT_EINVAL, "null argument");
  const long long n = s->site[0].size;
  const Batch b = batch_of(*s);
  apply_heff1(b, 0, one(s->A[0]), one(s->wv));
  double* ob = s->obs_ptr();
  launch_mdot(one<const double>(s->A[0]), n, 1, one<const double>(s->wv), n, 0, one(s->part), 1, ST());
  launch_dot_final(s->part, kRedBlocks, 1, ob, ST());
  launch_mdot(BPtr<const double>{}, 0, 0, one<const double>(s->A[0]), n, 1, one(s->part), 1, ST());
  launch_dot_final(s->part, kRedBlocks, 1, ob + 1, ST());
  launch_trace(s->d_trace, s->d_trace_start, s->N, s->d_sites, s->vtr, s->max_bond, ob + 2, ST());
  // <<rho|P|rho>>: transfer matrices on the (q, -q) blocks, E_0 = 1
  double* Ein = s->Ea;
  double* Eout = s->Eb;
  launch_fill(Ein, 1.0, 1, ST());
  for (int k = 0; k < s->N; ++k) {
    launch_gemm(s->swp1[k], s->tabs.dev, one(Slots{{Ein, s->A[k], s->Xs, nullptr}}), 1, TT_FP64, one(s->pws), ST());
    launch_gemm(s->swp2[k], s->tabs.dev, one(Slots{{s->A[k], s->Xs, Eout, nullptr}}), 1, TT_FP64, one(s->pws), ST());
    std::swap(Ein, Eout);
  }
  double swap_ov = 0.0;
  double h[4], lam;
  HIPX(hipMemcpyAsync(h, ob, 32, hipMemcpyDeviceToHost, ST()));
  HIPX(hipMemcpyAsync(&lam, s->lam_ptr(), 8, hipMemcpyDeviceToHost, ST()));
  HIPX(hipMemcpyAsync(&swap_ov, Ein, 8, hipMemcpyDeviceToHost, ST()));
  HIPX(hipStreamSynchronize(ST()));
  o->beta = s->beta;
  o->beta_phys = 2.0 * s->beta;
  o->lambda = lam;
  o->lnZ = 2.0 * lam;
  o->n_sites = s->N;
  o->f = -o->lnZ / (s->N * o->beta_phys);
  o->E = h[0] / h[1];
  o->e = o->E / s->N;
  o->lnZ_single = lam + h[2];
  // the right-canonical sites have unit norm: <<rho|rho>> = ||A_0||^2
  o->herm_defect = std::sqrt(std::max(0.0, 2.0 - 2.0 * swap_ov / h[1]));
  TT_REQUIRE(std::isfinite(o->lnZ) && std::isfinite(o->E), TT_ENUMERIC, "non-finite observables");
  ABI_END
}

int thermo_local_observables(tt_state* s, double* host_out2) {
  ABI_BEGIN
  TT_REQUIRE(s && host_out2, TT_EINVAL, "null argument");
  const double n = local_expectation(*s, 0) / s->N;
  const double docc = local_expectation(*s, 1) / s->N;
  TT_REQUIRE(std::isfinite(n) && std::isfinite(docc), TT_ENUMERIC, "non-finite observables");
  host_out2[0] = n;
  host_out2[1] = docc;
  ABI_END
}

int thermo_spin_correlation(tt_state* s, int d2, double* host_F, int* host_npairs) {
  ABI_BEGIN
  TT_REQUIRE(s && host_F, TT_EINVAL, "null argument");
  TT_REQUIRE(d2 >= 1, TT_EINVAL, "thermo_spin_correlation: d2 must be positive");
  const auto pairs = pairs_at_distance(s->lat, d2);
  TT_REQUIRE(!pairs.empty(), TT_EINVAL, "thermo_spin_correlation: no pair of sites at that distance");
  const int key = kObsSpinPairs + d2;
  auto it = s->obs.find(key);
  tt_state::ObsMpo& O = it != s->obs.end() ? it->second : build_obs_mpo(*s, key, make_spin_pair_mpo(s->N, pairs));
  const double F = obs_expectation(*s, O) / (double)pairs.size();
  TT_REQUIRE(std::isfinite(F), TT_ENUMERIC, "non-finite spin correlation");
  *host_F = F;
  if (host_npairs) *host_npairs = (int)pairs.size();
  ABI_END
}

int thermo_green_function(tt_state* s, double kx, double ky, double* host_G) {
  ABI_BEGIN
  TT_REQUIRE(s && host_G, TT_EINVAL, "null argument");
  TT_REQUIRE(std::isfinite(kx) && std::isfinite(ky), TT_EINVAL, "thermo_green_function: non-finite momentum");
  const double G = green_expectation(*s, kx, ky);
  TT_REQUIRE(std::isfinite(G), TT_ENUMERIC, "non-finite Green's function");
  *host_G = G;
  ABI_END
}

int thermo_pairing_order(tt_state* s, double* host_delta, int* host_nbonds) {
  ABI_BEGIN
  TT_REQUIRE(s && host_delta, TT_EINVAL, "null argument");
  TT_REQUIRE(s->opts.symmetry != 1, TT_EINVAL, "thermo_pairing_order: needs a state with symmetry = 0 or 2");
  const auto bonds = pairing_bonds(s->lat);
  TT_REQUIRE(!bonds.empty(), TT_EINVAL, "thermo_pairing_order: no bonds");
  auto it = s->obs.find(kObsPairing);
  // H - hp Delta_tot with t = U = mu = 0 and hp = -1 is Delta_tot itself
  tt_state::ObsMpo& O =
      it != s->obs.end() ? it->second : build_obs_mpo(*s, kObsPairing, make_hubbard_mpo(s->lat, 0.0, 0.0, 0.0, 0.0, -1.0));
  const double d = obs_expectation(*s, O) / (double)bonds.size();
  TT_REQUIRE(std::isfinite(d), TT_ENUMERIC, "non-finite pairing order");
  *host_delta = d;
  if (host_nbonds) *host_nbonds = (int)bonds.size();
  ABI_END
}

void tt_state_free(tt_state* s) {
  if (!s) return;
  (void)hipStreamSynchronize(ST());
  delete s;
}

int tt_state_info(const tt_state* s, int* n_sites, int* dims) {
  ABI_BEGIN
  TT_REQUIRE(s && n_sites, TT_EINVAL, "null argument");
  *n_sites = s->N;
  if (dims)
    for (int k = 0; k <= s->N; ++k) dims[k] = (int)s->bonds[k].total;
  ABI_END
}

int tt_state_bond_sectors(const tt_state* s, int k, int* nsec, int* qu, int* qd, int* dim) {
  ABI_BEGIN
  TT_REQUIRE(s && nsec, TT_EINVAL, "null argument");
  TT_REQUIRE(k >= 0 && k <= s->N, TT_EINVAL, "bond index out of range");
  const Bond& b = s->bonds[k];
  int ns = (int)b.secs.size();
  if (qu || qd || dim) {
    TT_REQUIRE(*nsec >= ns, TT_EINVAL, "sector arrays too small");
    for (int i = 0; i < ns; ++i) {
      if (qu) qu[i] = b.secs[i].q.first;
      if (qd) qd[i] = b.secs[i].q.second;
      if (dim) dim[i] = b.secs[i].dim;
    }
  }
  *nsec = ns;
  ABI_END
}

static void site_dense_map(const tt_state* s, int k, const std::function<void(long long, long long)>& f) {
  const SiteLayout& S = s->site[k];
  const Bond& bl = s->bonds[k];
  const Bond& br = s->bonds[k + 1];
  const long long Dr = br.total;
  for (int l = 0; l < S.nl; ++l)
    for (int g = 0; g < s->G.ng; ++g) {
      int r = S.rsec[l][g];
      if (r < 0) continue;
      int ns = (int)s->G.s[g].size();
      for (int x = 0; x < S.dl[l]; ++x)
        for (int si = 0; si < ns; ++si)
          for (int y = 0; y < br.secs[r].dim; ++y) {
            long long src = S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)si * br.secs[r].dim + y;
            long long dst = ((bl.secs[l].off + x) * 16 + s->G.s[g][si]) * Dr + br.secs[r].off + y;
            f(src, dst);
          }
    }
}

int tt_state_export_site(const tt_state* s, int k, double* host) {
  ABI_BEGIN
  TT_REQUIRE(s && host, TT_EINVAL, "null argument");
  TT_REQUIRE(k >= 0 && k < s->N, TT_EINVAL, "site index out of range");
  std::vector<double> packed(s->site[k].size);
  HIPX(hipMemcpyAsync(packed.data(), s->A[k], 8 * packed.size(), hipMemcpyDeviceToHost, ST()));
  HIPX(hipStreamSynchronize(ST()));
  long long tot = s->bonds[k].total * 16 * s->bonds[k + 1].total;
  std::memset(host, 0, 8 * tot);
  site_dense_map(s, k, [&](long long src, long long dst) { host[dst] = packed[src]; });
  ABI_END
}

int tt_state_import_site(tt_state* s, int k, const double* host) {
  ABI_BEGIN
  TT_REQUIRE(s && host, TT_EINVAL, "null argument");
  TT_REQUIRE(k >= 0 && k < s->N, TT_EINVAL, "site index out of range");
  std::vector<double> packed(s->site[k].size);
  bool finite = true;
  site_dense_map(s, k, [&](long long src, long long dst) {
    packed[src] = host[dst];
    finite = finite && std::isfinite(host[dst]);
  });
  TT_REQUIRE(finite, TT_ENUMERIC, "imported tensor holds NaN or Inf");
  HIPX(hipMemcpyAsync(s->A[k], packed.data(), 8 * packed.size(), hipMemcpyHostToDevice, ST()));
  HIPX(hipStreamSynchronize(ST()));
  ABI_END
}

static const char kMagic[8] = {'T', 'A', 'N', 'T', 'R', 'G', '0', '1'};

int tt_state_save(const tt_state* s, const char* path) {
  ABI_BEGIN
  TT_REQUIRE(s && path, TT_EINVAL, "null argument");
  FILE* f = std::fopen(path, "wb");
  TT_REQUIRE(f, TT_EIO, std::string("cannot open ") + path);
  std::unique_ptr<FILE, int (*)(FILE*)> guard(f, std::fclose);
  double lam = 0.0;
  HIPX(hipMemcpyAsync(&lam, const_cast<tt_state*>(s)->lam_ptr(), 8, hipMemcpyDeviceToHost, ST()));
  HIPX(hipStreamSynchronize(ST()));
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8;
  ok = ok && std::fwrite(&s->model, sizeof(tt_model), 1, f) == 1;
  ok = ok && std::fwrite(&s->opts, sizeof(tt_options), 1, f) == 1;
  ok = ok && std::fwrite(&s->beta, 8, 1, f) == 1;
  ok = ok && std::fwrite(&lam, 8, 1, f) == 1;
  ok = ok && std::fwrite(&s->sweeps, 8, 1, f) == 1;
  for (int k = 0; k <= s->N && ok; ++k) {
    int ns = (int)s->bonds[k].secs.size();
    ok = std::fwrite(&ns, 4, 1, f) == 1;
    for (auto& sec : s->bonds[k].secs) {
      int v[3] = {sec.q.first, sec.q.second, sec.dim};
      ok = ok && std::fwrite(v, 4, 3, f) == 3;
    }
  }
  for (int k = 0; k < s->N && ok; ++k) {
    std::vector<double> packed(s->site[k].size);
    HIPX(hipMemcpyAsync(packed.data(), s->A[k], 8 * packed.size(), hipMemcpyDeviceToHost, ST()));
    HIPX(hipStreamSynchronize(ST()));
    long long n = (long long)packed.size();
    ok = std::fwrite(&n, 8, 1, f) == 1 && std::fwrite(packed.data(), 8, n, f) == (size_t)n;
  }
  TT_REQUIRE(ok, TT_EIO, "write failed");
  ABI_END
}

int tt_state_load(const char* path, tt_state** out) {
  ABI_BEGIN
  TT_REQUIRE(path && out, TT_EINVAL, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  TT_REQUIRE(f, TT_EIO, std::string("cannot open ") + path);
  std::unique_ptr<FILE, int (*)(FILE*)> guard(f, std::fclose);
  char magic[8];
  tt_model m;
  tt_options o;
  double beta, lam;
  long long sweeps;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0;
  TT_REQUIRE(ok, TT_EIO, "not a saved tanTRG state");
  ok = std::fread(&m, sizeof(m), 1, f) == 1 && std::fread(&o, sizeof(o), 1, f) == 1 &&
       std::fread(&beta, 8, 1, f) == 1 && std::fread(&lam, 8, 1, f) == 1 && std::fread(&sweeps, 8, 1, f) == 1;
  TT_REQUIRE(ok, TT_EIO, "truncated state file");
  validate(m, o);
  check_device();
  auto s = std::make_unique<tt_state>();
  s->model = m;
  s->opts = o;
  s->lat = make_lattice(m.W, m.L, m.geometry);
  s->N = s->lat.N;
  s->mpo = make_hubbard_mpo(s->lat, m.t, m.tp, m.U, m.mu, m.hp);
  s->G = make_groups(o.symmetry);
  std::vector<std::map<Q, int>> dims(s->N + 1);
  for (int k = 0; k <= s->N; ++k) {
    int ns = 0;
    TT_REQUIRE(std::fread(&ns, 4, 1, f) == 1 && ns >= 1 && ns < 1000000, TT_EIO, "bad sector table");
    for (int i = 0; i < ns; ++i) {
      int v[3];
      TT_REQUIRE(std::fread(v, 4, 3, f) == 3 && v[2] >= 1, TT_EIO, "bad sector table");
      dims[k][{v[0], v[1]}] = v[2];
    }
  }
  build_layouts(*s, dims);
  require_sweep_plans(*s);
  alloc_state(*s);
  for (int k = 0; k < s->N; ++k) {
    long long n = 0;
    TT_REQUIRE(std::fread(&n, 8, 1, f) == 1 && n == s->site[k].size, TT_EIO, "site size mismatch");
    std::vector<double> packed(n);
    TT_REQUIRE(std::fread(packed.data(), 8, n, f) == (size_t)n, TT_EIO, "truncated site data");
    HIPX(hipMemcpyAsync(s->A[k], packed.data(), 8 * n, hipMemcpyHostToDevice, ST()));
  }
  HIPX(hipMemcpyAsync(s->lam_ptr(), &lam, 8, hipMemcpyHostToDevice, ST()));
  set_unit_env(s->Lenv[0], ST());
  s->lw_site = -1;
  set_unit_env(s->Renv[s->N], ST());
  for (int k = s->N - 1; k >= 1; --k) env_right(batch_of(*s), k);
  s->beta = beta;
  s->sweeps = sweeps;
  HIPX(hipStreamSynchronize(ST()));
  *out = s.release();
  ABI_END
}

int tt_heff_apply(int Dl, int Dr, int DH, const double* L, const double* W, const double* A, const double* R,
                  double* out, int precision, void* stream) {
  ABI_BEGIN
  TT_REQUIRE(Dl >= 1 && Dr >= 1 && DH >= 1, TT_EINVAL, "dimensions must be positive");
  TT_REQUIRE(L && W && A && R && out, TT_EINVAL, "null device pointer");
  TT_REQUIRE(precision >= TT_FP64 && precision <= TT_BF16X6, TT_EINVAL, "unknown precision");
  TT_REQUIRE((double)Dl * DH * 16 * Dr < 4.0e9, TT_EINVAL, "problem too large");
  hipStream_t saved = g_stream;
  if (stream) g_stream = (hipStream_t)stream;
  try {
    if (g_heff.Dl != Dl || g_heff.Dr != Dr || g_heff.DH != DH) build_heff_cache(Dl, Dr, DH);
    HeffCache& c = g_heff;
    hipStream_t st = ST();
    if (precision == TT_BF16X3 || precision == TT_BF16X6) {
      // split-BF16: every operand split once into BF16 planes (the split of L
      // and A counted with L.A, of W with the W stage, of R with .R), rows
      // contiguous in the contracted index and zero-padded to the GEMM's K
      // tile; the intermediates written as planes by the launches that
      // produce them.  Layouts (element offsets inside one plane):
      //   Lp[(x', a)][kp1]  = L[x'][a][x]          At[(s, y)][kp1] = A[x][s][y]
      //   T1[a][x'][s][y]   (the layout of the FP64 path)
      //   T2[(x', s)][kp3]  = T2[x'][s][b][y]      Rp[y'][kp3]     = R[y'][b][y]
      const int np = precision == TT_BF16X3 ? 2 : 3;
      const long long M1 = (long long)Dl * DH, N1 = 16LL * Dr, K3 = (long long)DH * Dr;
      auto pl = [](long long n) { return (n + 127) / 128 * 128; };   // plane strides: 256-byte multiples
      const long long sL = pl(M1 * c.kp1), sA = pl(N1 * c.kp1), sW = pl((long long)DH * 16 * DH),
                      sR = pl((long long)Dr * c.kp3), sT1 = pl(c.t1), sT2 = pl(16LL * Dl * c.kp3);
      const long long need = 2LL * np * (sL + sA + sW + sR + sT1 + sT2);
      if (need > c.plane_bytes) {
        dfree(c.planes);
        c.planes = nullptr;
        c.planes = dalloc(need);
        c.plane_bytes = need;
      }
      char* base = static_cast<char*>(c.planes);
      long long off = 0;
      auto carve = [&](long long n) { __bf16* q = reinterpret_cast<__bf16*>(base + off); off += 2LL * np * n; return q; };
      __bf16 *Lp = carve(sL), *Ap = carve(sA), *Wp = carve(sW), *Rp = carve(sR), *T1p = carve(sT1), *T2p = carve(sT2);
      HIPX(hipEventRecord(c.ev[0], st));
      launch_split_rows(L, M1, Dl, Dl, Lp, c.kp1, sL, precision, st);
      launch_split_t(A, Dl, (int)N1, Ap, c.kp1, sA, precision, st);
      BgArgs g1{};
      g1.A = Lp; g1.lda = c.kp1; g1.sa = sL;
      g1.B = Ap; g1.ldb = c.kp1; g1.sb = sA;
      g1.M = (int)M1; g1.N = (int)N1; g1.K = c.kp1;
      g1.C = T1p; g1.cdiv = DH; g1.ldc0 = (long long)Dl * N1; g1.ldc1 = N1; g1.sc = sT1; g1.cplanes = 1;
      launch_bgemm(g1, precision, st);
      HIPX(hipEventRecord(c.ev[1], st));
      if (DH <= wstage_planes_max_dh()) {   // FP32 vector kernel, bound by the planes' traffic
        launch_wstage_planes(T1p, sT1, W, DH, Dl, Dr, T2p, sT2, c.kp3, precision, st);
      } else {   // grouped GEMMs on W split into planes; T2's K padding cleared first
        launch_fill(reinterpret_cast<double*>(T2p), 0.0, (2LL * np * sT2) / 8, st);
        launch_split(W, (long long)DH * 16 * DH, Wp, sW, precision, st);
        Planes p2;
        p2.s[0] = sW; p2.s[1] = sT1; p2.s[2] = sT2; p2.c = 1;
        launch_gemm_planes(c.wgq, c.tabs.dev, Slots{{(double*)Wp, (double*)T1p, (double*)T2p, nullptr}}, p2,
                           precision, st);
      }
      HIPX(hipEventRecord(c.ev[2], st));
      launch_split_rows(R, Dr, (int)K3, K3, Rp, c.kp3, sR, precision, st);
      BgArgs g3{};
      g3.A = T2p; g3.lda = c.kp3; g3.sa = sT2;
      g3.B = Rp; g3.ldb = c.kp3; g3.sb = sR;
      g3.M = 16 * Dl; g3.N = Dr; g3.K = c.kp3;
      g3.C = out; g3.cdiv = 16 * Dl; g3.ldc0 = Dr; g3.ldc1 = 0; g3.sc = 0; g3.cplanes = 0;
      launch_bgemm(g3, precision, st);
      HIPX(hipEventRecord(c.ev[3], st));
    } else if ((precision == TT_FP64 || precision == TT_FP32) && dense_f64_applies(DH)) {
      const DenseF64Sizes z = dense_f64_sizes(Dl, Dr, DH);
      const long long need = z.lq + z.aq + z.rq + z.t2q + 4 * 32;
      if (need > c.f64_doubles) {
        dfree(c.f64);
        c.f64 = nullptr;
        c.f64 = (double*)dalloc(8 * need);
        c.f64_doubles = need;
      }
      auto al = [](long long n) { return (n + 31) / 32 * 32; };   // 256-byte aligned pieces
      DenseF64Bufs b{c.f64, c.f64 + al(z.lq), c.f64 + al(z.lq) + al(z.aq), c.T1,
                     c.f64 + al(z.lq) + al(z.aq) + al(z.rq)};
      if (precision == TT_FP64) {
        dense_apply_f64(Dl, Dr, DH, L, W, A, R, out, b, z, c.ev, st);
      } else {
        DenseF32Bufs f{(float*)b.Lq, (float*)b.Aq, (float*)b.Rq, (float*)b.T1, (float*)b.T2q};
        dense_apply_f32(Dl, Dr, DH, L, W, A, R, out, f, c.ev, st);
      }
    } else {
      HIPX(hipEventRecord(c.ev[0], st));
      launch_gemm(c.plan.s1, c.tabs.dev, one(Slots{{const_cast<double*>(L), const_cast<double*>(A), c.T1, nullptr}}), 1,
                  precision, one(c.pws), st);
      HIPX(hipEventRecord(c.ev[1], st));
      launch_gemm(c.wg, c.tabs.dev, one(Slots{{const_cast<double*>(W), c.T1, c.T2, nullptr}}), 1, precision, one(c.pws),
                  st);
      HIPX(hipEventRecord(c.ev[2], st));
      launch_gemm(c.plan.s3, c.tabs.dev, one(Slots{{c.T2, const_cast<double*>(R), out, nullptr}}), 1, precision,
                  one(c.pws), st);
      HIPX(hipEventRecord(c.ev[3], st));
    }
    c.timed = true;
  } catch (...) {
    g_stream = saved;
    throw;
  }
  g_stream = saved;
  ABI_END
}

int tt_heff_apply_noalloc(int Dl, int Dr, int DH, const double* L, const double* W, const double* A,
                          const double* R, double* out, int precision, void* stream) {
  ABI_BEGIN
  TT_REQUIRE(Dl >= 1 && Dr >= 1 && DH >= 1, TT_EINVAL, "dimensions must be positive");
  TT_REQUIRE(L && W && A && R && out, TT_EINVAL, "null device pointer");
  TT_REQUIRE(precision >= TT_FP64 && precision <= TT_BF16X6, TT_EINVAL, "unknown precision");
  TT_REQUIRE(!prof_enabled(), TT_EINVAL, "tt_heff_apply_noalloc: kernel profiling (which creates events) is on");
  // T1 and T2 alone take 16 Dl DH 16 Dr bytes: refuse what cannot fit before planning
  TT_REQUIRE(16.0 * Dl * DH * 16.0 * Dr <= (double)kScratchBytes, TT_EINVAL,
             "tt_heff_apply_noalloc: the intermediates need " + std::to_string(16.0 * Dl * DH * 16.0 * Dr) +
                 " bytes, more than the " + std::to_string(kScratchBytes) + "-byte scratch");
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  TT_REQUIRE(dev >= 0 && dev < kMaxDevices, TT_EDEVICE, "device index out of range");
  NoAllocDev& d = g_noalloc[dev];
  hipStream_t st = stream ? (hipStream_t)stream : ST();
  if (!d.base) {   // once per device, with that device current
    void* p = nullptr;
    HIPX(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    d.base = static_cast<char*>(p);
  }
  if (d.Dl != Dl || d.Dr != Dr || d.DH != DH) {
    d.Dl = d.Dr = d.DH = -1;
    d.host = heff_plans(Dl, Dr, DH);
    d.Dl_pending = Dl; d.Dr_pending = Dr; d.DH_pending = DH;
    const long long need = noalloc_layout(d, false, st);
    TT_REQUIRE(need <= kScratchBytes, TT_EINVAL,
               "tt_heff_apply_noalloc: the apply needs " + std::to_string(need) + " bytes of scratch, more than " +
                   std::to_string(kScratchBytes));
    noalloc_layout(d, true, st);
    d.Dl = Dl; d.Dr = Dr; d.DH = DH;
  }
  double* l = const_cast<double*>(L);
  double* w = const_cast<double*>(W);
  double* a = const_cast<double*>(A);
  double* r = const_cast<double*>(R);
  if (precision == TT_FP64 && dense_f64_applies(DH)) {   // the kernels of tt_heff_apply's FP64 path
    DenseF64Bufs b{d.Lq, d.Aq, d.Rq, d.T1, d.T2};
    dense_apply_f64(Dl, Dr, DH, L, W, A, R, out, b, dense_f64_sizes(Dl, Dr, DH), nullptr, st);
    return TT_OK;
  }
  if (precision == TT_FP32 && dense_f64_applies(DH)) {   // and of its FP32 path, in the same pieces
    DenseF32Bufs f{(float*)d.Lq, (float*)d.Aq, (float*)d.Rq, (float*)d.T1, (float*)d.T2};
    dense_apply_f32(Dl, Dr, DH, L, W, A, R, out, f, nullptr, st);
    return TT_OK;
  }
  launch_gemm(d.s1, d.tabs, one(Slots{{l, a, d.T1, nullptr}}), 1, precision, one(d.pws), st);
  launch_gemm(d.wg, d.tabs, one(Slots{{w, d.T1, d.T2, nullptr}}), 1, precision, one(d.pws), st);
  launch_gemm(d.s3, d.tabs, one(Slots{{d.T2, r, out, nullptr}}), 1, precision, one(d.pws), st);
  ABI_END
}

int tt_heff2_apply(int Dl, int Dr, int DH, const double* L, const double* W1, const double* W2, const double* C,
                   const double* R, double* out, int precision, void* stream) {
  ABI_BEGIN
  TT_REQUIRE(Dl >= 1 && Dr >= 1 && DH >= 1, TT_EINVAL, "dimensions must be positive");
  TT_REQUIRE(L && W1 && W2 && C && R && out, TT_EINVAL, "null device pointer");
  TT_REQUIRE(precision >= TT_FP64 && precision <= TT_BF16X6, TT_EINVAL, "unknown precision");
  TT_REQUIRE((double)Dl * DH * 256 * Dr < 4.0e9, TT_EINVAL, "problem too large");
  hipStream_t saved = g_stream;
  if (stream) g_stream = (hipStream_t)stream;
  try {
    if (g_heff2.Dl != Dl || g_heff2.Dr != Dr || g_heff2.DH != DH) build_heff2_cache(Dl, Dr, DH);
    Heff2Cache& c = g_heff2;
    hipStream_t st = ST();
    double* l = const_cast<double*>(L);
    double* w1 = const_cast<double*>(W1);
    double* w2 = const_cast<double*>(W2);
    double* a = const_cast<double*>(C);
    double* r = const_cast<double*>(R);
    launch_gemm(c.st[0], c.tabs.dev, one(Slots{{l, a, c.T1, nullptr}}), 1, precision, one(c.pws), st);
    launch_gemm(c.st[1], c.tabs.dev, one(Slots{{w1, c.T1, c.T2, nullptr}}), 1, precision, one(c.pws), st);
    launch_gemm(c.st[2], c.tabs.dev, one(Slots{{w2, c.T2, c.T1, nullptr}}), 1, precision, one(c.pws), st);
    launch_gemm(c.st[3], c.tabs.dev, one(Slots{{c.T1, r, out, nullptr}}), 1, precision, one(c.pws), st);
  } catch (...) {
    g_stream = saved;
    throw;
  }
  g_stream = saved;
  ABI_END
}

int tt_check_plans(const tt_model* model, const tt_options* opts, long long* violations, long long* work_doubles) {
  ABI_BEGIN
  TT_REQUIRE(model && opts && violations, TT_EINVAL, "null argument");
  auto s = make_host_state(*model, *opts);
  std::string rep;
  *violations = check_all_plans(*s, rep);
  if (work_doubles) {
    long long tot = 0;
    for (auto& l : s->site) tot += l.size;
    for (auto& e : s->env) tot += 2 * e.size;
    *work_doubles = tot;
  }
  if (*violations) g_err = rep;
  ABI_END
}

int tt_model_bond_sectors(const tt_model* model, const tt_options* opts, int k, int* nsec, int* qu, int* qd,
                          int* dim) {
  ABI_BEGIN
  TT_REQUIRE(model && opts && nsec, TT_EINVAL, "null argument");
  auto s = make_host_state(*model, *opts, false);
  return tt_state_bond_sectors(s.get(), k, nsec, qu, qd, dim);
  ABI_END
}

int tt_svd_lds_limit(long long max_doubles) {
  ABI_BEGIN
  TT_REQUIRE(max_doubles >= 0, TT_EINVAL, "tt_svd_lds_limit: negative size");
  g_svd_lds_limit = max_doubles;
  ABI_END
}

int tt_sweep_graphs(int on) {
  ABI_BEGIN
  g_graphs = on != 0;
  ABI_END
}

int tt_phase_timing(int on) {
  ABI_BEGIN
  g_phase = on != 0;
  ABI_END
}

int tt_profile_enable(int on) {
  ABI_BEGIN
  prof_enable(on != 0);
  ABI_END
}

int tt_profile_read(double* host_out72) {
  ABI_BEGIN
  static_assert(PROF_KINDS == 18, "tt_profile_read fills 18 kinds");
  TT_REQUIRE(host_out72, TT_EINVAL, "null argument");
  double out[PROF_KINDS][4];
  prof_read(out);
  for (int k = 0; k < PROF_KINDS; ++k)
    for (int j = 0; j < 4; ++j) host_out72[k * 4 + j] = out[k][j];
  ABI_END
}

// Entropy and specific heat per site from a series of bilayer observables
// (main text, Fig. 2(b); SM Fig. S1(c)): s = beta (e - f), C_e = -beta^2 de/dbeta
// with the slope of the quadratic through three neighbouring points (centred
// inside, one-sided at the ends; exact for quadratics).  Host arithmetic only.
int tt_thermo_derived(int n, const double* beta, const double* e, const double* f, double* c_out, double* s_out) {
  ABI_BEGIN
  TT_REQUIRE(n >= 3 && beta && e && f && c_out && s_out, TT_EINVAL, "tt_thermo_derived: need n >= 3 and non-null arrays");
  for (int i = 0; i < n; ++i) {
    TT_REQUIRE(std::isfinite(beta[i]) && std::isfinite(e[i]) && std::isfinite(f[i]), TT_EINVAL,
               "tt_thermo_derived: non-finite input");
    TT_REQUIRE(beta[i] > 0.0, TT_EINVAL, "tt_thermo_derived: beta must be positive");
    TT_REQUIRE(i == 0 || beta[i] > beta[i - 1], TT_EINVAL, "tt_thermo_derived: beta must increase strictly");
  }
  for (int i = 0; i < n; ++i) {
    const int a = i == 0 ? 0 : (i == n - 1 ? n - 3 : i - 1);   // nodes a, a+1, a+2
    double slope = 0.0;
    for (int p = 0; p < 3; ++p) {   // derivative of the Lagrange basis polynomial of node a+p at beta[i]
      const int k = a + p, q = a + (p + 1) % 3, r = a + (p + 2) % 3;
      slope += e[k] * ((beta[i] - beta[q]) + (beta[i] - beta[r])) / ((beta[k] - beta[q]) * (beta[k] - beta[r]));
    }
    c_out[i] = -beta[i] * beta[i] * slope;
    s_out[i] = beta[i] * (e[i] - f[i]);
  }
  ABI_END
}

int tt_heff_last_timing(double* ms4) {
  ABI_BEGIN
  TT_REQUIRE(ms4, TT_EINVAL, "null argument");
  TT_REQUIRE(g_heff.timed, TT_EINVAL, "no timed apply yet");
  HIPX(hipEventSynchronize(g_heff.ev[3]));
  float a, b, c, d;
  HIPX(hipEventElapsedTime(&a, g_heff.ev[0], g_heff.ev[1]));
  HIPX(hipEventElapsedTime(&b, g_heff.ev[1], g_heff.ev[2]));
  HIPX(hipEventElapsedTime(&c, g_heff.ev[2], g_heff.ev[3]));
  HIPX(hipEventElapsedTime(&d, g_heff.ev[0], g_heff.ev[3]));
  ms4[0] = a; ms4[1] = b; ms4[2] = c; ms4[3] = d;
  ABI_END
}

}  // extern "C"
