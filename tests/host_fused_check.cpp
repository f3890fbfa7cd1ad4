// Host-only check of the fused apply descriptors (FzPlan) of one site and of
// its left bond: a plain
// loop interpreter of their meaning,
//   out[x', y'] = sum_b sum_y (sum_t sum_x LW_t[x', x] x_t[x, y]) R[y', (b, y)],
// against the grouped GEMMs of the folded form (T2 = LW . x in passes, the
// cleared T2 blocks, then T2 . R^T) on random operands in their layouts; plus
// coverage: every element of the output site vector lies in exactly one
// output block, and the jobs tile every block's rows and columns exactly once
// (each tile as one unsplit job or as four parts of one workgroup).  No GPU
// code is involved.
//
// usage: host_fused_check W L geometry D sector_cap k   (prints one line, exit 0 on success)
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../paper_2212_11973_amd/csrc/plan.h"

using namespace tt;

// the tile planner in layout.cpp asks the kernels for LDS sizes; unused here
namespace tt { int gemm_smem_bytes(int) { return 0; } }

static std::mt19937_64 rng(4242);
static double rnd() { return std::uniform_real_distribution<double>(-1.0, 1.0)(rng); }

static long long at(long long tab, long long stride, int i, const std::vector<long long>& T) {
  return tab >= 0 ? T[tab + i] : (long long)i * stride;
}

static void run_gemm(const GemmPlan& p, const std::vector<long long>& T, std::vector<double>* slot[4]) {
  for (const GemmProb& g : p.probs)
    for (int m = 0; m < g.M; ++m)
      for (int n = 0; n < g.N; ++n) {
        double acc = 0.0;
        for (int k = 0; k < g.K; ++k)
          acc += slot[g.ia]->at(g.offA + at(g.tam, g.sam, m, T) + at(g.tak, g.sak, k, T)) *
                 slot[g.ib]->at(g.offB + at(g.tbk, g.sbk, k, T) + at(g.tbn, g.sbn, n, T));
        double& c = slot[g.ic]->at(g.offC + at(g.tcm, g.scm, m, T) + n);
        c = g.alpha * acc + (g.beta == 0.0 ? 0.0 : g.beta * c);
      }
}

static void run_w(const WPlan& p, const std::vector<double>& in, std::vector<double>& out) {
  for (const WTask& t : p.tasks)
    for (int i = 0; i < t.ni; ++i)
      for (int j = 0; j < t.nj; ++j) {
        double acc = 0.0;
        for (int q = t.t0; q < t.t0 + t.nt; ++q) {
          const WTerm& w = p.terms[q];
          acc += w.w * in.at(w.src + i * w.ssi + j * w.ssj);
        }
        out.at(t.dst + i * t.dsi + j * t.dsj) = acc;
      }
}

// out = the fused plan's result (every output block written from its b
// blocks and terms); returns the number of output elements not written
// exactly once
static long long fz_interpret(const FzPlan& F, const std::vector<double>& lw, const std::vector<double>& x,
                              const std::vector<double>& R, long long out_size, std::vector<double>& out) {
  out.assign(out_size, 0.0);
  std::vector<int> hits(out_size, 0);
  for (const FzOut& o : F.outs) {
    std::vector<double> acc((size_t)o.dp * o.dr, 0.0);
    for (int bi = 0; bi < o.nb; ++bi) {
      const FzB& b = F.bs.at(o.b0 + bi);
      std::vector<double> tb((size_t)o.dp * b.dc, 0.0);
      for (int ti = 0; ti < b.nt; ++ti) {
        const FzT& t = F.terms.at(b.t0 + ti);
        for (int i = 0; i < o.dp; ++i)
          for (int y = 0; y < b.dc; ++y) {
            double s = 0.0;
            for (int q = 0; q < t.dl; ++q) s += lw.at(t.lw + (long long)i * t.ldlw + q) * x.at(t.a + (long long)q * t.lda + y);
            tb[(size_t)i * b.dc + y] += s;
          }
      }
      for (int i = 0; i < o.dp; ++i)
        for (int yp = 0; yp < o.dr; ++yp) {
          double s = 0.0;
          for (int y = 0; y < b.dc; ++y) s += tb[(size_t)i * b.dc + y] * R.at(o.rrow + (long long)yp * o.ldr + b.rcol + y);
          acc[(size_t)i * o.dr + yp] += s;
        }
    }
    for (int i = 0; i < o.dp; ++i)
      for (int yp = 0; yp < o.dr; ++yp) {
        const long long e = o.out + (long long)i * o.ldo + yp;
        out.at(e) = acc[(size_t)i * o.dr + yp];
        hits.at(e)++;
      }
  }
  long long bad = 0;
  for (long long e = 0; e < out_size; ++e)
    if (hits[e] != 1) ++bad;
  return bad;
}

static double rel_err(const std::vector<double>& a, const std::vector<double>& b) {
  double e = 0.0, n = 0.0;
  for (size_t i = 0; i < a.size(); ++i) { e = std::max(e, std::fabs(a[i] - b[i])); n = std::max(n, std::fabs(b[i])); }
  return e / std::max(n, 1e-300);
}

// every (block, 16-row tile, kFzCols-column tile) exactly once, as one
// unsplit job or as the four parts of one workgroup
static long long check_jobs(const FzPlan& F) {
  std::map<std::array<int, 3>, int> seen;
  long long jbad = 0;
  if (F.jobs.size() % 4 || (long long)F.jobs.size() != 4LL * F.nblocks) ++jbad;
  for (size_t w = 0; w + 3 < F.jobs.size(); w += 4)
    for (int q = 0; q < 4; ++q) {
      const FzJob& j = F.jobs[w + q];
      if (j.o < 0) continue;
      if (j.nparts == 4 && j.part != q) ++jbad;
      if (j.nparts == 4 && (F.jobs[w].o != j.o || F.jobs[w].row0 != j.row0 || F.jobs[w].col0 != j.col0)) ++jbad;
      if (j.nparts == 1 || j.part == 0) seen[{j.o, j.row0, j.col0}]++;
    }
  long long tiles = 0;
  for (int oi = 0; oi < (int)F.outs.size(); ++oi)
    for (int r0 = 0; r0 < F.outs[oi].dp; r0 += 16)
      for (int c0 = 0; c0 < F.outs[oi].dr; c0 += kFzCols) {
        ++tiles;
        auto it = seen.find({oi, r0, c0});
        if (it == seen.end() || it->second != 1) ++jbad;
      }
  if ((long long)seen.size() != tiles) ++jbad;
  return jbad;
}

int main(int argc, char** argv) {
  if (argc < 7) { std::fprintf(stderr, "usage\n"); return 2; }
  const int W = std::atoi(argv[1]), Lx = std::atoi(argv[2]), geo = std::atoi(argv[3]);
  const int D = std::atoi(argv[4]), cap = std::atoi(argv[5]), k = std::atoi(argv[6]);
  Lattice lat = make_lattice(W, Lx, geo);
  const int N = lat.N;
  if (k < 0 || k + 1 > N) { std::fprintf(stderr, "bad k\n"); return 2; }
  Mpo mpo = make_hubbard_mpo(lat, 1.0, 0.0, 8.0, 1.5, 0.0);
  Rho0 r0 = make_rho0(mpo, 0.01, 1);
  const int mode = 1;
  Groups G = make_groups(mode);
  std::vector<std::map<Q, int>> n0(N + 1);
  for (int b = 0; b <= N; ++b)
    for (const Q& q : r0.q[b]) n0[b][project_charge(q, mode)]++;
  std::vector<std::map<Q, int>> dims = allocate_sectors(N, D, n0, cap, mode);
  std::vector<Bond> bonds(N + 1);
  for (int b = 0; b <= N; ++b)
    for (auto& kv : dims[b]) bonds[b].add(kv.first, kv.second);
  std::vector<std::vector<Q>> qH(N + 1);
  for (int b = 0; b < N; ++b)
    for (int a = 0; a < mpo.DH[b]; ++a) qH[b].push_back(project_charge(mpo.charge(b, a), mode));
  qH[N] = {Q{0, 0}};
  std::vector<std::vector<double>> Wt = mpo.W;
  {
    const int DL = mpo.DH[N - 1], DR = mpo.DH[N];
    std::vector<double> w((size_t)DL * 16, 0.0);
    for (int a = 0; a < DL; ++a)
      for (int q = 0; q < 16; ++q) w[(size_t)a * 16 + q] = mpo.W[N - 1][((size_t)a * 16 + q) * DR + 1];
    Wt[N - 1] = w;
  }
  const Bond &bl = bonds[k], &br = bonds[k + 1];
  const SiteLayout S = make_site_layout(bl, br, G);
  const EnvLayout ER = make_env_layout(br, qH[k + 1]);
  SiteTables tabs;
  SitePlan P = build_site_plan(k, bl, br, G, qH[k], qH[k + 1], Wt[k], Wt[k], tabs);
  const std::vector<long long>& T = tabs.host;
  const FzPlan& F = P.fz;

  std::vector<double> lw(std::max(P.lw_size, 1LL)), x(S.size), R(ER.size);
  for (auto* v : {&lw, &x, &R})
    for (double& e : *v) e = rnd();

  // the folded form's grouped GEMMs
  std::vector<double> t2(std::max(P.t2_size, 1LL), 0.0), ref(S.size, 0.0);
  {
    std::vector<double> none;
    for (int j = 0; j < P.n_s1w; ++j) {
      std::vector<double>* sl[4] = {&lw, &x, &t2, &none};
      run_gemm(P.s1w[j], T, sl);
      if (j == 0) run_w(P.t2zero, none, t2);
    }
    std::vector<double>* s3[4] = {&t2, &R, &ref, &none};
    run_gemm(P.s3, T, s3);
  }

  // the fused descriptors, interpreted
  std::vector<double> out;
  long long bad = fz_interpret(F, lw, x, R, S.size, out);
  if (bad) std::printf("MISMATCH coverage: %lld elements not written exactly once\n", bad);
  double worst = rel_err(out, ref);
  if (worst > 1e-12) std::printf("MISMATCH fused vs folded rel %.3e\n", worst);

  // the bond apply of the left bond: L . S into U, then U . R^T, against its fused plan
  {
    const EnvLayout EL = make_env_layout(bl, qH[k]);
    const BondMatLayout bm = make_bondmat_layout(bl);
    std::vector<double> Le(EL.size), Re(EL.size), Sm(bm.size), U(std::max(P.u_size, 1LL), 0.0), bref(bm.size, 0.0);
    for (auto* v : {&Le, &Re, &Sm})
      for (double& e : *v) e = rnd();
    std::vector<double> none;
    std::vector<double>* b1[4] = {&Le, &Sm, &U, &none};
    run_gemm(P.b1, T, b1);
    std::vector<double>* b2[4] = {&U, &Re, &bref, &none};
    run_gemm(P.b2, T, b2);
    std::vector<double> bout;
    const long long bbad = fz_interpret(P.fzb, Le, Sm, Re, bm.size, bout);
    if (bbad) std::printf("MISMATCH bond coverage: %lld\n", bbad);
    const double be = rel_err(bout, bref);
    if (be > 1e-12) std::printf("MISMATCH fused bond rel %.3e\n", be);
    bad += bbad;
    worst = std::max(worst, be);
    bad += check_jobs(P.fzb);
  }
  const long long jbad = check_jobs(F);
  if (jbad) std::printf("MISMATCH jobs %lld\n", jbad);
  int maxd = 0;
  for (auto& s : bl.secs) maxd = std::max(maxd, s.dim);
  for (auto& s : br.secs) maxd = std::max(maxd, s.dim);
  std::printf("fused k=%d Dl=%d Dr=%d max_sector=%d blocks=%zu b=%zu terms=%zu jobs=%zu worst=%.3e\n", k,
              (int)bl.total, (int)br.total, maxd, F.outs.size(), F.bs.size(), F.terms.size(), F.jobs.size(), worst);
  return (worst <= 1e-12 && bad == 0 && jbad == 0) ? 0 : 1;
}
