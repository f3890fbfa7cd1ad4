// Host-only check of the two-site (2-TDVP) descriptors: the planner's join,
// H^(2) and split tables are run through a plain loop interpreter of their
// semantics (grouped GEMM with index maps, weighted W-stage gathers) on random
// block-sparse operands and compared with the same contractions written
// densely over the global bond indices.  No GPU code is involved.
//
// usage: host_pair_check W L geometry D symmetry k   (prints one line, exit 0 on success)
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2212_11973_amd/csrc/plan.h"

using namespace tt;

// the tile planner in layout.cpp asks the kernels for LDS sizes; unused here
namespace tt { int gemm_smem_bytes(int) { return 0; } }

static std::mt19937_64 rng(12345);
static double rnd() { return std::uniform_real_distribution<double>(-1.0, 1.0)(rng); }

static long long at(long long tab, long long stride, int i, const std::vector<long long>& T) {
  return tab >= 0 ? T[tab + i] : (long long)i * stride;
}

// C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C(m, n) for every problem of the plan
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

// dst(i, j) = sum_t w_t src_t(i, j)
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

// one-sided Jacobi SVD of an r x c matrix (row-major), returns U (r x n), s, Vt (n x c), n = min(r, c)
static void svd(const std::vector<double>& M, int r, int c, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& Vt) {
  const bool tr = r < c;
  const int m = tr ? c : r, n = tr ? r : c;
  std::vector<double> X((size_t)m * n), V((size_t)n * n, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) {
      if (!tr) X[i + (size_t)j * m] = M[(size_t)i * c + j];
      else X[j + (size_t)i * m] = M[(size_t)i * c + j];
    }
  for (int i = 0; i < n; ++i) V[i + (size_t)i * n] = 1.0;
  for (int sw = 0; sw < 60; ++sw) {
    bool rot = false;
    for (int a = 0; a < n; ++a)
      for (int b = a + 1; b < n; ++b) {
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < m; ++i) {
          const double u = X[i + (size_t)a * m], v = X[i + (size_t)b * m];
          al += u * u; be += v * v; ga += u * v;
        }
        if (!(std::fabs(ga) > 1e-15 * std::sqrt(al * be))) continue;
        rot = true;
        const double z = (be - al) / (2 * ga);
        const double t = (z >= 0 ? 1.0 : -1.0) / (std::fabs(z) + std::hypot(1.0, z));
        const double cs = 1 / std::sqrt(1 + t * t), sn = cs * t;
        for (int i = 0; i < m; ++i) {
          const double u = X[i + (size_t)a * m], v = X[i + (size_t)b * m];
          X[i + (size_t)a * m] = cs * u - sn * v;
          X[i + (size_t)b * m] = sn * u + cs * v;
        }
        for (int i = 0; i < n; ++i) {
          const double u = V[i + (size_t)a * n], v = V[i + (size_t)b * n];
          V[i + (size_t)a * n] = cs * u - sn * v;
          V[i + (size_t)b * n] = sn * u + cs * v;
        }
      }
    if (!rot) break;
  }
  s.assign(n, 0.0);
  U.assign((size_t)r * n, 0.0);
  Vt.assign((size_t)n * c, 0.0);
  for (int j = 0; j < n; ++j) {
    double q = 0;
    for (int i = 0; i < m; ++i) q += X[i + (size_t)j * m] * X[i + (size_t)j * m];
    s[j] = std::sqrt(q);
    for (int i = 0; i < r; ++i) U[(size_t)i * n + j] = tr ? V[i + (size_t)j * n] : X[i + (size_t)j * m] / s[j];
    for (int i = 0; i < c; ++i) Vt[(size_t)j * c + i] = tr ? X[i + (size_t)j * m] / s[j] : V[i + (size_t)j * n];
  }
}

int main(int argc, char** argv) {
  if (argc < 7) { std::fprintf(stderr, "usage\n"); return 2; }
  const int W = std::atoi(argv[1]), Lx = std::atoi(argv[2]), geo = std::atoi(argv[3]);
  const int D = std::atoi(argv[4]), mode = std::atoi(argv[5]), k = std::atoi(argv[6]);
  Lattice lat = make_lattice(W, Lx, geo);
  const int N = lat.N;
  if (k < 0 || k + 2 > N) { std::fprintf(stderr, "bad k\n"); return 2; }
  Mpo mpo = make_hubbard_mpo(lat, 1.0, 0.0, 8.0, 1.5, 0.0);
  Rho0 r0 = make_rho0(mpo, 0.01, 1);
  Groups G = make_groups(mode);
  std::vector<std::map<Q, int>> n0(N + 1);
  for (int b = 0; b <= N; ++b)
    for (const Q& q : r0.q[b]) n0[b][project_charge(q, mode)]++;
  std::vector<std::map<Q, int>> dims;
  if (mode) {
    dims = allocate_sectors(N, D, n0, 0, mode);
  } else {
    dims.assign(N + 1, {});
    for (int b = 0; b <= N; ++b) {
      long long mx = 1;
      for (int i = 0; i < std::min(b, N - b) && mx < D; ++i) mx *= 16;
      dims[b][{0, 0}] = (int)std::max<long long>(std::min<long long>(D, mx), (long long)r0.q[b].size());
    }
  }
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
  const Bond &bl = bonds[k], &bm = bonds[k + 1], &br = bonds[k + 2];
  const SiteLayout SA = make_site_layout(bl, bm, G), SB = make_site_layout(bm, br, G);
  const EnvLayout EL = make_env_layout(bl, qH[k]), ER = make_env_layout(br, qH[k + 2]);
  SiteTables tabs;
  PairPlan P = build_pair_plan(bl, bm, br, G, qH[k], qH[k + 1], qH[k + 2], Wt[k], Wt[k + 1], SA, SB, tabs);
  const std::vector<long long>& T = tabs.host;
  const int DHl = (int)qH[k].size(), DHm = (int)qH[k + 1].size(), DHr = (int)qH[k + 2].size();
  const long long Dl = bl.total, Dm = bm.total, Dr = br.total;

  // random operands in their layouts, and their dense forms over global indices
  std::vector<double> Ak(SA.size), Bk(SB.size), Le(EL.size), Re(ER.size);
  for (auto* v : {&Ak, &Bk, &Le, &Re})
    for (double& x : *v) x = rnd();
  auto site_dense = [&](const SiteLayout& S, const Bond& L, const Bond& R, const std::vector<double>& v) {
    std::vector<double> d((size_t)L.total * 16 * R.total, 0.0);
    for (int l = 0; l < S.nl; ++l)
      for (int g = 0; g < G.ng; ++g) {
        const int r = S.rsec[l][g];
        if (r < 0) continue;
        for (int x = 0; x < S.dl[l]; ++x)
          for (int p = 0; p < (int)G.s[g].size(); ++p)
            for (int y = 0; y < R.secs[r].dim; ++y)
              d[((size_t)(L.secs[l].off + x) * 16 + G.s[g][p]) * R.total + R.secs[r].off + y] =
                  v[S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)p * R.secs[r].dim + y];
      }
    return d;
  };
  auto env_dense = [&](const EnvLayout& E, const Bond& B, int DH, const std::vector<double>& v) {
    std::vector<double> d((size_t)B.total * DH * B.total, 0.0);   // [bra][a][ket]
    for (int p = 0; p < E.np; ++p)
      for (int a = 0; a < DH; ++a) {
        const int x = E.csec[p][a];
        if (x < 0) continue;
        for (int i = 0; i < E.dp[p]; ++i)
          for (int j = 0; j < B.secs[x].dim; ++j)
            d[((size_t)(B.secs[p].off + i) * DH + a) * B.total + B.secs[x].off + j] =
                v[E.base[p] + (long long)i * E.K[p] + E.colb[p][a] + j];
      }
    return d;
  };
  // Theta in the pair layout <-> dense [Dl][16][16][Dr]
  auto pair_dense = [&](const std::vector<double>& v) {
    std::vector<double> d((size_t)Dl * 256 * Dr, 0.0);
    for (int l = 0; l < P.L.nl; ++l)
      for (int g1 = 0; g1 < G.ng; ++g1) {
        if (P.L.colg[l][g1] < 0) continue;
        const Q m = {bl.secs[l].q.first + G.delta[g1].first, bl.secs[l].q.second + G.delta[g1].second};
        const long long w = P.L.w(m);
        for (int p1 = 0; p1 < (int)G.s[g1].size(); ++p1)
          for (const MidBlock& mb : P.L.mid.at(m))
            for (int p2 = 0; p2 < (int)G.s[mb.g2].size(); ++p2)
              for (int x = 0; x < P.L.dl[l]; ++x)
                for (int y = 0; y < br.secs[mb.r].dim; ++y)
                  d[(((size_t)(bl.secs[l].off + x) * 16 + G.s[g1][p1]) * 16 + G.s[mb.g2][p2]) * Dr + br.secs[mb.r].off + y] =
                      v[P.L.base[l] + (long long)x * P.L.C[l] + P.L.colg[l][g1] + (long long)p1 * w + mb.off +
                        (long long)p2 * br.secs[mb.r].dim + y];
      }
    return d;
  };
  const std::vector<double> dA = site_dense(SA, bl, bm, Ak), dB = site_dense(SB, bm, br, Bk);
  const std::vector<double> dL = env_dense(EL, bl, DHl, Le), dR = env_dense(ER, br, DHr, Re);

  double worst = 0.0;
  auto cmp = [&](const std::vector<double>& a, const std::vector<double>& b, const char* what) {
    double e = 0.0, n = 0.0;
    for (size_t i = 0; i < a.size(); ++i) { e = std::max(e, std::fabs(a[i] - b[i])); n = std::max(n, std::fabs(b[i])); }
    const double rel = e / std::max(n, 1e-300);
    worst = std::max(worst, rel);
    if (rel > 1e-12) std::printf("MISMATCH %s rel %.3e\n", what, rel);
  };

  // join
  std::vector<double> th(P.L.size, 0.0);
  {
    std::vector<double> none;
    std::vector<double>* sl[4] = {&Ak, &Bk, &th, &none};
    run_gemm(P.join, T, sl);
  }
  std::vector<double> dth((size_t)Dl * 256 * Dr, 0.0);
  for (long long x = 0; x < Dl; ++x)
    for (int s1 = 0; s1 < 16; ++s1)
      for (long long mu = 0; mu < Dm; ++mu) {
        const double a = dA[((size_t)x * 16 + s1) * Dm + mu];
        if (a == 0.0) continue;
        for (int s2 = 0; s2 < 16; ++s2)
          for (long long y = 0; y < Dr; ++y)
            dth[(((size_t)x * 16 + s1) * 16 + s2) * Dr + y] += a * dB[((size_t)mu * 16 + s2) * Dr + y];
      }
  cmp(pair_dense(th), dth, "join");

  // H^(2) on a random Theta (every block of the layout, also middle charges the bond lacks)
  for (double& v : th) v = rnd();
  const std::vector<double> dx = pair_dense(th);
  std::vector<double> t1(P.t1_size, 0.0), t2(P.t2_size, 0.0), t3(P.t3_size, 0.0), out(P.L.size, 0.0);
  {
    std::vector<double> none;
    std::vector<double>* sl[4] = {&Le, &th, &t1, &none};
    run_gemm(P.s1, T, sl);
    run_w(P.w1, t1, t2);
    run_w(P.w2, t2, t3);
    std::vector<double>* s4[4] = {&t3, &Re, &out, &none};
    run_gemm(P.s4, T, s4);
  }
  auto wsup = [](const std::vector<double>& Wv, int DHo, int a, int so, int si, int b) {
    if ((so & 3) != (si & 3)) return 0.0;
    return Wv[(size_t)((((long long)a * 4 + (so >> 2)) * 4 + (si >> 2)) * DHo + b)];
  };
  // dense: X1[x'][a -> b][s1'][s2][y] then the site k+1 MPO, then R
  std::vector<double> u1((size_t)Dl * DHl * 256 * Dr, 0.0);   // L.x: [x'][a][s1 s2][y]
  for (long long xp = 0; xp < Dl; ++xp)
    for (int a = 0; a < DHl; ++a)
      for (long long x = 0; x < Dl; ++x) {
        const double lv = dL[((size_t)xp * DHl + a) * Dl + x];
        if (lv == 0.0) continue;
        for (size_t q = 0; q < (size_t)256 * Dr; ++q) u1[((size_t)xp * DHl + a) * 256 * Dr + q] += lv * dx[(size_t)x * 256 * Dr + q];
      }
  std::vector<double> u2((size_t)Dl * DHm * 256 * Dr, 0.0);   // [x'][b][s1' s2][y]
  for (long long xp = 0; xp < Dl; ++xp)
    for (int a = 0; a < DHl; ++a)
      for (int b = 0; b < DHm; ++b)
        for (int so = 0; so < 16; ++so)
          for (int si = 0; si < 16; ++si) {
            const double w = wsup(Wt[k], DHm, a, so, si, b);
            if (w == 0.0) continue;
            for (size_t q = 0; q < (size_t)16 * Dr; ++q)
              u2[(((size_t)xp * DHm + b) * 16 + so) * 16 * Dr + q] += w * u1[(((size_t)xp * DHl + a) * 16 + si) * 16 * Dr + q];
          }
  std::vector<double> u3((size_t)Dl * DHr * 256 * Dr, 0.0);   // [x'][c][s1'][s2'][y]
  for (long long xp = 0; xp < Dl; ++xp)
    for (int b = 0; b < DHm; ++b)
      for (int c = 0; c < DHr; ++c)
        for (int so = 0; so < 16; ++so)
          for (int si = 0; si < 16; ++si) {
            const double w = wsup(Wt[k + 1], DHr, b, so, si, c);
            if (w == 0.0) continue;
            for (int s1 = 0; s1 < 16; ++s1)
              for (long long y = 0; y < Dr; ++y)
                u3[((((size_t)xp * DHr + c) * 16 + s1) * 16 + so) * Dr + y] +=
                    w * u2[((((size_t)xp * DHm + b) * 16 + s1) * 16 + si) * Dr + y];
          }
  std::vector<double> dout((size_t)Dl * 256 * Dr, 0.0);
  for (long long xp = 0; xp < Dl; ++xp)
    for (int c = 0; c < DHr; ++c)
      for (int s12 = 0; s12 < 256; ++s12)
        for (long long yp = 0; yp < Dr; ++yp) {
          double acc = 0.0;
          for (long long y = 0; y < Dr; ++y)
            acc += u3[(((size_t)xp * DHr + c) * 256 + s12) * Dr + y] * dR[((size_t)yp * DHr + c) * Dr + y];
          dout[((size_t)xp * 256 + s12) * Dr + yp] += acc;
        }
  // the dense result restricted to the blocks the layout holds (the projection
  // onto the bonds' charge sectors): zero the blocks the layout lacks
  {
    std::vector<double> ones(P.L.size, 1.0);
    const std::vector<double> mask = pair_dense(ones);
    for (size_t i = 0; i < dout.size(); ++i) dout[i] *= mask[i];
  }
  cmp(pair_dense(out), dout, "heff2");

  // split tables: every task's rows are the (x, s1) rows of its middle charge,
  // columns the (s2, y) of that charge; a full-rank SVD of each task rebuilds Theta
  std::vector<double> rec((size_t)Dl * 256 * Dr, 0.0);
  long long rows_total = 0;
  for (size_t t = 0; t < P.svd.size(); ++t) {
    const SvdTask& st = P.svd[t];
    std::vector<double> M((size_t)st.R * st.w);
    for (int i = 0; i < st.R; ++i)
      for (int j = 0; j < st.w; ++j) M[(size_t)i * st.w + j] = th.at(T.at(st.rtab + i) + j);
    std::vector<double> U, s, Vt;
    svd(M, st.R, st.w, U, s, Vt);
    const int n = std::min(st.R, st.w);
    std::vector<double> Mr((size_t)st.R * st.w, 0.0);
    for (int i = 0; i < st.R; ++i)
      for (int j = 0; j < st.w; ++j) {
        double acc = 0.0;
        for (int q = 0; q < n; ++q) acc += U[(size_t)i * n + q] * s[q] * Vt[(size_t)q * st.w + j];
        Mr[(size_t)i * st.w + j] = acc;
      }
    // scatter back through the row groups (l, g1, s1 position) and the middle charge's columns
    const Q m = P.mq[t];
    int i = 0;
    for (const auto& rg : P.rowgroups[t]) {
      const int l = rg[0], g1 = rg[1], p1 = rg[2];
      for (int x = 0; x < bl.secs[l].dim; ++x, ++i)
        for (const MidBlock& mb : P.L.mid.at(m))
          for (int p2 = 0; p2 < (int)G.s[mb.g2].size(); ++p2)
            for (int y = 0; y < br.secs[mb.r].dim; ++y)
              rec[(((size_t)(bl.secs[l].off + x) * 16 + G.s[g1][p1]) * 16 + G.s[mb.g2][p2]) * Dr + br.secs[mb.r].off + y] =
                  Mr[(size_t)i * st.w + mb.off + (long long)p2 * br.secs[mb.r].dim + y];
    }
    if (i != st.R) { std::printf("MISMATCH split rows\n"); worst = 1.0; }
    rows_total += st.R;
  }
  cmp(rec, dx, "split");
  long long expect_rows = 0;
  for (int l = 0; l < P.L.nl; ++l)
    for (int g1 = 0; g1 < G.ng; ++g1)
      if (P.L.colg[l][g1] >= 0) expect_rows += (long long)bl.secs[l].dim * G.s[g1].size();
  if (rows_total != expect_rows) { std::printf("MISMATCH split coverage %lld %lld\n", rows_total, expect_rows); worst = 1.0; }
  std::printf("pair k=%d Dl=%lld Dm=%lld Dr=%lld theta=%lld tasks=%zu worst=%.3e\n", k, Dl, Dm, Dr, P.L.size,
              P.svd.size(), worst);
  return worst <= 1e-12 ? 0 : 1;
}
