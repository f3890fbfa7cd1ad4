// Block-sparse layouts and the descriptor lists of every contraction of one
// site.  Each contraction of the one-site sweep (SM Fig. optimalB(c,d) and the
// environment recursion) becomes a grouped GEMM over charge blocks, in the
// contraction order of SM Fig. Lanczos (L.A, then W, then R); with one sector
// per bond (no symmetry) each grouped GEMM is a single dense GEMM.
#include <algorithm>
#include <cmath>

#include "plan.h"

namespace tt {

static Q addq(Q a, Q b) { return {a.first + b.first, a.second + b.second}; }
static Q subq(Q a, Q b) { return {a.first - b.first, a.second - b.second}; }

SiteLayout make_site_layout(const Bond& left, const Bond& right, const Groups& G) {
  SiteLayout s;
  s.nl = (int)left.secs.size();
  s.dl.resize(s.nl);
  s.C.resize(s.nl);
  s.base.resize(s.nl);
  s.rsec.resize(s.nl);
  s.colb.resize(s.nl);
  long long pos = 0;
  for (int l = 0; l < s.nl; ++l) {
    s.dl[l] = left.secs[l].dim;
    int c = 0;
    for (int g = 0; g < 9; ++g) { s.rsec[l][g] = -1; s.colb[l][g] = -1; }
    for (int g = 0; g < G.ng; ++g) {
      int r = right.find(addq(left.secs[l].q, G.delta[g]));
      if (r < 0) continue;
      s.rsec[l][g] = r;
      s.colb[l][g] = c;
      c += (int)G.s[g].size() * right.secs[r].dim;
    }
    s.C[l] = c;
    s.base[l] = pos;
    pos += (long long)s.dl[l] * c;
  }
  s.size = pos;
  return s;
}

EnvLayout make_env_layout(const Bond& bond, const std::vector<Q>& qH) {
  EnvLayout e;
  e.np = (int)bond.secs.size();
  e.dp.resize(e.np);
  e.K.resize(e.np);
  e.base.resize(e.np);
  e.csec.assign(e.np, std::vector<int>(qH.size(), -1));
  e.colb.assign(e.np, std::vector<int>(qH.size(), -1));
  long long pos = 0;
  for (int p = 0; p < e.np; ++p) {
    e.dp[p] = bond.secs[p].dim;
    int c = 0;
    for (size_t a = 0; a < qH.size(); ++a) {
      int x = bond.find(subq(bond.secs[p].q, qH[a]));
      if (x < 0) continue;
      e.csec[p][a] = x;
      e.colb[p][a] = c;
      c += bond.secs[x].dim;
    }
    e.K[p] = c;
    e.base[p] = pos;
    pos += (long long)e.dp[p] * c;
  }
  e.size = pos;
  return e;
}

BondMatLayout make_bondmat_layout(const Bond& bond) {
  BondMatLayout b;
  long long pos = 0;
  for (auto& s : bond.secs) {
    b.off.push_back(pos);
    pos += (long long)s.dim * s.dim;
  }
  b.size = pos;
  return b;
}

static GemmProb gp(int M, int N, int K, int ia, int ib, int ic) {
  GemmProb p{};
  p.M = M; p.N = N; p.K = K;
  p.ia = ia; p.ib = ib; p.ic = ic;
  p.tam = p.tak = p.tbk = p.tbn = p.tcm = -1;
  p.alpha = 1.0; p.beta = 0.0;
  return p;
}

static void add_prob(GemmPlan& plan, const GemmProb& p) {
  if (p.M <= 0 || p.N <= 0) return;
  plan.probs.push_back(p);
  plan.flops += 2.0 * p.M * (double)p.N * p.K;
  plan.bytes += 8.0 * ((double)p.M * p.K + (double)p.K * p.N + (double)p.M * p.N);
}

// algorithmic traffic of a W stage: distinct source blocks read once, outputs written once
static void finish_wplan(WPlan& w) {
  std::vector<std::pair<long long, long long>> src;
  double out = 0.0;
  // byte offsets inside a block fit 32 bits unless some block spans 2^29
  // elements or more (then the kernel forms them in 64 bits)
  auto fits = [](long long ni, long long nj, long long si, long long sj) {
    return ni <= 0 || nj <= 0 || (ni - 1) * si + (nj - 1) * sj < (1LL << 29);
  };
  w.wide = false;
  for (auto& t : w.tasks) {
    if (!fits(t.ni, t.nj, t.dsi, t.dsj)) w.wide = true;
    for (int q = t.t0; q < t.t0 + t.nt; ++q)
      if (!fits(t.ni, t.nj, w.terms[q].ssi, w.terms[q].ssj)) w.wide = true;
    out += (double)t.ni * t.nj;
    for (int q = t.t0; q < t.t0 + t.nt; ++q) src.push_back({w.terms[q].src, (long long)t.ni * t.nj});
  }
  std::sort(src.begin(), src.end());
  src.erase(std::unique(src.begin(), src.end()), src.end());
  double in = 0.0;
  for (auto& s : src) in += (double)s.second;
  w.bytes = 8.0 * (in + out);
}

static void finish_qrplan(QRPlan& q) {
  for (auto& t : q.tasks) {
    double m = t.m, n = t.n;
    q.flops += 4.0 * m * n * n - 4.0 / 3.0 * n * n * n;
    q.bytes += 8.0 * (2.0 * m * n + n * n);
  }
}

int gemm_cfg_for(int M, int N) {
  if (M <= 32 && N <= 32) return 4;
  if (M <= 32) return 3;
  if (N <= 16) return 2;
  if (N <= 32) return 1;
  return 0;
}

static int wave_shape_for(int M, int N) {
  if (N <= 16) return 0;
  if (M <= 16) return 2;
  return 1;
}

// largest element offset of an index map over [0, n) (tables hold non-negative offsets)
static long long map_max(const std::vector<long long>* T, long long tab, long long stride, int n) {
  if (n <= 0) return 0;
  if (tab < 0) return (long long)(n - 1) * stride;
  long long m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, (*T)[tab + i]);
  return m;
}

void tile_plan(GemmPlan& p, const std::vector<long long>* tabs) {
  p.tiles.clear();
  p.splits.clear();
  p.jobs.clear();
  p.jobs_fine.clear();
  p.wave_blocks_fine = 0;
  p.pws_size = 0;
  p.smem_bytes = 0;
  p.red_bytes = 0;
  p.wave_blocks = 0;
  p.wave_flops = p.wave_bytes = 0;
  for (int c = 0; c < kGemmCfgs; ++c) p.cfg_flops[c] = p.cfg_bytes[c] = 0;
  // the wave kernel addresses operands with 32-bit byte offsets from each operand base
  const long long lim = 1LL << 29;
  // float operands (dt) are read and written by the wave GEMM only
  std::vector<char> wave(p.probs.size(), 0);
  for (size_t i = 0; i < p.probs.size(); ++i) {
    GemmProb& g = p.probs[i];
    g.dt = (p.slot_f32[g.ia] ? kDtA : 0) | (p.slot_f32[g.ib] ? kDtB : 0) | (p.slot_f32[g.ic] ? kDtC : 0);
    if (!p.wave_ok) {
      TT_REQUIRE(g.dt == 0, TT_EINVAL, "plan: float operands need the wave GEMM");
      continue;
    }
    if (g.dt == 0 && g.M >= kLdsMinMN && g.N >= kLdsMinMN && g.K >= kLdsMinK) continue;
    TT_REQUIRE(tabs != nullptr, TT_EINVAL, "plan: wave GEMM planning needs the index tables");
    const long long a = map_max(tabs, g.tam, g.sam, g.M) + map_max(tabs, g.tak, g.sak, g.K);
    const long long b = map_max(tabs, g.tbk, g.sbk, g.K) + map_max(tabs, g.tbn, g.sbn, g.N);
    const long long c = map_max(tabs, g.tcm, g.scm, g.M) + g.N;
    const bool fit = a < lim && b < lim && c < lim;
    TT_REQUIRE(fit || g.dt == 0, TT_EINVAL, "plan: float operands beyond 32-bit offsets");
    wave[i] = fit ? 1 : 0;
  }
  auto use_wave = [&](const GemmProb& g) { return wave[&g - p.probs.data()] != 0; };
  // wave jobs: split blocks (four K parts in one workgroup) first, then
  // unsplit blocks four to a workgroup.  fine: 16x16 blocks and K split from
  // four chunks on, for launches too small to fill the GPU otherwise.
  auto plan_jobs = [&](bool fine, std::vector<GemmJob>& jobs) {
    std::vector<GemmJob> single;
    jobs.clear();
    for (int i = 0; i < (int)p.probs.size(); ++i) {
      const GemmProb& g = p.probs[i];
      if (!use_wave(g) || g.M == 0 || g.N == 0) continue;
      const int sh = fine ? 3 : wave_shape_for(g.M, g.N);
      const int tm = (g.M + kWaveBM[sh] - 1) / kWaveBM[sh], tn = (g.N + kWaveBN[sh] - 1) / kWaveBN[sh];
      // every part then takes at least two (one when fine) 16-deep chunks
      const bool split = (g.K + 15) / 16 >= (fine ? 4 : 8);
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          if (split) {
            for (int q = 0; q < 4; ++q) jobs.push_back({i, a, b, sh, q, 4});
          } else {
            single.push_back({i, a, b, sh, 0, 1});
          }
        }
    }
    for (auto& j : single) jobs.push_back(j);
  };
  for (int i = 0; i < (int)p.probs.size(); ++i) {
    const GemmProb& g = p.probs[i];
    if (!use_wave(g) || g.M == 0 || g.N == 0) continue;
    p.wave_flops += 2.0 * g.M * g.N * g.K;
    p.wave_bytes += (g.dt & kDtA ? 4.0 : 8.0) * g.M * g.K + (g.dt & kDtB ? 4.0 : 8.0) * g.K * g.N +
                    (g.dt & kDtC ? 4.0 : 8.0) * g.M * g.N;
  }
  plan_jobs(false, p.jobs);
  p.jobs_fine.clear();
  if (!p.jobs.empty() && (long long)p.jobs.size() < kWaveMinJobs) {
    plan_jobs(true, p.jobs_fine);
    if (p.jobs_fine.size() <= p.jobs.size()) p.jobs_fine.clear();
  }
  for (auto* j : {&p.jobs, &p.jobs_fine})
    while (j->size() % 4) j->push_back({-1, 0, 0, 0, 0, 1});
  p.wave_blocks = (int)(p.jobs.size() / 4);
  p.wave_blocks_fine = (int)(p.jobs_fine.size() / 4);

  // LDS-staged tiles for the rest; K splitting only pays when the launch has
  // too few tiles to fill the GPU
  long long tiles0 = 0;
  for (auto& g : p.probs) {
    if (use_wave(g)) continue;
    int cfg = gemm_cfg_for(g.M, g.N);
    tiles0 += (long long)((g.M + kGemmBM[cfg] - 1) / kGemmBM[cfg]) * ((g.N + kGemmBN[cfg] - 1) / kGemmBN[cfg]);
  }
  const bool may_split = tiles0 < kSplitBelowTiles && !p.no_split;
  for (int i = 0; i < (int)p.probs.size(); ++i) {
    const GemmProb& g = p.probs[i];
    if (use_wave(g)) continue;
    int cfg = gemm_cfg_for(g.M, g.N);
    int BM = kGemmBM[cfg], BN = kGemmBN[cfg];
    int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
    int nk = may_split ? (g.K + kKSlice - 1) / kKSlice : 1;
    if (nk < 1) nk = 1;
    if (nk > kMaxKSplit) nk = kMaxKSplit;
    p.smem_bytes = std::max(p.smem_bytes, gemm_smem_bytes(cfg));
    p.cfg_flops[cfg] += 2.0 * g.M * g.N * g.K;
    p.cfg_bytes[cfg] += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N);
    if (nk > 1) p.red_bytes += 8.0 * ((double)nk * tm * tn * BM * BN + (double)g.M * g.N);
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        long long pw = -1;
        int sidx = -1;
        if (nk > 1) {
          pw = p.pws_size;
          p.pws_size += (long long)nk * BM * BN;
          sidx = (int)p.splits.size();
          p.splits.push_back({i, a, b, cfg, nk, 0, pw});
        }
        for (int ks = 0; ks < nk; ++ks) p.tiles.push_back({i, a, b, cfg, ks, nk, sidx, 0, pw});
      }
  }
  std::stable_sort(p.tiles.begin(), p.tiles.end(), [](const GemmTile& x, const GemmTile& y) { return x.cfg < y.cfg; });
  for (int c = 0; c <= kGemmCfgs; ++c) p.cfg_off[c] = 0;
  for (auto& t : p.tiles) p.cfg_off[t.cfg + 1]++;
  for (int c = 0; c < kGemmCfgs; ++c) p.cfg_off[c + 1] += p.cfg_off[c];
  p.ntiles = (int)p.tiles.size();
}

// MFMA instructions of one fused-apply job (16 rows, up to kFzCols columns)
// over all b blocks of output block o: per b and 16-wide y chunk, the
// 4-deep steps of every term, then the steps of the product with R
static double fz_steps(const FzPlan& F, const FzOut& o) {
  const int fn = (std::min(o.dr, kFzCols) + 15) / 16;
  double steps = 0.0;
  for (int bi = 0; bi < o.nb; ++bi) {
    const FzB& b = F.bs[o.b0 + bi];
    double k1 = 0.0;
    for (int t = b.t0; t < b.t0 + b.nt; ++t) k1 += (F.terms[t].dl + 3) / 4;
    steps += ((b.dc + 15) / 16) * k1 + (double)fn * ((b.dc + 3) / 4);
  }
  return steps;
}

// the jobs of a fused-apply plan: every (block, 16-row tile, kFzCols-column
// tile); a tile with enough work for every wave to take several b blocks
// becomes four K parts in one workgroup.  The heaviest first; split jobs stay
// in groups of four.
static void plan_fz_jobs(FzPlan& F) {
  struct JobW { FzJob j; double steps; };
  std::vector<JobW> split, single;
  for (int oi = 0; oi < (int)F.outs.size(); ++oi) {
    const FzOut& o = F.outs[oi];
    const double steps = fz_steps(F, o);
    const bool sp4 = o.nb >= 8 && steps >= 256.0;
    for (int r0 = 0; r0 < o.dp; r0 += 16)
      for (int c0 = 0; c0 < o.dr; c0 += kFzCols) {
        if (sp4) {
          for (int q = 0; q < 4; ++q) split.push_back({{oi, r0, c0, q, 4, 0}, steps});
        } else {
          single.push_back({{oi, r0, c0, 0, 1, 0}, steps});
        }
      }
  }
  std::stable_sort(single.begin(), single.end(), [](const JobW& a, const JobW& b) { return a.steps > b.steps; });
  std::vector<int> order(split.size() / 4);
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return split[4 * a].steps > split[4 * b].steps; });
  F.jobs.clear();
  for (int g : order)
    for (int q = 0; q < 4; ++q) F.jobs.push_back(split[4 * g + q].j);
  for (auto& j : single) F.jobs.push_back(j.j);
  while (F.jobs.size() % 4) F.jobs.push_back({-1, 0, 0, 0, 1, 0});
  F.nblocks = (int)(F.jobs.size() / 4);
}

// LW^{b,so,si}[x', x] = sum_a W[a,so,si,b] L^a[x', x] per bra sector p, and
// T2^{b,(so,sp)} = sum_si LW^{b,so,si} A^{(si,sp)} written into stage 3's T2
// layout (rows (p, g', x', s') of the right sector r' = p + Delta(so, sp),
// columns (b, y) of R's row block r').  For the Hubbard MPOs an output block
// (b, so) has 1.0-1.3 si terms on average, so T2 costs about the flops of L.A
// while T1 and the per-apply W stage disappear: the fold runs once per
// environment.  Problems are keyed by (pass j, l, si, sp): B is the block
// A^{(si,sp)} of left sector l, A the stacked LW rows of every (p, b, so) whose
// j-th term is (si, l); rows whose output block lies outside the truncated
// bond are dropped (the projection onto the kept space, as in the W stage).
static void build_lw_plans(SitePlan& P, const SiteLayout& S, const Bond& bl, const Bond& br, const Groups& G,
                           const EnvLayout& EL, const EnvLayout& ER, const std::vector<Q>& qHl,
                           const std::vector<Q>& qHr, const std::vector<double>& W, const std::vector<double>& Wp,
                           const std::vector<long long>& t2base, const std::vector<std::array<int, 9>>& rowpos2,
                           SiteTables& tabs) {
  const int DHl = (int)qHl.size(), DHr = (int)qHr.size();
  // charge of the ket operator |so><si| in the block structure's projection:
  // Delta(4 so + sp) - Delta(4 si + sp) for any ancilla sp
  auto dq = [&](int so, int si) { return subq(G.delta[G.group_of[4 * so]], G.delta[G.group_of[4 * si]]); };
  auto wat = [&](const std::vector<double>& T, int a, int so, int si, int b) {
    return T[(size_t)(((long long)a * 4 + so) * 4 + si) * DHr + b];
  };
  // groups of every bra sector p: (b, so, si) -> ket sector l and column base in LW
  struct Grp { int b, so, si, l; long long col; };
  std::vector<std::vector<Grp>> grp(S.nl);
  std::vector<long long> lwbase(S.nl, 0), lwK(S.nl, 0);
  std::vector<int> task_p;   // bra sector of every LW task
  long long pos = 0;
  for (int p = 0; p < S.nl; ++p) {
    long long c = 0;
    for (int b = 0; b < DHr; ++b)
      for (int so = 0; so < 4; ++so)
        for (int si = 0; si < 4; ++si) {
          const Q ql = subq(addq(bl.secs[p].q, dq(so, si)), qHr[b]);
          const int l = bl.find(ql);
          if (l < 0) continue;
          WTask t;
          t.t0 = (int)P.lw.terms.size();
          for (int a = 0; a < DHl; ++a) {
            const double w = wat(W, a, so, si, b);
            if (w == 0.0 && wat(Wp, a, so, si, b) == 0.0) continue;
            TT_REQUIRE(EL.csec[p][a] == l, TT_EINVAL, "plan: MPO entry breaks charge conservation (LW)");
            WTerm tm;
            tm.src = EL.base[p] + EL.colb[p][a];
            tm.ssi = EL.K[p];
            tm.ssj = 1;
            tm.w = w;
            P.lw.terms.push_back(tm);
            P.lw.widx.push_back((((long long)a * 4 + so) * 4 + si) * DHr + b);
          }
          t.nt = (int)P.lw.terms.size() - t.t0;
          if (t.nt == 0) continue;
          grp[p].push_back({b, so, si, l, c});
          t.dst = pos + c;   // lwbase[p] == pos while p's columns are laid out
          t.dsi = 0;         // p's row width, set once it is known
          t.dsj = 1;
          t.ni = S.dl[p];
          t.nj = bl.secs[l].dim;
          P.lw.tasks.push_back(t);
          task_p.push_back(p);
          c += bl.secs[l].dim;
        }
    lwbase[p] = pos;
    lwK[p] = c;
    pos += (long long)S.dl[p] * c;
  }
  for (size_t i = 0; i < P.lw.tasks.size(); ++i) P.lw.tasks[i].dsi = lwK[task_p[i]];
  P.lw_size = pos;
  for (auto& t : P.lw.tasks) P.lw.flops += 2.0 * t.nt * (double)t.ni * t.nj;

  // term lists of every output block (p, b, so, sp): si ascending, where the
  // group exists and A^{(si,sp)} has a block in left sector l
  struct Row { int p, b, so, sp, pass; const Grp* g; };
  std::vector<Row> rows;
  std::vector<char> written;   // per (p, b, s_out)
  auto widx3 = [&](int p, int b, int s) { return ((size_t)p * DHr + b) * 16 + s; };
  written.assign((size_t)S.nl * DHr * 16, 0);
  for (int p = 0; p < S.nl; ++p)
    for (int b = 0; b < DHr; ++b)
      for (int so = 0; so < 4; ++so)
        for (int sp = 0; sp < 4; ++sp) {
          const int s_out = 4 * so + sp, g_out = G.group_of[s_out];
          const int rq = S.rsec[p][g_out];
          if (rq < 0 || ER.csec[rq][b] < 0) continue;   // T2 has no such block
          int j = 0;
          for (const Grp& gr : grp[p]) {
            if (gr.b != b || gr.so != so) continue;
            const int s_in = 4 * gr.si + sp;
            if (S.rsec[gr.l][G.group_of[s_in]] < 0) continue;
            TT_REQUIRE(S.rsec[gr.l][G.group_of[s_in]] == ER.csec[rq][b], TT_EINVAL, "plan: inconsistent charges (LW)");
            TT_REQUIRE(j < SitePlan::kMaxLwPasses, TT_EINVAL, "plan: too many MPO terms per output block");
            rows.push_back({p, b, so, sp, j, &gr});
            ++j;
          }
          if (j > 0) written[widx3(p, b, s_out)] = 1;
        }
  // problems keyed by (pass, l, si, sp), rows in (p, b, so) order
  std::map<std::array<int, 4>, std::vector<const Row*>> probs;
  for (const Row& r : rows) probs[{r.pass, r.g->l, r.g->si, r.sp}].push_back(&r);
  P.n_s1w = 0;
  for (auto& kv : probs) {
    const int pass = kv.first[0], l = kv.first[1], si = kv.first[2], sp = kv.first[3];
    const int s_in = 4 * si + sp, g_in = G.group_of[s_in];
    const int r = S.rsec[l][g_in];
    std::vector<long long> arow, crow;
    for (const Row* rw : kv.second) {
      const int p = rw->p, s_out = 4 * rw->so + sp, g_out = G.group_of[s_out];
      const int rq = S.rsec[p][g_out];
      const int ns = (int)G.s[g_out].size();
      for (int x = 0; x < S.dl[p]; ++x) {
        arow.push_back(lwbase[p] + (long long)x * lwK[p] + rw->g->col);
        crow.push_back(t2base[rq] + ((long long)rowpos2[p][g_out] + (long long)x * ns + G.pos_of[s_out]) * ER.K[rq] +
                       ER.colb[rq][rw->b]);
      }
    }
    GemmProb g = gp((int)arow.size(), br.secs[r].dim, S.dl[l], 0, 1, 2);
    g.tam = tabs.add(arow); g.sak = 1;
    g.offB = S.base[l] + S.colb[l][g_in] + (long long)G.pos_of[s_in] * br.secs[r].dim;
    g.sbk = S.C[l]; g.sbn = 1;
    g.tcm = tabs.add(crow);
    g.beta = pass == 0 ? 0.0 : 1.0;
    add_prob(P.s1w[pass], g);
    P.n_s1w = std::max(P.n_s1w, pass + 1);
  }
  for (int j = 0; j < SitePlan::kMaxLwPasses; ++j) P.s1w[j].tag = TAG_LA;

  // the fused apply: one output block per (p, so, sp) that has a right sector;
  // per block the b of R's row block with at least one term, per b the terms
  // (b, so, si) of LW with the input block (l, 4 si + sp) in the same order as
  // the passes above.  A block with no b is written as zeros.
  {
    FzPlan& F = P.fz;
    F = FzPlan();
    for (int p = 0; p < S.nl; ++p)
      for (int so = 0; so < 4; ++so)
        for (int sp = 0; sp < 4; ++sp) {
          const int s_out = 4 * so + sp, g_out = G.group_of[s_out];
          const int rq = S.rsec[p][g_out];
          if (rq < 0) continue;
          FzOut o;
          o.dr = br.secs[rq].dim;
          o.out = S.base[p] + S.colb[p][g_out] + (long long)G.pos_of[s_out] * o.dr;
          o.ldo = S.C[p];
          o.dp = S.dl[p];
          o.rrow = ER.base[rq];
          o.ldr = ER.K[rq];
          o.b0 = (int)F.bs.size();
          o.nb = 0;
          for (int b = 0; b < DHr; ++b) {
            const int c = ER.csec[rq][b];
            if (c < 0) continue;
            FzB fb;
            fb.rcol = ER.colb[rq][b];
            fb.dc = br.secs[c].dim;
            fb.t0 = (int)F.terms.size();
            fb.nt = 0;
            fb.pad = 0;
            for (const Grp& gr : grp[p]) {
              if (gr.b != b || gr.so != so) continue;
              const int s_in = 4 * gr.si + sp, g_in = G.group_of[s_in];
              if (S.rsec[gr.l][g_in] < 0) continue;
              TT_REQUIRE(S.rsec[gr.l][g_in] == c, TT_EINVAL, "plan: inconsistent charges (fused apply)");
              FzT t;
              t.lw = lwbase[p] + gr.col;
              t.ldlw = (int)lwK[p];
              t.a = S.base[gr.l] + S.colb[gr.l][g_in] + (long long)G.pos_of[s_in] * fb.dc;
              t.lda = S.C[gr.l];
              t.dl = S.dl[gr.l];
              t.pad = 0;
              F.terms.push_back(t);
              ++fb.nt;
              F.flops += 2.0 * o.dp * (double)fb.dc * t.dl;
              F.bytes += 8.0 * ((double)o.dp * t.dl + (double)t.dl * fb.dc);
            }
            if (fb.nt == 0) continue;
            F.flops += 2.0 * o.dp * (double)fb.dc * o.dr;
            F.bytes += 8.0 * (double)o.dr * fb.dc;
            F.bs.push_back(fb);
            ++o.nb;
          }
          F.bytes += 8.0 * (double)o.dp * o.dr;
          F.outs.push_back(o);
        }
    plan_fz_jobs(F);
  }

  // T2 blocks that no term reaches are cleared (a task with no terms writes zeros)
  for (int rq = 0; rq < (int)br.secs.size(); ++rq)
    for (int p = 0; p < S.nl; ++p)
      for (int g = 0; g < G.ng; ++g) {
        if (S.rsec[p][g] != rq) continue;
        const int ns = (int)G.s[g].size();
        for (int si = 0; si < ns; ++si) {
          const int s_out = G.s[g][si];
          for (int b = 0; b < DHr; ++b) {
            const int c = ER.csec[rq][b];
            if (c < 0 || written[widx3(p, b, s_out)]) continue;
            WTask t;
            t.dst = t2base[rq] + (long long)(rowpos2[p][g] + si) * ER.K[rq] + ER.colb[rq][b];
            t.dsi = (long long)ns * ER.K[rq];
            t.dsj = 1;
            t.ni = S.dl[p];
            t.nj = br.secs[c].dim;
            t.t0 = 0;
            t.nt = 0;
            P.t2zero.tasks.push_back(t);
          }
        }
      }
  finish_wplan(P.lw);
  finish_wplan(P.t2zero);
}

SitePlan build_site_plan(int k, const Bond& bl, const Bond& br, const Groups& G,
                         const std::vector<Q>& qHl, const std::vector<Q>& qHr,
                         const std::vector<double>& W, const std::vector<double>& Wp, SiteTables& tabs,
                         bool super_op, bool with_lw) {
  (void)k;
  SitePlan P;
  const int DHl = (int)qHl.size(), DHr = (int)qHr.size();
  SiteLayout S = make_site_layout(bl, br, G);
  EnvLayout EL = make_env_layout(bl, qHl);
  EnvLayout ER = make_env_layout(br, qHr);
  // MPO entry for the super indices s_out, s_in (s = 4 sigma + sigma'): a
  // ket-only tensor W[a, so, si, b] leaves the ancilla sigma' unchanged; a
  // super-operator tensor holds all 16 x 16 entries
  // widx: the flat index of the entry in W, or -1 where it is zero by structure
  auto widx = [&](int a, int sout, int sin, int b) -> long long {
    if (super_op) return (((long long)a * 16 + sout) * 16 + sin) * DHr + b;
    if ((sout & 3) != (sin & 3)) return -1;
    return (((long long)a * 4 + (sout >> 2)) * 4 + (sin >> 2)) * DHr + b;
  };
  auto Wsup = [&](const std::vector<double>& T, int a, int sout, int sin, int b) -> double {
    const long long i = widx(a, sout, sin, b);
    return i < 0 ? 0.0 : T[(size_t)i];
  };
  const int nr = (int)br.secs.size();

  // ---------------- stage 1: T1_l[(a,x)][cols of A_l] = L[x,a,l-block] . A_l
  std::vector<long long> t1base(S.nl, 0);
  std::vector<std::vector<int>> rowbase1(S.nl, std::vector<int>(DHl, -1));
  long long pos = 0;
  for (int l = 0; l < S.nl; ++l) {
    std::vector<long long> rows;
    for (int a = 0; a < DHl; ++a) {
      int p = bl.find(addq(bl.secs[l].q, qHl[a]));
      if (p < 0 || EL.csec[p][a] != l) continue;
      rowbase1[l][a] = (int)rows.size();
      for (int x = 0; x < EL.dp[p]; ++x) rows.push_back(EL.base[p] + (long long)x * EL.K[p] + EL.colb[p][a]);
    }
    t1base[l] = pos;
    GemmProb g = gp((int)rows.size(), S.C[l], S.dl[l], 0, 1, 2);
    g.tam = tabs.add(rows); g.sak = 1;
    g.offB = S.base[l]; g.sbk = S.C[l]; g.sbn = 1;
    g.offC = pos; g.scm = S.C[l];
    add_prob(P.s1, g);
    pos += (long long)rows.size() * S.C[l];
  }
  P.t1_size = pos;
  P.s1.tag = TAG_LA; P.s3.tag = TAG_R; P.el.tag = TAG_ENVL; P.r1.tag = TAG_ENVR1; P.r3.tag = TAG_ENVR3;
  P.b1.tag = TAG_BOND; P.b2.tag = TAG_BOND; P.absL.tag = TAG_ABSORB; P.absR.tag = TAG_ABSORB;

  // ---------------- W stage: T2 grouped by the right bra sector r'
  // rows (p, g', x, s'), cols (b, y) as in the R environment of sector r'
  std::vector<long long> t2base(nr, 0);
  std::vector<int> nrows2(nr, 0);
  std::vector<std::vector<long long>> outrows(nr);   // row -> offset in the output site tensor
  std::vector<std::array<int, 9>> rowpos2(S.nl);
  for (int l = 0; l < S.nl; ++l) rowpos2[l].fill(-1);
  pos = 0;
  for (int r = 0; r < nr; ++r) {
    int cnt = 0;
    for (int p = 0; p < S.nl; ++p)
      for (int g = 0; g < G.ng; ++g) {
        if (S.rsec[p][g] != r) continue;
        rowpos2[p][g] = cnt;
        int ns = (int)G.s[g].size();
        for (int x = 0; x < S.dl[p]; ++x)
          for (int si = 0; si < ns; ++si)
            outrows[r].push_back(S.base[p] + (long long)x * S.C[p] + S.colb[p][g] + (long long)si * br.secs[r].dim);
        cnt += S.dl[p] * ns;
      }
    nrows2[r] = cnt;
    t2base[r] = pos;
    pos += (long long)cnt * ER.K[r];
  }
  P.t2_size = pos;
  for (int r = 0; r < nr; ++r) {
    for (int p = 0; p < S.nl; ++p)
      for (int g = 0; g < G.ng; ++g) {
        if (S.rsec[p][g] != r) continue;
        int ns = (int)G.s[g].size();
        for (int si = 0; si < ns; ++si) {
          int sp = G.s[g][si];   // output super index
          for (int b = 0; b < DHr; ++b) {
            int c = ER.csec[r][b];
            if (c < 0) continue;
            WTask t;
            t.dst = t2base[r] + (long long)(rowpos2[p][g] + si) * ER.K[r] + ER.colb[r][b];
            t.dsi = (long long)ns * ER.K[r];
            t.dsj = 1;
            t.ni = S.dl[p];
            t.nj = br.secs[c].dim;
            t.t0 = (int)P.w2.terms.size();
            for (int a = 0; a < DHl; ++a) {
              int l = EL.csec[p][a];
              if (l < 0) continue;
              for (int s = 0; s < 16; ++s) {
                double w = Wsup(W, a, sp, s, b);
                if (w == 0.0 && Wsup(Wp, a, sp, s, b) == 0.0) continue;
                int gg = G.group_of[s];
                TT_REQUIRE(S.rsec[l][gg] == c, TT_EINVAL, "plan: MPO entry breaks charge conservation");
                WTerm tm;
                tm.src = t1base[l] + (long long)rowbase1[l][a] * S.C[l] + S.colb[l][gg] +
                         (long long)G.pos_of[s] * br.secs[c].dim;
                tm.ssi = S.C[l];
                tm.ssj = 1;
                tm.w = w;
                P.w2.terms.push_back(tm);
                P.w2.widx.push_back(widx(a, sp, s, b));
              }
            }
            t.nt = (int)P.w2.terms.size() - t.t0;
            P.w2.flops += 2.0 * t.nt * (double)t.ni * t.nj;
            P.w2.tasks.push_back(t);
          }
        }
      }
  }

  // ---------------- the MPO folded into the left environment (ket-only MPOs)
  if (!super_op && with_lw) build_lw_plans(P, S, bl, br, G, EL, ER, qHl, qHr, W, Wp, t2base, rowpos2, tabs);

  // ---------------- stage 3: out rows (p,g',x,s') = T2_r' . R_r'^T ; env-left final
  for (int r = 0; r < nr; ++r) {
    if (nrows2[r] == 0) continue;
    long long tab = tabs.add(outrows[r]);
    GemmProb g = gp(nrows2[r], br.secs[r].dim, ER.K[r], 0, 1, 2);
    g.offA = t2base[r]; g.sam = ER.K[r]; g.sak = 1;
    g.offB = ER.base[r]; g.sbk = 1; g.sbn = ER.K[r];
    g.tcm = tab;
    add_prob(P.s3, g);
    // L_{k+1}[y'][(b,y)] = sum_rows A^L[row][y'] T2[row][(b,y)]
    GemmProb e = gp(br.secs[r].dim, ER.K[r], nrows2[r], 0, 1, 2);
    e.sam = 1; e.tak = tab;
    e.offB = t2base[r]; e.sbk = ER.K[r]; e.sbn = 1;
    e.offC = ER.base[r]; e.scm = ER.K[r];
    add_prob(P.el, e);
  }

  // ---------------- env-right stage 1': Y^T_c[(b,y')][(l,g,x,s)] = R[y',b,c-block] . A^T
  const int nc = nr;
  std::vector<long long> ybase(nc, 0);
  std::vector<int> ycols(nc, 0);
  std::vector<std::vector<int>> rowbaseY(nc, std::vector<int>(DHr, -1));
  std::vector<std::array<int, 9>> colposY(S.nl);
  for (int l = 0; l < S.nl; ++l) colposY[l].fill(-1);
  std::vector<std::vector<long long>> qrrows(nc);   // A rows grouped by right sector
  pos = 0;
  for (int c = 0; c < nc; ++c) {
    for (int l = 0; l < S.nl; ++l)
      for (int g = 0; g < G.ng; ++g) {
        if (S.rsec[l][g] != c) continue;
        colposY[l][g] = (int)qrrows[c].size();
        int ns = (int)G.s[g].size();
        for (int x = 0; x < S.dl[l]; ++x)
          for (int si = 0; si < ns; ++si)
            qrrows[c].push_back(S.base[l] + (long long)x * S.C[l] + S.colb[l][g] + (long long)si * br.secs[c].dim);
      }
    ycols[c] = (int)qrrows[c].size();
    std::vector<long long> rrows;
    for (int b = 0; b < DHr; ++b) {
      int rp = br.find(addq(br.secs[c].q, qHr[b]));
      if (rp < 0 || ER.csec[rp][b] != c) continue;
      rowbaseY[c][b] = (int)rrows.size();
      for (int y = 0; y < br.secs[rp].dim; ++y)
        rrows.push_back(ER.base[rp] + (long long)y * ER.K[rp] + ER.colb[rp][b]);
    }
    ybase[c] = pos;
    long long qtab = tabs.add(qrrows[c]);
    if (!rrows.empty() && ycols[c] > 0) {
      GemmProb g = gp((int)rrows.size(), ycols[c], br.secs[c].dim, 0, 1, 2);
      g.tam = tabs.add(rrows); g.sak = 1;
      g.sbk = 1; g.tbn = qtab;
      g.offC = pos; g.scm = ycols[c];
      add_prob(P.r1, g);
    }
    pos += (long long)rrows.size() * ycols[c];
    // QR of the rows of sector c (left-to-right gauge move)
    QRTask q{};
    q.m = ycols[c]; q.n = br.secs[c].dim; q.trans = 0;
    q.rbase = 0; q.rs = 0; q.cs = 1; q.rtab = qtab;
    q.ws = P.qr.ws_size;
    P.qr.ws_size += 2LL * q.m * q.n;
    P.qr.tasks.push_back(q);
    // absorb from the right: rows . S_c
    GemmProb ab = gp(ycols[c], br.secs[c].dim, br.secs[c].dim, 0, 1, 2);
    ab.tam = qtab; ab.sak = 1;
    ab.sbk = br.secs[c].dim; ab.sbn = 1;
    ab.tcm = qtab;
    add_prob(P.absR, ab);
  }
  P.y_size = pos;
  // S offsets of the right bond for QR outputs / absorbR
  {
    BondMatLayout bm = make_bondmat_layout(br);
    for (int c = 0; c < nc; ++c) P.qr.tasks[c].sdst = bm.off[c];
    int i = 0;
    for (int c = 0; c < nc; ++c)
      if (ycols[c] > 0) P.absR.probs[i++].offB = bm.off[c];
  }

  // ---------------- env-right W stage: Z_p[(g',s',y')][(a,x)]
  std::vector<long long> zbase(S.nl, 0);
  pos = 0;
  for (int p = 0; p < S.nl; ++p) {
    zbase[p] = pos;
    pos += (long long)S.C[p] * EL.K[p];
  }
  P.z_size = pos;
  for (int p = 0; p < S.nl; ++p)
    for (int g = 0; g < G.ng; ++g) {
      int rp = S.rsec[p][g];
      if (rp < 0) continue;
      int ns = (int)G.s[g].size();
      for (int si = 0; si < ns; ++si) {
        int sp = G.s[g][si];
        for (int a = 0; a < DHl; ++a) {
          int l = EL.csec[p][a];
          if (l < 0) continue;
          WTask t;
          t.dst = zbase[p] + ((long long)S.colb[p][g] + (long long)si * br.secs[rp].dim) * EL.K[p] + EL.colb[p][a];
          t.dsi = EL.K[p];
          t.dsj = 1;
          t.ni = br.secs[rp].dim;
          t.nj = S.dl[l];
          t.t0 = (int)P.wr.terms.size();
          for (int b = 0; b < DHr; ++b)
            for (int s = 0; s < 16; ++s) {
              double w = Wsup(W, a, sp, s, b);
              if (w == 0.0 && Wsup(Wp, a, sp, s, b) == 0.0) continue;
              int gg = G.group_of[s];
              int c = S.rsec[l][gg];
              if (c < 0) continue;   // the ket block (l, s) -> c is absent from the truncated bond
              TT_REQUIRE(rowbaseY[c][b] >= 0, TT_EINVAL, "plan: MPO entry breaks charge conservation");
              TT_REQUIRE(br.find(addq(br.secs[c].q, qHr[b])) == rp, TT_EINVAL, "plan: inconsistent charges");
              WTerm tm;
              tm.src = ybase[c] + (long long)rowbaseY[c][b] * ycols[c] + colposY[l][gg] + G.pos_of[s];
              tm.ssi = ycols[c];
              tm.ssj = (long long)G.s[gg].size();
              tm.w = w;
              P.wr.terms.push_back(tm);
              P.wr.widx.push_back(widx(a, sp, s, b));
            }
          t.nt = (int)P.wr.terms.size() - t.t0;
          P.wr.flops += 2.0 * t.nt * (double)t.ni * t.nj;
          P.wr.tasks.push_back(t);
        }
      }
    }
  // final: R_k[p] = A_p . Z_p
  for (int p = 0; p < S.nl; ++p) {
    GemmProb g = gp(S.dl[p], EL.K[p], S.C[p], 0, 1, 2);
    g.offA = S.base[p]; g.sam = S.C[p]; g.sak = 1;
    g.offB = zbase[p]; g.sbk = EL.K[p]; g.sbn = 1;
    g.offC = EL.base[p]; g.scm = EL.K[p];
    add_prob(P.r3, g);
  }

  // ---------------- LQ per left sector (right-to-left gauge move), absorb from the left
  {
    BondMatLayout bm = make_bondmat_layout(bl);
    for (int l = 0; l < S.nl; ++l) {
      QRTask q{};
      q.m = S.C[l]; q.n = S.dl[l]; q.trans = 1;
      q.rbase = S.base[l]; q.rs = 1; q.cs = S.C[l]; q.rtab = -1;
      q.sdst = bm.off[l];
      q.ws = P.lq.ws_size;
      P.lq.ws_size += 2LL * q.m * q.n;
      P.lq.tasks.push_back(q);
      GemmProb ab = gp(S.dl[l], S.C[l], S.dl[l], 0, 1, 2);
      ab.offA = bm.off[l]; ab.sam = S.dl[l]; ab.sak = 1;
      ab.offB = S.base[l]; ab.sbk = S.C[l]; ab.sbn = 1;
      ab.offC = S.base[l]; ab.scm = S.C[l];
      add_prob(P.absL, ab);
    }
    // ---------------- bond effective Hamiltonian on the left bond k
    // U[(a,x)][y] = L[x,a,q-block] . S_q written in environment layout; out_p = U_p . R_p^T
    for (int q = 0; q < (int)bl.secs.size(); ++q) {
      std::vector<long long> rows;
      for (int a = 0; a < DHl; ++a) {
        int p = bl.find(addq(bl.secs[q].q, qHl[a]));
        if (p < 0 || EL.csec[p][a] != q) continue;
        for (int x = 0; x < EL.dp[p]; ++x) rows.push_back(EL.base[p] + (long long)x * EL.K[p] + EL.colb[p][a]);
      }
      if (rows.empty()) continue;
      long long tab = tabs.add(rows);
      GemmProb g = gp((int)rows.size(), bl.secs[q].dim, bl.secs[q].dim, 0, 1, 2);
      g.tam = tab; g.sak = 1;
      g.offB = bm.off[q]; g.sbk = bl.secs[q].dim; g.sbn = 1;
      g.tcm = tab;
      add_prob(P.b1, g);
    }
    P.u_size = EL.size;
    for (int p = 0; p < EL.np; ++p) {
      GemmProb g = gp(EL.dp[p], EL.dp[p], EL.K[p], 0, 1, 2);
      g.offA = EL.base[p]; g.sam = EL.K[p]; g.sak = 1;
      g.offB = EL.base[p]; g.sbk = 1; g.sbn = EL.K[p];
      g.offC = bm.off[p]; g.scm = EL.dp[p];
      add_prob(P.b2, g);
    }
    // the same apply as one fused launch: out_p = sum_a (L^a_p S_q) (R^a_p)^T
    // with q = p - qH(a), one b block per a with the single term L^a_p . S_q
    // (slots: 0 = L env, 1 = S, 2 = R env, 3 = output S)
    FzPlan& F = P.fzb;
    F = FzPlan();
    for (int p = 0; p < EL.np; ++p) {
      FzOut o;
      o.out = bm.off[p]; o.ldo = EL.dp[p]; o.dp = o.dr = EL.dp[p];
      o.rrow = EL.base[p]; o.ldr = EL.K[p];
      o.b0 = (int)F.bs.size(); o.nb = 0;
      for (int a = 0; a < DHl; ++a) {
        const int q = EL.csec[p][a];
        if (q < 0) continue;
        const int dq = bl.secs[q].dim;
        FzB fb;
        fb.rcol = EL.colb[p][a]; fb.dc = dq; fb.t0 = (int)F.terms.size(); fb.nt = 1; fb.pad = 0;
        FzT t;
        t.lw = EL.base[p] + EL.colb[p][a]; t.ldlw = EL.K[p];
        t.a = bm.off[q]; t.lda = dq; t.dl = dq; t.pad = 0;
        F.terms.push_back(t);
        F.bs.push_back(fb);
        ++o.nb;
        F.flops += 2.0 * o.dp * (double)dq * dq + 2.0 * o.dp * (double)dq * o.dr;
        F.bytes += 8.0 * ((double)o.dp * dq + (double)dq * dq + (double)o.dr * dq);
      }
      F.bytes += 8.0 * (double)o.dp * o.dr;
      F.outs.push_back(o);
    }
    plan_fz_jobs(F);
  }
  finish_wplan(P.w2);
  finish_wplan(P.wr);
  finish_qrplan(P.qr);
  finish_qrplan(P.lq);
  // ---------------- trace transfer: the group with zero charge holds the diagonal s = (sigma, sigma)
  const int g0 = G.group_of[0];
  for (int l = 0; l < S.nl; ++l) {
    int r = S.rsec[l][g0];
    if (r < 0) continue;
    P.tr.push_back({S.base[l] + S.colb[l][g0], (long long)S.C[l], (long long)l, (long long)r});
  }
  return P;
}

// ---------------------------------------------------------------- 2-TDVP
// The two-site step of SM Sec. "2-TDVP in the initial stage" (Eq. S-2TDVP) in
// charge blocks: Theta = A_k A_{k+1}, then H^(2) Theta contracted as L.Theta,
// the MPO of site k, the MPO of site k+1, then .R (the order of SM Fig.
// Lanczos with one more W stage), and the SVD tasks of the split.
PairPlan build_pair_plan(const Bond& bl, const Bond& bm, const Bond& br, const Groups& G,
                         const std::vector<Q>& qHl, const std::vector<Q>& qHm, const std::vector<Q>& qHr,
                         const std::vector<double>& W1, const std::vector<double>& W2,
                         const SiteLayout& SA, const SiteLayout& SB, SiteTables& tabs) {
  PairPlan P;
  PairLayout& L = P.L;
  const int DHl = (int)qHl.size(), DHm = (int)qHm.size(), DHr = (int)qHr.size();
  const EnvLayout EL = make_env_layout(bl, qHl), ER = make_env_layout(br, qHr);
  // columns of a middle charge: (g2, s2, y) for every g2 that reaches the right bond
  auto width = [&](const Q& m) -> long long {
    auto it = L.width.find(m);
    if (it != L.width.end()) return it->second;
    std::vector<MidBlock> v;
    long long off = 0;
    for (int g2 = 0; g2 < G.ng; ++g2) {
      const int r = br.find(addq(m, G.delta[g2]));
      if (r < 0) continue;
      v.push_back({g2, r, off});
      off += (long long)G.s[g2].size() * br.secs[r].dim;
    }
    L.mid[m] = v;
    L.width[m] = off;
    return off;
  };
  auto midblock = [&](const Q& m, int g2) -> const MidBlock* {
    for (const MidBlock& b : L.mid.at(m))
      if (b.g2 == g2) return &b;
    return nullptr;
  };
  // ket-only MPO entry W[a, so, si, b] between super indices (the ancilla is unchanged)
  auto wsup = [](const std::vector<double>& W, int DHo, int a, int sout, int sin, int b) -> double {
    if ((sout & 3) != (sin & 3)) return 0.0;
    return W[(size_t)((((long long)a * 4 + (sout >> 2)) * 4 + (sin >> 2)) * DHo + b)];
  };

  // ---------------- layout of Theta
  L.nl = (int)bl.secs.size();
  L.dl.resize(L.nl);
  L.C.resize(L.nl);
  L.base.resize(L.nl);
  L.colg.resize(L.nl);
  long long pos = 0;
  for (int l = 0; l < L.nl; ++l) {
    L.dl[l] = bl.secs[l].dim;
    L.colg[l].fill(-1);
    long long c = 0;
    for (int g1 = 0; g1 < G.ng; ++g1) {
      const long long w = width(addq(bl.secs[l].q, G.delta[g1]));
      if (w == 0) continue;
      L.colg[l][g1] = c;
      c += (long long)G.s[g1].size() * w;
    }
    L.C[l] = c;
    L.base[l] = pos;
    pos += (long long)L.dl[l] * c;
  }
  L.size = pos;
  // column of (s1, s2, y = 0) in the row block of l
  auto tcol = [&](int l, int s1, int s2) -> long long {
    const int g1 = G.group_of[s1];
    const Q m = addq(bl.secs[l].q, G.delta[g1]);
    const MidBlock* b = midblock(m, G.group_of[s2]);
    TT_REQUIRE(L.colg[l][g1] >= 0 && b, TT_EINVAL, "pair plan: no such block");
    return L.colg[l][g1] + (long long)G.pos_of[s1] * L.w(m) + b->off +
           (long long)G.pos_of[s2] * br.secs[b->r].dim;
  };
  P.join.tag = TAG_ABSORB;
  P.s1.tag = TAG_LA;
  P.s4.tag = TAG_R;

  // ---------------- join: Theta(l; s1, :) = A_k(l; s1, mu) . A_{k+1}(m; mu, :)
  for (int l = 0; l < L.nl; ++l)
    for (int g1 = 0; g1 < G.ng; ++g1) {
      const int mi = SA.rsec[l][g1];
      if (mi < 0) continue;
      TT_REQUIRE(L.colg[l][g1] >= 0 && bm.secs[mi].q == addq(bl.secs[l].q, G.delta[g1]), TT_EINVAL,
                 "pair plan: inconsistent middle bond");
      const long long w = L.w(bm.secs[mi].q);
      TT_REQUIRE(SB.C[mi] == w, TT_EINVAL, "pair plan: right site columns differ from the two-site layout");
      const int dm = bm.secs[mi].dim;
      for (int p1 = 0; p1 < (int)G.s[g1].size(); ++p1) {
        GemmProb g = gp(L.dl[l], (int)w, dm, 0, 1, 2);
        g.offA = SA.base[l] + SA.colb[l][g1] + (long long)p1 * dm; g.sam = SA.C[l]; g.sak = 1;
        g.offB = SB.base[mi]; g.sbk = SB.C[mi]; g.sbn = 1;
        g.offC = L.base[l] + L.colg[l][g1] + (long long)p1 * w; g.scm = L.C[l];
        add_prob(P.join, g);
      }
    }

  // ---------------- s1: T1_l[(a, x')][cols of Theta_l] = L^a . Theta_l
  std::vector<long long> t1base(L.nl, 0);
  std::vector<std::vector<int>> rowbase1(L.nl, std::vector<int>(DHl, -1));
  pos = 0;
  for (int l = 0; l < L.nl; ++l) {
    std::vector<long long> rows;
    for (int a = 0; a < DHl; ++a) {
      const int p = bl.find(addq(bl.secs[l].q, qHl[a]));
      if (p < 0 || EL.csec[p][a] != l) continue;
      rowbase1[l][a] = (int)rows.size();
      for (int x = 0; x < EL.dp[p]; ++x) rows.push_back(EL.base[p] + (long long)x * EL.K[p] + EL.colb[p][a]);
    }
    t1base[l] = pos;
    if (rows.empty() || L.C[l] == 0) continue;
    GemmProb g = gp((int)rows.size(), (int)L.C[l], L.dl[l], 0, 1, 2);
    g.tam = tabs.add(rows); g.sak = 1;
    g.offB = L.base[l]; g.sbk = L.C[l]; g.sbn = 1;
    g.offC = pos; g.scm = L.C[l];
    add_prob(P.s1, g);
    pos += (long long)rows.size() * L.C[l];
  }
  P.t1_size = pos;

  // ---------------- w1: T2_p[x'][(s1', b, cols of m)] = sum W_k[a, so1, si1, b] T1,
  // m = p - qH(b) + Delta(s1') the (unchanged) middle ket charge
  std::vector<long long> t2base(L.nl, 0), K2(L.nl, 0);
  std::vector<long long> col2((size_t)L.nl * 16 * DHm, -1);
  auto c2 = [&](int p, int s1, int b) -> long long& { return col2[((size_t)p * 16 + s1) * DHm + b]; };
  auto mid_of = [&](int p, int s1, int b) { return addq(subq(bl.secs[p].q, qHm[b]), G.delta[G.group_of[s1]]); };
  pos = 0;
  for (int p = 0; p < L.nl; ++p) {
    long long c = 0;
    for (int g1 = 0; g1 < G.ng; ++g1)
      for (int s1 : G.s[g1])
        for (int b = 0; b < DHm; ++b) {
          const long long w = width(mid_of(p, s1, b));
          if (w == 0) continue;
          c2(p, s1, b) = c;
          c += w;
        }
    K2[p] = c;
    t2base[p] = pos;
    pos += (long long)L.dl[p] * c;
  }
  P.t2_size = pos;
  for (int p = 0; p < L.nl; ++p)
    for (int g1 = 0; g1 < G.ng; ++g1)
      for (int so : G.s[g1])
        for (int b = 0; b < DHm; ++b) {
          if (c2(p, so, b) < 0) continue;
          const Q m = mid_of(p, so, b);
          WTask t;
          t.dst = t2base[p] + c2(p, so, b);
          t.dsi = K2[p];
          t.dsj = 1;
          t.ni = L.dl[p];
          t.nj = (int)L.w(m);
          t.t0 = (int)P.w1.terms.size();
          for (int a = 0; a < DHl; ++a) {
            const int l = EL.csec[p][a];
            if (l < 0) continue;
            for (int si = (so & 3); si < 16; si += 4) {
              const double w = wsup(W1, DHm, a, so, si, b);
              if (w == 0.0) continue;
              const int gi = G.group_of[si];
              TT_REQUIRE(addq(bl.secs[l].q, G.delta[gi]) == m && L.colg[l][gi] >= 0 && rowbase1[l][a] >= 0,
                         TT_EINVAL, "pair plan: MPO entry breaks charge conservation (site k)");
              WTerm tm;
              tm.src = t1base[l] + (long long)rowbase1[l][a] * L.C[l] + L.colg[l][gi] + (long long)G.pos_of[si] * L.w(m);
              tm.ssi = L.C[l];
              tm.ssj = 1;
              tm.w = w;
              P.w1.terms.push_back(tm);
            }
          }
          t.nt = (int)P.w1.terms.size() - t.t0;
          P.w1.flops += 2.0 * t.nt * (double)t.ni * t.nj;
          P.w1.tasks.push_back(t);
        }

  // ---------------- w2: T3 grouped by the right bra sector r', rows (p, s1', s2', x'),
  // columns (c, y) as in R's row block r'
  const int nr = (int)br.secs.size();
  struct Row3 { int p, s1, s2; long long row; };
  std::vector<std::vector<Row3>> rows3(nr);
  std::vector<long long> t3base(nr, 0), nrows3(nr, 0);
  for (int p = 0; p < L.nl; ++p)
    for (int g1 = 0; g1 < G.ng; ++g1) {
      if (L.colg[p][g1] < 0) continue;
      const Q m = addq(bl.secs[p].q, G.delta[g1]);
      for (int s1 : G.s[g1])
        for (const MidBlock& mb : L.mid.at(m))
          for (int s2 : G.s[mb.g2]) {
            rows3[mb.r].push_back({p, s1, s2, nrows3[mb.r]});
            nrows3[mb.r] += L.dl[p];
          }
    }
  pos = 0;
  for (int r = 0; r < nr; ++r) {
    t3base[r] = pos;
    pos += nrows3[r] * ER.K[r];
  }
  P.t3_size = pos;
  for (int r = 0; r < nr; ++r)
    for (const Row3& rw : rows3[r]) {
      const int so2 = rw.s2;
      for (int c = 0; c < DHr; ++c) {
        const int ry = ER.csec[r][c];
        if (ry < 0) continue;
        WTask t;
        t.dst = t3base[r] + rw.row * ER.K[r] + ER.colb[r][c];
        t.dsi = ER.K[r];
        t.dsj = 1;
        t.ni = L.dl[rw.p];
        t.nj = br.secs[ry].dim;
        t.t0 = (int)P.w2.terms.size();
        for (int b = 0; b < DHm; ++b) {
          if (c2(rw.p, rw.s1, b) < 0) continue;
          const Q m = mid_of(rw.p, rw.s1, b);
          for (int si = (so2 & 3); si < 16; si += 4) {
            const double w = wsup(W2, DHr, b, so2, si, c);
            if (w == 0.0) continue;
            const MidBlock* mb = midblock(m, G.group_of[si]);
            if (!mb) continue;   // the ket block (m, s2) does not reach the right bond
            TT_REQUIRE(mb->r == ry, TT_EINVAL, "pair plan: MPO entry breaks charge conservation (site k+1)");
            WTerm tm;
            tm.src = t2base[rw.p] + c2(rw.p, rw.s1, b) + mb->off + (long long)G.pos_of[si] * br.secs[ry].dim;
            tm.ssi = K2[rw.p];
            tm.ssj = 1;
            tm.w = w;
            P.w2.terms.push_back(tm);
          }
        }
        t.nt = (int)P.w2.terms.size() - t.t0;
        P.w2.flops += 2.0 * t.nt * (double)t.ni * t.nj;
        P.w2.tasks.push_back(t);
      }
    }

  // ---------------- s4: out rows (p, s1', s2', x') = T3_r' . R_r'^T
  for (int r = 0; r < nr; ++r) {
    if (nrows3[r] == 0) continue;
    std::vector<long long> crow;
    crow.reserve((size_t)nrows3[r]);
    for (const Row3& rw : rows3[r]) {
      const long long col = tcol(rw.p, rw.s1, rw.s2);
      for (int x = 0; x < L.dl[rw.p]; ++x) crow.push_back(L.base[rw.p] + (long long)x * L.C[rw.p] + col);
    }
    GemmProb g = gp((int)nrows3[r], br.secs[r].dim, (int)ER.K[r], 0, 1, 2);
    g.offA = t3base[r]; g.sam = ER.K[r]; g.sak = 1;
    g.offB = ER.base[r]; g.sbk = 1; g.sbn = ER.K[r];
    g.tcm = tabs.add(crow);
    add_prob(P.s4, g);
  }

  // ---------------- split: one task per middle charge
  for (const auto& kv : L.width) {
    const Q& m = kv.first;
    const long long w = kv.second;
    if (w == 0) continue;
    std::vector<std::array<int, 3>> rg;
    std::vector<long long> rows;
    for (int l = 0; l < L.nl; ++l)
      for (int g1 = 0; g1 < G.ng; ++g1) {
        if (L.colg[l][g1] < 0 || addq(bl.secs[l].q, G.delta[g1]) != m) continue;
        for (int p1 = 0; p1 < (int)G.s[g1].size(); ++p1) {
          rg.push_back({l, g1, p1});
          for (int x = 0; x < L.dl[l]; ++x)
            rows.push_back(L.base[l] + (long long)x * L.C[l] + L.colg[l][g1] + (long long)p1 * w);
        }
      }
    if (rows.empty()) continue;
    TT_REQUIRE(rows.size() < (1u << 30) && w < (1LL << 30), TT_EINVAL, "pair plan: split block too large");
    SvdTask t;
    t.R = (int)rows.size();
    t.w = (int)w;
    t.rtab = tabs.add(rows);
    t.ws = P.svd_ws;
    t.sig = P.svd_nsig;
    const long long mn = std::min<long long>(t.R, t.w), mx = std::max<long long>(t.R, t.w);
    P.svd_ws += mx * mn + mn * mn;
    P.svd_nsig += mn;
    P.svd.push_back(t);
    P.mq.push_back(m);
    P.rowgroups.push_back(rg);
  }
  finish_wplan(P.w1);
  finish_wplan(P.w2);
  P.join.no_split = P.s1.no_split = P.s4.no_split = true;
  P.join.wave_ok = P.s1.wave_ok = P.s4.wave_ok = true;
  return P;
}

}  // namespace tt
