// Model builder: lattice and snake order, the finite-state-machine MPO of the
// Hubbard Hamiltonian, U(1)xU(1) bond sectors and the padding noise.
//
// Paper: Eq. (3) (Hubbard model), main-text Hubbard paragraph (cylinders
// periodic across the width, open squares), Fig. 1a (snake path down one
// column, across at the bottom, up the next).  The MPO construction itself is
// only cited by the paper; the bond-state convention below is shared with
// every other builder of this MPO so that padded tensors coincide:
//   bond 0: [start]; bond N: [start, done]; ks = N/2;
//   0 < k <= ks: [start, src(i,type) for pending sources i ascending, done]
//   ks < k < N : [start, dst(j,type) for pending destinations j ascending, done]
// type in (c+_up P, c+_dn P, P c_up, P c_dn).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <set>

#include "tt_internal.h"

namespace tt {

Lattice make_lattice(int W, int L, int geometry) {
  TT_REQUIRE(W >= 1 && L >= 1, TT_EINVAL, "lattice: W and L must be positive");
  TT_REQUIRE(geometry >= 0 && geometry <= 2, TT_EINVAL, "lattice: unknown geometry");
  TT_REQUIRE(geometry != TT_CHAIN || W == 1, TT_EINVAL, "lattice: a chain has W = 1");
  Lattice lat{W, L, geometry, W * L, {}};
  TT_REQUIRE(lat.N >= 2, TT_EINVAL, "lattice: need at least two sites");
  // snake: column x top-down (y = W-1..0) when x is even, bottom-up when odd
  std::vector<int> idx(W * L);
  int n = 0;
  for (int x = 0; x < L; ++x)
    for (int r = 0; r < W; ++r) {
      int y = (x % 2 == 0) ? (W - 1 - r) : r;
      idx[x * W + y] = n++;
    }
  std::set<std::pair<int, int>> e;
  auto add = [&](int a, int b) { e.insert({std::min(a, b), std::max(a, b)}); };
  for (int x = 0; x < L; ++x)
    for (int y = 0; y < W; ++y) {
      int me = idx[x * W + y];
      if (x + 1 < L) add(me, idx[(x + 1) * W + y]);
      if (y + 1 < W) add(me, idx[x * W + y + 1]);
      else if (geometry == TT_CYLINDER && W >= 3) add(me, idx[x * W + 0]);
    }
  lat.bonds.assign(e.begin(), e.end());
  return lat;
}

// local operators in the basis {0, up, dn, updn}, |updn> = c+_up c+_dn |0>
namespace {
struct M4 { double v[4][4]; };
M4 zero4() { M4 m{}; return m; }
M4 mul(const M4& a, const M4& b) {
  M4 r = zero4();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 4; ++k) r.v[i][j] += a.v[i][k] * b.v[k][j];
  return r;
}
M4 transpose(const M4& a) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.v[i][j] = a.v[j][i];
  return r;
}
struct LocalOps {
  M4 id, par, cdu, cdd, cu, cd, onsite;
  M4 left[4], right[4];
  M4 pleft[4], pright[4];   // pairing channels: (a P)_i ... b_j
};
LocalOps local_ops(double U, double mu) {
  LocalOps o;
  o.id = zero4(); o.par = zero4(); o.cdu = zero4(); o.cdd = zero4(); o.onsite = zero4();
  for (int i = 0; i < 4; ++i) o.id.v[i][i] = 1.0;
  o.par.v[0][0] = 1; o.par.v[1][1] = -1; o.par.v[2][2] = -1; o.par.v[3][3] = 1;
  o.cdu.v[1][0] = 1; o.cdu.v[3][2] = 1;       // c+_up
  o.cdd.v[2][0] = 1; o.cdd.v[3][1] = -1;      // c+_dn (passes the up mode)
  o.cu = transpose(o.cdu);
  o.cd = transpose(o.cdd);
  for (int s = 0; s < 4; ++s) {
    int nu = s & 1, nd = s >> 1;
    o.onsite.v[s][s] = U * nu * nd - mu * (nu + nd);
  }
  // c+_i c_j = (c+ P)_i P... (c)_j ;  c+_j c_i = (P c)_i P... (c+)_j
  o.left[0] = mul(o.cdu, o.par); o.right[0] = o.cu;
  o.left[1] = mul(o.cdd, o.par); o.right[1] = o.cd;
  o.left[2] = mul(o.par, o.cu);  o.right[2] = o.cdu;
  o.left[3] = mul(o.par, o.cd);  o.right[3] = o.cdd;
  // pairing: c_i,dn c_j,up, c_i,up c_j,dn, c+_i,dn c+_j,up, c+_i,up c+_j,dn
  o.pleft[0] = mul(o.cd, o.par);  o.pright[0] = o.cu;
  o.pleft[1] = mul(o.cu, o.par);  o.pright[1] = o.cd;
  o.pleft[2] = mul(o.cdd, o.par); o.pright[2] = o.cdu;
  o.pleft[3] = mul(o.cdu, o.par); o.pright[3] = o.cdd;
  return o;
}
// signs of the pairing channels in
// c_i,dn c_j,up - c_i,up c_j,dn - c+_i,dn c+_j,up + c+_i,up c+_j,dn
const double kPairSign[4] = {1.0, -1.0, -1.0, 1.0};
// channel charges: the hopping channels 0..3 (c+_up, c+_dn, c_up, c_dn at the
// source), the spin channels 4..6 (Sz, S+, S- at the source), the pairing
// channels 7..10 (c_dn, c_up, c+_dn, c+_up at the source)
const Q kChannelQ[11] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}, {0, 0}, {1, -1}, {-1, 1},
                         {0, -1}, {-1, 0}, {0, 1}, {1, 0}};
}  // namespace

Q Mpo::charge(int k, int a) const {
  const MpoState& s = states[k][a];
  if (s.kind < 2) return {0, 0};
  return kChannelQ[s.type];
}

std::vector<std::pair<std::pair<int, int>, double>> pairing_bonds(const Lattice& lat) {
  std::vector<std::pair<std::pair<int, int>, double>> out;
  for (auto& b : lat.bonds) {
    const int xi = b.first / lat.W, xj = b.second / lat.W;   // column along the length
    out.push_back({b, xi != xj ? 1.0 : -1.0});
  }
  return out;
}

Mpo make_hubbard_mpo(const Lattice& lat, double t, double tp, double U, double mu, double hp) {
  const int N = lat.N;
  Mpo m;
  m.N = N;
  // hopping amplitude of every coupled pair (i < j): t on nearest neighbours,
  // tp on next-nearest (diagonal) neighbours when tp != 0 (SM Eq. S1)
  std::map<std::pair<int, int>, double> hop, pair;
  for (auto& b : lat.bonds) hop[b] = t;
  if (tp != 0.0)
    for (auto& b : pairs_at_distance(lat, 2)) hop[b] = tp;
  // pairing field -hp Delta_tot: amplitude -hp s_ij / (2 sqrt 2) per bond
  if (hp != 0.0)
    for (auto& b : pairing_bonds(lat)) pair[b.first] = -hp * b.second / (2.0 * std::sqrt(2.0));
  std::vector<int> types = {0, 1, 2, 3};
  if (hp != 0.0) types.insert(types.end(), {7, 8, 9, 10});
  // amplitude of channel type ty between i < j (with the channel's sign)
  auto coef = [&](int i, int j, int ty) {
    const std::pair<int, int> key{std::min(i, j), std::max(i, j)};
    if (ty < 4) {
      auto it = hop.find(key);
      return it == hop.end() ? 0.0 : -it->second;
    }
    auto it = pair.find(key);
    return it == pair.end() ? 0.0 : it->second * kPairSign[ty - 7];
  };
  std::vector<std::set<int>> later(N), earlier(N);   // coupled sites j > i, i < j
  for (auto* mp : {&hop, &pair})
    for (auto& kv : *mp) {
      later[kv.first.first].insert(kv.first.second);
      earlier[kv.first.second].insert(kv.first.first);
    }
  const int ks = N / 2;
  m.states.resize(N + 1);
  m.states[0] = {{0, -1, -1}};
  m.states[N] = {{0, -1, -1}, {1, -1, -1}};
  for (int k = 1; k < N; ++k) {
    auto& st = m.states[k];
    st.push_back({0, -1, -1});
    if (k <= ks) {
      for (int i = 0; i < k; ++i) {
        bool pending = !later[i].empty() && *later[i].rbegin() >= k;
        if (pending)
          for (int ty : types) st.push_back({2, i, ty});
      }
    } else {
      for (int j = k; j < N; ++j) {
        bool pending = !earlier[j].empty() && *earlier[j].begin() < k;
        if (pending)
          for (int ty : types) st.push_back({3, j, ty});
      }
    }
    st.push_back({1, -1, -1});
  }
  for (int k = 0; k <= N; ++k) m.DH.push_back((int)m.states[k].size());
  LocalOps o = local_ops(U, mu);
  auto left = [&](int ty) -> const M4& { return ty < 4 ? o.left[ty] : o.pleft[ty - 7]; };
  auto right = [&](int ty) -> const M4& { return ty < 4 ? o.right[ty] : o.pright[ty - 7]; };
  m.W.resize(N);
  for (int k = 0; k < N; ++k) {
    const auto& Ls = m.states[k];
    const auto& Rs = m.states[k + 1];
    int DL = (int)Ls.size(), DR = (int)Rs.size();
    std::vector<double> Wk((size_t)DL * 16 * DR, 0.0);
    auto find = [&](int kind, int site, int type) {
      for (int b = 0; b < DR; ++b)
        if (Rs[b].kind == kind && (kind < 2 || (Rs[b].site == site && Rs[b].type == type))) return b;
      return -1;
    };
    auto put = [&](int a, int b, const M4& op, double c) {
      for (int so = 0; so < 4; ++so)
        for (int si = 0; si < 4; ++si)
          Wk[(((size_t)a * 4 + so) * 4 + si) * DR + b] += c * op.v[so][si];
    };
    int bstart = find(0, -1, -1), bdone = find(1, -1, -1);
    for (int a = 0; a < DL; ++a) {
      const MpoState& s = Ls[a];
      if (s.kind == 0) {
        put(a, bstart, o.id, 1.0);
        if (bdone >= 0) put(a, bdone, o.onsite, 1.0);
        for (int ty : types) {
          int b = find(2, k, ty);
          if (b >= 0) put(a, b, left(ty), 1.0);
          for (int j : later[k]) {
            int bd = find(3, j, ty);
            if (bd >= 0) put(a, bd, left(ty), coef(k, j, ty));
          }
        }
      } else if (s.kind == 1) {
        put(a, bdone, o.id, 1.0);
      } else if (s.kind == 2) {
        int b = find(2, s.site, s.type);
        if (b >= 0) put(a, b, o.par, 1.0);
        for (int j : later[s.site]) {
          if (j <= k) continue;
          int bd = find(3, j, s.type);
          if (bd >= 0) put(a, bd, o.par, coef(s.site, j, s.type));
        }
        if (later[s.site].count(k)) put(a, bdone, right(s.type), coef(s.site, k, s.type));
      } else {
        if (s.site == k) {
          put(a, bdone, right(s.type), 1.0);
        } else {
          int b = find(3, s.site, s.type);
          TT_REQUIRE(b >= 0, TT_EINVAL, "mpo: lost destination channel");
          put(a, b, o.par, 1.0);
        }
      }
    }
    m.W[k] = std::move(Wk);
  }
  return m;
}

Q project_charge(Q q, int mode) {
  if (mode == 0) return {0, 0};
  if (mode == 2) return {q.first - q.second, 0};
  return q;
}

Groups make_groups(int mode) {
  Groups g;
  g.group_of.assign(16, 0);
  g.pos_of.assign(16, 0);
  if (mode == 2) {   // Sz only: five groups by the super charge du - dd
    g.ng = 5;
    for (int sz = -2; sz <= 2; ++sz) g.delta.push_back({sz, 0});
    g.s.resize(5);
    for (int s = 0; s < 16; ++s) {
      int sig = s / 4, sp = s % 4;
      int du = (sig & 1) - (sp & 1), dd = (sig >> 1) - (sp >> 1);
      int gi = du - dd + 2;
      g.group_of[s] = gi;
      g.pos_of[s] = (int)g.s[gi].size();
      g.s[gi].push_back(s);
    }
    return g;
  }
  if (mode == 0) {
    g.ng = 1;
    g.delta = {{0, 0}};
    g.s.resize(1);
    for (int s = 0; s < 16; ++s) { g.s[0].push_back(s); g.pos_of[s] = s; }
    return g;
  }
  g.ng = 9;
  for (int du = -1; du <= 1; ++du)
    for (int dd = -1; dd <= 1; ++dd) g.delta.push_back({du, dd});
  g.s.resize(9);
  for (int s = 0; s < 16; ++s) {
    int sig = s / 4, sp = s % 4;
    int du = (sig & 1) - (sp & 1), dd = (sig >> 1) - (sp >> 1);
    int gi = (du + 1) * 3 + (dd + 1);
    g.group_of[s] = gi;
    g.pos_of[s] = (int)g.s[gi].size();
    g.s[gi].push_back(s);
  }
  return g;
}

uint64_t splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double noise_uniform(uint64_t seed, int site, uint64_t flat) {
  uint64_t n = (uint64_t)site * (1ULL << 40) + flat + 1ULL;
  uint64_t z = splitmix64(seed + n * 0x9E3779B97F4A7C15ULL);
  double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u - 1.0;
}

namespace {
using u128 = unsigned __int128;
const u128 kSat = ((u128)1) << 120;
u128 sat_mul(u128 a, u128 b) {
  if (a == 0 || b == 0) return 0;
  if (a >= kSat || b >= kSat) return kSat;
  if (a > kSat / b) return kSat;
  u128 r = a * b;
  return r > kSat ? kSat : r;
}
// binomial C(n, k) saturated at 2^120 (Pascal's triangle, cached)
u128 binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  static std::vector<std::vector<u128>> tri;
  while ((int)tri.size() <= n) {
    int r = (int)tri.size();
    std::vector<u128> row(r + 1, 1);
    for (int i = 1; i < r; ++i) {
      u128 v = tri[r - 1][i - 1] + tri[r - 1][i];
      row[i] = v > kSat ? kSat : v;
    }
    tri.push_back(std::move(row));
  }
  return tri[n][k];
}
u128 count_side(int n, Q q) {
  if (std::abs(q.first) > n || std::abs(q.second) > n) return 0;
  return sat_mul(binom(2 * n, n + q.first), binom(2 * n, n + q.second));
}
}  // namespace

std::vector<std::map<Q, int>> allocate_sectors(int N, int D, const std::vector<std::map<Q, int>>& n0,
                                               int sector_cap, int mode) {
  std::vector<std::map<Q, int>> dims(N + 1);
  dims[0][{0, 0}] = 1;
  dims[N][{0, 0}] = 1;
  const bool sz = mode == 2;
  std::vector<Q> sc;  // the 16 local super-index charges
  for (int s = 0; s < 16; ++s) {
    int sig = s / 4, sp = s % 4;
    sc.push_back(project_charge({(sig & 1) - (sp & 1), (sig >> 1) - (sp >> 1)}, mode));
  }
  // super states of charge q on n sites: comb(2n, n + a) comb(2n, n + b), or
  // comb(4n, 2n + a) with the Sz charge alone
  auto count = [&](int n, Q q) -> u128 {
    if (!sz) return count_side(n, q);
    return std::abs(q.first) > 2 * n ? 0 : binom(4 * n, 2 * n + q.first);
  };
  for (int k = 1; k < N; ++k) {
    int h = std::min(k, N - k);
    std::vector<Q> qs;
    if (sz) {
      for (int a = -2 * h; a <= 2 * h; ++a) qs.push_back({a, 0});
    } else {
      for (int a = -h; a <= h; ++a)
        for (int b = -h; b <= h; ++b) qs.push_back({a, b});
    }
    std::map<Q, u128> dmax;
    u128 tot = 0;
    for (auto q : qs) {
      u128 v = std::min(count(k, q), count(N - k, q));
      dmax[q] = v;
      tot = tot + v;
      if (tot > kSat) tot = kSat;
    }
    std::map<Q, int> d;
    if (tot <= (u128)D) {
      for (auto q : qs) d[q] = (int)dmax[q];
    } else {
      int hw = std::min(h, 14);
      std::map<Q, u128> w, cap;
      for (auto q : qs) {
        u128 v = 0;
        if (sz) {
          if (std::abs(q.first) <= 2 * hw) v = binom(4 * hw, 2 * hw + q.first);
        } else if (std::abs(q.first) <= hw && std::abs(q.second) <= hw) {
          v = binom(2 * hw, hw + q.first) * binom(2 * hw, hw + q.second);
        }
        w[q] = v;
        cap[q] = (sector_cap <= 0) ? dmax[q] : std::min(dmax[q], (u128)sector_cap);
      }
      // largest-remainder split of D over the free sectors; sectors above their
      // cap are fixed at the cap and the remainder is split again
      std::map<Q, long long> fixed, base;
      while (true) {
        long long Dfree = D;
        for (auto& kv : fixed) Dfree -= kv.second;
        std::vector<Q> freeq;
        u128 wt = 0;
        for (auto q : qs)
          if (!fixed.count(q)) { freeq.push_back(q); wt += w[q]; }
        base.clear();
        if (wt == 0 || Dfree <= 0) {
          for (auto q : freeq) base[q] = 0;
        } else {
          std::vector<std::pair<u128, Q>> rem;
          long long used = 0;
          for (auto q : freeq) {
            u128 num = (u128)Dfree * w[q];
            base[q] = (long long)(num / wt);
            used += base[q];
            rem.push_back({num % wt, q});
          }
          std::sort(rem.begin(), rem.end(), [](const std::pair<u128, Q>& x, const std::pair<u128, Q>& y) {
            if (x.first != y.first) return x.first > y.first;
            return x.second < y.second;
          });
          long long left = Dfree - used;
          for (long long i = 0; i < left && i < (long long)rem.size(); ++i) base[rem[i].second] += 1;
        }
        bool over = false;
        for (auto q : freeq)
          if ((u128)base[q] > cap[q]) { fixed[q] = (long long)cap[q]; over = true; }
        if (!over) break;
      }
      for (auto& kv : fixed) base[kv.first] = kv.second;
      for (auto q : qs) {
        long long v = base[q];
        auto it = n0[k].find(q);
        if (it != n0[k].end()) v = std::max<long long>(v, it->second);
        if ((u128)v > dmax[q]) v = (long long)dmax[q];
        d[q] = (int)v;
      }
    }
    for (auto& kv : d)
      if (kv.second > 0) dims[k][kv.first] = kv.second;
  }
  bool changed = true;
  auto get = [&](int k, Q q) {
    auto it = dims[k].find(q);
    return it == dims[k].end() ? 0 : it->second;
  };
  while (changed) {
    changed = false;
    for (int k = 1; k < N; ++k)
      for (auto& kv : dims[k]) {
        long long rows = 0;
        for (auto c : sc) rows += get(k - 1, {kv.first.first - c.first, kv.first.second - c.second});
        if (kv.second > rows) { kv.second = (int)rows; changed = true; }
      }
    for (int k = N - 1; k >= 1; --k)
      for (auto& kv : dims[k]) {
        long long cols = 0;
        for (auto c : sc) cols += get(k + 1, {kv.first.first + c.first, kv.first.second + c.second});
        if (kv.second > cols) { kv.second = (int)cols; changed = true; }
      }
    for (int k = 1; k < N; ++k)
      for (auto it = dims[k].begin(); it != dims[k].end();)
        it = (it->second <= 0) ? dims[k].erase(it) : std::next(it);
  }
  return dims;
}

// Pairs (i, j), i < j, of chain indices at squared lattice distance d2: dx^2 +
// dy^2, dy the short way round a cylinder's width (W >= 3).  Coordinates
// follow the snake: column x = n / W, top-down for even x, bottom-up for odd.
std::vector<std::pair<int, int>> pairs_at_distance(const Lattice& lat, int d2) {
  const int W = lat.W;
  auto xy = [&](int n, int& x, int& y) {
    x = n / W;
    const int r = n % W;
    y = (x % 2 == 0) ? W - 1 - r : r;
  };
  std::vector<std::pair<int, int>> out;
  for (int i = 0; i < lat.N; ++i)
    for (int j = i + 1; j < lat.N; ++j) {
      int xi, yi, xj, yj;
      xy(i, xi, yi);
      xy(j, xj, yj);
      int dy = std::abs(yi - yj);
      if (lat.geometry == TT_CYLINDER && W >= 3) dy = std::min(dy, W - dy);
      if ((xi - xj) * (xi - xj) + dy * dy == d2) out.push_back({i, j});
    }
  return out;
}

// Sum over pairs (i < j) of S_i . S_j = Sz_i Sz_j + (S+_i S-_j + S-_i S+_j)/2
// (the spin correlation of main text Fig. 2(c)) as an MPO: channels start,
// src(i, type) for every site i < k that has a partner j >= k (type Sz, S+,
// S-: spin channels 4..6), and done.  Spin operators are bosonic (no string).
Mpo make_spin_pair_mpo(int N, const std::vector<std::pair<int, int>>& pairs) {
  std::vector<std::set<int>> later(N);
  for (auto& p : pairs) later[p.first].insert(p.second);
  Mpo m;
  m.N = N;
  m.states.resize(N + 1);
  for (int k = 0; k <= N; ++k) {
    auto& st = m.states[k];
    st.push_back({0, -1, -1});
    for (int i = 0; i < k && k < N; ++i)
      if (!later[i].empty() && *later[i].rbegin() >= k)
        for (int ty = 4; ty < 7; ++ty) st.push_back({2, i, ty});
    if (k > 0) st.push_back({1, -1, -1});
  }
  for (int k = 0; k <= N; ++k) m.DH.push_back((int)m.states[k].size());
  M4 id = zero4(), sz = zero4(), sp = zero4(), sm = zero4();
  for (int i = 0; i < 4; ++i) id.v[i][i] = 1.0;
  sz.v[1][1] = 0.5; sz.v[2][2] = -0.5;
  sp.v[1][2] = 1.0;   // |up><dn|
  sm.v[2][1] = 1.0;
  const M4* left[3] = {&sz, &sp, &sm};
  const M4* right[3] = {&sz, &sm, &sp};
  const double coef[3] = {1.0, 0.5, 0.5};
  m.W.resize(N);
  for (int k = 0; k < N; ++k) {
    const auto& Ls = m.states[k];
    const auto& Rs = m.states[k + 1];
    const int DL = (int)Ls.size(), DR = (int)Rs.size();
    std::vector<double> Wk((size_t)DL * 16 * DR, 0.0);
    auto find = [&](int kind, int site, int type) {
      for (int b = 0; b < DR; ++b)
        if (Rs[b].kind == kind && (kind < 2 || (Rs[b].site == site && Rs[b].type == type))) return b;
      return -1;
    };
    auto put = [&](int a, int b, const M4& op, double c) {
      for (int so = 0; so < 4; ++so)
        for (int si = 0; si < 4; ++si) Wk[(((size_t)a * 4 + so) * 4 + si) * DR + b] += c * op.v[so][si];
    };
    const int bstart = find(0, -1, -1), bdone = find(1, -1, -1);
    for (int a = 0; a < DL; ++a) {
      const MpoState& s = Ls[a];
      if (s.kind == 0) {
        put(a, bstart, id, 1.0);
        for (int ty = 4; ty < 7; ++ty) {
          const int b = find(2, k, ty);
          if (b >= 0) put(a, b, *left[ty - 4], 1.0);
        }
      } else if (s.kind == 1) {
        put(a, bdone, id, 1.0);
      } else {
        const int b = find(2, s.site, s.type);
        if (b >= 0) put(a, b, id, 1.0);
        if (later[s.site].count(k)) put(a, bdone, *right[s.type - 4], coef[s.type - 4]);
      }
    }
    m.W[k] = Wk;
  }
  return m;
}

// Sum of one on-site operator over all sites, sum_i op_i (a diagonal 4x4 in
// the local basis {0, up, dn, updn}), as an MPO with two channels per bond:
// start (identity so far) and done (op placed).  Bond 0 has start only, bond N
// start and done, like the Hamiltonian.
Mpo make_local_sum_mpo(int N, const double op[4]) {
  Mpo m;
  m.N = N;
  m.states.resize(N + 1);
  m.states[0] = {{0, -1, -1}};
  for (int k = 1; k <= N; ++k) m.states[k] = {{0, -1, -1}, {1, -1, -1}};
  for (int k = 0; k <= N; ++k) m.DH.push_back((int)m.states[k].size());
  m.W.resize(N);
  for (int k = 0; k < N; ++k) {
    const int DL = m.DH[k], DR = m.DH[k + 1];
    std::vector<double> Wk((size_t)DL * 16 * DR, 0.0);
    for (int s = 0; s < 4; ++s) {
      Wk[(((size_t)0 * 4 + s) * 4 + s) * DR + 0] = 1.0;    // start -> start: identity
      Wk[(((size_t)0 * 4 + s) * 4 + s) * DR + 1] = op[s];  // start -> done: the operator
      if (DL == 2) Wk[(((size_t)1 * 4 + s) * 4 + s) * DR + 1] = 1.0;   // done -> done
    }
    m.W[k] = Wk;
  }
  return m;
}

// Matsubara Green's function at half the imaginary time (main text,
// Fermi-surface paragraph), as a super-operator MPO on the super index
// s = 4 sigma + sigma' (16 x 16 local matrices, ld = 16):
//   X(k) = sum_s sum_{r,r'} cos(k.(r - r')) c+_{rs} (x) (c_{r's})^T ,
// <<rho|X|rho>> = sum_{rr'} cos(k.(r - r')) Tr[rho c+_r rho c_r'] (the Choi map
// sends A rho B to (A (x) B^T)|rho>>, SM Sec. II.A).  With the Jordan-Wigner
// strings c+_r = P..P c+ at r and (c_r')^T = P..P c+ at r' (c^T = c+ for the
// real local matrices, P diagonal), so every pair is a product of local
// (ket op) (x) (ancilla op); cos(k.(r - r')) = cos cos + sin sin splits it into
// separable terms.  Bond states: start (P (x) P), the placed-ket channels
// (1 (x) P) and placed-ancilla channels (P (x) 1) per spin and per cos|sin
// (site = 0|1, type 0..3: ket up, ket dn, ancilla up, ancilla dn, whose charge
// is that of the channel table), done (1 (x) 1).  r = (x, y): x along the
// length, y across the width, in the snake order.  pattern = true puts 1 in
// place of every cos and sin (the nonzero pattern for any k).
Mpo make_green_mpo(const Lattice& lat, double kx, double ky, bool pattern) {
  const int N = lat.N, W = lat.W;
  const LocalOps o = local_ops(0.0, 0.0);
  Mpo m;
  m.N = N;
  m.ld = 16;
  m.states.resize(N + 1);
  m.states[0] = {{0, -1, -1}};
  for (int k = 1; k <= N; ++k) {
    m.states[k] = {{0, -1, -1}};
    for (int ty = 0; ty < 4; ++ty)
      for (int f = 0; f < 2; ++f) m.states[k].push_back({2, f, ty});
    m.states[k].push_back({1, -1, -1});
  }
  for (int k = 0; k <= N; ++k) m.DH.push_back((int)m.states[k].size());
  const M4* cdag[2] = {&o.cdu, &o.cdd};
  m.W.resize(N);
  for (int q = 0; q < N; ++q) {
    const int x = q / W, rr = q % W, y = (x % 2 == 0) ? (W - 1 - rr) : rr;
    const double th = kx * x + ky * y;
    const double trig[2] = {pattern ? 1.0 : std::cos(th), pattern ? 1.0 : std::sin(th)};
    const auto& Ls = m.states[q];
    const auto& Rs = m.states[q + 1];
    const int DL = (int)Ls.size(), DR = (int)Rs.size();
    std::vector<double> Wk((size_t)DL * 256 * DR, 0.0);
    auto find = [&](int kind, int f, int type) {
      for (int b = 0; b < DR; ++b)
        if (Rs[b].kind == kind && (kind < 2 || (Rs[b].site == f && Rs[b].type == type))) return b;
      return -1;
    };
    // W[a, 4 so + ao, 4 si + ai, b] += c ket[so][si] anc[ao][ai]
    auto put = [&](int a, int b, const M4& ket, const M4& anc, double c) {
      if (b < 0) return;
      for (int so = 0; so < 4; ++so)
        for (int si = 0; si < 4; ++si)
          for (int ao = 0; ao < 4; ++ao)
            for (int ai = 0; ai < 4; ++ai)
              Wk[(((size_t)a * 16 + 4 * so + ao) * 16 + 4 * si + ai) * DR + b] += c * ket.v[so][si] * anc.v[ao][ai];
    };
    const int bstart = find(0, -1, -1), bdone = find(1, -1, -1);
    for (int a = 0; a < DL; ++a) {
      const MpoState& s = Ls[a];
      if (s.kind == 0) {
        put(a, bstart, o.par, o.par, 1.0);
        for (int sp = 0; sp < 2; ++sp) {
          for (int f = 0; f < 2; ++f) {
            put(a, find(2, f, sp), *cdag[sp], o.par, trig[f]);
            put(a, find(2, f, 2 + sp), o.par, *cdag[sp], trig[f]);
          }
          put(a, bdone, *cdag[sp], *cdag[sp], 1.0);
        }
      } else if (s.kind == 1) {
        put(a, bdone, o.id, o.id, 1.0);
      } else if (s.type < 2) {   // ket operator placed
        put(a, find(2, s.site, s.type), o.id, o.par, 1.0);
        put(a, bdone, o.id, *cdag[s.type], trig[s.site]);
      } else {                   // ancilla operator placed
        put(a, find(2, s.site, s.type), o.par, o.id, 1.0);
        put(a, bdone, *cdag[s.type - 2], o.id, trig[s.site]);
      }
    }
    m.W[q] = Wk;
  }
  return m;
}

namespace {
// Ordered modified Gram-Schmidt (two passes) over the columns cols[j] (each
// of length m): dependent columns (residual <= tol x own norm) are dropped.
// Returns the kept orthonormal columns; R (kept x n) holds the coefficients,
// cols[j] = sum_i Q[i] R[i][j].  A residual within a factor 10 of the
// threshold is an error (the decision would rest on rounding).
constexpr double kSettnTol = 1e-8;
std::vector<std::vector<double>> mgs_keep(const std::vector<std::vector<double>>& cols,
                                          std::vector<std::vector<double>>& R) {
  const size_t n = cols.size();
  std::vector<std::vector<double>> Q;
  std::vector<std::vector<double>> Rc(n);   // per column: coefficients on Q (grows)
  std::vector<int> pivot(n, -1);
  for (size_t j = 0; j < n; ++j) {
    std::vector<double> v = cols[j];
    double n0 = 0.0;
    for (double x : v) n0 += x * x;
    n0 = std::sqrt(n0);
    std::vector<double> coef(Q.size(), 0.0);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t i = 0; i < Q.size(); ++i) {
        double c = 0.0;
        for (size_t r = 0; r < v.size(); ++r) c += Q[i][r] * v[r];
        coef[i] += c;
        for (size_t r = 0; r < v.size(); ++r) v[r] -= c * Q[i][r];
      }
    double nv = 0.0;
    for (double x : v) nv += x * x;
    nv = std::sqrt(nv);
    Rc[j] = coef;
    if (n0 == 0.0) continue;
    if (nv > 0.1 * kSettnTol * n0 && nv <= 10.0 * kSettnTol * n0) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "SETTN start: a Gram-Schmidt residual (%.3e of its column) is too close to "
                    "the threshold (change taylor_order or beta0)", nv / n0);
      throw Error(TT_EINVAL, msg);
    }
    if (nv > kSettnTol * n0) {
      for (double& x : v) x /= nv;
      Q.push_back(v);
      pivot[j] = (int)Q.size() - 1;
      Rc[j].push_back(nv);
    }
  }
  R.assign(Q.size(), std::vector<double>(n, 0.0));
  for (size_t j = 0; j < n; ++j)
    for (size_t i = 0; i < Rc[j].size() && i < Q.size(); ++i) R[i][j] = Rc[j][i];
  return Q;
}
}  // namespace

Rho0 make_rho0(const Mpo& H, double beta0, int order) {
  const int N = H.N;
  Rho0 r;
  r.A.resize(N);
  r.q.resize(N + 1);
  std::vector<std::vector<Q>> ch(N + 1);
  for (int k = 0; k <= N; ++k)
    for (int a = 0; a < H.DH[k]; ++a) ch[k].push_back(H.charge(k, a));
  std::vector<int> D(N + 1);
  if (order == 1) {
    for (int k = 0; k < N; ++k) {
      r.q[k] = ch[k];
      D[k] = H.DH[k];
    }
    const int DR = H.DH[N];
    for (int k = 0; k < N - 1; ++k) r.A[k] = H.W[k];
    std::vector<double> last((size_t)H.DH[N - 1] * 16, 0.0);
    for (int a = 0; a < H.DH[N - 1]; ++a)
      for (int q = 0; q < 16; ++q)
        last[(size_t)a * 16 + q] = H.W[N - 1][((size_t)a * 16 + q) * DR + 0] - beta0 * H.W[N - 1][((size_t)a * 16 + q) * DR + 1];
    r.A[N - 1] = last;
    r.q[N] = {Q{0, 0}};
    return r;
  }
  // product MPO of `order` copies: state (a1..an) -> index ((a1 * DH + a2) * DH + ...)
  for (int k = 0; k <= N; ++k) {
    long long d = 1;
    for (int i = 0; i < order; ++i) d *= H.DH[k];
    TT_REQUIRE(d <= 8192, TT_EINVAL, "SETTN start: the product MPO bond is too large (lower taylor_order)");
    D[k] = (int)d;
    std::vector<Q> qs(1, Q{0, 0});
    for (int i = 0; i < order; ++i) {
      std::vector<Q> nq;
      for (const Q& x : qs)
        for (const Q& y : ch[k]) nq.push_back({x.first + y.first, x.second + y.second});
      qs = nq;
    }
    r.q[k] = qs;
  }
  long long total = 0;
  for (int k = 0; k < N; ++k) total += (long long)D[k] * 16 * D[k + 1];
  TT_REQUIRE(total <= (1LL << 28), TT_EINVAL, "SETTN start: the product MPO is too large (lower taylor_order)");
  for (int k = 0; k < N; ++k) {
    TT_REQUIRE((long long)D[k] * 16 * D[k + 1] <= (1LL << 26), TT_EINVAL,
               "SETTN start: the product MPO tensor is too large (lower taylor_order)");
    const int DL1 = H.DH[k], DR1 = H.DH[k + 1];
    std::vector<double> P = H.W[k];   // [A][so][si][B], sizes dl x 4 x 4 x dr
    long long dl = DL1, dr = DR1;
    for (int f = 1; f < order; ++f) {
      std::vector<double> Pn((size_t)(dl * DL1) * 16 * (dr * DR1), 0.0);
      for (long long A = 0; A < dl; ++A)
        for (int so = 0; so < 4; ++so)
          for (int t = 0; t < 4; ++t)
            for (long long B = 0; B < dr; ++B) {
              const double p = P[((A * 4 + so) * 4 + t) * dr + B];
              if (p == 0.0) continue;
              for (int a = 0; a < DL1; ++a)
                for (int si = 0; si < 4; ++si)
                  for (int b = 0; b < DR1; ++b) {
                    const double w = H.W[k][(((size_t)a * 4 + t) * 4 + si) * DR1 + b];
                    if (w == 0.0) continue;
                    Pn[(((A * DL1 + a) * 4 + so) * 4 + si) * (dr * DR1) + (B * DR1 + b)] += p * w;
                  }
            }
      P.swap(Pn);
      dl *= DL1;
      dr *= DR1;
    }
    r.A[k] = P;
  }
  {   // boundary vector: a tuple with m factors done stands for H^m
    const int nR = H.DH[N];   // start, done
    const int M = D[N];
    std::vector<double> bv(M);
    for (int idx = 0; idx < M; ++idx) {
      int m = 0, x = idx;
      for (int i = 0; i < order; ++i) { m += (x % nR == 1); x /= nR; }
      double c = 1.0, binom = 1.0;
      for (int i = 1; i <= m; ++i) c *= -beta0 / i;
      for (int i = 1; i <= m; ++i) binom = binom * (order - m + i) / i;
      bv[idx] = c / binom;
    }
    const int dl = D[N - 1];
    std::vector<double> last((size_t)dl * 16, 0.0);
    for (int a = 0; a < dl; ++a)
      for (int q = 0; q < 16; ++q) {
        double v = 0.0;
        for (int b = 0; b < M; ++b) v += r.A[N - 1][((size_t)a * 16 + q) * M + b] * bv[b];
        last[(size_t)a * 16 + q] = v;
      }
    r.A[N - 1] = last;
    D[N] = 1;
    r.q[N] = {Q{0, 0}};
  }
  // exact reduction, left to right over the columns of the left unfoldings
  for (int k = 0; k < N - 1; ++k) {
    const int a = D[k], b = D[k + 1];
    std::set<Q> qs(r.q[k + 1].begin(), r.q[k + 1].end());
    std::vector<std::vector<double>> newcols, coef;   // coef: rows of C (new x old b)
    std::vector<Q> newq;
    for (const Q& qq : qs) {
      std::vector<int> J;
      for (int j = 0; j < b; ++j)
        if (r.q[k + 1][j] == qq) J.push_back(j);
      std::vector<std::vector<double>> cols(J.size(), std::vector<double>((size_t)a * 16));
      for (size_t c = 0; c < J.size(); ++c)
        for (long long row = 0; row < (long long)a * 16; ++row) cols[c][row] = r.A[k][row * b + J[c]];
      std::vector<std::vector<double>> R;
      auto Qm = mgs_keep(cols, R);
      for (size_t i = 0; i < Qm.size(); ++i) {
        newcols.push_back(Qm[i]);
        std::vector<double> crow(b, 0.0);
        for (size_t c = 0; c < J.size(); ++c) crow[J[c]] = R[i][c];
        coef.push_back(crow);
        newq.push_back(qq);
      }
    }
    const int nb = (int)newcols.size();
    std::vector<double> Ak((size_t)a * 16 * nb);
    for (long long row = 0; row < (long long)a * 16; ++row)
      for (int c = 0; c < nb; ++c) Ak[row * nb + c] = newcols[c][row];
    const int bn = D[k + 2];
    std::vector<double> An((size_t)nb * 16 * bn, 0.0);   // C . A_{k+1}
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < b; ++j) {
        const double c = coef[i][j];
        if (c == 0.0) continue;
        const double* src = &r.A[k + 1][(size_t)j * 16 * bn];
        double* dst = &An[(size_t)i * 16 * bn];
        for (long long e = 0; e < 16LL * bn; ++e) dst[e] += c * src[e];
      }
    r.A[k] = Ak;
    r.A[k + 1] = An;
    D[k + 1] = nb;
    r.q[k + 1] = newq;
  }
  // right to left over the rows of the right unfoldings
  for (int k = N - 1; k >= 1; --k) {
    const int a = D[k], b = D[k + 1];
    std::set<Q> qs(r.q[k].begin(), r.q[k].end());
    std::vector<std::vector<double>> newrows, coef;   // coef: rows of C (new x old a)
    std::vector<Q> newq;
    for (const Q& qq : qs) {
      std::vector<int> J;
      for (int j = 0; j < a; ++j)
        if (r.q[k][j] == qq) J.push_back(j);
      std::vector<std::vector<double>> cols(J.size());
      for (size_t c = 0; c < J.size(); ++c)
        cols[c].assign(r.A[k].begin() + (size_t)J[c] * 16 * b, r.A[k].begin() + (size_t)(J[c] + 1) * 16 * b);
      std::vector<std::vector<double>> R;
      auto Qm = mgs_keep(cols, R);
      for (size_t i = 0; i < Qm.size(); ++i) {
        newrows.push_back(Qm[i]);
        std::vector<double> crow(a, 0.0);
        for (size_t c = 0; c < J.size(); ++c) crow[J[c]] = R[i][c];
        coef.push_back(crow);
        newq.push_back(qq);
      }
    }
    const int na = (int)newrows.size();
    std::vector<double> Ak((size_t)na * 16 * b);
    for (int i = 0; i < na; ++i) std::copy(newrows[i].begin(), newrows[i].end(), Ak.begin() + (size_t)i * 16 * b);
    const int ap = D[k - 1];
    std::vector<double> Ap((size_t)ap * 16 * na, 0.0);   // A_{k-1} . C^T
    for (long long row = 0; row < (long long)ap * 16; ++row)
      for (int j = 0; j < a; ++j) {
        const double v = r.A[k - 1][row * a + j];
        if (v == 0.0) continue;
        for (int i = 0; i < na; ++i) Ap[row * na + i] += v * coef[i][j];
      }
    r.A[k] = Ak;
    r.A[k - 1] = Ap;
    D[k] = na;
    r.q[k] = newq;
  }
  return r;
}

}  // namespace tt
