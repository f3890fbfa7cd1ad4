// Internal declarations of the tanTRG library (host side).
#pragma once
#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tantrg.h"

namespace tt {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define TT_REQUIRE(cond, code, msg)                     \
  do {                                                  \
    if (!(cond)) throw ::tt::Error((code), (msg));      \
  } while (0)

using Q = std::pair<int, int>;  // (n_up, n_dn) charge

// ------------------------------------------------------------------ model
struct Lattice {
  int W, L, geometry, N;
  std::vector<std::pair<int, int>> bonds;      // i < j, chain indices
};
Lattice make_lattice(int W, int L, int geometry);

// One MPO bond state: kind 0 start, 1 done, 2 source channel, 3 destination channel
struct MpoState { int kind, site, type; };

struct Mpo {
  int N;
  std::vector<std::vector<MpoState>> states;   // per bond 0..N (bond N: start, done)
  int ld = 4;                                  // local operator size: 4 (ket only) or 16 (super index)
  std::vector<std::vector<double>> W;          // W[k][((a*ld+so)*ld+si)*DHr + b]
  std::vector<int> DH;                         // per bond
  Q charge(int k, int a) const;
};
Mpo make_hubbard_mpo(const Lattice& lat, double t, double tp, double U, double mu, double hp);
std::vector<std::pair<std::pair<int, int>, double>> pairing_bonds(const Lattice& lat);   // bonds with s_ij
Mpo make_local_sum_mpo(int N, const double op[4]);   // sum_i op_i, op diagonal
std::vector<std::pair<int, int>> pairs_at_distance(const Lattice& lat, int d2);
Mpo make_spin_pair_mpo(int N, const std::vector<std::pair<int, int>>& pairs);   // sum over pairs of S_i . S_j
Mpo make_green_mpo(const Lattice& lat, double kx, double ky, bool pattern);      // super-operator of G(k, beta/2)

// The start rho0 as a super-MPS on the host: A[k] = [D_k][16][D_{k+1}] (bond N
// has one state) and the charge of every bond state (bonds 0..N).  order 1:
// 1 - beta0 H; order > 1: the SETTN polynomial sum_{n <= order} (-beta0 H)^n / n!
// from the product MPO, reduced exactly to linearly independent bond states.
struct Rho0 {
  std::vector<std::vector<double>> A;
  std::vector<std::vector<Q>> q;
};
Rho0 make_rho0(const Mpo& H, double beta0, int order);

// ------------------------------------------------------------------ sectors
struct Sector { Q q; int dim; long long off; };
struct Bond {
  std::vector<Sector> secs;
  long long total = 0;
  std::map<Q, int> index;
  int find(Q q) const { auto it = index.find(q); return it == index.end() ? -1 : it->second; }
  void add(Q q, int dim) { index[q] = (int)secs.size(); secs.push_back({q, dim, total}); total += dim; }
};

// super-index groups: 9 charge groups (symmetric) or one group of all 16
struct Groups {
  int ng;
  std::vector<Q> delta;                 // per group
  std::vector<std::vector<int>> s;      // super indices s = 4*sigma + sigma' per group
  std::vector<int> group_of, pos_of;    // per s
};
// block structure: 0 none (one sector), 1 U(1)charge x U(1)spin, 2 U(1) of
// q_up - q_dn alone (charges (sz, 0))
Groups make_groups(int mode);
Q project_charge(Q q, int mode);

uint64_t splitmix64(uint64_t x);
double noise_uniform(uint64_t seed, int site, uint64_t flat);

// sector dimensions of bonds 0..N for a target D (n0: rho0 states per charge)
std::vector<std::map<Q, int>> allocate_sectors(int N, int D, const std::vector<std::map<Q, int>>& n0,
                                               int sector_cap, int mode = 1);

}  // namespace tt
