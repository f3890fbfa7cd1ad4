"""U(1)charge x U(1)spin bond sectors and the padded initial state (oracle;
test infrastructure only).

The density operator commutes with N_up and N_down (main text: the spin and
charge symmetries live in the grand-canonical MPO), so a super-MPS tensor
A[x, (sigma, sigma'), y] is non-zero only when
    q(y) = q(x) + q(sigma) - q(sigma'),   q = (n_up, n_dn),
with q(bond 0) = q(bond N) = (0, 0).  The local super-index charge
Delta(s) = q(sigma) - q(sigma') takes 9 values: (0,0) four times, the four
(+-1,0), (0,+-1) twice each, the four (+-1,+-1) once each.

Reading for growing rho0 = 1 - beta0 H (bond D_H) to a target D with the
one-site method, which cannot grow bonds by itself (the paper grows them
with the two-site update in its initial stage): pad every bond to D, fill
the new charge-allowed entries with small seeded noise, canonicalise.

Sector dimensions at bond k (0 < k < N) for a target D:
* maximal dimension of sector q: Dmax_k(q) = min(cL, cR) with
  cL = C(2k, k+q_up) C(2k, k+q_dn) and cR the same with k -> N-k (the number
  of left / right super-index configurations of charge +-q);
* if sum_q Dmax_k(q) <= D every sector is maximal;
* else sizes proportional to w(q) = C(2h, h+q_up) C(2h, h+q_dn),
  h = min(k, N-k, 14), by the largest-remainder rule in exact integers (ties
  to the lexicographically smaller q), with every sector capped at
  c(q) = min(Dmax_k(q), sector_cap) (sector_cap = 0: no cap): sectors whose
  share exceeds their cap are fixed at the cap and the rest of D is shared
  again among the others, until no share exceeds its cap; then every sector
  is raised to the number of rho0 states of charge q;
* then capped, until nothing changes, by the rows a left-to-right QR can
  supply (sum_Delta n(Delta) d_{k-1}(q - Delta)) and by the columns a
  right-to-left LQ can supply (sum_Delta n(Delta) d_{k+1}(q + Delta)).
Bond index order: sectors sorted by (q_up, q_dn); inside a sector, first the
rho0 states of that charge in MPO bond-state order, then the padding.
Without symmetry (dense), every bond is one block of min(D, 16^min(k,N-k))
states (never below the rho0 bond), rho0 states first.

Noise (padding entries only, i.e. x or y is a padding state, and, with
symmetry, charge-allowed): pad_eps * (2u - 1), u in [0, 1) from SplitMix64
(Steele, Lea & Flood 2014): output n of seed is mix(seed + n*0x9E3779B97F4A7C15)
with n = site*2^40 + flat + 1, flat = (x*16 + s)*D_{k+1} + y, and u the top
53 bits times 2^-53.
"""
from functools import lru_cache
from math import comb as _comb

import numpy as np


@lru_cache(maxsize=None)
def comb(n, k):
    return _comb(n, k)

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def s_charge(s):
    sig, sigp = s // 4, s % 4
    return ((sig & 1) - (sigp & 1), (sig >> 1) - (sigp >> 1))


S_CHARGES = [s_charge(s) for s in range(16)]


def project(q, mode):
    """A (q_up, q_dn) charge in the block structure of ``mode``: "u1u1" keeps
    both U(1) charges; "sz" keeps only q_up - q_dn (as (sz, 0)), the one left
    when a pairing field breaks the particle numbers."""
    return tuple(q) if mode == "u1u1" else (q[0] - q[1], 0)


def s_charges(mode):
    return [project(c, mode) for c in S_CHARGES]


def splitmix64(x):
    z = x & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def noise_uniform(seed, site, flat):
    """Vectorised SplitMix64 draw in [-1, 1) for integer array ``flat``."""
    flat = np.asarray(flat, dtype=np.uint64)
    with np.errstate(over="ignore"):
        n = np.uint64(site) * np.uint64(1 << 40) + flat + np.uint64(1)
        z = np.uint64(seed & MASK) + n * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def _dmax(N, k, q, mode="u1u1"):
    """Number of super basis states of charge q on the k sites left of the
    bond (or the N - k right of it, whichever is smaller): per site the
    super charge of (n_up, n_dn) is a difference of two local values, so k
    sites give comb(2k, k + a) comb(2k, k + b); with the Sz charge alone,
    comb(4k, 2k + a)."""
    a, b = q
    m = N - k
    def cnt(n):
        if mode == "sz":
            return comb(4 * n, 2 * n + a) if abs(a) <= 2 * n else 0
        if abs(a) > n or abs(b) > n:
            return 0
        return comb(2 * n, n + a) * comb(2 * n, n + b)
    return min(cnt(k), cnt(m))


def _share(D, qs, w):
    """Largest-remainder split of D proportional to w (exact integers)."""
    tot = sum(w[q] for q in qs)
    if tot == 0 or D <= 0:
        return {q: 0 for q in qs}
    base = {q: (D * w[q]) // tot for q in qs}
    rem = {q: (D * w[q]) % tot for q in qs}
    left = D - sum(base.values())
    for q in sorted(qs, key=lambda q: (-rem[q], q))[:left]:
        base[q] += 1
    return base


def allocate_sectors(N, D, n0, sector_cap=0, mode="u1u1"):
    """Sector dimensions per bond.  n0[k] maps charge -> number of rho0
    states.  Returns a list over bonds 0..N of dicts {q: dim} (nonzero).
    mode "sz": charges (sz, 0) of the Sz-only block structure."""
    dims = [{(0, 0): 1}]
    sc = s_charges(mode)
    for k in range(1, N):
        h = min(k, N - k)
        if mode == "sz":
            qs = [(a, 0) for a in range(-2 * h, 2 * h + 1)]
        else:
            qs = [(a, b) for a in range(-h, h + 1) for b in range(-h, h + 1)]
        dmax = {q: _dmax(N, k, q, mode) for q in qs}
        if sum(dmax.values()) <= D:
            d = dict(dmax)
        else:
            hw = min(h, 14)
            w = {}
            for q in qs:
                a, b = q
                if mode == "sz":
                    w[q] = comb(4 * hw, 2 * hw + a) if abs(a) <= 2 * hw else 0
                else:
                    w[q] = (comb(2 * hw, hw + a) * comb(2 * hw, hw + b)
                            if abs(a) <= hw and abs(b) <= hw else 0)
            cap = {q: dmax[q] if sector_cap <= 0 else min(dmax[q], sector_cap) for q in qs}
            fixed = {}
            while True:
                free = [q for q in qs if q not in fixed]
                base = _share(D - sum(fixed.values()), free, w)
                over = [q for q in free if base[q] > cap[q]]
                if not over:
                    break
                for q in over:
                    fixed[q] = cap[q]
            base.update(fixed)
            d = {q: min(max(base[q], n0[k].get(q, 0)), dmax[q]) for q in qs}
        dims.append({q: v for q, v in d.items() if v > 0})
    dims.append({(0, 0): 1})
    # consistency caps
    changed = True
    while changed:
        changed = False
        for k in range(1, N):
            for q in list(dims[k]):
                rows = sum(dims[k - 1].get((q[0] - c[0], q[1] - c[1]), 0)
                           for c in sc)
                if dims[k][q] > rows:
                    dims[k][q] = rows
                    changed = True
        for k in range(N - 1, 0, -1):
            for q in list(dims[k]):
                cols = sum(dims[k + 1].get((q[0] + c[0], q[1] + c[1]), 0)
                           for c in sc)
                if dims[k][q] > cols:
                    dims[k][q] = cols
                    changed = True
        for k in range(1, N):
            dims[k] = {q: v for q, v in dims[k].items() if v > 0}
    return dims


class BondLayout:
    """Dense embedding of a padded bond: charge per index, rho0 slot map."""

    def __init__(self, charges, rho0_index, is_pad):
        self.charges = charges          # list of q per bond index
        self.rho0_index = rho0_index    # rho0 bond state j -> padded index
        self.is_pad = np.array(is_pad, dtype=bool)

    @property
    def dim(self):
        return len(self.charges)


def bond_layouts(rho0_charges, N, D, symmetric, sector_cap=0, mode="u1u1"):
    """Layouts of bonds 0..N.  rho0_charges[k] = charge per rho0 bond state
    (as (q_up, q_dn); projected onto the block structure of ``mode``)."""
    layouts = []
    if symmetric:
        rho0_charges = [[project(q, mode) for q in qk] for qk in rho0_charges]
        n0 = []
        for k in range(N + 1):
            cnt = {}
            for q in rho0_charges[k]:
                cnt[q] = cnt.get(q, 0) + 1
            n0.append(cnt)
        dims = allocate_sectors(N, D, n0, sector_cap, mode)
        for k in range(N + 1):
            secs = sorted(dims[k])
            off, p = {}, 0
            for q in secs:
                off[q] = p
                p += dims[k][q]
            charges = [q for q in secs for _ in range(dims[k][q])]
            used = {q: 0 for q in secs}
            rho0_index = []
            is_pad = [True] * p
            for q in rho0_charges[k]:
                if used.get(q, 0) >= dims[k].get(q, 0):
                    raise ValueError("rho0 does not fit the sectors of bond %d" % k)
                idx = off[q] + used[q]
                used[q] += 1
                rho0_index.append(idx)
                is_pad[idx] = False
            layouts.append(BondLayout(charges, rho0_index, is_pad))
    else:
        for k in range(N + 1):
            n = len(rho0_charges[k])
            dmax = 16 ** min(k, N - k)
            d = max(min(D, dmax), n)
            layouts.append(BondLayout([(0, 0)] * d, list(range(n)),
                                      [False] * n + [True] * (d - n)))
    return layouts


def padded_rho0(A0, layouts, symmetric, pad_eps, seed, mode="u1u1"):
    """Embed rho0 tensors into the padded bonds and add the seeded noise."""
    out = []
    for k, a in enumerate(A0):
        Ll, Lr = layouts[k], layouts[k + 1]
        Dl, Dr = Ll.dim, Lr.dim
        A = np.zeros((Dl, 16, Dr))
        a16 = a.reshape(a.shape[0], 16, a.shape[3])
        A[np.ix_(Ll.rho0_index, range(16), Lr.rho0_index)] = a16
        if pad_eps != 0.0:
            x, s, y = np.meshgrid(np.arange(Dl), np.arange(16), np.arange(Dr),
                                  indexing="ij")
            mask = Ll.is_pad[x] | Lr.is_pad[y]
            if symmetric:
                ql = np.array(Ll.charges)
                qr = np.array(Lr.charges)
                sc = np.array(s_charges(mode))
                ok = ((ql[x, 0] + sc[s, 0] == qr[y, 0]) &
                      (ql[x, 1] + sc[s, 1] == qr[y, 1]))
                mask &= ok
            flat = (x * 16 + s) * Dr + y
            A[mask] = pad_eps * noise_uniform(seed, k, flat[mask])
        out.append(A.reshape(Dl, 4, 4, Dr))
    return out
