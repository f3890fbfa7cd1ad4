"""Sector-blocked exact diagonalisation of the Hubbard model (oracle).

Paper: Eq. (3), H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i n_iu n_id
- mu sum_i n_i, on the lattices of ``oracle.lattice``; the density operator
rho = exp(-beta H) and the bilayer identity rho(beta) = rho(beta/2)
rho(beta/2)^dagger of SM Sec. II.A.

Fock basis: 2N fermion modes ordered (site 0 up, site 0 down, site 1 up, ...)
along the snake; a basis state is prod_m (c+_m)^{n_m} |vac> with the
creation operators applied in increasing mode order (leftmost first).  The
dense index of a state is sum_i sigma_i 4^(N-1-i), sigma_i = n_iu + 2 n_id,
i.e. the local basis {0, up, down, updown} with |updown> = c+_u c+_d |0>.

H commutes with N_up and N_down, so it is built and diagonalised block by
block over (N_up, N_down).
"""
from itertools import product

import numpy as np

from . import lattice


def _mode(site, spin):
    return 2 * site + spin


def _index(occ, N):
    """Dense index of an occupation tuple (length 2N)."""
    idx = 0
    for i in range(N):
        idx = idx * 4 + occ[2 * i] + 2 * occ[2 * i + 1]
    return idx


def _hop(occ, m, n):
    """Apply c+_m c_n to a basis state.  Returns (sign, new_occ) or None."""
    if occ[n] == 0:
        return None
    occ = list(occ)
    sign = (-1) ** sum(occ[:n])          # c_n passes the occupied modes left of n
    occ[n] = 0
    if occ[m] == 1:
        return None
    sign *= (-1) ** sum(occ[:m])         # c+_m passes the occupied modes left of m
    occ[m] = 1
    return sign, tuple(occ)


def _spin_flip(occ, i, j):
    """S+_i S-_j = (c+_{i up} c_{i dn}) (c+_{j dn} c_{j up}) on a basis state
    (S-_j applied first).  Returns (sign, new_occ) or None."""
    r = _hop(occ, _mode(j, 1), _mode(j, 0))
    if r is None:
        return None
    s1, occ1 = r
    r = _hop(occ1, _mode(i, 0), _mode(i, 1))
    if r is None:
        return None
    s2, occ2 = r
    return s1 * s2, occ2


def _annihilate(occ, m):
    """Apply c_m to a basis state.  Returns (sign, new_occ) or None."""
    if occ[m] == 0:
        return None
    sign = (-1) ** sum(occ[:m])
    occ = list(occ)
    occ[m] = 0
    return sign, tuple(occ)


class Hubbard:
    """Eq. (3) on a snake-ordered lattice; sector-blocked Hamiltonian."""

    def __init__(self, W, L, geometry, t=1.0, U=8.0, mu=0.0, tp=0.0):
        self.W, self.L, self.geometry = W, L, geometry
        self.t, self.U, self.mu, self.tp = float(t), float(U), float(mu), float(tp)
        self.N = W * L
        self.bonds = lattice.nn_bonds(W, L, geometry)
        # hopping amplitude per coupled pair: t on bonds, tp on diagonals (SM Eq. S1)
        self.hops = [(i, j, self.t) for (i, j) in self.bonds]
        if self.tp != 0.0:
            self.hops += [(i, j, self.tp) for (i, j) in lattice.nnn_bonds(W, L, geometry)]

    def _diag(self, occ):
        e = 0.0
        for i in range(self.N):
            nu, nd = occ[2 * i], occ[2 * i + 1]
            e += self.U * nu * nd - self.mu * (nu + nd)
        return e

    def sector_states(self, nup, ndn):
        N = self.N
        states = []
        for occ in product((0, 1), repeat=2 * N):
            if sum(occ[0::2]) == nup and sum(occ[1::2]) == ndn:
                states.append(occ)
        return states

    def sector_hamiltonian(self, nup, ndn):
        """Dense H restricted to the (N_up, N_down) block, and the dense indices."""
        states = self.sector_states(nup, ndn)
        pos = {s: k for k, s in enumerate(states)}
        H = np.zeros((len(states), len(states)))
        for k, occ in enumerate(states):
            H[k, k] += self._diag(occ)
            for (i, j, amp) in self.hops:
                for spin in (0, 1):
                    mi, mj = _mode(i, spin), _mode(j, spin)
                    for (m, n) in ((mi, mj), (mj, mi)):
                        r = _hop(occ, m, n)
                        if r is not None:
                            sgn, new = r
                            H[pos[new], k] += -amp * sgn
        idx = np.array([_index(s, self.N) for s in states], dtype=np.int64)
        return H, idx

    def sector_spin_pairs(self, nup, ndn, pairs, zz_only=False):
        """Dense sum over pairs of S_i . S_j = Sz_i Sz_j + (S+_i S-_j + S-_i S+_j)/2
        on the (N_up, N_down) block (the operator conserves both), with
        Sz = (n_up - n_dn)/2; zz_only keeps the Sz Sz part."""
        states = self.sector_states(nup, ndn)
        pos = {s: k for k, s in enumerate(states)}
        O = np.zeros((len(states), len(states)))
        for k, occ in enumerate(states):
            for (i, j) in pairs:
                O[k, k] += 0.25 * (occ[2 * i] - occ[2 * i + 1]) * (occ[2 * j] - occ[2 * j + 1])
                if zz_only:
                    continue
                for (a, b) in ((i, j), (j, i)):
                    r = _spin_flip(occ, a, b)
                    if r is not None:
                        sgn, new = r
                        O[pos[new], k] += 0.5 * sgn
        return O

    def dense_spin_pairs(self, pairs):
        """The full 4^N x 4^N matrix of sum over pairs of S_i . S_j (small N)."""
        N = self.N
        O = np.zeros((4 ** N, 4 ** N))
        for nup in range(N + 1):
            for ndn in range(N + 1):
                _, idx = self.sector_hamiltonian(nup, ndn)
                O[np.ix_(idx, idx)] = self.sector_spin_pairs(nup, ndn, pairs)
        return O

    def dense_hamiltonian(self):
        """Full 4^N x 4^N H in the dense basis (small N only)."""
        N = self.N
        H = np.zeros((4 ** N, 4 ** N))
        for nup in range(N + 1):
            for ndn in range(N + 1):
                h, idx = self.sector_hamiltonian(nup, ndn)
                H[np.ix_(idx, idx)] = h
        return H

    def spectrum(self):
        """All eigenvalues with their (N_up, N_down) labels."""
        N = self.N
        evals, nups, ndns = [], [], []
        for nup in range(N + 1):
            for ndn in range(N + 1):
                h, _ = self.sector_hamiltonian(nup, ndn)
                e = np.linalg.eigvalsh(h)
                evals.append(e)
                nups.append(np.full(e.size, nup))
                ndns.append(np.full(e.size, ndn))
        return np.concatenate(evals), np.concatenate(nups), np.concatenate(ndns)

    def dense_annihilator(self, site, spin):
        """The full 4^N x 4^N matrix of c_{site, spin} (small N)."""
        N = self.N
        C = np.zeros((4 ** N, 4 ** N))
        for occ in product((0, 1), repeat=2 * N):
            r = _annihilate(occ, _mode(site, spin))
            if r is not None:
                C[_index(r[1], N), _index(occ, N)] = r[0]
        return C

    def dense_function(self, fn):
        """The full 4^N x 4^N matrix fn(H), built block by block from the
        eigen-decomposition of every (N_up, N_down) block (small N)."""
        N = self.N
        M = np.zeros((4 ** N, 4 ** N))
        for nup in range(N + 1):
            for ndn in range(N + 1):
                h, idx = self.sector_hamiltonian(nup, ndn)
                E, V = np.linalg.eigh(h)
                M[np.ix_(idx, idx)] = (V * fn(E)) @ V.T
        return M

    def hopping_matrix(self):
        """Single-particle matrix h with H(U=0) = sum_s c+_s h c_s."""
        h = -self.mu * np.eye(self.N)
        for (i, j, amp) in self.hops:
            h[i, j] -= amp
            h[j, i] -= amp
        return h


def _logsumexp(x):
    m = np.max(x)
    return m + np.log(np.sum(np.exp(x - m)))


def thermal_physical(E, beta):
    """Exact ln Z(beta) and energy <H> for rho = exp(-beta H)."""
    x = -beta * E
    lnZ = _logsumexp(x)
    w = np.exp(x - lnZ)
    return lnZ, float(np.sum(w * E))


def start_poly(E, beta0, order=1):
    """The start rho0 on the eigenvalues: sum_{n <= order} (-beta0 E)^n / n!
    (order 1: the linear start 1 - beta0 E; higher orders: SETTN, SM I.E)."""
    a = np.zeros_like(np.asarray(E, dtype=float))
    term = np.ones_like(a)
    for n in range(order + 1):
        if n:
            term = term * (-beta0 * np.asarray(E, dtype=float)) / n
        a = a + term
    return a


def same_ode_bilayer(E, beta0, beta, order=1):
    """Exact values reached by the flow d rho/d beta = -H rho from the linear
    start rho(beta0) = 1 - beta0 H (main text, noninteracting-benchmark
    paragraph): rho(beta) = exp(-(beta-beta0) H) (1 - beta0 H).

    Bilayer (SM Sec. II.A): Z_bl = ||rho(beta)||_F^2 is the partition function
    at the physical inverse temperature 2*beta, and
    E_bl = <<rho|H (x) 1|rho>> / <<rho|rho>>.
    Returns (ln Z_bl, E_bl).  order > 1: the start is the Taylor polynomial
    of ``start_poly``.
    """
    a = start_poly(E, beta0, order)
    x = 2.0 * np.log(np.abs(a)) - 2.0 * (beta - beta0) * E
    lnZ = _logsumexp(x)
    w = np.exp(x - lnZ)
    return lnZ, float(np.sum(w * E))


def same_ode_bilayer_thermo(E, beta0, beta, N):
    """Per-site thermodynamics of the bilayer values at beta_phys = 2*beta
    for the same flow as ``same_ode_bilayer`` (weights w_n proportional to
    (1 - beta0 E_n)^2 exp(-2 (beta - beta0) E_n)):
    e = <E>_w / N, f = -ln Z_bl / (N beta_phys), the entropy s = beta_phys
    (e - f) and the specific heat C_e = -beta_phys de/dln(beta_phys) (main
    text, Fig. 2(b)).  d ln w_n / d beta = -2 E_n, so de/d beta_phys =
    -Var_w(E) / N and C_e = beta_phys^2 Var_w(E) / N.
    Returns a dict with beta_phys, e, f, s, c."""
    lnZ, En = same_ode_bilayer(E, beta0, beta)
    a = 1.0 - beta0 * E
    x = 2.0 * np.log(np.abs(a)) - 2.0 * (beta - beta0) * E
    w = np.exp(x - _logsumexp(x))
    var = float(np.sum(w * (E - En) ** 2))
    bp = 2.0 * beta
    e = En / N
    f = -lnZ / (N * bp)
    return {"beta_phys": bp, "e": e, "f": f, "s": bp * (e - f), "c": bp * bp * var / N}


def free_fermion_entropy_heat(h, beta):
    """U = 0 closed forms per mode pair (both spins): with f_k the Fermi
    function of eps_k = eig(h), S = 2 sum_k [-f ln f - (1-f) ln(1-f)] and
    C = 2 beta^2 sum_k eps_k^2 f_k (1 - f_k).  Returns (S, C) (totals)."""
    eps = np.linalg.eigvalsh(h)
    fk = 1.0 / (np.exp(beta * eps) + 1.0)
    ent = -(fk * np.log(fk) + (1.0 - fk) * np.log1p(-fk))
    return 2.0 * float(np.sum(ent)), 2.0 * beta * beta * float(np.sum(eps * eps * fk * (1.0 - fk)))


def same_ode_bilayer_spin_pairs(model, beta0, beta, pairs, zz_only=False):
    """Bilayer value at 2*beta of the spin correlation averaged over pairs,
    F = sum_pairs <S_i . S_j> / len(pairs) (main text, Fig. 2(c)), with
    <O> = Tr(O rho^2) / Tr(rho^2) for rho = exp(-(beta-beta0) H)(1 - beta0 H):
    sum_k w_k <k|O|k> over the eigenvectors of every (N_up, N_down) block."""
    xs, os_ = [], []
    for nup in range(model.N + 1):
        for ndn in range(model.N + 1):
            h, _ = model.sector_hamiltonian(nup, ndn)
            E, V = np.linalg.eigh(h)
            O = model.sector_spin_pairs(nup, ndn, pairs, zz_only)
            a = 1.0 - beta0 * E
            xs.append(2.0 * np.log(np.abs(a)) - 2.0 * (beta - beta0) * E)
            os_.append(np.einsum("fk,fg,gk->k", V, O, V))
    x, o = np.concatenate(xs), np.concatenate(os_)
    w = np.exp(x - _logsumexp(x))
    return float(np.sum(w * o)) / len(pairs)


def free_fermion_spin_pairs(h, beta, pairs):
    """U = 0 closed form (Wick): with the one-particle density matrix
    G = (exp(beta h) + 1)^-1 per spin, <S_i . S_j> = -(3/2) G_ij^2 for i != j
    (Sz Sz gives -G_ij^2/2, the spin-flip pair -G_ij^2).  Averaged over pairs."""
    eps, U = np.linalg.eigh(h)
    G = (U / (np.exp(beta * eps) + 1.0)) @ U.T
    return float(np.mean([-1.5 * G[i, j] ** 2 for (i, j) in pairs]))


def same_ode_single(E, beta0, beta, order=1):
    """ln Tr rho(beta) for rho(beta) = exp(-(beta-beta0) H) rho0, rho0 the
    start of ``start_poly``."""
    a = start_poly(E, beta0, order)
    x = -(beta - beta0) * E
    m = np.max(x)
    return m + np.log(np.sum(a * np.exp(x - m)))


def free_fermion_lnZ(h, beta):
    """U = 0 closed form: ln Z = 2 sum_k ln(1 + exp(-beta eps_k)), eps = eig(h)."""
    eps = np.linalg.eigvalsh(h)
    return 2.0 * float(np.sum(np.logaddexp(0.0, -beta * eps)))


def free_fermion_energy(h, beta):
    """U = 0 closed form: <H> = 2 sum_k eps_k f(eps_k)."""
    eps = np.linalg.eigvalsh(h)
    return 2.0 * float(np.sum(eps / (np.exp(beta * eps) + 1.0)))


def same_ode_bilayer_local(model, beta0, beta):
    """Density and double occupancy per site, bilayer values at 2*beta:
    <O> = Tr(O rho^2) / Tr(rho^2) for rho = exp(-(beta-beta0) H) (1 - beta0 H)
    (SM Sec. II.A), O = sum_i n_i or sum_i n_iu n_id.  Both are diagonal in
    the Fock basis, so <k|O|k> = sum_f |V_fk|^2 O_f over each eigenvector.
    Returns (n, docc)."""
    N = model.N
    xs, ns, ds = [], [], []
    for nup in range(N + 1):
        for ndn in range(N + 1):
            h, _ = model.sector_hamiltonian(nup, ndn)
            states = model.sector_states(nup, ndn)
            docc = np.array([sum(o[2 * i] * o[2 * i + 1] for i in range(N)) for o in states], dtype=float)
            E, V = np.linalg.eigh(h)
            a = 1.0 - beta0 * E
            xs.append(2.0 * np.log(np.abs(a)) - 2.0 * (beta - beta0) * E)
            ns.append(np.full(E.size, float(nup + ndn)))
            ds.append((V ** 2).T @ docc)
    x, n, d = np.concatenate(xs), np.concatenate(ns), np.concatenate(ds)
    w = np.exp(x - _logsumexp(x))
    return float(np.sum(w * n)) / N, float(np.sum(w * d)) / N



# ---------------------------------------------------------------- Matsubara G
def momentum_phases(W, L, k):
    """k . r for every chain index, r = (x, y) the lattice coordinates of the
    snake order (x along the length L, y across the width W)."""
    return np.array([k[0] * x + k[1] * y for (x, y) in lattice.snake_order(W, L)])


def green_k(model, rho, k):
    """Single-particle Matsubara Green's function at half the imaginary time
    of a density operator (main text, Fermi-surface paragraph):
    G(k, beta/2) = sum_s Tr[rho c+_ks rho c_ks] / Tr[rho rho], with
    c_ks = N^-1/2 sum_r exp(-i k.r) c_rs.  For rho = exp(-beta H / 2) this is
    sum_s <exp(beta H/2) c+_ks exp(-beta H/2) c_ks>_beta; for a bilayer state
    rho(beta) it is the value at beta_phys = 2 beta.  Complex arithmetic as
    written; the imaginary part vanishes for a real symmetric rho."""
    N = model.N
    ph = momentum_phases(model.W, model.L, k)
    num = 0.0 + 0.0j
    for spin in (0, 1):
        ck = sum(np.exp(-1j * ph[r]) * model.dense_annihilator(r, spin) for r in range(N)) / np.sqrt(N)
        num += np.trace(rho @ ck.conj().T @ rho @ ck)
    den = np.trace(rho @ rho)
    assert abs(num.imag) <= 1e-12 * max(1.0, abs(num.real))
    return float(num.real / den)


def thermal_green(model, beta, k):
    """G(k, beta/2) of the thermal state exp(-beta H)."""
    return green_k(model, model.dense_function(lambda E: np.exp(-0.5 * beta * E)), k)


def same_ode_bilayer_green(model, beta0, beta, k):
    """G(k, beta_phys/2) at beta_phys = 2 beta for the flow of
    ``same_ode_bilayer``: rho(beta) = exp(-(beta-beta0) H) (1 - beta0 H)."""
    return green_k(model, model.dense_function(lambda E: np.exp(-(beta - beta0) * E) * (1.0 - beta0 * E)), k)


def free_fermion_green(h, W, L, beta, k):
    """U = 0 closed form: with h = sum_m eps_m phi_m phi_m^T,
    <c+_r(beta/2) c_r'> = sum_m phi_m(r) phi_m(r') exp(beta eps_m / 2) f(eps_m)
    = sum_m phi_m(r) phi_m(r') / (2 cosh(beta eps_m / 2)), so
    G(k, beta/2) = (2/N) sum_m |sum_r exp(i k.r) phi_m(r)|^2 / (2 cosh(beta eps_m / 2))
    (both spins)."""
    eps, phi = np.linalg.eigh(h)
    ph = momentum_phases(W, L, k)
    amp = np.abs(np.exp(1j * ph) @ phi) ** 2
    return 2.0 * float(np.sum(amp / (2.0 * np.cosh(0.5 * beta * eps)))) / h.shape[0]


def atomic_green(U, mu, beta):
    """t = 0 closed form (every k): one site with energies 0, -mu (twice),
    U - 2 mu; per spin Tr[exp(-beta H/2) c+ exp(-beta H/2) c] collects the
    pairs (0 -> s) and (other spin -> both), so
    G = 2 [exp(beta mu / 2) + exp(-beta (U - 3 mu) / 2)] / Z_site."""
    z = 1.0 + 2.0 * np.exp(beta * mu) + np.exp(-beta * (U - 2.0 * mu))
    return 2.0 * (np.exp(0.5 * beta * mu) + np.exp(-0.5 * beta * (U - 3.0 * mu))) / z


# ---------------------------------------------------------------- pairing field
def pairing_bonds(W, L, geometry):
    """Nearest-neighbour bonds (i < j) with the d-wave form factor s_ij: +1 for
    a bond along the length (x), -1 across the width (y) (main text, d-wave
    pairing paragraph)."""
    order = lattice.snake_order(W, L)
    out = []
    for (i, j) in lattice.nn_bonds(W, L, geometry):
        (xi, _), (xj, _) = order[i], order[j]
        out.append((i, j, 1.0 if xi != xj else -1.0))
    return out


def dense_pairing(model):
    """Delta_tot = sum_<ij> s_ij (Delta_ij + Delta_ij^+)/2 with
    Delta_ij = (c_i,dn c_j,up - c_i,up c_j,dn)/sqrt 2, as a dense 4^N matrix."""
    N = model.N
    C = {(i, s): model.dense_annihilator(i, s) for i in range(N) for s in (0, 1)}
    out = np.zeros((4 ** N, 4 ** N))
    for (i, j, s) in pairing_bonds(model.W, model.L, model.geometry):
        d = (C[(i, 1)] @ C[(j, 0)] - C[(i, 0)] @ C[(j, 1)]) / np.sqrt(2.0)
        out += s * (d + d.T) / 2.0
    return out


def dense_hamiltonian_with_pairing(model, hp):
    """H - hp Delta_tot as a dense matrix (the field breaks N_up, N_down)."""
    return model.dense_hamiltonian() - hp * dense_pairing(model)


def same_ode_bilayer_pairing(model, hp, beta0, beta):
    """Bilayer values at beta_phys = 2 beta for rho(beta) = exp(-(beta-beta0) H)
    (1 - beta0 H), H with the pairing field: (ln Z_bl, E_bl, Delta_p) with
    Delta_p = <Delta_tot> / N_p, <O> = Tr(O rho^2) / Tr(rho^2)."""
    H = dense_hamiltonian_with_pairing(model, hp)
    E, V = np.linalg.eigh(H)
    a = 1.0 - beta0 * E
    x = 2.0 * np.log(np.abs(a)) - 2.0 * (beta - beta0) * E
    lnZ = _logsumexp(x)
    w = np.exp(x - lnZ)
    Dt = dense_pairing(model)
    d = np.einsum("fk,fg,gk->k", V, Dt, V)
    nb = len(pairing_bonds(model.W, model.L, model.geometry))
    return lnZ, float(np.sum(w * E)), float(np.sum(w * d)) / nb


def thermal_pairing(model, hp, beta):
    """Exact thermal (ln Z, Delta_p) of exp(-beta (H - hp Delta_tot)), dense."""
    H = dense_hamiltonian_with_pairing(model, hp)
    E, V = np.linalg.eigh(H)
    x = -beta * E
    lnZ = _logsumexp(x)
    w = np.exp(x - lnZ)
    d = np.einsum("fk,fg,gk->k", V, dense_pairing(model), V)
    nb = len(pairing_bonds(model.W, model.L, model.geometry))
    return lnZ, float(np.sum(w * d)) / nb


def bdg_pairing(model, hp, beta):
    """U = 0 closed form (Bogoliubov-de Gennes).  With the Nambu spinor
    psi = (c_up, c+_dn), H = psi^+ H_B psi + Tr h, H_B = [[h, K], [K, -h]],
    h the hopping matrix (with -mu) and K_ij = K_ji = -hp s_ij / (2 sqrt 2)
    on the bonds (from c_i,dn c_j,up + c_j,dn c_i,up = psi^+_{N+i} psi_j +
    psi^+_{N+j} psi_i).  With <psi^+_a psi_b> = [f(H_B)]_ba:
    ln Z = -beta Tr h + sum_n ln(1 + exp(-beta E_n)) over the 2N eigenvalues,
    <Delta_tot> = sum_<ij> s_ij / sqrt 2 (<psi^+_{N+i} psi_j> + <psi^+_{N+j} psi_i>).
    Returns (ln Z, Delta_p)."""
    assert model.U == 0.0
    N = model.N
    h = model.hopping_matrix()
    K = np.zeros((N, N))
    bonds = pairing_bonds(model.W, model.L, model.geometry)
    for (i, j, s) in bonds:
        K[i, j] = K[j, i] = -hp * s / (2.0 * np.sqrt(2.0))
    HB = np.block([[h, K], [K, -h]])
    E, U = np.linalg.eigh(HB)
    f = 1.0 / (np.exp(beta * E) + 1.0)
    G = (U * f) @ U.T                      # G[b, a] = <psi^+_a psi_b>
    lnZ = -beta * np.trace(h) + float(np.sum(np.logaddexp(0.0, -beta * E)))
    tot = sum(s / np.sqrt(2.0) * (G[j, N + i] + G[i, N + j]) for (i, j, s) in bonds)
    return lnZ, float(tot) / len(bonds)
