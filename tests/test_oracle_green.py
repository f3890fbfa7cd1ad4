"""Pins of the oracle's Matsubara Green's function at half the imaginary time,
G(k, beta/2) = sum_s <exp(beta H/2) c+_ks exp(-beta H/2) c_ks> (main text,
Fermi-surface paragraph): the U = 0 closed form, the atomic limit, infinite
temperature, and the super-operator MPO against the dense ED operators
(occupation-number signs on one side, Jordan-Wigner matrices on the other)."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo, tdvp

KS = [(0.0, 0.0), (np.pi, 0.0), (0.7, np.pi), (np.pi / 2, 2 * np.pi / 3)]


@pytest.mark.parametrize("W,L,geo", [(1, 4, lattice.CHAIN), (2, 2, lattice.OPEN_SQUARE), (1, 5, lattice.CHAIN)])
@pytest.mark.parametrize("beta", [0.4, 3.0])
def test_free_fermion_closed_form(W, L, geo, beta):
    h = ed.Hubbard(W, L, geo, t=1.0, U=0.0, mu=0.35)
    for k in KS:
        got = ed.thermal_green(h, beta, k)
        want = ed.free_fermion_green(h.hopping_matrix(), W, L, beta, k)
        assert abs(got - want) < 1e-12, (k, got, want)


@pytest.mark.parametrize("U,mu,beta", [(5.0, 1.2, 0.9), (8.0, 4.0, 2.5), (3.0, -0.5, 1.7)])
def test_atomic_limit(U, mu, beta):
    # t = 0: sites decouple, G_rr' = delta_rr' G_site, the same value for every k
    h = ed.Hubbard(1, 3, lattice.CHAIN, t=0.0, U=U, mu=mu)
    want = ed.atomic_green(U, mu, beta)
    for k in KS:
        assert abs(ed.thermal_green(h, beta, k) - want) < 1e-12


def test_infinite_temperature_and_bounds():
    # rho = 1: Tr[c+_k c_k] / 4^N = 1/2 per spin for a normalised mode
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=1.0, U=6.0, mu=1.0)
    for k in KS:
        assert abs(ed.thermal_green(h, 0.0, k) - 1.0) < 1e-13
        # 0 <= G <= 1: G = ||rho^1/4 c_k rho^1/4||^2 per spin, bounded by
        # sqrt(<c+c><cc+>) <= 1/2
        g = ed.thermal_green(h, 2.0, k)
        assert 0.0 < g <= 1.0


def _choi(rho, N):
    """|rho>> with site-major super index s_i = 4 sigma_i + sigma'_i."""
    T = rho.reshape([4] * (2 * N))
    perm = [q for i in range(N) for q in (i, N + i)]
    return T.transpose(perm).reshape(-1)


def _mpo_apply(Ws, v, N):
    """X|v>> for a super-operator MPO with boundary bonds of dimension 1."""
    V = v.reshape(1, 1, 16, 16 ** (N - 1))
    for q, Wq in enumerate(Ws):
        V = np.einsum("bpsr,bosc->cpor", V, Wq)
        c, P, o, R = V.shape
        if q + 1 < N:
            V = V.reshape(c, P * o, 16, R // 16)
        else:
            V = V.reshape(c, P * o)
    return V[0]


@pytest.mark.parametrize("W,L,geo,U,mu", [(1, 4, lattice.CHAIN, 4.0, 0.3), (2, 2, lattice.OPEN_SQUARE, 8.0, 1.5),
                                          (1, 3, lattice.CHAIN, 2.0, -0.7)])
def test_mpo_matches_dense_operators(W, L, geo, U, mu):
    h = ed.Hubbard(W, L, geo, t=1.0, U=U, mu=mu)
    N = h.N
    rho = h.dense_function(lambda E: np.exp(-0.6 * E) * (1.0 - 0.02 * E))
    v = _choi(rho, N)
    for k in KS:
        Xv = _mpo_apply(mpo.green_mpo(W, L, k), v, N)
        got = float(v @ Xv) / (N * float(v @ v))
        assert abs(got - ed.green_k(h, rho, k)) < 1e-12, k


@pytest.mark.parametrize("beta", [0.5, 2.0])
def test_mpo_free_fermion_closed_form(beta):
    # pins the MPO alone: rho = exp(-beta H/2) at U = 0 against the closed form
    W, L = 2, 2
    h = ed.Hubbard(W, L, lattice.OPEN_SQUARE, t=1.0, U=0.0, mu=-0.3)
    v = _choi(h.dense_function(lambda E: np.exp(-0.5 * beta * E)), 4)
    for k in KS:
        Xv = _mpo_apply(mpo.green_mpo(W, L, k), v, 4)
        got = float(v @ Xv) / (4 * float(v @ v))
        assert abs(got - ed.free_fermion_green(h.hopping_matrix(), W, L, beta, k)) < 1e-12


@pytest.mark.parametrize("W,L,geo,U,mu,sym", [(1, 4, 0, 4.0, 0.0, True), (2, 2, 2, 8.0, 1.5, True),
                                               (1, 4, 0, 4.0, 0.7, False)])
def test_oracle_state_exact_at_maximal_bond(W, L, geo, U, mu, sym):
    # the super-MPS expectation of the oracle state at untruncated bonds equals
    # the same-flow ED value (bilayer, beta_phys = 2 beta)
    b0 = 0.01
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu)
    st = tdvp.initial_state(m, b0, 16 ** 8, sym)
    for _ in range(6):
        st.sweep(0.05)
    h = ed.Hubbard(W, L, geo, 1.0, U, mu)
    for k in KS[:3]:
        got = st.super_expectation(mpo.green_mpo(W, L, k)) / (W * L)
        want = ed.same_ode_bilayer_green(h, b0, st.beta, k)
        assert abs(got - want) <= 1e-10, (k, got, want)
