"""Pins of the oracle's d-wave pairing field -hp Delta_tot (main text, pairing
paragraph): the U = 0 Bogoliubov-de Gennes closed form, the MPO against the
dense ED operator, the zero of <Delta> without a field, linear response, and
the flow at untruncated bonds."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo, tdvp


def test_pairing_bonds_form_factor():
    b = ed.pairing_bonds(2, 2, lattice.OPEN_SQUARE)
    # snake order (x, y): 0 (0,1), 1 (0,0), 2 (1,0), 3 (1,1): two vertical, two horizontal bonds
    assert sorted(b) == [(0, 1, -1.0), (0, 3, 1.0), (1, 2, 1.0), (2, 3, -1.0)]
    assert all(s == 1.0 for (_, _, s) in ed.pairing_bonds(1, 5, lattice.CHAIN))


@pytest.mark.parametrize("W,L,geo,mu,hp,beta", [(1, 4, lattice.CHAIN, 0.3, 0.2, 1.3), (2, 2, lattice.OPEN_SQUARE, -0.5, 0.5, 2.0),
                                                (1, 5, lattice.CHAIN, 0.0, 0.1, 0.7), (1, 3, lattice.CHAIN, 0.4, 0.3, 1.1)])
def test_ed_matches_bdg_closed_form(W, L, geo, mu, hp, beta):
    h = ed.Hubbard(W, L, geo, 1.0, 0.0, mu)
    lnZ, d = ed.thermal_pairing(h, hp, beta)
    lnZ_b, d_b = ed.bdg_pairing(h, hp, beta)
    assert abs(lnZ - lnZ_b) < 1e-11
    assert abs(d - d_b) < 1e-12


@pytest.mark.parametrize("W,L,geo,hp", [(1, 4, lattice.CHAIN, 0.3), (2, 2, lattice.OPEN_SQUARE, 0.5),
                                        (1, 3, lattice.CHAIN, -0.7), (2, 2, lattice.OPEN_SQUARE, 0.0)])
def test_mpo_contracts_to_ed_operator(W, L, geo, hp):
    h = ed.Hubbard(W, L, geo, 1.0, 4.0, 0.3)
    m = mpo.HubbardMPO(W, L, geo, 1.0, 4.0, 0.3, hp=hp)
    assert np.abs(mpo.mpo_to_dense(m.mpo_for_env()) - ed.dense_hamiltonian_with_pairing(h, hp)).max() < 1e-13
    # with t = U = mu = 0 and hp = -1 the MPO is Delta_tot itself
    d = mpo.HubbardMPO(W, L, geo, 0.0, 0.0, 0.0, hp=-1.0)
    assert np.abs(mpo.mpo_to_dense(d.mpo_for_env()) - ed.dense_pairing(h)).max() < 1e-13


def test_no_field_no_order_and_linear_response():
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, 1.0, 6.0, 1.0)
    assert abs(ed.thermal_pairing(h, 0.0, 1.5)[1]) < 1e-14
    # Delta_p is odd in hp and linear at small hp: chi = Delta_p / hp converges
    d1 = ed.thermal_pairing(h, 1e-3, 1.5)[1]
    d2 = ed.thermal_pairing(h, 2e-3, 1.5)[1]
    dm = ed.thermal_pairing(h, -1e-3, 1.5)[1]
    assert abs(d1 + dm) < 1e-14
    assert d1 > 0.0
    assert abs(d2 / 2e-3 - d1 / 1e-3) < 1e-4 * abs(d1 / 1e-3)


@pytest.mark.parametrize("W,L,geo,U,mu,hp", [(1, 4, lattice.CHAIN, 4.0, 0.3, 0.3), (2, 2, lattice.OPEN_SQUARE, 8.0, 1.5, 0.5)])
def test_oracle_flow_exact_at_maximal_bond(W, L, geo, U, mu, hp):
    b0 = 0.01
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu, hp=hp)
    st = tdvp.initial_state(m, b0, 16 ** 8, False)
    for _ in range(6):
        st.sweep(0.05)
    lnZ, E, dp = ed.same_ode_bilayer_pairing(ed.Hubbard(W, L, geo, 1.0, U, mu), hp, b0, st.beta)
    o = st.observables()
    nb = len(ed.pairing_bonds(W, L, geo))
    got = st.expectation(mpo.HubbardMPO(W, L, geo, 0.0, 0.0, 0.0, hp=-1.0).mpo_for_env()) / nb
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - E) <= 1e-10 * max(abs(E), 1e-2)
    assert abs(got - dp) <= 1e-10


@pytest.mark.parametrize("W,L,geo,U,mu,hp", [(1, 4, lattice.CHAIN, 4.0, 0.3, 0.3), (2, 2, lattice.OPEN_SQUARE, 8.0, 1.5, 0.5)])
def test_sz_block_structure_flow_exact_at_maximal_bond(W, L, geo, U, mu, hp):
    # the pairing field conserves q_up - q_dn: blocks by that charge alone
    # (charges (sz, 0)) hold the flow exactly at untruncated bonds
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu, hp=hp)
    st = tdvp.initial_state(m, 0.01, 16 ** 8, True, mode="sz")
    assert all(q[1] == 0 for lay in st.layouts for q in lay.charges)
    for _ in range(6):
        st.sweep(0.05)
    lnZ, E, dp = ed.same_ode_bilayer_pairing(ed.Hubbard(W, L, geo, 1.0, U, mu), hp, 0.01, st.beta)
    o = st.observables()
    nb = len(ed.pairing_bonds(W, L, geo))
    got = st.expectation(mpo.HubbardMPO(W, L, geo, 0.0, 0.0, 0.0, hp=-1.0).mpo_for_env()) / nb
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - E) <= 1e-10 * max(abs(E), 1e-2)
    assert abs(got - dp) <= 1e-10


def test_sz_sector_counts():
    # the Sz-only counts are the sums of the U(1)xU(1) counts over q_up - q_dn
    from oracle import charges
    for N, k in [(6, 2), (8, 3), (10, 5)]:
        h = min(k, N - k)
        for a in range(-2 * h, 2 * h + 1):
            left = sum(charges.comb(2 * k, k + u) * charges.comb(2 * k, k + u - a)
                       for u in range(-k, k + 1) if abs(u - a) <= k)
            right = sum(charges.comb(2 * (N - k), N - k + u) * charges.comb(2 * (N - k), N - k + u - a)
                        for u in range(-(N - k), N - k + 1) if abs(u - a) <= N - k)
            assert charges._dmax(N, k, (a, 0), "sz") == min(left, right)
