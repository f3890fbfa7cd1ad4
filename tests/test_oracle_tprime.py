"""Pins of the next-nearest hopping t' (SM Eq. S1) in the oracle: the 2x2
plaquette's single-particle levels, the MPO against the Fock-space H, charge
conservation, the U = 0 closed form and the broken particle-hole symmetry."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo

TP_CASES = [(2, 2, lattice.OPEN_SQUARE, 1.0, 8.0, 1.3, -0.25), (3, 2, lattice.CYLINDER, 0.7, 2.0, -0.5, 0.3),
            (2, 3, lattice.OPEN_SQUARE, 1.0, 8.0, 4.0, -0.25), (3, 2, lattice.CYLINDER, 1.0, 0.0, 0.2, -0.4)]


def test_plaquette_single_particle_levels():
    # 2x2 plaquette: a ring of four bonds t and two diagonals t'.  The ring's
    # Bloch phases k = 0, pi/2, pi, 3pi/2 give -2t cos k; the diagonal joins
    # opposite corners, adding -t' e^{2ik} = -t', +t', -t', +t'.
    t, tp = 1.0, -0.25
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=t, U=0.0, mu=0.0, tp=tp).hopping_matrix()
    want = sorted([-2 * t - tp, tp, tp, 2 * t - tp])
    assert np.allclose(np.linalg.eigvalsh(h), want, atol=1e-14)
    assert lattice.nnn_bonds(2, 2, lattice.OPEN_SQUARE) == [(0, 2), (1, 3)]
    assert lattice.nnn_bonds(1, 6, lattice.CHAIN) == []


@pytest.mark.parametrize("W,L,geo,t,U,mu,tp", TP_CASES)
def test_mpo_equals_fock_hamiltonian_with_tprime(W, L, geo, t, U, mu, tp):
    Hd = ed.Hubbard(W, L, geo, t, U, mu, tp=tp).dense_hamiltonian()
    m = mpo.HubbardMPO(W, L, geo, t, U, mu, tp=tp)
    assert np.abs(mpo.mpo_to_dense(m.mpo_for_env()) - Hd).max() < 1e-13
    for k, Wk in enumerate(m.W):
        qa, qb = m.bond_charges(k), m.bond_charges(k + 1)
        for a, so, si, b in zip(*np.nonzero(Wk)):
            qo, qi = mpo.local_charge(so), mpo.local_charge(si)
            assert (qa[a][0] + qo[0] - qi[0], qa[a][1] + qo[1] - qi[1]) == qb[b]


def test_tprime_zero_leaves_the_mpo_unchanged():
    a = mpo.HubbardMPO(4, 4, lattice.CYLINDER, 1.0, 8.0, 1.5)
    b = mpo.HubbardMPO(4, 4, lattice.CYLINDER, 1.0, 8.0, 1.5, tp=0.0)
    assert a.states == b.states and all(np.array_equal(x, y) for x, y in zip(a.W, b.W))
    c = mpo.HubbardMPO(4, 4, lattice.CYLINDER, 1.0, 8.0, 1.5, tp=-0.25)
    assert max(len(s) for s in c.states) > max(len(s) for s in a.states)


@pytest.mark.parametrize("beta", [0.3, 2.0])
def test_free_fermion_closed_form_with_tprime(beta):
    h = ed.Hubbard(2, 3, lattice.OPEN_SQUARE, t=1.0, U=0.0, mu=0.2, tp=-0.3)
    E, _, _ = h.spectrum()
    lnZ, En = ed.thermal_physical(E, beta)
    hm = h.hopping_matrix()
    assert abs(lnZ - ed.free_fermion_lnZ(hm, beta)) < 1e-10 * abs(lnZ)
    assert abs(En - ed.free_fermion_energy(hm, beta)) < 1e-10 * max(1.0, abs(En))


def test_tprime_breaks_half_filling_at_mu_u_over_2():
    # on the bipartite square lattice mu = U/2 is half filling for t' = 0; the
    # diagonal hopping joins sites of one sublattice and breaks that symmetry
    U, beta = 8.0, 2.0
    for tp, exact in ((0.0, True), (-0.25, False)):
        h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=1.0, U=U, mu=U / 2, tp=tp)
        E, nu, nd = h.spectrum()
        w = np.exp(-beta * (E - E.min()))
        n = float(np.sum(w * (nu + nd)) / np.sum(w)) / h.N
        assert (abs(n - 1.0) < 1e-12) == exact
