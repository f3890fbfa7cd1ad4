"""Pins of the oracle's spin correlation F(d) = average over pairs at distance
d of <S_i . S_j> (main text, Fig. 2(c)): the U = 0 Wick closed form, spin
rotation symmetry, the Hubbard dimer's singlet, infinite temperature, the
pair lists, and the MPO against the dense ED operator."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo


def test_pairs_at_distance():
    # nearest neighbours are the lattice bonds; a cylinder wraps the short way
    for W, L, geo in [(1, 6, lattice.CHAIN), (3, 3, lattice.CYLINDER), (4, 4, lattice.CYLINDER), (2, 3, lattice.OPEN_SQUARE)]:
        assert lattice.pairs_at_distance(W, L, geo, 1) == lattice.nn_bonds(W, L, geo)
    # open 2x2 square: two diagonals; 4-wide cylinder: dy = 2 both ways
    assert len(lattice.pairs_at_distance(2, 2, lattice.OPEN_SQUARE, 2)) == 2
    assert len(lattice.pairs_at_distance(4, 1, lattice.CYLINDER, 4)) == 2
    assert lattice.pairs_at_distance(1, 5, lattice.CHAIN, 9) == [(0, 3), (1, 4)]


@pytest.mark.parametrize("W,L,geo,d2", [(1, 5, lattice.CHAIN, 1), (1, 5, lattice.CHAIN, 4),
                                        (2, 3, lattice.OPEN_SQUARE, 2), (3, 2, lattice.CYLINDER, 1)])
@pytest.mark.parametrize("beta_phys", [0.3, 2.0])
def test_free_fermion_wick(W, L, geo, d2, beta_phys):
    h = ed.Hubbard(W, L, geo, t=1.0, U=0.0, mu=0.4)
    pairs = lattice.pairs_at_distance(W, L, geo, d2)
    got = ed.same_ode_bilayer_spin_pairs(h, 0.0, beta_phys / 2, pairs)
    want = ed.free_fermion_spin_pairs(h.hopping_matrix(), beta_phys, pairs)
    assert abs(got - want) < 1e-12


@pytest.mark.parametrize("beta0,beta", [(0.0, 0.7), (0.01, 1.5)])
def test_spin_rotation_symmetry(beta0, beta):
    # H commutes with total spin: <S_i . S_j> = 3 <Sz_i Sz_j> (checks the
    # fermion signs of the spin-flip part against the diagonal part)
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=1.0, U=6.0, mu=2.1)
    for d2 in (1, 2):
        pairs = lattice.pairs_at_distance(2, 2, lattice.OPEN_SQUARE, d2)
        full = ed.same_ode_bilayer_spin_pairs(h, beta0, beta, pairs)
        zz = ed.same_ode_bilayer_spin_pairs(h, beta0, beta, pairs, zz_only=True)
        assert abs(full - 3.0 * zz) < 1e-12


def test_dimer_singlet_and_infinite_temperature():
    U, t = 8.0, 1.0
    h = ed.Hubbard(1, 2, lattice.CHAIN, t=t, U=U, mu=U / 2)
    pairs = [(0, 1)]
    # the half-filled ground state is a singlet a|S> + b|D>: singly occupied
    # singlet |S> (S_1 . S_2 = -3/4) mixed with the doubly occupied |D> by the
    # hopping; in the basis (|S>, |D>) H = [[0, -2t], [-2t, U]], so
    # E0 = (U - sqrt(U^2 + 16 t^2))/2 and |a|^2 = 1/(1 + E0^2/(4 t^2)).  The
    # triplet lies about 4t^2/U higher: negligible at beta_phys = 50.
    E0 = (U - np.sqrt(U * U + 16 * t * t)) / 2
    want = -0.75 / (1.0 + E0 * E0 / (4 * t * t))
    assert abs(ed.same_ode_bilayer_spin_pairs(h, 0.0, 25.0, pairs) - want) < 1e-9
    assert abs(ed.same_ode_bilayer_spin_pairs(h, 0.0, 0.0, pairs)) < 1e-14


@pytest.mark.parametrize("W,L,geo,d2", [(1, 4, lattice.CHAIN, 1), (1, 4, lattice.CHAIN, 9),
                                        (2, 2, lattice.OPEN_SQUARE, 2), (3, 2, lattice.CYLINDER, 1)])
def test_mpo_contracts_to_ed_operator(W, L, geo, d2):
    h = ed.Hubbard(W, L, geo, t=1.0, U=3.0, mu=0.5)
    pairs = lattice.pairs_at_distance(W, L, geo, d2)
    M = mpo.mpo_to_dense(mpo.spin_pair_mpo(h.N, pairs))
    assert np.abs(M - h.dense_spin_pairs(pairs)).max() < 1e-14
