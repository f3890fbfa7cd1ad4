"""Pins of the exact-diagonalisation oracle against closed forms and
invariants fixed by the paper's model (Eq. 3) and by textbook results."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ed, lattice

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _eval(expr, t, U):
    return float(eval(expr.replace("^", "**"), {"sqrt": math.sqrt, "t": t, "U": U}))


def test_dimer_spectrum_matches_textbook_closed_form():
    g = json.load(open(os.path.join(GOLD, "hubbard_dimer.json")))
    t, U = g["t"], g["U"]
    h = ed.Hubbard(1, 2, lattice.CHAIN, t=t, U=U, mu=0.0)
    for key, exprs in g["sectors"].items():
        nu, nd = map(int, key.split(","))
        H, _ = h.sector_hamiltonian(nu, nd)
        got = np.sort(np.linalg.eigvalsh(H))
        want = np.sort([_eval(e, t, U) for e in exprs])
        assert np.allclose(got, want, atol=1e-12), key


@pytest.mark.parametrize("W,L,geo", [(1, 5, 0), (2, 3, 2), (3, 2, 1), (2, 2, 2)])
@pytest.mark.parametrize("beta", [0.1, 1.0, 3.0])
def test_free_fermion_closed_form(W, L, geo, beta):
    h = ed.Hubbard(W, L, geo, t=1.0, U=0.0, mu=0.37)
    E, _, _ = h.spectrum()
    lnZ, En = ed.thermal_physical(E, beta)
    hm = h.hopping_matrix()
    assert abs(lnZ - ed.free_fermion_lnZ(hm, beta)) < 1e-10 * abs(lnZ)
    assert abs(En - ed.free_fermion_energy(hm, beta)) < 1e-10 * max(1.0, abs(En))


def test_infinite_temperature_trace_and_entropy():
    g = json.load(open(os.path.join(GOLD, "paper_values.json")))
    h = ed.Hubbard(2, 2, 2, t=1.0, U=8.0, mu=1.0)
    E, _, _ = h.spectrum()
    assert E.size == g["local_dim"]["value"] ** h.N
    lnZ, _ = ed.thermal_physical(E, 0.0)
    assert abs(lnZ / h.N - g["entropy_per_site_infinite_T"]["value"]) < 1e-14


@pytest.mark.parametrize("W,L,geo", [(1, 4, 0), (2, 2, 2), (2, 3, 2)])
@pytest.mark.parametrize("beta", [0.3, 2.0, 6.0])
def test_half_filling_particle_hole(W, L, geo, beta):
    U = 8.0
    h = ed.Hubbard(W, L, geo, t=1.0, U=U, mu=U / 2)
    E, nu, nd = h.spectrum()
    x = -beta * E
    w = np.exp(x - x.max())
    n = float(np.sum(w * (nu + nd)) / np.sum(w)) / h.N
    assert abs(n - 1.0) < 1e-12


def test_snake_order_and_bonds():
    # Fig. 1a: columns of W sites traversed alternately down and up
    assert lattice.snake_order(3, 2) == [(0, 2), (0, 1), (0, 0), (1, 0), (1, 1), (1, 2)]
    # 4x4 cylinder: 2 W L bonds (periodic across, open along) minus the open ends
    b = lattice.nn_bonds(4, 4, lattice.CYLINDER)
    assert len(b) == 4 * 4 + 4 * 3
    # 4x4 open square: 2 * 4 * 3 bonds
    assert len(lattice.nn_bonds(4, 4, lattice.OPEN_SQUARE)) == 24
    # W = 2 cylinders get no doubled wrap bond
    assert lattice.nn_bonds(2, 3, lattice.CYLINDER) == lattice.nn_bonds(2, 3, lattice.OPEN_SQUARE)


def test_same_ode_reference_at_start():
    h = ed.Hubbard(1, 3, 0, t=1.0, U=4.0, mu=0.3)
    Hd = h.dense_hamiltonian()
    E, _, _ = h.spectrum()
    b0 = 0.02
    rho0 = np.eye(Hd.shape[0]) - b0 * Hd
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, b0)
    assert abs(lnZ - np.log(np.sum(rho0 * rho0))) < 1e-12
    assert abs(Ebl - np.trace(rho0 @ Hd @ rho0) / np.sum(rho0 * rho0)) < 1e-12
    assert abs(ed.same_ode_single(E, b0, b0) - np.log(np.trace(rho0))) < 1e-12
    # and after evolving: rho(beta) = expm(-(beta-b0) H) rho0
    from scipy.linalg import expm
    rb = expm(-(0.7 - b0) * Hd) @ rho0
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, 0.7)
    assert abs(lnZ - np.log(np.sum(rb * rb))) < 1e-10
    assert abs(Ebl - np.trace(rb.T @ Hd @ rb) / np.sum(rb * rb)) < 1e-10
