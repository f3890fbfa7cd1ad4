"""Pins of the oracle's entropy and specific heat (main text, Fig. 2(b) and
SM Fig. S1(c)): U = 0 closed forms, a brute-force derivative of the energy,
and the infinite-temperature limits."""
import math

import numpy as np
import pytest

from oracle import ed, lattice


@pytest.mark.parametrize("W,L,geo", [(1, 5, lattice.CHAIN), (2, 3, lattice.OPEN_SQUARE), (3, 2, lattice.CYLINDER)])
@pytest.mark.parametrize("beta_phys", [0.2, 1.0, 4.0])
def test_free_fermion_entropy_and_heat(W, L, geo, beta_phys):
    # beta0 = 0: the bilayer weights are exp(-beta_phys E), the Gibbs ensemble
    h = ed.Hubbard(W, L, geo, t=1.0, U=0.0, mu=0.37)
    E, _, _ = h.spectrum()
    th = ed.same_ode_bilayer_thermo(E, 0.0, beta_phys / 2.0, h.N)
    S, C = ed.free_fermion_entropy_heat(h.hopping_matrix(), beta_phys)
    assert abs(th["s"] - S / h.N) < 1e-10
    assert abs(th["c"] - C / h.N) < 1e-10


@pytest.mark.parametrize("beta0", [0.0, 0.01])
@pytest.mark.parametrize("beta", [0.05, 0.4, 1.5])
def test_specific_heat_is_minus_beta_squared_energy_slope(beta0, beta):
    # brute force: Richardson-extrapolated central differences of e(beta_phys)
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=1.0, U=8.0, mu=1.3)
    E, _, _ = h.spectrum()
    def e_at(bp):
        return ed.same_ode_bilayer(E, beta0, bp / 2.0)[1] / h.N
    bp = 2.0 * beta
    d = []
    for hstep in (1e-3, 5e-4):
        d.append((e_at(bp + hstep) - e_at(bp - hstep)) / (2 * hstep))
    slope = (4 * d[1] - d[0]) / 3
    th = ed.same_ode_bilayer_thermo(E, beta0, beta, h.N)
    assert abs(th["c"] - (-bp * bp * slope)) < 1e-8 * max(1.0, th["c"])
    assert th["c"] >= 0.0


def test_infinite_temperature_limits():
    # beta -> 0: entropy ln 4 per site (four local states), no specific heat
    h = ed.Hubbard(1, 4, lattice.CHAIN, t=1.0, U=4.0, mu=0.0)
    E, _, _ = h.spectrum()
    th = ed.same_ode_bilayer_thermo(E, 0.0, 1e-9, h.N)
    assert abs(th["s"] - math.log(4.0)) < 1e-7
    assert th["c"] < 1e-12


def test_entropy_decreases_on_cooling():
    h = ed.Hubbard(2, 2, lattice.OPEN_SQUARE, t=1.0, U=8.0, mu=4.0)
    E, _, _ = h.spectrum()
    s = [ed.same_ode_bilayer_thermo(E, 0.0, b, h.N)["s"] for b in np.linspace(0.05, 5.0, 40)]
    assert all(s[i + 1] < s[i] for i in range(len(s) - 1))
    assert s[-1] > 0.0
