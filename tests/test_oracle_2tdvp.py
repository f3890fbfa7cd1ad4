"""Pins of the oracle's 2-TDVP sweep (SM Sec. "2-TDVP in the initial stage",
Eq. S-2TDVP): exact at full bonds against the same-flow ED, adaptive bond
growth from the bare start, truncation by D_max."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo, tdvp


@pytest.mark.parametrize("W,L,geo,U,mu", [(2, 2, lattice.OPEN_SQUARE, 8.0, 1.5), (1, 4, lattice.CHAIN, 4.0, 0.3)])
def test_exact_from_full_bonds(W, L, geo, U, mu):
    # zero-padded full bonds: the two-site splitting is then exact
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu)
    st = tdvp.initial_state(m, 0.01, 16 ** 8, False)
    E, _, _ = ed.Hubbard(W, L, geo, 1.0, U, mu).spectrum()
    for _ in range(4):
        st.sweep2(0.05, 10 ** 6)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, 0.01, st.beta)
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - Ebl) <= 1e-10 * abs(Ebl)


def test_bonds_grow_from_the_bare_start():
    # the chain's rho0 = 1 - beta0 H has bonds D_H = 6; the two-site updates
    # grow them to the full 16 / 256 / 16 and the flow is exact
    m = mpo.HubbardMPO(1, 4, lattice.CHAIN, 1.0, 4.0, 0.3)
    st = tdvp.initial_state(m, 0.01, 1, False)
    assert st.dims() == [1, 6, 6, 6, 1]
    E, _, _ = ed.Hubbard(1, 4, lattice.CHAIN, 1.0, 4.0, 0.3).spectrum()
    for _ in range(6):
        st.sweep2(0.05, 10 ** 6)
    assert st.dims() == [1, 16, 256, 16, 1]
    lnZ, _ = ed.same_ode_bilayer(E, 0.01, st.beta)
    assert abs(st.observables()["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)


def test_truncation_caps_the_bonds():
    m = mpo.HubbardMPO(1, 5, lattice.CHAIN, 1.0, 4.0, 0.3)
    st = tdvp.initial_state(m, 0.01, 1, False)
    E, _, _ = ed.Hubbard(1, 5, lattice.CHAIN, 1.0, 4.0, 0.3).spectrum()
    for _ in range(4):
        st.sweep2(0.1, 12)
    assert max(st.dims()) == 12
    # the truncated state stays close to the exact flow at this temperature
    lnZ, Ebl = ed.same_ode_bilayer(E, 0.01, st.beta)
    o = st.observables()
    assert abs(o["E"] - Ebl) <= 1e-2 * abs(Ebl)
    # and the centre is normalised with right-orthonormal sites behind it
    for k in range(1, 5):
        a = st.A[k].reshape(st.A[k].shape[0], -1)
        assert np.allclose(a @ a.T, np.eye(a.shape[0]), atol=1e-12)
