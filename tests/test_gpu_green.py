"""GPU parity of the Matsubara Green's function G(k, beta_phys/2) (bilayer
value at beta_phys = 2 beta; a super-operator MPO acting on the ket and the
ancilla index) with ED at untruncated bonds and with the oracle at truncated
bonds (same initial tensors)."""
import math

import pytest

from oracle import ed, mpo as ompo, tdvp as otd
from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu

TOL = 1e-10           # G is of order one; absolute
KS = [(0.0, 0.0), (math.pi, 0.0), (0.7, math.pi), (math.pi / 2, 2 * math.pi / 3)]


@pytest.mark.parametrize("W,L,geo,U,mu,sym", [(1, 4, T.TT_CHAIN, 4.0, 0.0, 1),
                                               (1, 4, T.TT_CHAIN, 4.0, 0.7, 0),
                                               (2, 2, T.TT_OPEN_SQUARE, 8.0, 1.5, 1)])
def test_green_matches_ed_untruncated(W, L, geo, U, mu, sym):
    print("green ed", W, L, geo, sym, flush=True)
    b0 = 0.01
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=256, symmetry=sym, beta0=b0))
    h = ed.Hubbard(W, L, geo, 1.0, U, mu)
    for step in range(9):
        if step % 4 == 0:
            beta = st.observables()["beta"]
            for k in KS:
                G = st.green_function(*k)
                ref = ed.same_ode_bilayer_green(h, b0, beta, k)
                assert abs(G - ref) <= TOL, (step, k, G, ref)
        st.sweep(0.05)
    st.free()


def test_green_rejects_non_finite_momentum():
    st = T.State.init(T.model(1, 4, T.TT_CHAIN, 1.0, 4.0, 0.0), T.options(D=16, symmetry=1, beta0=0.01))
    with pytest.raises(T.TTError):
        st.green_function(float("nan"), 0.0)
    with pytest.raises(T.TTError):
        st.green_function(0.0, float("inf"))
    st.free()


@pytest.mark.parametrize("W,L,geo,U,mu,D,sym,pad", [(2, 3, T.TT_OPEN_SQUARE, 8.0, 1.0, 20, 1, 0.3),
                                                    (3, 3, T.TT_CYLINDER, 8.0, 2.0, 24, 1, 0.3),
                                                    (1, 6, T.TT_CHAIN, 4.0, 0.3, 12, 0, 1e-3)])
def test_green_matches_oracle_truncated(W, L, geo, U, mu, D, sym, pad):
    print("green oracle", W, L, geo, D, flush=True)
    b0 = 0.01
    mm = ompo.HubbardMPO(W, L, geo, 1.0, U, mu)
    ost = otd.initial_state(mm, b0, D, bool(sym), pad_eps=pad, seed=11, sector_cap=64)
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=D, symmetry=sym, beta0=b0, pad_eps=pad, seed=11))
    for _ in range(2):
        st.sweep(0.1)
        ost.sweep(0.1)
    first = None
    for k in KS[1:] + KS[1:2]:
        G = st.green_function(*k)
        ref = ost.super_expectation(ompo.green_mpo(W, L, k)) / (W * L)
        assert abs(G - ref) <= TOL, (k, G, ref)
        if first is None:
            first = G
    # returning to the first momentum rewrites the same weights: same value
    assert G == first
    st.free()


def test_full_size_cylinder_green_function():
    # 4x16 cylinder at D = 2000 (the sweep workload) at beta_phys ~ 0.1:
    # 0 < G <= 1 (G = ||rho^1/4 c_k rho^1/4||^2 summed over spins, each at most
    # 1/2), close to its infinite-temperature value 1
    print("green 4x16", flush=True)
    st = T.State.init(T.model(4, 16, T.TT_CYLINDER, 1.0, 8.0, 1.5),
                      T.options(D=2000, symmetry=1, beta0=0.05 / 4096, pad_eps=1e-3, seed=1))
    st.sweep(0.05)
    for k in [(0.0, 0.0), (math.pi, math.pi / 2), (math.pi / 2, math.pi)]:
        G = st.green_function(*k)
        assert 0.8 < G <= 1.0, (k, G)
    st.free()
