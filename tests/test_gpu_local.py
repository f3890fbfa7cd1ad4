"""GPU parity of the local observables (density n and double occupancy D_n at
beta_phys = 2 beta) with ED at untruncated bonds and with the oracle at
truncated bonds (same initial tensors)."""
import numpy as np
import pytest

from oracle import ed, mpo as ompo, tdvp as otd
from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu

TOL = 1e-10           # per-site quantities of order one, absolute
N_OP = [0.0, 1.0, 1.0, 2.0]
D_OP = [0.0, 0.0, 0.0, 1.0]


@pytest.mark.parametrize("W,L,geo,U,mu,sym", [(1, 4, T.TT_CHAIN, 4.0, 0.0, 1), (1, 4, T.TT_CHAIN, 4.0, 0.7, 0),
                                               (2, 2, T.TT_OPEN_SQUARE, 8.0, 1.5, 1)])
def test_local_observables_match_ed_untruncated(W, L, geo, U, mu, sym):
    b0 = 0.01
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=256, symmetry=sym, beta0=b0))
    h = ed.Hubbard(W, L, geo, 1.0, U, mu)
    for step in range(12):
        if step % 4 == 0:
            lo = st.local_observables()
            beta = st.observables()["beta"]
            n_ref, d_ref = ed.same_ode_bilayer_local(h, b0, beta)
            assert abs(lo["n"] - n_ref) <= TOL, (step, lo, n_ref)
            assert abs(lo["docc"] - d_ref) <= TOL, (step, lo, d_ref)
        st.sweep(0.05)
    st.free()


def test_half_filling_density_is_one():
    # particle-hole symmetry at mu = U/2, untruncated: n = 1
    st = T.State.init(T.model(1, 4, T.TT_CHAIN, 1.0, 6.0, 3.0), T.options(D=256, symmetry=1, beta0=0.01))
    for _ in range(10):
        st.sweep(0.1)
    assert abs(st.local_observables()["n"] - 1.0) < 1e-11
    st.free()


@pytest.mark.parametrize("W,L,geo,U,mu,D,sym,pad", [(2, 3, T.TT_OPEN_SQUARE, 8.0, 1.0, 20, 1, 0.3),
                                                     (3, 3, T.TT_CYLINDER, 8.0, 2.0, 24, 1, 0.3),
                                                     (1, 6, T.TT_CHAIN, 4.0, 0.3, 12, 0, 1e-3)])
def test_local_observables_match_oracle_truncated(W, L, geo, U, mu, D, sym, pad):
    b0 = 0.01
    mm = ompo.HubbardMPO(W, L, geo, 1.0, U, mu)
    ost = otd.initial_state(mm, b0, D, bool(sym), pad_eps=pad, seed=11, sector_cap=64)
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=D, symmetry=sym, beta0=b0, pad_eps=pad, seed=11))
    for _ in range(2):
        st.sweep(0.1)
        ost.sweep(0.1)
    N = W * L
    lo = st.local_observables()
    n_ref = ost.expectation(ompo.local_sum_mpo(N, N_OP)) / N
    d_ref = ost.expectation(ompo.local_sum_mpo(N, D_OP)) / N
    assert abs(lo["n"] - n_ref) <= TOL, (lo, n_ref)
    assert abs(lo["docc"] - d_ref) <= TOL, (lo, d_ref)
    st.free()
