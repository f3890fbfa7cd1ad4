"""Pins of the oracle's local observables (density and double occupancy at
beta_phys = 2 beta, SM Sec. II.A bilayer; main text Fig. 2 for D_n)."""
import os
import sys

import numpy as np
import pytest
from scipy.linalg import expm

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import ed, mpo, tdvp  # noqa: E402

N_OP = [0.0, 1.0, 1.0, 2.0]
D_OP = [0.0, 0.0, 0.0, 1.0]


def _dense_diag(N, op):
    """sum_i op_i as the diagonal of the 4^N dense operator (index sum sigma_i 4^(N-1-i))."""
    d = np.zeros(4 ** N)
    for idx in range(4 ** N):
        x = idx
        for i in range(N):
            d[idx] += op[x % 4]
            x //= 4
    return d


@pytest.mark.parametrize("N", [1, 3, 4])
def test_local_sum_mpo_equals_dense_operator(N):
    for op in (N_OP, D_OP, [0.3, -1.0, 2.0, 0.5]):
        got = mpo.mpo_to_dense(mpo.local_sum_mpo(N, op))
        assert np.abs(got - np.diag(_dense_diag(N, op))).max() < 1e-14


def test_ed_local_infinite_temperature():
    # rho = 1: every one of the 4^N states has weight 1 -> n = 1, D_n = 1/4
    h = ed.Hubbard(2, 2, 2, 1.0, 8.0, 1.3)
    n, d = ed.same_ode_bilayer_local(h, 0.0, 0.0)
    assert abs(n - 1.0) < 1e-14 and abs(d - 0.25) < 1e-14


@pytest.mark.parametrize("beta", [0.3, 1.5, 4.0])
def test_ed_local_half_filling_and_brute_force(beta):
    # particle-hole symmetry: n = 1 at mu = U/2 for any beta
    h = ed.Hubbard(1, 4, 0, 1.0, 6.0, 3.0)
    n, _ = ed.same_ode_bilayer_local(h, 0.01, beta)
    assert abs(n - 1.0) < 1e-12
    # brute force: dense expm for the same-ODE density operator, away from half filling
    h = ed.Hubbard(1, 4, 0, 1.0, 4.0, 0.7)
    H = h.dense_hamiltonian()
    b0 = 0.01
    rho = expm(-(beta - b0) * H) @ (np.eye(256) - b0 * H)
    r2 = rho @ rho.T
    for op, val in zip((N_OP, D_OP), ed.same_ode_bilayer_local(h, b0, beta)):
        want = np.sum(_dense_diag(4, op) * np.diag(r2)) / np.trace(r2) / 4
        assert abs(val - want) < 1e-12 * max(abs(want), 1e-2)


@pytest.mark.parametrize("W,L,geo,U,mu,sym", [(1, 4, 0, 4.0, 0.0, True), (2, 2, 2, 8.0, 1.5, True),
                                               (1, 4, 0, 4.0, 0.7, False)])
def test_oracle_local_observables_exact_at_maximal_bond(W, L, geo, U, mu, sym):
    b0 = 0.01
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu)
    st = tdvp.initial_state(m, b0, 16 ** 8, sym)
    for _ in range(10):
        st.sweep(0.05)
    N = W * L
    n = st.expectation(mpo.local_sum_mpo(N, N_OP)) / N
    d = st.expectation(mpo.local_sum_mpo(N, D_OP)) / N
    n_ref, d_ref = ed.same_ode_bilayer_local(ed.Hubbard(W, L, geo, 1.0, U, mu), b0, st.beta)
    # per-site quantities of order one: the FP64 bar 1e-10, absolute
    assert abs(n - n_ref) <= 1e-10
    assert abs(d - d_ref) <= 1e-10
