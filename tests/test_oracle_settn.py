"""Pins of the oracle's SETTN start rho0 = sum_{n <= Nc} (-beta0 H)^n / n!
(SM I.E): the dense Taylor polynomial, the Taylor remainder bound against
exp(-beta0 H), the exact bond reduction (charges, sizes, minimality against
the dense Schmidt ranks), and the flow from it at untruncated bonds."""
import math

import numpy as np
import pytest

from oracle import charges, ed, lattice, mpo, tdvp


def _dense_poly(H, beta0, order):
    return sum(np.linalg.matrix_power(-beta0 * H, n) / math.factorial(n) for n in range(order + 1))


@pytest.mark.parametrize("W,L,geo", [(1, 4, lattice.CHAIN), (2, 2, lattice.OPEN_SQUARE), (1, 3, lattice.CHAIN)])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_contracts_to_taylor_polynomial(W, L, geo, order):
    h = ed.Hubbard(W, L, geo, 1.0, 5.0, 0.7)
    A, _ = mpo.settn_rho0(mpo.HubbardMPO(W, L, geo, 1.0, 5.0, 0.7), 0.2, order)
    H = h.dense_hamiltonian()
    assert np.abs(mpo.mpo_to_dense(A) - _dense_poly(H, 0.2, order)).max() < 1e-13


@pytest.mark.parametrize("W,L,geo,order", [(2, 2, lattice.OPEN_SQUARE, 1), (2, 2, lattice.OPEN_SQUARE, 2),
                                           (2, 2, lattice.OPEN_SQUARE, 3), (1, 4, lattice.CHAIN, 4)])
def test_taylor_remainder_bound(W, L, geo, order):
    # ||rho0 - exp(-beta0 H)||_2 <= (beta0 ||H||)^(order+1) / (order+1)! x exp(beta0 ||H||)
    b0 = 0.05
    h = ed.Hubbard(W, L, geo, 1.0, 6.0, 1.0)
    A, _ = mpo.settn_rho0(mpo.HubbardMPO(W, L, geo, 1.0, 6.0, 1.0), b0, order)
    rho0 = mpo.mpo_to_dense(A)
    Hn = np.abs(np.linalg.eigvalsh(h.dense_hamiltonian())).max()
    ex = h.dense_function(lambda E: np.exp(-b0 * E))
    err = np.linalg.norm(rho0 - ex, 2)
    bound = (b0 * Hn) ** (order + 1) / math.factorial(order + 1) * math.exp(b0 * Hn)
    assert err <= bound
    # and not far below it: the leading neglected term is of that order
    assert err >= 1e-3 * bound


def _schmidt_ranks(M, N):
    """Operator Schmidt ranks of a 4^N x 4^N operator over every cut."""
    T = M.reshape([4] * (2 * N))
    perm = [q for i in range(N) for q in (i, N + i)]
    v = T.transpose(perm).reshape([16] * N)
    out = []
    for k in range(1, N):
        s = np.linalg.svd(v.reshape(16 ** k, -1), compute_uv=False)
        out.append(int(np.sum(s > 1e-10 * s[0])))
    return out


@pytest.mark.parametrize("W,L,geo,order", [(1, 4, lattice.CHAIN, 2), (1, 4, lattice.CHAIN, 3),
                                           (2, 2, lattice.OPEN_SQUARE, 2), (1, 5, lattice.CHAIN, 2)])
def test_reduction_is_exact_minimal_and_charge_conserving(W, L, geo, order):
    m = mpo.HubbardMPO(W, L, geo, 1.0, 4.0, 0.3)
    A, Q = mpo.settn_rho0(m, 0.1, order)
    N = W * L
    # bond sizes equal the operator Schmidt ranks of the dense polynomial
    H = ed.Hubbard(W, L, geo, 1.0, 4.0, 0.3).dense_hamiltonian()
    assert [a.shape[0] for a in A[1:]] == _schmidt_ranks(_dense_poly(H, 0.1, order), N)
    # every nonzero entry conserves the charge q(left) + q(s) = q(right)
    Qs = list(Q) + [[(0, 0)]]
    for k, a in enumerate(A):
        a16 = a.reshape(a.shape[0], 16, a.shape[3])
        for (x, s, y) in zip(*np.nonzero(np.abs(a16) > 1e-14)):
            ql, qr, qs = Qs[k][x], Qs[k + 1][y], charges.s_charge(s)
            assert (ql[0] + qs[0], ql[1] + qs[1]) == tuple(qr)


def test_product_size_guard():
    # Nc = 4 on a 2x2 square: the product bond exceeds 8192 states
    with pytest.raises(ValueError):
        mpo.settn_rho0(mpo.HubbardMPO(2, 2, lattice.OPEN_SQUARE, 1.0, 4.0, 0.0), 0.05, 4)


def test_mgs_threshold_guard():
    # a second column independent by 1e-8 relative sits inside the guard band
    rng = np.random.default_rng(0)
    u = rng.standard_normal(8)
    w = rng.standard_normal(8)
    M = np.stack([u, u + 1e-8 * w], axis=1)
    with pytest.raises(ValueError):
        mpo._mgs_keep(M, mpo.SETTN_TOL)
    Q, R = mpo._mgs_keep(np.stack([u, 2.0 * u, w], axis=1), mpo.SETTN_TOL)
    assert Q.shape[1] == 2
    assert np.abs(Q @ R - np.stack([u, 2.0 * u, w], axis=1)).max() < 1e-14


@pytest.mark.parametrize("W,L,geo,order,sym", [(1, 4, lattice.CHAIN, 2, True), (2, 2, lattice.OPEN_SQUARE, 3, True),
                                               (1, 4, lattice.CHAIN, 3, False)])
def test_flow_from_settn_start_exact_at_maximal_bond(W, L, geo, order, sym):
    b0 = 0.1
    m = mpo.HubbardMPO(W, L, geo, 1.0, 4.0, 0.3)
    E, _, _ = ed.Hubbard(W, L, geo, 1.0, 4.0, 0.3).spectrum()
    st = tdvp.initial_state(m, b0, 16 ** 8, sym, taylor_order=order)
    for _ in range(4):
        st.sweep(0.1)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, o["beta"], order)
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - Ebl) <= 1e-10 * max(abs(Ebl), 1e-2)
    assert abs(o["lnZ_single"] - ed.same_ode_single(E, b0, o["beta"], order)) <= 1e-10 * max(abs(o["lnZ_single"]), 1e-2)
