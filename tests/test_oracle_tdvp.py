"""Pins of the oracle's one-site TDVP machinery: Lanczos exponential against
scipy's expm, contractions against brute-force loops, QR/LQ conventions,
exactness at untruncated bonds against ED (SM Sec. II.E: the splitting is
exact on the affine tangent space), second-order Lie-Trotter scaling at a
truncated bond (SM Sec. I, Fig. S7(c)), and charge conservation."""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import charges, ed, mpo, tdvp

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return 0.5 * (M + M.T)


@pytest.mark.parametrize("t,K", [(-0.05, 8), (0.05, 8), (-0.3, 20), (0.2, 16)])
def test_lanczos_expm_matches_scipy(t, K):
    M = _sym(120, 1) / np.sqrt(120)
    v = np.random.default_rng(2).standard_normal(120)
    got, info = tdvp.lanczos_expm(lambda x: M @ x, v, t, K)
    want = expm(t * M) @ v
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    assert info["k"] == K


def test_lanczos_lucky_breakdown_is_exact():
    # v lies in a 3-dimensional invariant subspace: Krylov stops at 3, result exact
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    lam = np.concatenate([[0.3, -1.1, 2.0], rng.standard_normal(47)])
    M = (Q * lam) @ Q.T
    v = Q[:, :3] @ np.array([1.0, -0.5, 0.25])
    got, info = tdvp.lanczos_expm(lambda x: M @ x, v, -0.7, 8)
    assert info["k"] == 3
    assert np.linalg.norm(got - expm(-0.7 * M) @ v) < 1e-12


def test_lanczos_zero_vector():
    got, info = tdvp.lanczos_expm(lambda x: 2 * x, np.zeros(5), 1.0, 4)
    assert np.all(got == 0) and info["k"] == 0


@pytest.mark.parametrize("m,n", [(40, 7), (16, 16), (64, 1)])
def test_qr_lq_conventions(m, n):
    M = np.random.default_rng(m * n).standard_normal((m, n))
    Q, R = tdvp.qr_pos(M)
    assert np.allclose(Q @ R, M, atol=1e-13)
    assert np.allclose(Q.T @ Q, np.eye(n), atol=1e-13)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    Lm, Qr = tdvp.lq_pos(M.T)
    assert np.allclose(Lm @ Qr, M.T, atol=1e-13)
    assert np.allclose(Qr @ Qr.T, np.eye(n), atol=1e-13)
    assert np.all(np.diag(Lm) >= 0) and np.allclose(np.triu(Lm, 1), 0)


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_contractions_against_loops():
    Dl, Dr, DH = 3, 2, 2
    L, W, A, R = _rand((Dl, DH, Dl), 1), _rand((DH, 4, 4, DH), 2), _rand((Dl, 4, 4, Dr), 3), _rand((Dr, DH, Dr), 4)
    out = np.zeros((Dl, 4, 4, Dr))
    for x, so, sp, y, a, al, si, b, be in itertools.product(
            range(Dl), range(4), range(4), range(Dr), range(DH), range(Dl), range(4), range(DH), range(Dr)):
        out[x, so, sp, y] += L[x, a, al] * A[al, si, sp, be] * W[a, so, si, b] * R[y, b, be]
    assert np.allclose(tdvp.heff1(L, W, R, A), out, atol=1e-12)
    Lnew = np.zeros((Dr, DH, Dr))
    for x2, so, sp, y2, a, x, si, y, b in itertools.product(
            range(Dl), range(4), range(4), range(Dr), range(DH), range(Dl), range(4), range(Dr), range(DH)):
        Lnew[y2, b, y] += A[x2, so, sp, y2] * L[x2, a, x] * A[x, si, sp, y] * W[a, so, si, b]
    assert np.allclose(tdvp.env_left(L, A, W), Lnew, atol=1e-12)
    Rn = np.zeros((Dl, DH, Dl))
    for x2, so, sp, y2, a, x, si, y, b in itertools.product(
            range(Dl), range(4), range(4), range(Dr), range(DH), range(Dl), range(4), range(Dr), range(DH)):
        Rn[x2, a, x] += A[x2, so, sp, y2] * W[a, so, si, b] * A[x, si, sp, y] * R[y2, b, y]
    assert np.allclose(tdvp.env_right(R, A, W), Rn, atol=1e-12)
    S = _rand((Dl, Dl), 5)
    L2, R2 = _rand((Dl, DH, Dl), 6), _rand((Dl, DH, Dl), 7)
    o0 = np.zeros((Dl, Dl))
    for x, y, a, al, be in itertools.product(range(Dl), range(Dl), range(DH), range(Dl), range(Dl)):
        o0[x, y] += L2[x, a, al] * S[al, be] * R2[y, a, be]
    assert np.allclose(tdvp.heff0(L2, R2, S), o0, atol=1e-12)


def _max_d_state(W, L, geo, t, U, mu, beta0):
    m = mpo.HubbardMPO(W, L, geo, t, U, mu)
    return tdvp.initial_state(m, beta0, 16 ** 8, False), m


def test_energy_and_norm_match_dense_operator():
    W, L, geo, t, U, mu, b0 = 1, 4, 0, 1.0, 4.0, 0.3, 0.01
    st, m = _max_d_state(W, L, geo, t, U, mu, b0)
    st.sweep(0.2, K=16)
    # dense rho from the super-MPS: A[x, so, si, y]
    M = st.A[0][0].transpose(2, 0, 1)
    for a in st.A[1:]:
        T = np.tensordot(M, a, axes=([0], [0])).transpose(4, 0, 2, 1, 3)
        M = T.reshape(T.shape[0], T.shape[1] * T.shape[2], T.shape[3] * T.shape[4])
    rho = M[0] * np.exp(st.lam)
    Hd = ed.Hubbard(W, L, geo, t, U, mu).dense_hamiltonian()
    o = st.observables()
    assert abs(o["lnZ"] - np.log(np.sum(rho * rho))) < 1e-11
    assert abs(o["E"] - np.trace(rho.T @ Hd @ rho) / np.sum(rho * rho)) < 1e-11
    assert abs(o["lnZ_single"] - np.log(np.trace(rho))) < 1e-11
    # rho is symmetric and equals expm(-(beta-b0)H)(1-b0 H)
    want = expm(-(st.beta - b0) * Hd) @ (np.eye(256) - b0 * Hd)
    assert np.abs(rho - want).max() < 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("W,L,geo,U,mu,sym", [(1, 4, 0, 4.0, 0.0, False), (1, 4, 0, 4.0, 0.0, True),
                                               (2, 2, 2, 8.0, 4.0, True), (1, 4, 0, 0.0, 0.5, False)])
def test_untruncated_tdvp_is_exact(W, L, geo, U, mu, sym):
    b0, db, n = 0.01, 0.05, 12
    m = mpo.HubbardMPO(W, L, geo, 1.0, U, mu)
    st = tdvp.initial_state(m, b0, 16 ** 8, sym)
    E, _, _ = ed.Hubbard(W, L, geo, 1.0, U, mu).spectrum()
    for _ in range(n):
        st.sweep(db)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, st.beta)
    assert abs(o["lnZ"] - lnZ) <= 1e-10 * abs(lnZ)
    assert abs(o["E"] - Ebl) <= 1e-10 * max(abs(Ebl), 1e-2)
    assert abs(o["lnZ_single"] - ed.same_ode_single(E, b0, st.beta)) <= 1e-10 * abs(lnZ)


def test_untruncated_u0_tracks_free_fermions():
    # U=0: same-ODE result differs from the closed form only by the linear start
    b0 = 1e-4
    m = mpo.HubbardMPO(1, 4, 0, 1.0, 0.0, 0.2)
    st = tdvp.initial_state(m, b0, 16 ** 8, False)
    for _ in range(10):
        st.sweep(0.05)
    hm = ed.Hubbard(1, 4, 0, 1.0, 0.0, 0.2).hopping_matrix()
    lnZ = ed.free_fermion_lnZ(hm, 2 * st.beta)
    assert abs(st.observables()["lnZ"] - lnZ) < 1e-6 * abs(lnZ)


def test_second_order_lie_trotter_at_truncated_bond():
    # as in SM Fig. S7(c): evolve one state to a common beta with small steps,
    # then continue with steps tau, tau/2, tau/4 and compare f
    import copy
    g = json.load(open(os.path.join(GOLD, "paper_values.json")))["lie_trotter_order"]
    m = mpo.HubbardMPO(1, 6, 0, 1.0, 2.0, 0.0)
    base = tdvp.initial_state(m, 0.01, 12, False, pad_eps=1e-3, seed=7)
    assert max(base.dims()) == 12
    for _ in range(20):
        base.sweep(0.05, K=16)
    fs = []
    for db in (0.4, 0.2, 0.1):
        st = copy.deepcopy(base)
        for _ in range(int(round(1.6 / db))):
            st.sweep(db, K=16)
        fs.append(st.observables()["f"])
    alpha = np.log2(abs((fs[0] - fs[1]) / (fs[1] - fs[2])))
    assert abs(alpha - g["value"]) < g["tol"], (fs, alpha)


def _dense(st):
    M = st.A[0][0].transpose(2, 0, 1)
    for a in st.A[1:]:
        T = np.tensordot(M, a, axes=([0], [0])).transpose(4, 0, 2, 1, 3)
        M = T.reshape(T.shape[0], T.shape[1] * T.shape[2], T.shape[3] * T.shape[4])
    return M[0]


def test_symmetric_padding_conserves_charge_through_sweeps():
    m = mpo.HubbardMPO(2, 3, 2, 1.0, 8.0, 1.0)
    st = tdvp.initial_state(m, 0.01, 40, True, pad_eps=1e-3, seed=3)
    for _ in range(2):
        st.sweep(0.1)
    # blockwise QR/LQ keeps every charge-forbidden entry exactly zero
    sc = np.array(charges.S_CHARGES)
    for k, A in enumerate(st.A):
        ql = np.array(st.layouts[k].charges)
        qr = np.array(st.layouts[k + 1].charges)
        A3 = A.reshape(A.shape[0], 16, A.shape[3])
        x, s, y = np.nonzero(A3)
        assert np.all(ql[x] + sc[s] == qr[y])
    rho = _dense(st)
    n = np.arange(4 ** m.N)
    qu = np.zeros_like(n)
    qd = np.zeros_like(n)
    for k in range(m.N):
        sig = (n // 4 ** (m.N - 1 - k)) % 4
        qu += sig & 1
        qd += sig >> 1
    ok = (qu[:, None] == qu[None, :]) & (qd[:, None] == qd[None, :])
    # the operator commutes with N_up and N_dn up to rounding
    assert np.abs(rho[~ok]).max() == 0.0


def test_canonical_form_after_sweep():
    m = mpo.HubbardMPO(2, 3, 2, 1.0, 8.0, 1.0)
    st = tdvp.initial_state(m, 0.01, 40, True, pad_eps=1e-4, seed=5)
    st.sweep(0.1)
    assert abs(np.linalg.norm(st.A[0]) - 1) < 1e-12
    for A in st.A[1:]:
        M = A.reshape(A.shape[0], -1)
        assert np.allclose(M @ M.T, np.eye(A.shape[0]), atol=1e-12)


def test_two_site_generator_against_loops():
    Dl, Dr, DH = 2, 2, 2
    L, R = _rand((Dl, DH, Dl), 11), _rand((Dr, DH, Dr), 12)
    W1, W2 = _rand((DH, 4, 4, DH), 13), _rand((DH, 4, 4, DH), 14)
    C = _rand((Dl, 4, 4, 4, 4, Dr), 15)
    out = np.zeros((Dl, 4, 4, 4, 4, Dr))
    for x, so1, sp1, so2, sp2, y in itertools.product(range(Dl), range(4), range(4), range(4), range(4), range(Dr)):
        v = 0.0
        for a, al, si1, b, si2, c, be in itertools.product(range(DH), range(Dl), range(4), range(DH), range(4),
                                                          range(DH), range(Dr)):
            v += L[x, a, al] * C[al, si1, sp1, si2, sp2, be] * W1[a, so1, si1, b] * W2[b, so2, si2, c] * R[y, c, be]
        out[x, so1, sp1, so2, sp2, y] = v
    assert np.allclose(tdvp.heff2(L, W1, W2, R, C), out, atol=1e-12)


def test_two_site_generator_is_h_on_a_two_site_system():
    # N = 2 with trivial environments: H^(2) C is (H (x) 1)|rho>> for the dense
    # two-site H of ED and any two-site super tensor C (Choi map, SM Sec. II.A)
    h = ed.Hubbard(1, 2, 0, 1.0, 5.0, 0.7)
    Ws = mpo.HubbardMPO(1, 2, 0, 1.0, 5.0, 0.7).mpo_for_env()
    C = _rand((1, 4, 4, 4, 4, 1), 16)
    one = np.ones((1, 1, 1))
    got = tdvp.heff2(one, Ws[0], Ws[1], one, C)[0, :, :, :, :, 0]      # so1 sp1 so2 sp2
    rho = C[0, :, :, :, :, 0].transpose(0, 2, 1, 3).reshape(16, 16)   # (s1 s2), (s1' s2')
    want = (h.dense_hamiltonian() @ rho).reshape(4, 4, 4, 4).transpose(0, 2, 1, 3)
    assert np.abs(got - want).max() < 1e-13
