"""Pins of the block-sparse oracle (``oracle.blocked``): every contraction
against the dense oracle's on random charge-conserving tensors, the blockwise
start against the dense start entry for entry, whole sweeps against the dense
oracle on truncated lattices (gauge-invariant outputs, 1e-12), and exactness
at untruncated bonds against exact diagonalisation (SM Sec. II.E: the
splitting is exact on the affine tangent space)."""
import numpy as np
import pytest

from oracle import blocked, ed, mpo, tdvp

S = blocked.S_CHARGES


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-2)


def _dense_env(E, bond, qH):
    """Dense [D, DH, D] environment from blocks E[a][q'] (bra sector q', ket
    sector q' - qH(a))."""
    out = np.zeros((bond.dim, len(qH), bond.dim))
    for a, Ea in enumerate(E):
        for qp, blk in Ea.items():
            q = blocked.qsub(qp, qH[a])
            out[bond.off(qp):bond.off(qp) + blk.shape[0], a, bond.off(q):bond.off(q) + blk.shape[1]] = blk
    return out


def _random_env(bond, qH, rng):
    """Random environment blocks E[a][q'] of shape d(q') x d(q' - qH(a))."""
    E = [dict() for _ in qH]
    for a, qa in enumerate(qH):
        for qp in bond.sec:
            q = blocked.qsub(qp, qa)
            if q in bond.sec:
                E[a][qp] = rng.standard_normal((bond.d(qp), bond.d(q)))
    return E


def _random_site(st, k, rng):
    A = {s: {} for s in range(16)}
    for (q, s, qr, dl, dr, off) in st.layout[k].blocks:
        A[s][q] = rng.standard_normal((dl, dr))
    return A


def _dense_site(st, k, A):
    keep = st.A[k]
    st.A[k] = A
    out = st.to_dense(k)
    st.A[k] = keep
    return out


@pytest.fixture(scope="module")
def chain_state():
    m = mpo.HubbardMPO(1, 6, 0, t=1.0, U=8.0, mu=1.5)
    return m, blocked.initial_state(m, 0.01, 40, pad_eps=1e-3, seed=1)


def test_contractions_match_dense_on_random_tensors(chain_state):
    m, st = chain_state
    rng = np.random.default_rng(7)
    k = 2
    bl, br = st.bonds[k], st.bonds[k + 1]
    qHl, qHr = st.qH[k], st.qH[k + 1]
    W = st.W[k]
    L = _random_env(bl, qHl, rng)
    R = _random_env(br, qHr, rng)
    A = _random_site(st, k, rng)
    Ld, Rd, Ad = _dense_env(L, bl, qHl), _dense_env(R, br, qHr), _dense_site(st, k, A)
    # H^(1) A (SM Fig. optimalB(c))
    got = _dense_site(st, k, blocked.heff1(L, qHl, W, R, qHr, A))
    want = tdvp.heff1(Ld, W, Rd, Ad)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # environments (left from L_k, right from R_{k+1})
    Ln = _dense_env(blocked.env_left(L, qHl, A, W, len(qHr)), br, qHr)
    want = tdvp.env_left(Ld, Ad, W)
    assert np.abs(Ln - want).max() <= 1e-12 * np.abs(want).max()
    Rn = _dense_env(blocked.env_right(R, qHr, A, W, qHl), bl, qHl)
    want = tdvp.env_right(Rd, Ad, W)
    assert np.abs(Rn - want).max() <= 1e-12 * np.abs(want).max()
    # H^(0) S on bond k (SM Fig. optimalB(d)), with R taken on the same bond
    R0 = _random_env(bl, qHl, rng)
    R0d = _dense_env(R0, bl, qHl)
    Sb = {q: rng.standard_normal((bl.d(q), bl.d(q))) for q in bl.sec}
    Sd = np.zeros((bl.dim, bl.dim))
    for q, blk in Sb.items():
        Sd[bl.off(q):bl.off(q) + blk.shape[0], bl.off(q):bl.off(q) + blk.shape[1]] = blk
    got = blocked.heff0(L, R0, qHl, Sb)
    Gd = np.zeros_like(Sd)
    for q, blk in got.items():
        Gd[bl.off(q):bl.off(q) + blk.shape[0], bl.off(q):bl.off(q) + blk.shape[1]] = blk
    want = tdvp.heff0(Ld, R0d, Sd)
    assert np.abs(Gd - want).max() <= 1e-12 * np.abs(want).max()


def test_gauge_moves_match_dense(chain_state):
    _, st = chain_state
    rng = np.random.default_rng(8)
    k = 2
    A = _random_site(st, k, rng)
    Ad = _dense_site(st, k, A)
    Dl, _, _, Dr = Ad.shape
    ql = st.bonds[k].layout.charges
    qr = st.bonds[k + 1].layout.charges
    # QR: A reshaped (D_l 16) x D_r
    row_q = [(a[0] + c[0], a[1] + c[1]) for a in ql for c in S]
    Qd, Rd = tdvp.qr_pos_blocked(Ad.reshape(Dl * 16, Dr), row_q, qr)
    Qb, Sb = blocked.qr_site(A, st.bonds[k + 1])
    assert np.abs(_dense_site(st, k, Qb).reshape(Dl * 16, Dr) - Qd).max() < 1e-12
    for q, blk in Sb.items():
        o = st.bonds[k + 1].off(q)
        assert np.abs(blk - Rd[o:o + blk.shape[0], o:o + blk.shape[1]]).max() < 1e-12
    # LQ: A reshaped D_l x (16 D_r)
    col_q = [(b[0] - c[0], b[1] - c[1]) for c in S for b in qr]
    Ld, Qd = tdvp.lq_pos_blocked(Ad.reshape(Dl, 16 * Dr), ql, col_q)
    Lb, Qb = blocked.lq_site(A, st.bonds[k])
    assert np.abs(_dense_site(st, k, Qb).reshape(Dl, 16 * Dr) - Qd).max() < 1e-12
    for q, blk in Lb.items():
        o = st.bonds[k].off(q)
        assert np.abs(blk - Ld[o:o + blk.shape[0], o:o + blk.shape[1]]).max() < 1e-12


@pytest.mark.parametrize("W,L,geo,D,cap,nsw", [
    (1, 6, 0, 40, 0, 2),        # chain
    (3, 2, 1, 60, 0, 2),        # 3x2 cylinder
    (2, 3, 2, 30, 0, 2),        # 2x3 open square
    (4, 4, 1, 40, 8, 1),        # 4x4 cylinder with a sector cap
])
def test_sweeps_match_dense_oracle(W, L, geo, D, cap, nsw):
    m = mpo.HubbardMPO(W, L, geo, t=1.0, U=8.0, mu=1.5)
    dn = tdvp.initial_state(m, 0.01, D, True, pad_eps=1e-3, seed=1, sector_cap=cap)
    bl = blocked.initial_state(m, 0.01, D, pad_eps=1e-3, seed=1, sector_cap=cap)
    # the blockwise start is the dense start entry for entry
    for k in range(dn.N):
        assert np.abs(dn.A[k] - bl.to_dense(k)).max() < 1e-14
    assert abs(dn.lam - bl.lam) < 1e-14
    for _ in range(nsw):
        dn.sweep(0.05)
        bl.sweep(0.05)
        od, ob = dn.observables(), bl.observables()
        for key in ("lnZ", "E", "lnZ_single", "f"):
            assert _rel(ob[key], od[key]) < 1e-12, (key, ob[key], od[key])


def test_untruncated_chain_matches_ed():
    """At maximal bonds [1,16,256,16,1] the sweep is exact (SM Sec. II.E), so
    the block-sparse oracle reproduces the same-ODE ED values."""
    W_, L_, t, U, mu, b0 = 1, 4, 1.0, 4.0, 0.0, 0.01
    m = mpo.HubbardMPO(W_, L_, 0, t=t, U=U, mu=mu)
    st = blocked.initial_state(m, b0, 256)
    assert [b.dim for b in st.bonds] == [1, 16, 256, 16, 1]
    E, _, _ = ed.Hubbard(W_, L_, 0, t, U, mu).spectrum()
    for _ in range(20):
        st.sweep(0.05)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, o["beta"])
    assert _rel(o["lnZ"], lnZ) < 1e-10
    assert _rel(o["E"], Ebl) < 1e-10


def test_hermiticity_defect_pins():
    """||rho - rho^T|| / ||rho||: zero for the symmetric start and for the exact
    flow at untruncated bonds (rho(beta) = exp(-(beta - beta0) H)(1 - beta0 H)
    is symmetric); at a truncated bond equal to the brute-force value of the
    dense operator, and the same in blocks and dense."""
    from oracle import mpo as om
    m = om.HubbardMPO(1, 4, 0, t=1.0, U=4.0, mu=0.3)
    st = tdvp.initial_state(m, 0.01, 256, True)
    assert st.herm_defect() < 1e-7
    for _ in range(5):
        st.sweep(0.1)
    assert st.herm_defect() < 1e-7
    # truncated, padded: brute force from the dense operator
    dn = tdvp.initial_state(m, 0.01, 12, True, pad_eps=0.3, seed=5)
    bl = blocked.initial_state(m, 0.01, 12, pad_eps=0.3, seed=5)
    for _ in range(2):
        dn.sweep(0.1)
        bl.sweep(0.1)
    rho = om.mpo_to_dense(dn.A)
    want = np.linalg.norm(rho - rho.T) / np.linalg.norm(rho)
    assert want > 1e-6
    assert abs(dn.herm_defect() - want) <= 1e-8 * max(want, 1.0)
    assert abs(bl.herm_defect() - dn.herm_defect()) <= 1e-10
