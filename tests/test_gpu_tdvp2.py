"""2-TDVP on the GPU (SM Sec. "2-TDVP in the initial stage", Eq. S-2TDVP):
tdvp_sweep2 from the bare rho0, with the split's SVD in every charge sector
of the middle bond, against the dense oracle's sweep2 (same flow, same
truncation rule) and against exact diagonalisation at full bonds; then the
switch to the one-site sweep on the grown bonds."""
import numpy as np
import pytest

from oracle import ed, lattice, mpo as ompo, tdvp
from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _rel(a, b, floor=1e-2):
    return abs(a - b) / max(abs(b), floor)


def _bare(W, L, geo, U, mu, b0=0.01):
    """GPU and oracle states at the bare rho0 = 1 - beta0 H (no padding)."""
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=1, symmetry=1, beta0=b0, pad_eps=0.0))
    ost = tdvp.initial_state(ompo.HubbardMPO(W, L, geo, 1.0, U, mu), b0, 1, False)
    return st, ost


def test_bonds_grow_from_the_bare_start_to_the_exact_flow():
    # the chain's rho0 has bonds D_H = 6; two-site updates grow them to the
    # full 16 / 256 / 16, where the flow is exact
    W, L, U, mu = 1, 4, 4.0, 0.3
    st, _ = _bare(W, L, T.TT_CHAIN, U, mu)
    assert st.info()[1] == [1, 6, 6, 6, 1]
    E, _, _ = ed.Hubbard(W, L, lattice.CHAIN, 1.0, U, mu).spectrum()
    for i in range(6):
        s = st.sweep2(0.05, 10 ** 6, 0.0, stats=True)
        print("sweep2", i, st.info()[1], "discarded", s.discarded, flush=True)
    assert st.info()[1] == [1, 16, 256, 16, 1]
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, 0.01, o["beta"])
    assert _rel(o["lnZ"], lnZ) <= TOL and _rel(o["E"], Ebl) <= TOL
    # and the one-site sweep continues on the grown bonds
    for _ in range(4):
        st.sweep(0.05)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, 0.01, o["beta"])
    assert _rel(o["lnZ"], lnZ) <= TOL and _rel(o["E"], Ebl) <= TOL
    st.free()


@pytest.mark.parametrize("W,L,geo,U,mu,cutoff,dbeta,n", [
    (1, 5, T.TT_CHAIN, 8.0, 1.5, 1e-6, 0.1, 3),
    (2, 3, T.TT_OPEN_SQUARE, 8.0, 1.5, 1e-5, 0.1, 1),
    (1, 6, T.TT_CHAIN, 4.0, 0.3, 1e-6, 0.1, 2),
])
def test_truncated_growth_matches_the_dense_oracle(W, L, geo, U, mu, cutoff, dbeta, n):
    print("sweep2 vs oracle", W, L, geo, cutoff, flush=True)
    st, ost = _bare(W, L, geo, U, mu)
    for i in range(n):
        s = st.sweep2(dbeta, 10 ** 6, cutoff, stats=True)
        ost.sweep2(dbeta, 10 ** 6, cutoff)
        print(i, st.info()[1], ost.dims(), "discarded", s.discarded, flush=True)
        assert st.info()[1] == ost.dims()
        assert 0.0 <= s.discarded < 1e-6
    o, oo = st.observables(), ost.observables()
    for key in ("lnZ", "E", "lnZ_single"):
        assert _rel(o[key], oo[key]) <= TOL, (key, o[key], oo[key])
    # the one-site sweep on the grown bonds, both sides
    for _ in range(2):
        st.sweep(dbeta)
        ost.sweep(dbeta)
    o, oo = st.observables(), ost.observables()
    for key in ("lnZ", "E", "lnZ_single"):
        assert _rel(o[key], oo[key]) <= TOL, (key, o[key], oo[key])
    st.free()


def test_d_max_caps_the_bonds_and_keeps_the_gauge():
    W, L, U, mu = 1, 5, 4.0, 0.3
    st, _ = _bare(W, L, T.TT_CHAIN, U, mu)
    E, _, _ = ed.Hubbard(W, L, lattice.CHAIN, 1.0, U, mu).spectrum()
    for _ in range(4):
        s = st.sweep2(0.1, 12, 0.0, stats=True)
    dims = st.info()[1]
    assert max(dims) == 12
    assert s.discarded > 0.0
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, 0.01, o["beta"])
    assert _rel(o["E"], Ebl) <= 1e-2        # the truncated state stays close to the exact flow
    # centre at site 0, right-orthonormal sites behind it
    for k in range(1, L):
        a = st.export_site(k).reshape(dims[k], -1)
        assert np.allclose(a @ a.T, np.eye(dims[k]), atol=1e-12)
    # the centre carries the kept weight of the last split (normalised into
    # Lambda by the next exponential, as in the oracle's flow)
    a0 = st.export_site(0).ravel()
    assert 1.0 - s.discarded - 1e-12 <= np.dot(a0, a0) <= 1.0 + 1e-12
    st.free()


def test_refuses_what_it_cannot_run():
    m = T.model(1, 4, T.TT_CHAIN, 1.0, 4.0, 0.3)
    st = T.State.init(m, T.options(D=1, symmetry=1, beta0=0.01, precision=T.TT_FP32))
    with pytest.raises(T.TTError) as e:
        st.sweep2(0.05, 100)
    assert e.value.code == T.TT_EINVAL
    st.free()
    st = T.State.init(m, T.options(D=1, symmetry=1, beta0=0.01))
    for bad in ((0.05, 0, 0.0), (0.05, 10, -1.0), (float("nan"), 10, 0.0)):
        with pytest.raises(T.TTError) as e:
            st.sweep2(*bad)
        assert e.value.code == T.TT_EINVAL
    st.sweep2(0.05, 100)                        # the state is untouched by the refusals
    assert st.info()[1][2] > 6
    st.free()


def _grow(limit, W=1, L=6, geo=T.TT_CHAIN, U=4.0, mu=0.3, cutoff=1e-6, dbeta=0.1, n=2):
    T.tt_svd_lds_limit(limit)
    try:
        st, _ = _bare(W, L, geo, U, mu)
        for _ in range(n):
            st.sweep2(dbeta, 10 ** 6, cutoff)
        dims = st.info()[1]
        return st, dims
    finally:
        T.tt_svd_lds_limit(0)


def test_spread_svd_rounds_equal_the_workgroup_form():
    # every block through the rounds spread over the GPU (limit 1) against the
    # default (every block of this chain fits one workgroup's LDS): the same
    # pairs in the same order with the same arithmetic
    print("spread SVD vs one workgroup, 1x6 chain", flush=True)
    a, da = _grow(0)
    b, db = _grow(1)
    try:
        assert da == db
        oa, ob = a.observables(), b.observables()
        for key in ("lnZ", "E", "lnZ_single"):
            assert _rel(oa[key], ob[key]) <= 1e-13, (key, oa[key], ob[key])
        for k in range(len(da) - 1):
            assert np.allclose(a.export_site(k), b.export_site(k), rtol=0, atol=1e-12), k
    finally:
        a.free()
        b.free()


def test_spread_svd_growth_matches_the_dense_oracle():
    print("spread SVD vs oracle, 2x3 square", flush=True)
    W, L, geo, U, mu, cutoff, dbeta = 2, 3, T.TT_OPEN_SQUARE, 8.0, 1.5, 1e-5, 0.1
    st, dims = _grow(1, W, L, geo, U, mu, cutoff, dbeta, 1)
    _, ost = _bare(W, L, geo, U, mu)
    ost.sweep2(dbeta, 10 ** 6, cutoff)
    try:
        assert dims == ost.dims()
        o, oo = st.observables(), ost.observables()
        for key in ("lnZ", "E", "lnZ_single"):
            assert _rel(o[key], oo[key]) <= TOL, (key, o[key], oo[key])
    finally:
        st.free()
