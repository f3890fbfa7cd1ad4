"""GPU parity of the one-site TDVP sweep through the C ABI against the oracle:
exact diagonalisation at untruncated bonds (SM Sec. II.E: the splitting is
exact on the affine tangent space) and the oracle's own sweep at truncated
bonds (gauge-invariant observables)."""
import copy
import os

import numpy as np
import pytest

from oracle import ed, mpo as ompo, tdvp as otd
from paper_2212_11973_amd import tantrg as T
from paper_2212_11973_amd import workloads as WL

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _rel(a, b, floor=1e-2):
    return abs(a - b) / max(abs(b), floor)


@pytest.mark.parametrize("sym", [1, 0])
def test_config1_chain4_matches_ed(sym):
    c = WL.MODELS["chain4"]
    print("chain4 sym", sym, flush=True)
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    st = T.State.init(m, T.options(D=c["D"], symmetry=sym, beta0=c["beta0"], krylov_dim=c["krylov"]))
    n, dims = st.info()
    assert dims == [1, 16, 256, 16, 1]
    E, _, _ = ed.Hubbard(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]).spectrum()
    worst = 0.0
    for step in range(c["nsteps"]):
        st.sweep(c["dbeta"])
        if step % 50 == 0 or step == c["nsteps"] - 1:
            o = st.observables()
            lnZ, Ebl = ed.same_ode_bilayer(E, c["beta0"], o["beta"])
            N = n
            f_ref = -lnZ / (N * 2 * o["beta"])
            worst = max(worst, _rel(o["f"], f_ref), _rel(o["E"] / N, Ebl / N))
            assert _rel(o["f"], f_ref) <= TOL_FP64, (step, o["f"], f_ref)
            assert _rel(o["e"], Ebl / N) <= TOL_FP64, (step, o["e"], Ebl / N)
            assert _rel(o["lnZ_single"], ed.same_ode_single(E, c["beta0"], o["beta"])) <= TOL_FP64
    assert abs(o["beta"] - 4.0) < 1e-9
    print("config1 worst rel err", worst)
    st.free()


def test_hermiticity_defect_matches_the_oracle():
    """||rho - rho^T|| / ||rho|| by transfer matrices on (q, -q) blocks: zero at
    untruncated bonds (the exact flow keeps rho symmetric), and the oracle's
    value on a padded truncated state (dense and Sz-free U(1) blocks)."""
    c = WL.MODELS["chain4"]
    st = T.State.init(T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]),
                      T.options(D=256, symmetry=1, beta0=c["beta0"]))
    for _ in range(5):
        st.sweep(0.1)
    assert st.observables()["herm_defect"] < 1e-7
    st.free()
    for sym in (1, 0):
        mm = ompo.HubbardMPO(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0)
        ost = otd.initial_state(mm, 0.01, 20, bool(sym), pad_eps=0.3, seed=11, sector_cap=64)
        st = T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0),
                          T.options(D=20, symmetry=sym, beta0=0.01, pad_eps=0.3, seed=11))
        for _ in range(2):
            st.sweep(0.1)
            ost.sweep(0.1)
        g, hd = st.observables()["herm_defect"], ost.herm_defect()
        assert hd > 1e-4
        assert abs(g - hd) <= 1e-8 + 1e-6 * hd, (sym, g, hd)
        st.free()


@pytest.mark.parametrize("W,L,geo,U,mu", [(2, 2, T.TT_OPEN_SQUARE, 8.0, 4.0), (1, 4, T.TT_CHAIN, 0.0, 0.3)])
def test_untruncated_2d_and_free_fermions_match_ed(W, L, geo, U, mu):
    b0 = 0.01
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=256, symmetry=1, beta0=b0))
    E, _, _ = ed.Hubbard(W, L, geo, 1.0, U, mu).spectrum()
    for _ in range(20):
        st.sweep(0.05)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, o["beta"])
    assert _rel(o["lnZ"], lnZ) <= TOL_FP64
    assert _rel(o["E"], Ebl) <= TOL_FP64
    st.free()


TRUNC = [
    # (W, L, geo, U, mu, D, sym, pad_eps, sweeps, dbeta)
    (1, 6, T.TT_CHAIN, 4.0, 0.0, 12, 0, 1e-3, 3, 0.1),
    (2, 3, T.TT_OPEN_SQUARE, 8.0, 1.0, 20, 1, 0.3, 3, 0.1),
    (3, 3, T.TT_CYLINDER, 8.0, 2.0, 24, 1, 0.3, 2, 0.1),
]


@pytest.mark.parametrize("W,L,geo,U,mu,D,sym,pad,ns,db", TRUNC)
def test_truncated_sweeps_match_oracle(W, L, geo, U, mu, D, sym, pad, ns, db):
    print("trunc", W, L, geo, D, sym, pad, flush=True)
    b0 = 0.01
    mm = ompo.HubbardMPO(W, L, geo, 1.0, U, mu)
    ost = otd.initial_state(mm, b0, D, bool(sym), pad_eps=pad, seed=11, sector_cap=64)
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu),
                      T.options(D=D, symmetry=sym, beta0=b0, pad_eps=pad, seed=11))
    assert st.info()[1] == ost.dims()
    o0 = st.observables()
    r0 = ost.observables()
    assert _rel(o0["lnZ"], r0["lnZ"]) <= TOL_FP64
    assert _rel(o0["E"], r0["E"]) <= TOL_FP64
    for _ in range(ns):
        st.sweep(db)
        ost.sweep(db)
    o, r = st.observables(), ost.observables()
    assert _rel(o["lnZ"], r["lnZ"]) <= TOL_FP64, (o["lnZ"], r["lnZ"])
    assert _rel(o["E"], r["E"]) <= TOL_FP64, (o["E"], r["E"])
    assert _rel(o["lnZ_single"], r["lnZ_single"]) <= TOL_FP64
    assert _rel(o["f"], r["f"]) <= TOL_FP64
    # the centre tensor's singular values are gauge invariant
    A0 = st.export_site(0).reshape(1 * 16, -1)
    sv = np.linalg.svd(A0, compute_uv=False)
    sv_ref = np.linalg.svd(ost.A[0].reshape(16, -1), compute_uv=False)
    assert np.abs(sv - sv_ref).max() <= 1e-9 * sv_ref.max()
    st.free()


def test_state_is_canonical_and_charge_conserving():
    st = T.State.init(T.model(3, 3, T.TT_CYLINDER, 1.0, 8.0, 2.0),
                      T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=3))
    st.sweep(0.1)
    n, dims = st.info()
    A0 = st.export_site(0)
    assert abs(np.linalg.norm(A0) - 1.0) < 1e-12
    for k in range(1, n):
        A = st.export_site(k).reshape(dims[k], -1)
        assert np.abs(A @ A.T - np.eye(dims[k])).max() < 1e-12
    st.free()


def test_save_load_resume_is_bitwise(tmp_path):
    m = T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0)
    o = T.options(D=20, symmetry=1, beta0=0.01, pad_eps=0.3, seed=5)
    a = T.State.init(m, o)
    a.sweep(0.1)
    p = str(tmp_path / "s.bin")
    T.tt_state_save(a.h, p)
    b = T.State(T.tt_state_load(p))
    for s in (a, b):
        s.sweep(0.1)
        s.sweep(0.1)
    oa, ob = a.observables(), b.observables()
    assert oa["lnZ"] == ob["lnZ"] and oa["E"] == ob["E"]
    for k in range(a.info()[0]):
        assert np.array_equal(a.export_site(k), b.export_site(k))
    a.free(); b.free()


def test_runs_are_deterministic():
    m = T.model(3, 3, T.TT_CYLINDER, 1.0, 8.0, 2.0)
    o = T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=3)
    res = []
    for _ in range(2):
        s = T.State.init(m, o)
        s.sweep(0.1)
        res.append((s.observables(), [s.export_site(k) for k in range(s.info()[0])]))
        s.free()
    assert res[0][0] == res[1][0]
    for x, y in zip(res[0][1], res[1][1]):
        assert np.array_equal(x, y)


def test_batch_equals_single_sweeps():
    m1 = T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0)
    m2 = T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 3.0)
    o = T.options(D=20, symmetry=1, beta0=0.01, pad_eps=0.3, seed=5)
    a, b = T.State.init(m1, o), T.State.init(m2, o)
    c, d = T.State.init(m1, o), T.State.init(m2, o)
    T.tdvp_sweep_batch([a.h, b.h], 0.1)
    c.sweep(0.1)
    d.sweep(0.1)
    assert a.observables() == c.observables()
    assert b.observables() == d.observables()
    for s in (a, b, c, d):
        s.free()


def test_import_export_roundtrip():
    m = T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0)
    st = T.State.init(m, T.options(D=20, symmetry=1, beta0=0.01, pad_eps=0.3, seed=5))
    A = st.export_site(2)
    T.tt_state_import_site(st.h, 2, A)
    assert np.array_equal(st.export_site(2), A)
    bad = A.copy()
    bad.flat[np.flatnonzero(A)[0]] = np.nan
    with pytest.raises(T.TTError) as e:
        T.tt_state_import_site(st.h, 2, bad)
    assert e.value.code == T.TT_ENUMERIC
    st.free()


# mixed-precision sweeps against the FP64 references: the bulk contractions in
# FP32 / split-BF16, Lanczos scalars, QR and Lambda in FP64
TOL_MIXED = 1e-6


BF16X3_MISSES_BAR = pytest.mark.xfail(
    strict=True, reason="bf16x3 (two BF16 parts per operand, 16 mantissa bits) misses the 1e-6 mixed bar: "
    "measured on the chain against ED after 100 sweeps, rel err f 1.45e-6, E/N 7.7e-6")


@pytest.mark.parametrize("prec", [T.TT_FP32, T.TT_BF16X6, pytest.param(T.TT_BF16X3, marks=BF16X3_MISSES_BAR)])
def test_mixed_precision_chain4_vs_ed(prec):
    c = WL.MODELS["chain4"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    st = T.State.init(m, T.options(D=c["D"], symmetry=1, beta0=c["beta0"], krylov_dim=c["krylov"], precision=prec))
    E, _, _ = ed.Hubbard(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]).spectrum()
    errs = []
    for step in range(100):
        st.sweep(c["dbeta"])
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, c["beta0"], o["beta"])
    f_ref = -lnZ / (4 * 2 * o["beta"])
    errs = (_rel(o["f"], f_ref), _rel(o["e"], Ebl / 4))
    print("precision", prec, "rel err f, e", errs)
    st.free()
    assert errs[0] <= TOL_MIXED and errs[1] <= TOL_MIXED, errs


@pytest.mark.parametrize("prec", [T.TT_FP32, T.TT_BF16X6, pytest.param(T.TT_BF16X3, marks=pytest.mark.xfail(
    strict=False, reason="bf16x3 misses the 1e-6 mixed bar on the chain (see above); here measured, not required"))])
def test_mixed_precision_truncated_vs_oracle(prec):
    W, L, geo, U, mu, D, pad = 3, 3, T.TT_CYLINDER, 8.0, 2.0, 24, 0.3
    b0 = 0.01
    mm = ompo.HubbardMPO(W, L, geo, 1.0, U, mu)
    ost = otd.initial_state(mm, b0, D, True, pad_eps=pad, seed=11, sector_cap=64)
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu),
                      T.options(D=D, symmetry=1, beta0=b0, pad_eps=pad, seed=11, precision=prec))
    for _ in range(2):
        st.sweep(0.1)
        ost.sweep(0.1)
    o, r = st.observables(), ost.observables()
    print("precision", prec, "rel err f, e vs the oracle", _rel(o["f"], r["f"]), _rel(o["e"], r["e"]))
    st.free()
    assert _rel(o["f"], r["f"]) <= TOL_MIXED, (o["f"], r["f"])
    assert _rel(o["e"], r["e"]) <= TOL_MIXED, (o["e"], r["e"])


def _grouped_launches(fn):
    T.tt_profile_enable(True)
    fn()
    T.tt_profile_enable(False)
    return T.tt_profile_read()["gemm"]["launches"]


def test_batch_shares_launches_and_matches_single_sweeps():
    # a mu-scan: identical plans, different couplings -> one launch per contraction for the whole batch
    mus = [0.7, 1.3, 2.1, 2.9, 3.6]
    o = T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=7)
    batch = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    single = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    n_batch = _grouped_launches(lambda: T.tdvp_sweep_batch([s.h for s in batch], 0.05))
    n_one = _grouped_launches(lambda: single[0].sweep(0.05))
    assert n_batch == n_one
    for s in single[1:]:
        s.sweep(0.05)
    T.tdvp_sweep_batch([s.h for s in batch], 0.05)
    for s in single:
        s.sweep(0.05)
    for a, b in zip(batch, single):
        assert a.observables() == b.observables()
        for k in range(a.info()[0]):
            assert np.array_equal(a.export_site(k), b.export_site(k))
    for s in batch + single:
        s.free()


def test_batch_with_different_plans_falls_back_to_groups():
    # a different D gives different plans: that state runs in its own group
    m = [T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu) for mu in (1.0, 4.0, 1.0)]
    opts = [T.options(D=d, symmetry=1, beta0=0.01, pad_eps=0.3, seed=5) for d in (20, 20, 16)]
    batch = [T.State.init(mm, oo) for mm, oo in zip(m, opts)]
    single = [T.State.init(mm, oo) for mm, oo in zip(m, opts)]
    T.tdvp_sweep_batch([s.h for s in batch], 0.1)
    for s in single:
        s.sweep(0.1)
    for a, b in zip(batch, single):
        assert a.observables() == b.observables()
    for s in batch + single:
        s.free()


def test_batch_rejects_duplicates():
    st = T.State.init(T.model(1, 4, T.TT_CHAIN, 1.0, 4.0, 0.0), T.options(D=16, symmetry=1, beta0=0.01))
    with pytest.raises(T.TTError) as e:
        T.tdvp_sweep_batch([st.h, st.h], 0.1)
    assert e.value.code == T.TT_EINVAL
    st.free()


def test_full_size_workload_properties():
    # the benchmark's workload and launch configuration (4x16 cylinder, D=2000, FP64):
    # properties that hold at any size, checked on sampled rows
    c = WL.MODELS["cl4x16"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    o = T.options(D=c["D"], symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"])
    a, b = T.State.init(m, o), T.State.init(m, o)
    for st in (a, b):
        st.sweep(c["dbeta"])
    oa, ob = a.observables(), b.observables()
    assert oa == ob                                   # deterministic at full size
    assert all(np.isfinite([oa["lnZ"], oa["E"], oa["f"], oa["lnZ_single"]]))
    assert abs(oa["beta"] - (c["beta0"] + c["dbeta"])) < 1e-12
    n, dims = a.info()
    assert max(dims) == c["D"]
    rng = np.random.default_rng(0)
    A0 = a.export_site(0)
    assert abs(np.linalg.norm(A0) - 1.0) < 1e-12      # the centre carries the norm
    for k in (1, n // 2, n - 1):                      # right-canonical sites: orthonormal rows
        A = a.export_site(k).reshape(dims[k], -1)
        rows = rng.choice(dims[k], size=min(48, dims[k]), replace=False)
        G = A[rows] @ A[rows].T
        assert np.abs(G - np.eye(len(rows))).max() < 1e-11, k
    a.free()
    b.free()


def test_uncapped_full_size_wide_lq_blocks_are_orthonormal():
    # the benchmark's workload without the sector cap: sectors of up to 195
    # states, so 14 sites at each end hold LQ blocks of 69-195 rows that the
    # global-memory (wide) QR factors; after a sweep every site k >= 1 is
    # right-canonical, checked on all rows of sites with such blocks
    c = WL.MODELS["cl4x16"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    o = T.options(D=c["D"], symmetry=1, beta0=c["beta0"], pad_eps=1e-3, seed=1, krylov_dim=c["krylov"],
                  sector_cap=0)
    st = T.State.init(m, o)
    n, dims = st.info()
    widest = {k: max(d for _, d in st.sectors(k)) for k in range(n + 1)}
    assert widest[3] > 64 and widest[n - 3] > 64                      # the wide form is exercised
    print("uncapped 4x16 D=2000, widest sectors", widest[3], widest[n - 3], flush=True)
    st.sweep(c["dbeta"])
    ob = st.observables()
    assert all(np.isfinite([ob["lnZ"], ob["E"], ob["f"]]))
    for k in (3, 5, n - 5, n - 3):
        A = st.export_site(k).reshape(dims[k], -1)
        G = A @ A.T
        assert np.abs(G - np.eye(dims[k])).max() < 1e-11, k
    st.free()
