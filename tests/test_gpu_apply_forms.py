"""The forms of the site apply (tt_tune_apply): the contraction order of SM
Fig. Lanczos (L.A, the MPO stage, .R), the MPO folded into the left
environment (LW = sum_a W L^a once per environment, then LW.A, .R), and the
fused kernel LW.A.R with T2 kept in registers.  Each is held to exact
diagonalisation at untruncated bonds (SM Sec. II.E) and to the block-sparse
oracle at truncated bonds; the autotuned mix too."""
import pytest

from oracle import blocked, ed, mpo as ompo
from paper_2212_11973_amd import tantrg as T
from paper_2212_11973_amd import workloads as WL

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _rel(a, b, floor=1e-2):
    return abs(a - b) / max(abs(b), floor)


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_untruncated_chain_matches_ed_in_every_form(mode):
    c = WL.MODELS["chain4"]
    m = T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"])
    st = T.State.init(m, T.options(D=c["D"], symmetry=1, beta0=c["beta0"], krylov_dim=c["krylov"]))
    print("chain4 mode", mode, flush=True)
    forms = st.tune_apply(mode)
    assert len(forms) == 4 and set(forms) <= {0, 1, 2, 4, 5, 6}
    if mode in (1, 4):
        assert forms == [{1: 1, 4: 6}[mode]] * 4
    E, _, _ = ed.Hubbard(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]).spectrum()
    for _ in range(40):
        st.sweep(c["dbeta"])
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, c["beta0"], o["beta"])
    assert _rel(o["lnZ"], lnZ) <= TOL_FP64 and _rel(o["E"], Ebl) <= TOL_FP64
    st.free()


@pytest.mark.parametrize("W,L,geo,D,sym,cap", [(3, 3, T.TT_CYLINDER, 40, 1, 64), (1, 8, T.TT_CHAIN, 600, 1, 64),
                                              (2, 3, T.TT_OPEN_SQUARE, 30, 0, 64), (1, 8, T.TT_CHAIN, 600, 1, 0)])
def test_forms_agree_with_each_other_and_the_oracle(W, L, geo, D, sym, cap):
    print("forms", W, L, geo, D, sym, cap, flush=True)
    U, mu, b0, pad, seed = 8.0, 1.5, 0.01, 1e-3, 3
    opts = T.options(D=D, symmetry=sym, beta0=b0, pad_eps=pad, seed=seed, sector_cap=cap)
    sts = {}
    for mode in (0, 1, 2, 4):
        sts[mode] = T.State.init(T.model(W, L, geo, 1.0, U, mu), opts)
        sts[mode].tune_apply(mode)
    ost = None
    if sym == 1:
        ost = blocked.initial_state(ompo.HubbardMPO(W, L, geo, 1.0, U, mu), b0, D, pad_eps=pad, seed=seed,
                                    sector_cap=cap)
    for _ in range(2):
        for st in sts.values():
            st.sweep(0.05)
        if ost is not None:
            ost.sweep(0.05)
    obs = {m: st.observables() for m, st in sts.items()}
    for key in ("lnZ", "E", "lnZ_single"):
        assert _rel(obs[1][key], obs[0][key]) <= 1e-12, key
        assert _rel(obs[2][key], obs[0][key]) <= 1e-12, key
        assert _rel(obs[4][key], obs[0][key]) <= 1e-12, key
        if ost is not None:
            assert _rel(obs[1][key], ost.observables()[key]) <= TOL_FP64, key
            assert _rel(obs[4][key], ost.observables()[key]) <= TOL_FP64, key
    for st in sts.values():
        st.free()


def test_batch_needs_equal_forms_and_stays_bit_exact():
    mus = [0.7, 1.3, 2.1]
    o = T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=7)
    batch = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    single = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    for s in batch + single:
        s.tune_apply(1)
    for _ in range(2):
        T.tdvp_sweep_batch([s.h for s in batch], 0.05)
        for s in single:
            s.sweep(0.05)
    for a, b in zip(batch, single):
        assert a.observables() == b.observables()
    batch[1].tune_apply(0)                      # a state with other forms runs in its own group
    T.tdvp_sweep_batch([s.h for s in batch], 0.05)
    for s in batch + single:
        s.free()


def test_fused_batch_is_bit_exact_and_refused_below_fp64():
    mus = [0.7, 1.3, 2.1]
    o = T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=7)
    batch = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    single = [T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, mu), o) for mu in mus]
    for s in batch + single:
        assert s.tune_apply(4) == [6] * 6
    for _ in range(2):
        T.tdvp_sweep_batch([s.h for s in batch], 0.05)
        for s in single:
            s.sweep(0.05)
    for a, b in zip(batch, single):
        assert a.observables() == b.observables()
    for s in batch + single:
        s.free()
    s32 = T.State.init(T.model(2, 3, T.TT_OPEN_SQUARE, 1.0, 8.0, 1.0),
                       T.options(D=24, symmetry=1, beta0=0.01, pad_eps=0.3, seed=7, precision=T.TT_FP32))
    with pytest.raises(T.TTError):
        s32.tune_apply(4)
    assert all(f in (0, 1) for f in s32.tune_apply(2))   # no fused form below FP64
    with pytest.raises(T.TTError):
        s32.tune_apply(3, [2] * 6)
    s32.free()
