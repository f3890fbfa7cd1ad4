"""GPU parity of sweeps of the t-t' Hubbard model (SM Eq. S1: next-nearest
hopping t' on the diagonal neighbours) with ED at untruncated bonds and with
the oracle at truncated bonds (same initial tensors)."""
import pytest

from oracle import ed, mpo as ompo, tdvp as otd
from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-2)


# (the 2x3 lattice's wider spectrum needs a smaller step for Krylov dimension 8
# to stay below the tolerance)
@pytest.mark.parametrize("W,L,geo,U,mu,tp,sym,D,db", [(2, 2, T.TT_OPEN_SQUARE, 8.0, 1.5, -0.25, 1, 256, 0.05),
                                                       (2, 2, T.TT_OPEN_SQUARE, 4.0, 0.5, 0.3, 0, 256, 0.05),
                                                       (2, 3, T.TT_OPEN_SQUARE, 8.0, 2.0, -0.25, 1, 4096, 0.02)])
def test_tprime_sweeps_match_ed_untruncated(W, L, geo, U, mu, tp, sym, D, db):
    print("tprime ed", W, L, geo, tp, sym, flush=True)
    b0 = 0.01
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu, tp), T.options(D=D, symmetry=sym, beta0=b0))
    h = ed.Hubbard(W, L, geo, 1.0, U, mu, tp=tp)
    E, _, _ = h.spectrum()
    for _ in range(6):
        st.sweep(db)
    o = st.observables()
    lnZ, Ebl = ed.same_ode_bilayer(E, b0, o["beta"])
    assert _rel(o["lnZ"], lnZ) <= TOL_FP64, (o["lnZ"], lnZ)
    assert _rel(o["E"], Ebl) <= TOL_FP64, (o["E"], Ebl)
    assert _rel(o["lnZ_single"], ed.same_ode_single(E, b0, o["beta"])) <= TOL_FP64
    st.free()


@pytest.mark.parametrize("W,L,geo,U,mu,tp,D,sym,pad", [(2, 3, T.TT_OPEN_SQUARE, 8.0, 1.0, -0.25, 20, 1, 0.3),
                                                        (3, 3, T.TT_CYLINDER, 8.0, 2.0, 0.2, 24, 1, 0.3)])
def test_tprime_truncated_sweeps_match_oracle(W, L, geo, U, mu, tp, D, sym, pad):
    print("tprime trunc", W, L, geo, tp, D, flush=True)
    b0 = 0.01
    mm = ompo.HubbardMPO(W, L, geo, 1.0, U, mu, tp=tp)
    ost = otd.initial_state(mm, b0, D, bool(sym), pad_eps=pad, seed=11, sector_cap=64)
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu, tp),
                      T.options(D=D, symmetry=sym, beta0=b0, pad_eps=pad, seed=11))
    assert st.info()[1] == ost.dims()
    for _ in range(2):
        st.sweep(0.1)
        ost.sweep(0.1)
    o, r = st.observables(), ost.observables()
    assert _rel(o["lnZ"], r["lnZ"]) <= TOL_FP64, (o["lnZ"], r["lnZ"])
    assert _rel(o["E"], r["E"]) <= TOL_FP64, (o["E"], r["E"])
    assert _rel(o["f"], r["f"]) <= TOL_FP64
    st.free()
