"""GPU parity with the block-sparse oracle at sizes where the dense oracle
cannot go: the 4x16 cylinder at D = 2000 (the headline workload, against the
stored values of tests/golden/make_blocked_golden.py) and an 8-site chain at
D = 1000 run in-process, whose QR blocks reach 64 columns in four row chunks
(capped sectors) or go to the global-memory QR (uncapped sectors, up to 98
columns).  Gauge-invariant outputs (SM Sec. II.A bilayer values and the
single-layer trace), FP64 to 1e-10; the FP32 mode to the mixed-path bar of
1e-6 against the same FP64 oracle values."""
import json
import os

import pytest

from oracle import blocked, charges, mpo as ompo
from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "blocked_cl4x16_d2000.json")
TOL_FP64 = 1e-10
TOL_MIXED = 1e-6
KEYS = ("lnZ", "f", "E", "e", "lnZ_single")


def _rel(a, b, floor=1e-2):
    return abs(a - b) / max(abs(b), floor)


def _qr_classes(st):
    """(columns, chunks) of every QR and LQ block of the oracle state's bonds,
    with the row-chunk rule of the GPU's register QR (chunks of at most 256
    rows, stacks of at most 256 rows, blocks of at most 64 columns)."""
    out = []
    S = charges.S_CHARGES
    for k in range(st.N):
        bl, br = st.bonds[k].sec, st.bonds[k + 1].sec
        shapes = [(n, sum(bl.get((c[0] - s[0], c[1] - s[1]), (0, 0))[1] for s in S)) for c, (_, n) in br.items()]
        shapes += [(n, sum(br.get((l[0] + s[0], l[1] + s[1]), (0, 0))[1] for s in S)) for l, (_, n) in bl.items()]
        for n, m in shapes:
            nc = -(-m // 256)
            out.append((n, nc if n <= 64 and nc * n <= 256 and m // nc >= n else 0))
    return out


@pytest.mark.parametrize("cap", [64, 0])
def test_mid_size_chain_matches_blocked_oracle(cap):
    W, L, geo, U, mu, D, b0, pad, seed = 1, 8, 0, 8.0, 1.5, 1000, 0.01, 1e-3, 1
    print("chain8 D=1000 cap", cap, flush=True)
    ost = blocked.initial_state(ompo.HubbardMPO(W, L, geo, 1.0, U, mu), b0, D, pad_eps=pad, seed=seed,
                                sector_cap=cap)
    cls = _qr_classes(ost)
    if cap == 64:
        assert any(n == 64 and nc == 4 for n, nc in cls)          # 64 columns, four chunks, 256-row stack
    else:
        assert any(n > 64 for n, nc in cls)                       # the global-memory QR
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu),
                      T.options(D=D, symmetry=1, beta0=b0, pad_eps=pad, seed=seed, sector_cap=cap))
    n, dims = st.info()
    assert dims == [b.dim for b in ost.bonds]
    for k in range(n + 1):
        assert st.sectors(k) == [(q, d) for q, (_, d) in sorted(ost.bonds[k].sec.items())]
    for sw in range(2):
        st.sweep(0.05)
        ost.sweep(0.05)
        g, o = st.observables(), ost.observables()
        for key in KEYS:
            assert _rel(g[key], o[key]) <= TOL_FP64, (sw, key, g[key], o[key])
    hd = ost.herm_defect()           # the swap overlap's defect: sqrt amplifies rounding near zero
    assert abs(g["herm_defect"] - hd) <= 1e-8 + 1e-6 * hd, (g["herm_defect"], hd)
    st.free()


def _golden():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("prec,tol,mode", [(T.TT_FP64, TOL_FP64, 0), (T.TT_FP64, TOL_FP64, 2),
                                           (T.TT_FP64, TOL_FP64, 4), (T.TT_FP32, TOL_MIXED, 2)])
def test_headline_cylinder_matches_blocked_oracle(prec, tol, mode):
    """4x16 cylinder, D = 2000, sector cap 64 (the timed workload): the start
    and two sweeps of d_beta = 0.05 against the block-sparse oracle's stored
    values, in the paper's contraction order everywhere (mode 0) and with the
    apply forms the autotuner picks (mode 2, as the benchmark runs), and with
    the fused apply at every site (mode 4)."""
    g = _golden()
    c = g["case"]
    print("cl4x16 D=2000 precision", prec, flush=True)
    st = T.State.init(T.model(c["W"], c["L"], c["geometry"], c["t"], c["U"], c["mu"]),
                      T.options(D=c["D"], symmetry=1, beta0=c["beta0"], pad_eps=c["pad_eps"], seed=c["seed"],
                                krylov_dim=c["krylov"], sector_cap=c["sector_cap"], precision=prec))
    assert st.info()[1] == g["bond_dims"]
    forms = st.tune_apply(mode)
    print("site forms (0 / 1 / 2):", [sum(f & 3 == i for f in forms) for i in (0, 1, 2)],
          "fused bonds:", sum(f >> 2 for f in forms), flush=True)
    worst = {}
    done = 0
    for rec in g["records"]:
        while done < rec["sweeps"]:
            st.sweep(c["dbeta"])
            done += 1
        o = st.observables()
        assert abs(o["beta"] - rec["beta"]) < 1e-12
        for key in KEYS:
            err = _rel(o[key], rec[key])
            worst[key] = max(worst.get(key, 0.0), err)
            assert err <= tol, (rec["sweeps"], key, o[key], rec[key])
    print("worst relative error vs the oracle:", worst)
    st.free()
