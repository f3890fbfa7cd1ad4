"""Sweeps replayed from a captured hipGraph equal uncaptured sweeps bit for
bit: every replay is checked against the eager state, with the program's own
eager work (observables, synchronising) between replays, and a change of the
step forces a new capture."""
import numpy as np
import pytest

from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,L,geo,D,sym,pad", [(3, 3, T.TT_CYLINDER, 24, 1, 0.3), (1, 6, T.TT_CHAIN, 12, 0, 1e-3)])
def test_graph_sweeps_equal_eager_sweeps(W, L, geo, D, sym, pad):
    print("graph", W, L, geo, D, sym, flush=True)
    m = T.model(W, L, geo, 1.0, 8.0, 1.5)
    o = T.options(D=D, symmetry=sym, beta0=0.01, pad_eps=pad, seed=5)
    a, b = T.State.init(m, o), T.State.init(m, o)
    try:
        for step, db in enumerate([0.1, 0.1, 0.1, 0.05, 0.05, 0.1]):
            T.tt_sweep_graphs(False)
            a.sweep(db)
            T.tt_sweep_graphs(True)
            b.sweep(db)
            T.tt_sweep_graphs(False)
            oa, ob = a.observables(), b.observables()
            for key in ("beta", "lnZ", "E", "lnZ_single"):
                assert oa[key] == ob[key], (step, key, oa[key], ob[key])
            n, _ = a.info()
            for k in (0, n // 2, n - 1):
                assert np.array_equal(a.export_site(k), b.export_site(k)), (step, k)
    finally:
        T.tt_sweep_graphs(False)
        a.free()
        b.free()
