"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(HIP sources built for the host only, no GPU needed): the MPO and start builders, the
sector allocation, every planner and the descriptor bounds checks run for the
workloads' lattices and options, and the argument checks reject bad input,
in a process that preloads the ASan runtime.  Any report aborts that process."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent("""
    from paper_2212_11973_amd import tantrg as T
    T.lib(init_torch=False)
    cases = [  # (W, L, geometry, D, symmetry, cap, taylor order, tp, hp)
        (1, 6, T.TT_CHAIN, 40, 1, 64, 1, 0.0, 0.0),
        (1, 8, T.TT_CHAIN, 1000, 1, 0, 1, 0.0, 0.0),
        (2, 3, T.TT_OPEN_SQUARE, 40, 0, 64, 1, 0.0, 0.0),
        (4, 4, T.TT_CYLINDER, 200, 1, 64, 2, 0.0, 0.0),
        (3, 4, T.TT_OPEN_SQUARE, 100, 1, 5, 1, 0.3, 0.0),
        (4, 6, T.TT_CYLINDER, 300, 2, 64, 1, 0.0, 0.01),
        (4, 16, T.TT_CYLINDER, 2000, 1, 64, 1, 0.0, 0.0),
    ]
    for (W, L, geo, D, sym, cap, order, tp, hp) in cases:
        m = T.model(W, L, geo, 1.0, 8.0, 1.5, tp=tp, hp=hp)
        o = T.options(D=D, symmetry=sym, sector_cap=cap, taylor_order=order, beta0=2.0 ** -10)
        v, work, rep = T.tt_check_plans(m, o)
        assert v == 0, rep
        assert T.tt_model_bond_sectors(m, o, L * W // 2)
    for field, value in (("precision", 7), ("krylov_dim", 0), ("D", 0), ("symmetry", 3)):
        o = T.options(D=32)
        setattr(o, field, value)
        try:
            T.tt_check_plans(T.model(1, 4, T.TT_CHAIN), o)
        except T.TTError as e:
            assert e.code == T.TT_EINVAL
        else:
            raise AssertionError("accepted " + field)
    print("host checks ok")
""")


def test_host_code_under_asan_and_ubsan():
    from paper_2212_11973_amd import build as B
    lib = B.host_sanitized_cached()
    env = dict(os.environ)
    env.update(TANTRG_LIB=lib, LD_PRELOAD=B.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "host checks ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
