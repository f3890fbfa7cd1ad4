"""The two-site (2-TDVP) descriptors on the host: tests/host_pair_check.cpp
links the planner (layout.cpp, model.cpp) without any GPU code, runs the
join, H^(2) and split descriptors through a loop interpreter of their
semantics on random block-sparse operands and compares them with dense
contractions over the global bond indices (SM Eq. S-2TDVP)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2212_11973_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("pair") / "host_pair_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", out, os.path.join(HERE, "host_pair_check.cpp"),
                    os.path.join(CSRC, "layout.cpp"), os.path.join(CSRC, "model.cpp")], check=True)
    return out


# (W, L, geometry, D, symmetry, k): chain ends and middle, the 2x3 square,
# a full middle bond, one dense sector, Sz-only blocks
CASES = [(1, 4, 0, 12, 1, 0), (1, 4, 0, 12, 1, 1), (1, 4, 0, 12, 1, 2), (2, 3, 2, 20, 1, 2),
         (1, 5, 0, 30, 1, 1), (1, 4, 0, 300, 1, 1), (1, 4, 0, 40, 0, 1), (2, 2, 2, 30, 2, 1)]


@pytest.mark.parametrize("W,L,geo,D,sym,k", CASES)
def test_pair_descriptors_match_dense_contractions(checker, W, L, geo, D, sym, k):
    r = subprocess.run([checker, str(W), str(L), str(geo), str(D), str(sym), str(k)], capture_output=True, text=True,
                       timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "worst=" in r.stdout
