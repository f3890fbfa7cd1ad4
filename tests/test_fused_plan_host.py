"""The fused one-site apply's descriptors on the host: tests/host_fused_check.cpp
links the planner (layout.cpp, model.cpp) without any GPU code, interprets the
fused output blocks, b blocks and terms on random operands and compares them
with the grouped GEMMs of the folded form (LW . A in passes, then . R; SM Fig.
Lanczos with the MPO summed into L), and checks that the output blocks cover
the site vector and the jobs tile every block exactly once."""
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
    out = str(tmp_path_factory.mktemp("fused") / "host_fused_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", out, os.path.join(HERE, "host_fused_check.cpp"),
                    os.path.join(CSRC, "layout.cpp"), os.path.join(CSRC, "model.cpp")], check=True)
    return out


# (W, L, geometry, D, sector cap, k): chain ends and middle, the 2x3 square,
# the 3x4 cylinder, an 8-site chain at D = 1000 with capped (64) and uncapped
# (98-state) sectors, so that output blocks span two column tiles
CASES = [(1, 4, 0, 12, 0, 0), (1, 4, 0, 12, 0, 3), (1, 6, 0, 40, 0, 2), (2, 3, 2, 60, 0, 2),
         (3, 4, 1, 300, 64, 5), (1, 8, 0, 1000, 64, 3), (1, 8, 0, 1000, 0, 4)]


@pytest.mark.parametrize("W,L,geo,D,cap,k", CASES)
def test_fused_descriptors_match_the_folded_form(checker, W, L, geo, D, cap, k):
    r = subprocess.run([checker, str(W), str(L), str(geo), str(D), str(cap), str(k)], capture_output=True,
                       text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "worst=" in r.stdout
