"""The sine and cosine of the move angles used by the sweep kernels (csrc/muca_trig.h), built for
the host from the same source and checked against long double sinl / cosl: below one unit in
the last place, sin^2 + cos^2 = 1 without bias (a bias would stretch or shrink the bonds that a
crankshaft rotation keeps at unit length, Sec. 2), odd / even symmetry."""
import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1702_01770_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("trig") / "move_trig_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(HERE, "cpp", "move_trig_check.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, n, lo, hi):
    out = subprocess.run([exe, str(n), repr(lo), repr(hi)], check=True, capture_output=True,
                         text=True).stdout
    return json.loads(out)


@pytest.mark.parametrize("lo,hi", [(-3.141592653589793, 6.283185307179586),   # every move angle
                                   (-1e-3, 1e-3),                               # tiny rotations
                                   (0.7, 0.9), (1.5, 1.65)])                    # quadrant edges
def test_sincos_move_within_one_ulp(checker, lo, hi):
    r = _run(checker, 400000, lo, hi)
    assert r["max_ulp_sin"] < 1.0 and r["max_ulp_cos"] < 1.0, r
    assert r["max_norm_err"] <= 3.5e-16, r
    assert abs(r["mean_norm_err"]) < 2e-17, r
    assert r["max_sym_err"] == 0.0, r
