"""The logarithm of the hybrid Monte Carlo acceptance test (csrc/muca_logu.h, ln u against
H0 - H1), built for the host from the same source and checked against long double logl: below
one unit in the last place on the kernel's own uniform draws, on the smallest of them, on every
power of two and around the reduction's edges (sqrt(1/2), 1, sqrt(2)).  A dropped series term, a
wrong reduction edge or a wrong ln 2 split each fail one of these."""
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
    exe = str(tmp_path_factory.mktemp("logu") / "log_unit_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(HERE, "cpp", "log_unit_check.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, *args):
    out = subprocess.run([exe, *map(str, args)], check=True, capture_output=True,
                         text=True).stdout
    return json.loads(out)


@pytest.mark.parametrize("args", [("uniform", 1000000),              # the kernel's draws
                                  ("smallest", 100000),              # (k + 1/2) 2^-32, k small
                                  ("pow2",),                         # e ln 2 alone
                                  ("range", 400000, 0.70, 0.72),     # below / above sqrt(1/2)
                                  ("range", 400000, 0.999, 1.0),     # f -> 0
                                  ("range", 400000, 1.40, 1.42),     # near sqrt(2)
                                  ("range", 400000, 1e-300, 1e300)])  # every exponent
def test_log_unit_within_one_ulp(checker, args):
    r = _run(checker, *args)
    assert r["max_ulp"] < 1.0, r
    assert r["mean_ulp"] < 0.3, r
