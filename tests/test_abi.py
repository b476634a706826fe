"""The C-ABI library loads without a GPU and exports every function include/muca.h declares,
with plain C types only."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muca.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("muca_", "microcanonical_"))))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("muca_init", "muca_sweep", "muca_update_weights", "microcanonical_analyze",
                     "muca_energy_fwd", "muca_energy_bwd", "muca_destroy"):
        assert required in names


def test_header_signatures_are_plain_c():
    txt = open(HEADER).read()
    for bad in ("torch", "at::", "hipStream_t", "std::", "Tensor"):
        assert bad not in re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    r = subprocess.run(["gcc", "-fsyntax-only", "-x", "c", "-std=c99", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_loads_and_exports_every_declared_symbol():
    import paper_1702_01770_amd as P
    lib = os.path.join(ROOT, "paper_1702_01770_amd", "libmuca.so")
    if not os.path.exists(lib):
        pytest.skip("libmuca.so not built (run __graft_entry__.build())")
    P.load()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(P._lib.EXPORTS) == set(_declared())


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_1702_01770_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        L.load()


def test_init_rejects_an_unbounded_crank_angle():
    """The configuration is validated before any device call: a crankshaft range beyond what the
    sweep kernels' move-angle sincos covers (|crank_max| <= 1e5) is refused with MUCA_E_INVAL."""
    import numpy as np
    import paper_1702_01770_amd as P
    lib = os.path.join(ROOT, "paper_1702_01770_amd", "libmuca.so")
    if not os.path.exists(lib):
        pytest.skip("libmuca.so not built (run __graft_entry__.build())")
    pos = np.stack([np.arange(6.0), np.zeros(6), np.zeros(6)], axis=1)
    for bad in (1e6, float("inf"), float("nan")):
        with pytest.raises(RuntimeError, match="crank_max"):
            P.Muca([1], [6], [0, 1, 0, 1, 0, 1], pos, np.array([[1.0, -0.5], [-0.5, 0.5]]),
                   [-10.0], [200], walkers_per_system=1, crank_max=bad)
