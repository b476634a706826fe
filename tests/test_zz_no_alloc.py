"""The allocation-free reweighting entry point (muca_reweight_fwd_noalloc: the workspace is a
static per-GPU array inside the library) against the allocating muca_reweight_fwd on the same
inputs, through the C ABI: two calls in a row, the second smaller (fewer samples, fewer
temperatures), each bit-identical to the allocating call and within rounding of the FP64 oracle;
an input whose workspace exceeds the static array is rejected on the host."""
import numpy as np
import pytest

from oracle import reweight as RW

pytestmark = pytest.mark.gpu


def _inputs(n, n_t, seed):
    rng = np.random.default_rng(seed)
    E = rng.uniform(-40.0, 5.0, n)                      # energies of a 76-bead system's window
    lnw0 = 0.8 * E + rng.normal(scale=0.5, size=n)      # MUCA weights roughly flattening E
    temps = np.linspace(0.1, 1.0, n_t)
    return E, lnw0, temps


def _run(P, torch, E, lnw0, temps, noalloc):
    dev = torch.device("cuda", 0)
    e = torch.from_numpy(E).to(dev)
    l0 = torch.from_numpy(lnw0).to(dev)
    nt = len(temps)
    mean = torch.full((nt,), float("nan"), dtype=torch.float64, device=dev)
    cv = torch.full((nt,), float("nan"), dtype=torch.float64, device=dev)
    mom = torch.full((nt, 3), float("nan"), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    if noalloc:
        P.reweight_fwd_noalloc(e.data_ptr(), l0.data_ptr(), len(E), temps, mean.data_ptr(),
                               cv.data_ptr(), mom.data_ptr(), st)
    else:
        nb = P.reweight_workspace_bytes(len(E), nt)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        P.reweight_fwd(e.data_ptr(), l0.data_ptr(), len(E), temps, mean.data_ptr(),
                       cv.data_ptr(), mom.data_ptr(), ws.data_ptr(), nb, st)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), cv.cpu().numpy(), mom.cpu().numpy()


def test_noalloc_reweight_matches_allocating_entry_point_twice():
    import torch
    import paper_1702_01770_amd as P
    P.load()
    for n, n_t, seed in ((1_000_000, 64, 11), (37_777, 17, 12)):
        print(f"case n={n} n_t={n_t} seed={seed}", flush=True)
        E, lnw0, temps = _inputs(n, n_t, seed)
        ref = _run(P, torch, E, lnw0, temps, noalloc=False)
        got = _run(P, torch, E, lnw0, temps, noalloc=True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)                  # same kernels, fixed-order sums
        m_o, cv_o = RW.canonical(E, lnw0, temps)
        assert np.allclose(got[0], m_o, rtol=1e-10, atol=1e-10)
        assert np.allclose(got[1], cv_o, rtol=1e-8, atol=1e-10)


def test_noalloc_reweight_rejects_inputs_beyond_the_static_workspace():
    """5e6 samples at 256 temperatures need about 40 MB of workspace: rejected before any
    launch, and the pointers (real device buffers of the claimed size) are never touched."""
    import torch
    import paper_1702_01770_amd as P
    P.load()
    n, n_t = 5_000_000, 256
    assert P.reweight_workspace_bytes(n, n_t) > (4 << 20)
    dev = torch.device("cuda", 0)
    e = torch.zeros(n, dtype=torch.float64, device=dev)
    out = torch.zeros((n_t, 5), dtype=torch.float64, device=dev)
    with pytest.raises(P.MucaError, match="static"):
        P.reweight_fwd_noalloc(e.data_ptr(), e.data_ptr(), n, np.linspace(0.1, 1.0, n_t),
                               out[:, 0].data_ptr(), out[:, 1].data_ptr(), out[:, 2].data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
