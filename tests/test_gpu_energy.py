"""GPU energy forward/backward and reweighting (C ABI + autograd wrappers) against the FP64 oracle:
energies of identical FP32 configurations within 1e-5 of the term scale, dE/dx and dE/dtheta
against the oracle's analytic FP64 gradient, reweighted <E>_T and C_V(T) and their theta
gradients against the oracle's fluctuation formulas, and finite differences in theta."""
import dataclasses

import numpy as np
import pytest

import workloads
from oracle import reweight as R

pytestmark = pytest.mark.gpu

TEMPS = np.linspace(0.1, 1.0, 64)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1702_01770_amd as P
    from paper_1702_01770_amd import autograd as AG
    P.load()
    return P, AG, torch


def _configs(orc, wl, n_cfg, sweeps_between=3, seed_walker=0, scale=1.0):
    """Configurations from an oracle walker at flat weights, plus random chains."""
    s = orc.System.from_workload(wl)
    sp = wl.systems[0]
    W = orc.Weights(sp.e_lo, wl.bin_width, sp.n_bins)
    w = orc.Walker(s, workloads.initial_positions(wl)[0], seed_walker, wl.seed)
    H = np.zeros(sp.n_bins, np.uint64)
    xs = []
    for _ in range(n_cfg):
        w.run(W, orc.move_params(wl), sweeps_between, H)
        xs.append(w.pos.copy())
    return np.array(xs) * scale


def _ctx(P, wl):
    return P.Muca.from_workload(wl, workloads.initial_positions(wl), walkers=1)


@pytest.mark.parametrize("make", [workloads.cross_seeding, workloads.aggregation,
                                  lambda: workloads.batched_chains(n_seq=1, n_min=40, n_max=40)])
def test_energy_and_gradients_vs_oracle(env, orc, make):
    P, AG, torch = env
    wl = make()
    xs = _configs(orc, wl, 64)
    xs[32:] = workloads.random_bond_chains(5, 32, wl.systems[0].chain_len, box_len=wl.box_len) * 1.03
    x32 = xs.astype(np.float32)
    x64 = x32.astype(np.float64)                     # both sides see identical coordinates
    theta = np.array([-0.45, 0.55, wl.k_bend + 0.02, wl.k_tors + 0.05])
    cl = np.array([[1.0, theta[0]], [theta[0], theta[1]]])
    s = orc.System(wl.systems[0].chain_len, wl.systems[0].types, cl, wl.k_lj_intra,
                   wl.k_lj_inter, theta[2], theta[3], wl.box_kind, wl.box_len)
    m = _ctx(P, wl)
    xt = torch.tensor(x32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    xt.requires_grad_(True)
    E = AG.EnergyFn.apply(xt, th, m, 0)
    ge = torch.linspace(-1.0, 2.0, len(xs), dtype=torch.float64, device="cuda")
    (E * ge).sum().backward()
    Eg = E.detach().cpu().numpy()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    gth = th.grad.cpu().numpy()
    gth_ref = np.zeros(4)
    for i in range(len(xs)):
        e64, grad, dth = s.energy_grad(x64[i])
        _, _, scale = s.energy_parts(x64[i])
        assert abs(Eg[i] - e64) <= 1e-5 * scale, (i, Eg[i], e64, scale)
        gref = ge[i].item() * grad
        gsc = np.abs(gref).max() + 1e-30
        assert np.max(np.abs(gx[i] - gref)) <= 2e-4 * gsc, (i, np.max(np.abs(gx[i] - gref)), gsc)
        gth_ref += ge[i].item() * dth
    assert np.allclose(gth, gth_ref, rtol=1e-4, atol=1e-6 * np.abs(gth_ref).max())
    m.close()


def _multi_chain(n_chains, chain_len, box_len):
    """n_chains copies of one seeded sequence in a periodic cube (bending + torsion)."""
    base = workloads.aggregation()
    rng = np.random.default_rng([1702, 11])
    seq = workloads.ab_sequence(rng, chain_len)
    lens = [chain_len] * n_chains
    e_lo, n_bins = workloads.default_window(sum(lens), 0.25)   # window table fits in LDS
    sp = workloads.SystemSpec(chain_len=lens, types=np.concatenate([seq] * n_chains), e_lo=e_lo,
                              n_bins=n_bins)
    return dataclasses.replace(base, name="multi", systems=[sp], box_len=box_len, k_tors=0.1,
                               bin_width=0.25, walkers_per_system=1)


@pytest.mark.parametrize("make,n_cfg", [
    (lambda: workloads.single_chain(n=3), 1),                 # smallest chain, one configuration
    (lambda: workloads.single_chain(n=3), 7),
    (lambda: workloads.single_chain(n=4), 5),                 # even N: the d = N/2 pair class
    (lambda: workloads.single_chain(n=65), 61),               # odd N above one wave, ragged count
    (lambda: _multi_chain(8, 16, 30.0), 9),                   # 128 beads (maximum), periodic
    (lambda: _multi_chain(3, 3, 12.0), 6),                    # chains of 3 (no torsion term)
])
def test_energy_edge_shapes(env, orc, make, n_cfg):
    """Energy, dE/dx and dE/dtheta on arbitrary overlap-free chains for the smallest and largest
    systems, odd and even N and configuration counts that leave a workgroup partly empty."""
    P, AG, torch = env
    wl = make()
    sp = wl.systems[0]
    xs = workloads.random_bond_chains(29, n_cfg, sp.chain_len, box_len=wl.box_len)
    x32 = xs.astype(np.float32)
    x64 = x32.astype(np.float64)
    theta = np.array([-0.4, 0.6, wl.k_bend + 0.01, wl.k_tors + 0.03])
    cl = np.array([[1.0, theta[0]], [theta[0], theta[1]]])
    s = orc.System(sp.chain_len, sp.types, cl, wl.k_lj_intra, wl.k_lj_inter, theta[2], theta[3],
                   wl.box_kind, wl.box_len)
    m = _ctx(P, wl)
    xt = torch.tensor(x32, device="cuda", requires_grad=True)
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    E = AG.EnergyFn.apply(xt, th, m, 0)
    ge = torch.linspace(0.5, 1.5, n_cfg, dtype=torch.float64, device="cuda")
    (E * ge).sum().backward()
    Eg = E.detach().cpu().numpy()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    gth_ref = np.zeros(4)
    for i in range(n_cfg):
        e64, grad, dth = s.energy_grad(x64[i])
        _, _, scale = s.energy_parts(x64[i])
        assert abs(Eg[i] - e64) <= 1e-5 * scale, (i, Eg[i], e64, scale)
        gref = ge[i].item() * grad
        gsc = np.abs(gref).max() + 1e-30
        assert np.max(np.abs(gx[i] - gref)) <= 2e-4 * gsc
        gth_ref += ge[i].item() * dth
    assert np.allclose(th.grad.cpu().numpy(), gth_ref, rtol=1e-4,
                       atol=1e-6 * np.abs(gth_ref).max() + 1e-12)
    m.close()


def test_energy_kernels_are_deterministic(env, orc):
    """Every sum runs in a fixed order: two calls give bit-identical energies and gradients."""
    P, AG, torch = env
    wl = workloads.cross_seeding()
    xs = workloads.random_bond_chains(31, 203, wl.systems[0].chain_len, box_len=wl.box_len)
    m = _ctx(P, wl)
    xt = torch.tensor(xs.astype(np.float32), device="cuda")
    theta = np.array([-0.5, 0.5, wl.k_bend, wl.k_tors])
    ge = torch.linspace(-1.0, 1.0, len(xs), dtype=torch.float64, device="cuda")
    out = []
    for _ in range(2):
        E = torch.empty(len(xs), dtype=torch.float64, device="cuda")
        gx = torch.empty_like(xt)
        gth = torch.empty(4, dtype=torch.float64, device="cuda")
        m.energy_fwd_ptr(0, xt.data_ptr(), len(xs), theta, E.data_ptr())
        m.energy_bwd_ptr(0, xt.data_ptr(), len(xs), theta, ge.data_ptr(), gx.data_ptr(),
                         gth.data_ptr())
        m.synchronize()
        out.append((E.cpu().numpy(), gx.cpu().numpy(), gth.cpu().numpy()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    m.close()


def test_reweighting_forward_backward_vs_oracle(env):
    P, AG, torch = env
    rng = np.random.default_rng(3)
    n = 100_000
    E = rng.normal(-20.0, 6.0, size=n)
    lnw0 = 0.9 * E + rng.normal(scale=0.5, size=n)          # a MUCA-like sampling weight
    G = rng.normal(size=(n, 4))
    Et = torch.tensor(E, device="cuda", requires_grad=True)
    lt = torch.tensor(lnw0, device="cuda")
    mean, cv = AG.ReweightFn.apply(Et, lt, TEMPS)
    m_ref, cv_ref = R.canonical(E, lnw0, TEMPS)
    assert np.allclose(mean.detach().cpu().numpy(), m_ref, rtol=1e-11, atol=1e-11)
    assert np.allclose(cv.detach().cpu().numpy(), cv_ref, rtol=1e-9, atol=1e-10)
    gm = rng.normal(size=64)
    gc = rng.normal(size=64)
    (mean * torch.tensor(gm, device="cuda")).sum().add_(
        (cv * torch.tensor(gc, device="cuda")).sum()).backward()
    gE = Et.grad.cpu().numpy()
    dm, dcv = R.canonical_grad(E, G, lnw0, TEMPS)
    lhs = gE @ G
    rhs = gm @ dm + gc @ dcv
    assert np.allclose(lhs, rhs, rtol=1e-8, atol=1e-8 * np.abs(rhs).max())


def test_reweighted_gradients_end_to_end_and_finite_differences(env, orc):
    """d<E>_T/dtheta and dC_V/dtheta through EnergyFn + ReweightFn against the oracle's
    fluctuation formulas on the oracle's FP64 energies, and against finite differences."""
    P, AG, torch = env
    wl = workloads.cross_seeding()
    xs = _configs(orc, wl, 400, sweeps_between=2).astype(np.float32)
    theta = np.array([-0.5, 0.5, wl.k_bend, wl.k_tors])
    s = orc.System.from_workload(wl)
    x64 = xs.astype(np.float64)
    E0 = s.energy_many(x64)
    lnw0 = np.zeros(len(xs))                                # flat sampling weights
    temps = np.array([0.5, 1.0, 2.0, 4.0])
    m = _ctx(P, wl)
    xt = torch.tensor(xs, device="cuda")
    lt = torch.tensor(lnw0, device="cuda")

    def obs(th_np, grad=False):
        th = torch.tensor(th_np, dtype=torch.float64, device="cuda", requires_grad=grad)
        mean, cv = AG.reweighted_observables(xt, th, lt, temps, m)
        return th, mean, cv

    th, mean, cv = obs(theta, grad=True)
    jac_mean = np.stack([torch.autograd.grad(mean[i], th, retain_graph=True)[0].cpu().numpy()
                         for i in range(len(temps))])
    jac_cv = np.stack([torch.autograd.grad(cv[i], th, retain_graph=True)[0].cpu().numpy()
                       for i in range(len(temps))])
    G = np.array([s.energy_grad(x)[2] for x in x64])
    dm_ref, dcv_ref = R.canonical_grad(E0, G, lnw0, temps)
    assert np.allclose(jac_mean, dm_ref, rtol=2e-4, atol=1e-4 * np.abs(dm_ref).max())
    assert np.allclose(jac_cv, dcv_ref, rtol=2e-3, atol=1e-3 * np.abs(dcv_ref).max())
    for t in range(4):
        h = 1e-3
        d = np.zeros(4)
        d[t] = h
        _, mp, cp = obs(theta + d)
        _, mm, cm = obs(theta - d)
        fd_m = (mp - mm).cpu().numpy() / (2 * h)
        fd_c = (cp - cm).cpu().numpy() / (2 * h)
        assert np.allclose(jac_mean[:, t], fd_m, rtol=2e-3, atol=2e-3 * np.abs(fd_m).max() + 1e-9)
        assert np.allclose(jac_cv[:, t], fd_c, rtol=1e-2, atol=1e-2 * np.abs(fd_c).max() + 1e-9)
    m.close()
