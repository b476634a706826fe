"""Hybrid Monte Carlo under multicanonical weights, FP64 reference (test infrastructure: only
tests/, the smoke check and the benchmark's CPU baseline use it).

The paper names hybrid MCMC as the faster evolution algorithm it plans to add (Sec. 5).  This
reference defines the variant the library implements, in the variables in which the paper's
chains have no constraint forces: every chain is its first bead o_c plus unit bond vectors
u_j = x_j - x_{j-1} (indexed by the bead j that ends the bond).  A trajectory samples
pi(x) ~ W(E(x)) = exp(ln W(E(x))) (Eq. 8) with respect to the freely-jointed reference measure
(uniform first bead, every bond uniform on the unit sphere), the measure the single-bead moves
sample as well:

  potential U = -ln W(E), kinetic K = |p|^2 / 2 summed over origins and bonds;
  bead forces F_j = -dU/dx_j = -beta(E) dE/dx_j, beta(E) the slope of -ln W in the bin of E
    (edge bins extended outside the window);
  generalized forces G_j = sum of F_i over the beads i >= j of the chain (for the first bead:
    the chain's total force, acting on o_c; otherwise the force on bond u_j);
  leapfrog with geodesic drift (Byrne and Girolami, Geodesic Monte Carlo on embedded
    manifolds, 2013): half kick p_j += h/2 G_j (bonds: G_j minus its component along u_j),
    drift o_c += h p_c and each bond turns along its great circle,
      u <- u cos(|w| h) + (w / |w|) sin(|w| h),  w <- w cos(|w| h) - u |w| sin(|w| h),
    then u renormalised and w projected on the tangent plane, positions rebuilt by summing the
    bonds along each chain, forces recomputed, half kick;
  Metropolis on H = U + K: accept iff ln v < H_old - H_new; a final energy outside the window
    or a bead outside the steric sphere rejects.  H_old uses the energy recomputed from the
    starting coordinates, so H is a function of the state; after a rejection the walker keeps
    that energy.

Random numbers (Philox4x32-10, walker key as for the moves, trajectory counter T):
  momentum of vector j: block (j, lo32(T), hi32(T), 7), uniforms a_i = (x_i + 1/2) 2^-32,
    z0 = sqrt(-2 ln a0) cos(2 pi a1), z1 = sqrt(-2 ln a0) sin(2 pi a1),
    z2 = sqrt(-2 ln a2) cos(2 pi a3); origins take z, bonds z - (z.u) u;
  acceptance: block (0, lo32(T), hi32(T), 8), word 0.
One histogram count per trajectory, at the energy after the decision.
"""
from __future__ import annotations

import numpy as np

from . import System, Weights, philox

TWO_PI = 2.0 * np.pi


def _uniform(x):
    return (x.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


class HmcWalker:
    def __init__(self, system: System, pos, walker_id: int, seed: int):
        self.s = system
        self.pos = np.array(pos, dtype=np.float64)
        self.energy = system.energy(self.pos)
        self.k0 = seed & 0xFFFFFFFF
        self.k1 = ((seed >> 32) & 0xFFFFFFFF) ^ (walker_id & 0xFFFFFFFF)
        self.traj = 0
        self.accepted = 0
        self.window_rejects = 0
        starts = np.asarray(system.chain_start[:-1])
        self.first = np.zeros(system.n_beads, bool)
        self.first[starts] = True
        self.chain_of = np.repeat(np.arange(len(system.chain_len)), system.chain_len)

    # ---- pieces of a trajectory ----
    def momenta(self, v, T):
        n = self.s.n_beads
        ctr = np.zeros((n, 4), np.uint32)
        ctr[:, 0] = np.arange(n)
        ctr[:, 1] = T & 0xFFFFFFFF
        ctr[:, 2] = (T >> 32) & 0xFFFFFFFF
        ctr[:, 3] = 7
        a = _uniform(philox(self.k0, self.k1, ctr))
        r0 = np.sqrt(-2.0 * np.log(a[:, 0]))
        r2 = np.sqrt(-2.0 * np.log(a[:, 2]))
        z = np.stack([r0 * np.cos(TWO_PI * a[:, 1]), r0 * np.sin(TWO_PI * a[:, 1]),
                      r2 * np.cos(TWO_PI * a[:, 3])], axis=1)
        dot = np.sum(z * v, axis=1)
        return np.where(self.first[:, None], z, z - dot[:, None] * v)

    def vectors(self, pos):
        """Origins (first beads) and unit bonds ending at every other bead."""
        v = pos.copy()
        v[~self.first] = pos[~self.first] - pos[np.nonzero(~self.first)[0] - 1]
        return v

    def positions(self, v):
        """Segmented prefix sums of the vectors along each chain."""
        pos = np.empty_like(v)
        for c, (a, b) in enumerate(zip(self.s.chain_start[:-1], self.s.chain_start[1:])):
            pos[a:b] = np.cumsum(v[a:b], axis=0)
        return pos

    def gen_forces(self, pos, W: Weights):
        """(E, G): energy and generalized forces (suffix sums of -beta(E) dE/dx per chain)."""
        e, g, _ = self.s.energy_grad(pos)
        k = int(np.clip(np.floor((e - W.e_lo) * (1.0 / W.bin_width)), 0, W.n_bins - 1))
        f = -W.beta[k] * g
        G = np.empty_like(f)
        for a, b in zip(self.s.chain_start[:-1], self.s.chain_start[1:]):
            G[a:b] = np.cumsum(f[a:b][::-1], axis=0)[::-1]
        return e, G

    def kick(self, v, mom, G, h):
        dot = np.sum(G * v, axis=1)
        tang = np.where(self.first[:, None], G, G - dot[:, None] * v)
        return mom + h * tang

    def drift(self, v, mom, h):
        v2, m2 = v.copy(), mom.copy()
        v2[self.first] = v[self.first] + h * mom[self.first]
        bonds = ~self.first
        u, w = v[bonds], mom[bonds]
        speed = np.linalg.norm(w, axis=1)
        c, s = np.cos(speed * h), np.sin(speed * h)
        safe = np.where(speed > 0.0, speed, 1.0)
        un = u * c[:, None] + (w / safe[:, None]) * s[:, None]
        wn = w * c[:, None] - u * (speed * s)[:, None]
        un /= np.linalg.norm(un, axis=1)[:, None]
        wn -= np.sum(wn * un, axis=1)[:, None] * un
        v2[bonds], m2[bonds] = un, wn
        return v2, m2

    def leapfrog(self, v, mom, W: Weights, n_steps: int, h: float):
        """n_steps leapfrog steps from (v, mom); returns (v, mom, positions)."""
        pos = self.positions(v)
        _, G = self.gen_forces(pos, W)
        for _ in range(n_steps):
            mom = self.kick(v, mom, G, 0.5 * h)
            v, mom = self.drift(v, mom, h)
            pos = self.positions(v)
            _, G = self.gen_forces(pos, W)
            mom = self.kick(v, mom, G, 0.5 * h)
        return v, mom, pos

    # ---- one trajectory ----
    def trajectory(self, W: Weights, n_steps: int, h: float, hist=None, sphere_r2: float = 0.0,
                   record=None):
        T = self.traj
        v = self.vectors(self.pos)
        mom = self.momenta(v, T)
        # H is a function of the state: the start's energy is recomputed from its coordinates
        # (a running energy handed over by the sweeps need not be the FP64 one); a rejected
        # trajectory keeps that recomputed energy
        e0 = self.s.energy(self.pos)
        lnw = lambda e: _lnw(W, e)
        H0 = -lnw(e0) + 0.5 * float(np.sum(mom * mom))
        v, mom, pos = self.leapfrog(v, mom, W, n_steps, h)
        e1 = self.s.energy(pos)
        t = (e1 - W.e_lo) * (1.0 / W.bin_width)
        inwin = 0.0 <= t < W.n_bins
        inside = sphere_r2 <= 0.0 or float(np.max(np.sum(pos * pos, axis=1))) <= sphere_r2
        H1 = (-lnw(e1) if inwin else np.inf) + 0.5 * float(np.sum(mom * mom))
        ra = philox(self.k0, self.k1, np.array([0, T & 0xFFFFFFFF, (T >> 32) & 0xFFFFFFFF, 8],
                                               np.uint32))
        accept = inwin and inside and (np.log(_uniform(ra[:1])[0]) < H0 - H1)
        if not inwin:
            self.window_rejects += 1
        if record is not None:
            record.append(dict(H0=H0, H1=H1, e1=e1, accept=accept, pos=pos.copy()))
        if accept:
            self.pos = pos
            self.energy = e1
            self.accepted += 1
        else:
            self.energy = e0
        if hist is not None:
            k = int(np.floor((self.energy - W.e_lo) * (1.0 / W.bin_width)))
            hist[min(max(k, 0), W.n_bins - 1)] += 1
        self.traj += 1
        return accept

    def run(self, W: Weights, n_traj: int, n_steps: int, h: float, hist=None,
            sphere_r2: float = 0.0, accept_log=None):
        for i in range(n_traj):
            a = self.trajectory(W, n_steps, h, hist, sphere_r2)
            if accept_log is not None and i < len(accept_log):
                accept_log[i] = 1 if a else 0


def _lnw(W: Weights, e: float) -> float:
    """ln W(E) = -beta_k E + alpha_k in the bin of E (edge bins extended)."""
    k = int(np.clip(np.floor((e - W.e_lo) * (1.0 / W.bin_width)), 0, W.n_bins - 1))
    return -W.beta[k] * e + W.alpha[k]
