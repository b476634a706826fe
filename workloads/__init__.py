"""Seeded synthetic inputs for the multicanonical AB-chain workloads.

This module only *generates inputs*: sequences, chain lengths, couplings, energy windows,
initial coordinates and run-length parameters.  It holds none of the method's arithmetic
(no energies, moves, weights or analysis), so both the FP64 oracle and the HIP library can
consume it without sharing any computation.

Stand-ins for the paper's inputs (PHAST, arXiv:1702.01770, Sec. 4):
  * the paper maps PDB entries to A/B strings with a hydrophobicity scale (Sec. 3.1); those files
    are not available, so sequences are drawn at random with ~60 % A, matching the 33-60 % A of
    the printed 9-10 bead sequences (Sec. 4.1, 4.2);
  * couplings follow the printed AB-limit parameter file (Sec. 4: r0 = 1, kappa_F = 0,
    kappa_C = 0.25, kappa_LJ_intra = kappa_LJ_inter = 4) and Eq. (1) for C_LJ;
  * the paper's steric sphere is replaced by a periodic cube for the aggregation workloads;
  * paper_system() runs the A/B strings the paper prints for its aggregation and cross-seeding
    examples (Sec. 4.1, 4.2) in the paper's steric spheres, with its chain-level moves.

Every generator takes an explicit integer seed and uses numpy's PCG64 stream, so every workload
is reproducible bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TYPE_A = 0
TYPE_B = 1

# Eq. (1): C_LJ(A,A) = +1, C_LJ(B,B) = +1/2, C_LJ(A,B) = C_LJ(B,A) = -1/2.
C_LJ_PAPER = np.array([[1.0, -0.5], [-0.5, 0.5]], dtype=np.float64)

BOX_NONE = 0
BOX_SPHERE = 1          # steric sphere of radius box_len about the origin
BOX_PERIODIC = 2        # periodic cube of edge box_len

PREC_FP64 = 0
PREC_FP32_SPLIT = 1


@dataclass
class SystemSpec:
    """One simulated system: M chains of given lengths and A/B types."""
    chain_len: List[int]
    types: np.ndarray                  # uint8, concatenated over chains
    e_lo: float                        # lower edge of the energy window
    n_bins: int                        # number of bins of width `bin_width`

    @property
    def n_beads(self) -> int:
        return int(sum(self.chain_len))

    @property
    def n_chains(self) -> int:
        return len(self.chain_len)


@dataclass
class Workload:
    """Everything a run needs: systems, couplings, box, move sizes, walkers, seed."""
    name: str
    systems: List[SystemSpec]
    walkers_per_system: int
    c_lj: np.ndarray = field(default_factory=lambda: C_LJ_PAPER.copy())
    k_lj_intra: float = 4.0
    k_lj_inter: float = 4.0
    k_bend: float = 0.25
    k_tors: float = 0.0
    box_kind: int = BOX_NONE
    box_len: float = 0.0
    bin_width: float = 0.05
    precision: int = PREC_FP64
    resync_sweeps: int = 0
    crank_max: float = np.pi / 3.0
    cap_rho: float = 0.8
    trans_max: float = 0.3
    rigid_per_sweep: int = 0
    pivot_per_sweep: int = 0           # pivots after every sweep
    pivot_max: float = np.pi / 6.0     # pivot angle uniform in [-pivot_max, pivot_max]
    rotate_per_sweep: int = 0          # rigid chain rotations after every sweep (multi-chain)
    rotate_max: float = np.pi / 6.0
    beta_min: float = 0.0              # weight recursion keeps beta_k in [beta_min, beta_max]
    beta_max: float = 0.0              # (off unless beta_max > beta_min)
    seed: int = 1702
    n_iter: int = 10
    n_sweeps: int = 100000

    @property
    def n_systems(self) -> int:
        return len(self.systems)

    @property
    def n_types(self) -> int:
        return int(self.c_lj.shape[0])


def ab_sequence(rng: np.random.Generator, length: int, frac_a: float = 0.6) -> np.ndarray:
    """Random A/B string (0 = A, 1 = B), each monomer A with probability `frac_a`."""
    return np.where(rng.random(length) < frac_a, TYPE_A, TYPE_B).astype(np.uint8)


def default_window(n_beads: int, bin_width: float = 0.05):
    """Energy window [-4 N, +N) in units of the LJ well depth, as (e_lo, n_bins)."""
    e_lo = -4.0 * n_beads
    n_bins = int(round(5.0 * n_beads / bin_width))
    return e_lo, n_bins


def straight_chains(chain_len, box_kind=BOX_NONE, box_len=0.0) -> np.ndarray:
    """Initial coordinates: every chain straight along +x with unit bonds.

    Chains are placed on a square grid in the (y, z) plane with spacing box_len / ceil(sqrt(M))
    (or 4 bond lengths without a box), centred in the box; in a sphere the grid (spacing 2) and
    every chain are centred on the origin.  Returns float64 [N, 3].
    """
    m = len(chain_len)
    side = int(np.ceil(np.sqrt(m)))
    spacing = {BOX_PERIODIC: box_len / side, BOX_SPHERE: 2.0}.get(box_kind, 4.0)
    out = []
    for c, n in enumerate(chain_len):
        gy, gz = c % side, c // side
        x0 = {BOX_PERIODIC: (box_len - (n - 1)) / 2.0, BOX_SPHERE: -(n - 1) / 2.0}.get(box_kind, 0.0)
        y = (gy + 0.5) * spacing
        z = (gz + 0.5) * spacing
        if box_kind == BOX_SPHERE:
            y -= side * spacing / 2.0
            z -= side * spacing / 2.0
        for i in range(n):
            out.append((x0 + i, y, z))
    return np.asarray(out, dtype=np.float64)


def _single_chain_system(types: np.ndarray, bin_width: float) -> SystemSpec:
    e_lo, n_bins = default_window(len(types), bin_width)
    return SystemSpec(chain_len=[len(types)], types=types, e_lo=e_lo, n_bins=n_bins)


def single_chain(seed: int = 1702, n: int = 13, walkers: int = 1, precision: int = PREC_FP64,
                 n_iter: int = 10, n_sweeps: int = 100000) -> Workload:
    """One AB chain of N beads (default N = 13), FP64, one walker."""
    rng = np.random.default_rng([seed, 0])
    sys_ = _single_chain_system(ab_sequence(rng, n), 0.05)
    return Workload(name=f"single_chain_n{n}", systems=[sys_], walkers_per_system=walkers,
                    precision=precision, seed=seed, n_iter=n_iter, n_sweeps=n_sweeps)


def batched_chains(seed: int = 1702, n_seq: int = 32, n_min: int = 13, n_max: int = 55,
                   walkers: int = 4096, precision: int = PREC_FP32_SPLIT,
                   n_iter: int = 10, n_sweeps: int = 100000) -> Workload:
    """`n_seq` single-chain systems with lengths uniform in [n_min, n_max], walkers spread evenly."""
    rng = np.random.default_rng([seed, 1])
    lens = rng.integers(n_min, n_max + 1, size=n_seq)
    systems = [_single_chain_system(ab_sequence(rng, int(n)), 0.05) for n in lens]
    return Workload(name=f"batched_{n_seq}seq_{n_min}-{n_max}", systems=systems,
                    walkers_per_system=walkers // n_seq, precision=precision, seed=seed,
                    resync_sweeps=100 if precision == PREC_FP32_SPLIT else 0,
                    n_iter=n_iter, n_sweeps=n_sweeps)


def chains_of_lengths(lengths, seed: int = 1702, walkers: int = 4,
                      precision: int = PREC_FP64) -> Workload:
    """Single-chain systems of the given lengths (seeded A/B sequences), `walkers` per system."""
    rng = np.random.default_rng([seed, 7])
    systems = [_single_chain_system(ab_sequence(rng, int(n)), 0.05) for n in lengths]
    return Workload(name="chains_" + "_".join(str(int(n)) for n in lengths), systems=systems,
                    walkers_per_system=walkers, precision=precision, seed=seed,
                    resync_sweeps=100 if precision == PREC_FP32_SPLIT else 0)


def aggregation(seed: int = 1702, walkers: int = 1024, precision: int = PREC_FP32_SPLIT,
                n_iter: int = 10, n_sweeps: int = 10000) -> Workload:
    """Four identical 9-bead chains in a periodic cube of edge 20, intra + inter LJ."""
    rng = np.random.default_rng([seed, 2])
    seq = ab_sequence(rng, 9)
    lens = [9, 9, 9, 9]
    e_lo, n_bins = default_window(sum(lens))
    sys_ = SystemSpec(chain_len=lens, types=np.concatenate([seq] * 4), e_lo=e_lo, n_bins=n_bins)
    return Workload(name="aggregation_4x9_L20", systems=[sys_], walkers_per_system=walkers,
                    box_kind=BOX_PERIODIC, box_len=20.0, precision=precision, resync_sweeps=100,
                    rigid_per_sweep=1, seed=seed, n_iter=n_iter, n_sweeps=n_sweeps)


def cross_seeding(seed: int = 1702, walkers: int = 4096, precision: int = PREC_FP32_SPLIT,
                  n_iter: int = 10, n_sweeps: int = 10000) -> Workload:
    """4 chains of a 9-bead sequence X + 4 chains of a 10-bead sequence Y (76 beads), periodic
    cube of edge 25, bending and torsion couplings drawn from U[0.2, 0.3] and U[0, 0.2]."""
    rng = np.random.default_rng([seed, 3])
    seq_x = ab_sequence(rng, 9)
    seq_y = ab_sequence(rng, 10)
    k_bend = float(rng.uniform(0.2, 0.3))
    k_tors = float(rng.uniform(0.0, 0.2))
    lens = [9] * 4 + [10] * 4
    types = np.concatenate([seq_x] * 4 + [seq_y] * 4)
    e_lo, n_bins = default_window(sum(lens))
    sys_ = SystemSpec(chain_len=lens, types=types, e_lo=e_lo, n_bins=n_bins)
    return Workload(name="cross_seeding_4x9+4x10_L25", systems=[sys_], walkers_per_system=walkers,
                    k_bend=k_bend, k_tors=k_tors, box_kind=BOX_PERIODIC, box_len=25.0,
                    precision=precision, resync_sweeps=100, rigid_per_sweep=1, seed=seed,
                    n_iter=n_iter, n_sweeps=n_sweeps)


def confined(seed: int = 1702, n_chains: int = 2, chain_len: int = 9, radius: float = 6.0,
             walkers: int = 256, precision: int = PREC_FP32_SPLIT, n_iter: int = 10,
             n_sweeps: int = 10000) -> Workload:
    """`n_chains` copies of one `chain_len`-bead sequence in a steric sphere of the given radius
    (the paper's container, Sec. 4), intra + inter LJ, rigid translations; a small radius makes
    the wall matter."""
    rng = np.random.default_rng([seed, 4])
    seq = ab_sequence(rng, chain_len)
    lens = [chain_len] * n_chains
    e_lo, n_bins = default_window(sum(lens))
    sys_ = SystemSpec(chain_len=lens, types=np.concatenate([seq] * n_chains), e_lo=e_lo,
                      n_bins=n_bins)
    return Workload(name=f"confined_{n_chains}x{chain_len}_R{radius:g}", systems=[sys_],
                    walkers_per_system=walkers, box_kind=BOX_SPHERE, box_len=radius,
                    precision=precision, resync_sweeps=100, rigid_per_sweep=1, seed=seed,
                    n_iter=n_iter, n_sweeps=n_sweeps)


# A/B strings and sphere radii of the paper's example systems (Sec. 4.1: the A-beta(25-33)
# dimer in a sphere of radius 40; Sec. 4.2: A-beta(25-33) cross-seeded by human or rat
# IAPP(20-29), two chains of each, in a sphere of radius 20).
PAPER_SYSTEMS = {
    "abeta_dimer": (["BBBBBAAAB", "BBBBBAAAB"], 40.0),
    "cross_human": (["BBBABAAABB", "BBBABAAABB", "BBBBBAAAB", "BBBBBAAAB"], 20.0),
    "cross_rat": (["BBBABAAAAA", "BBBABAAAAA", "BBBBBAAAB", "BBBBBAAAB"], 20.0),
}


def ab_from_string(seq: str) -> np.ndarray:
    """'A'/'B' letters to type codes."""
    return np.array([TYPE_A if c == "A" else TYPE_B for c in seq], dtype=np.uint8)


def paper_system(name: str = "cross_human", walkers: int = 4096,
                 precision: int = PREC_FP32_SPLIT, pivot_per_sweep: int = 1,
                 rotate_per_sweep: int = 1, bin_width: float = 0.05, seed: int = 1702,
                 beta_max: float = 6.0, n_iter: int = 10, n_sweeps: int = 10000,
                 e_hi: Optional[float] = None) -> Workload:
    """One of PAPER_SYSTEMS in its steric sphere with the paper's move set: single-bead moves,
    rigid translations, pivots and rigid chain rotations (the last two per sweep as given).
    The weight recursion is bounded to inverse temperatures [0, beta_max]: the steep slopes that
    sparse first-iteration tails produce would otherwise be copied to every lower bin and
    freeze the walkers there.  e_hi (total energy) moves the window's upper edge from +N."""
    seqs, radius = PAPER_SYSTEMS[name]
    types = np.concatenate([ab_from_string(q) for q in seqs])
    lens = [len(q) for q in seqs]
    e_lo, n_bins = default_window(sum(lens), bin_width)
    if e_hi is not None:
        n_bins = int(round((e_hi - e_lo) / bin_width))
    sys_ = SystemSpec(chain_len=lens, types=types, e_lo=e_lo, n_bins=n_bins)
    return Workload(name=f"paper_{name}_R{radius:g}", systems=[sys_], walkers_per_system=walkers,
                    box_kind=BOX_SPHERE, box_len=radius, bin_width=bin_width,
                    precision=precision, resync_sweeps=100, rigid_per_sweep=1,
                    pivot_per_sweep=pivot_per_sweep, rotate_per_sweep=rotate_per_sweep,
                    beta_min=0.0, beta_max=beta_max, seed=seed, n_iter=n_iter,
                    n_sweeps=n_sweeps)


def initial_positions(wl: Workload) -> List[np.ndarray]:
    """Per-system initial coordinates (float64 [N, 3]); every walker of a system starts there."""
    return [straight_chains(s.chain_len, wl.box_kind, wl.box_len) for s in wl.systems]


def random_bond_chains(seed: int, n_cfg: int, chain_len, box_len: float = 0.0,
                       min_dist: float = 0.85) -> np.ndarray:
    """`n_cfg` configurations of chains grown from random unit bond directions, each new bead
    redrawn until it keeps a distance >= `min_dist` from every bead placed before it (minimum
    image in a box).  Returns float64 [n_cfg, N, 3]; the first bead of a chain is uniform in the
    box (or at (0, 4c, 0) without a box).  Used as arbitrary, overlap-free test geometries."""
    rng = np.random.default_rng([seed, 7])
    n = int(sum(chain_len))
    out = np.empty((n_cfg, n, 3))

    def too_close(x, placed):
        if not placed:
            return False
        d = np.asarray(placed) - x
        if box_len > 0:
            d -= box_len * np.rint(d / box_len)
        return bool(np.min(np.einsum("ij,ij->i", d, d)) < min_dist * min_dist)

    for k in range(n_cfg):
        placed = []
        for c, L in enumerate(chain_len):
            while True:
                start = (rng.uniform(0, box_len, size=3) if box_len > 0
                         else np.array([0.0, 4.0 * c, 0.0]))
                if not too_close(start, placed):
                    break
            placed.append(start)
            for _ in range(L - 1):
                for _attempt in range(1000):
                    v = rng.normal(size=3)
                    x = placed[-1] + v / np.linalg.norm(v)
                    if not too_close(x, placed):
                        break
                placed.append(x)
        out[k] = np.asarray(placed)
    return out
