"""Seeded generators for the synthetic polypeptide workloads.

Recipe (every array is drawn from its own ``numpy.random.Generator(PCG64)``):

* 20 residue types, each with 10 atom slots (N, H, CA, HA, CB, HB1, HB2, HB3,
  C, O).  Per type: a net charge drawn from {-1, 0, +1}; ten slot charges drawn
  uniformly in [-0.5, 0.5], shifted to that net charge and then clipped and
  redistributed until every |q| <= 0.5 e; per slot a Lennard-Jones sigma in
  [1.8, 4.0] A and well depth in [0.02, 0.2] kcal/mol; one hydrophobicity in
  [-4.5, 4.5] per type.
* Sequences are uniform over the 20 types.
* Initial dihedrals (phi, psi) are uniform in (-pi, pi] unless a stored compact
  globule is requested.
* Batches: lengths uniform in [50, 600] residues, one seed per chain.
* Serving: Poisson arrivals (exponential gaps) and lognormal lengths
  (median 200, sigma 0.6) clipped to [30, 2000].
* Polyalanine: one fixed Ala-like residue type with element-typical constants
  (listed in ``alanine_like_types``); batches of 10-20 residue chains with
  phi, psi uniform in [-90, 90] degrees.
* Monte Carlo moves: per trial a few random joints with uniform offsets, and
  one uniform number for the Metropolis test.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

N_TYPES = 20
ATOMS_PER_RES = 10
TYPE_TABLE_SEED = 0x1712
BASE_SEED = 1712050120

_DATA_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "data")


@dataclass(frozen=True)
class ResidueTypes:
    """Per-type, per-slot force-field inputs.  Shapes: q, sigma, eps: (20, 10); hydro: (20,)."""

    q: np.ndarray
    sigma: np.ndarray
    eps: np.ndarray
    hydro: np.ndarray


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _charges(rng: np.random.Generator) -> np.ndarray:
    q_net = float(rng.integers(-1, 2))
    q = rng.uniform(-0.5, 0.5, ATOMS_PER_RES)
    q += (q_net - q.sum()) / ATOMS_PER_RES
    for _ in range(100):
        q = np.clip(q, -0.5, 0.5)
        diff = q_net - q.sum()
        if abs(diff) < 1e-15:
            break
        free = (q < 0.5) if diff > 0 else (q > -0.5)
        q[free] += diff / free.sum()
    q = np.clip(q, -0.5, 0.5)
    q[np.argmax(np.where(np.abs(q) < 0.5, 1.0, 0.0))] += q_net - q.sum()
    return q


def residue_types(seed: int = TYPE_TABLE_SEED) -> ResidueTypes:
    rng = _rng(seed)
    q = np.empty((N_TYPES, ATOMS_PER_RES))
    for t in range(N_TYPES):
        q[t] = _charges(rng)
    sigma = rng.uniform(1.8, 4.0, (N_TYPES, ATOMS_PER_RES))
    eps = rng.uniform(0.02, 0.2, (N_TYPES, ATOMS_PER_RES))
    hydro = rng.uniform(-4.5, 4.5, N_TYPES)
    return ResidueTypes(q=q, sigma=sigma, eps=eps, hydro=hydro)


def config_seed(config: int, chain: int = 0) -> int:
    """Base seed of workload ``config`` (1-based); chain ``b`` of a batch adds 1000*b."""
    return BASE_SEED + int(config) + 1000 * int(chain)


def sequence(m: int, seed: int) -> np.ndarray:
    return _rng(seed * 2 + 1).integers(0, N_TYPES, int(m)).astype(np.int32)


def random_dihedrals(m: int, seed: int) -> np.ndarray:
    """(phi_1, psi_1, ..., phi_m, psi_m), each uniform in (-pi, pi]."""
    u = _rng(seed * 2 + 2).uniform(0.0, 2.0 * np.pi, 2 * int(m))
    return np.pi - u


def random_chi(m: int, seed: int) -> np.ndarray:
    """(chi_1, ..., chi_m), side-chain angles, each uniform in (-pi, pi]."""
    u = _rng(seed * 2 + 3).uniform(0.0, 2.0 * np.pi, int(m))
    return np.pi - u


def batch_lengths(n_chains: int, seed: int, lo: int = 50, hi: int = 600) -> np.ndarray:
    return _rng(seed).integers(lo, hi + 1, int(n_chains)).astype(np.int32)


def serving_jobs(n_jobs: int, seed: int, rate: float = 50.0, median: float = 200.0,
                 sigma: float = 0.6, lo: int = 30, hi: int = 2000):
    """Arrival times (s, increasing) and residue counts of a Poisson job stream."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, int(n_jobs))
    arrivals = np.cumsum(gaps) - gaps[0]
    lengths = np.clip(np.rint(np.exp(rng.normal(np.log(median), sigma, int(n_jobs)))), lo, hi)
    return arrivals, lengths.astype(np.int32)


def alanine_like_types() -> ResidueTypes:
    """One residue type shaped like alanine, for the polyalanine experiments.

    Slots N, H, CA, HA, CB, HB1-3, C, O.  Charges give the backbone amide its
    dipole (N -0.40, H +0.25, C +0.50, O -0.50 e) and the CH3 group a small
    polarity; the residue is neutral.  Lennard-Jones sigma and well depth are
    element-typical round values (C 3.4 A / 0.09, N 3.25 A / 0.17,
    O 3.0 A / 0.21 kcal/mol, H on carbon 2.5 A, H on nitrogen 1.1 A,
    both 0.02 kcal/mol).  Hydrophobicity +1.8 (alanine on the Kyte-Doolittle
    scale).  These are not the force-field tables of any published model.
    """
    q = np.array([[-0.40, 0.25, 0.05, 0.05, -0.10, 0.05, 0.05, 0.05, 0.50, -0.50]])
    sigma = np.array([[3.25, 1.10, 3.40, 2.50, 3.40, 2.50, 2.50, 2.50, 3.40, 3.00]])
    eps = np.array([[0.17, 0.02, 0.09, 0.02, 0.09, 0.02, 0.02, 0.02, 0.09, 0.21]])
    return ResidueTypes(q=q, sigma=sigma, eps=eps, hydro=np.array([1.8]))


def polyala_starts(n_chains: int, seed: int, lo: int = 10, hi: int = 20, max_deg: float = 90.0):
    """Residue counts uniform in [lo, hi] and, per chain, (phi_1, psi_1, ...)
    uniform in [-max_deg, +max_deg] degrees (radians)."""
    rng = _rng(seed)
    lengths = rng.integers(lo, hi + 1, int(n_chains)).astype(np.int32)
    lim = np.radians(max_deg)
    thetas = [rng.uniform(-lim, lim, 2 * int(m)) for m in lengths]
    return lengths, thetas


def mc_moves(n_trials: int, n_joints: int, seed: int, n_moved: int = 2, max_rad: float = 0.5):
    """Monte Carlo perturbations [n_trials, n_joints]: per trial, n_moved
    distinct joints drawn uniformly get an offset uniform in [-max_rad,
    max_rad]; the others stay 0.  Also the trials' Metropolis uniforms
    [n_trials] in [0, 1).  Returns (delta, u)."""
    rng = _rng(seed)
    d = np.zeros((int(n_trials), int(n_joints)))
    k = min(int(n_moved), int(n_joints))
    for t in range(int(n_trials)):
        js = rng.choice(int(n_joints), size=k, replace=False)
        d[t, js] = rng.uniform(-max_rad, max_rad, k)
    u = rng.uniform(0.0, 1.0, int(n_trials))
    return d, u


def load_globule(m: int) -> np.ndarray:
    """Stored compact-globule dihedrals for an m-residue chain of ``sequence(m, config_seed(c))``.

    The files are inputs written once by ``oracle/make_globules.py``; they are
    read here, never computed.
    """
    path = os.path.join(_DATA_DIR, f"globule_m{int(m)}.npy")
    if not os.path.exists(path):
        raise FileNotFoundError(f"no stored globule for m={m}: {path}")
    th = np.load(path, allow_pickle=False)
    if th.shape != (2 * int(m),):
        raise ValueError(f"{path}: shape {th.shape}, expected {(2 * int(m),)}")
    return th.astype(np.float64)
