"""Energy landscapes: the KCM energy terms over a grid of dihedral values.

A scan fixes every joint (the joint mask of the problem statement, Sec. 4)
and evaluates the Coulomb, Lennard-Jones and solvation energies of the chain
at each requested set of dihedrals: a Ramachandran map of a residue pair, or
a hinge scan of one or more joints of a longer chain.  The conformations of
a scan are spread over a pool of chains that one ``kcm_step`` call advances
together, so each call evaluates a whole batch of grid points on the device
(one iteration with every joint fixed leaves the dihedrals unchanged and
reports the energies of the conformation the forces were taken at).

Everything runs through the C ABI; this module only marshals the grid.
"""
from __future__ import annotations

import itertools

import numpy as np


class EnergyScanner:
    """A pool of ``batch`` copies of one chain with every joint fixed."""

    def __init__(self, res_type, residue_types, params=None, batch: int = 256, stream=None,
                 side_chains: bool = False):
        from . import kcm

        if batch < 1:
            raise ValueError("batch must be positive")
        self.kcm = kcm
        self.params = params if params is not None else kcm.kcm_default_params()
        self.stream = stream
        self.res_type = np.ascontiguousarray(res_type, dtype=np.int32)
        self.n_joints = (3 if side_chains else 2) * self.res_type.size
        mask = np.zeros(self.n_joints, np.uint8)
        self.pool = [kcm.Chain(self.res_type, residue_types, self.params, joint_mask=mask, stream=stream,
                               side_chains=side_chains)
                     for _ in range(batch)]

    def energies(self, thetas) -> np.ndarray:
        """thetas: [G, J] dihedrals (J = 2 n_res, or 3 n_res with side chains);
        returns [G, 3] (elec, vdw, cav) energies."""
        th = np.asarray(thetas, dtype=np.float64)
        if th.ndim != 2 or th.shape[1] != self.n_joints:
            raise ValueError(f"thetas must have shape [G, {self.n_joints}]")
        if not np.all(np.isfinite(th)):
            raise ValueError("thetas must be finite")
        out = np.zeros((th.shape[0], 3))
        B = len(self.pool)
        for g0 in range(0, th.shape[0], B):
            part = th[g0:g0 + B]
            chains = self.pool[:part.shape[0]]
            held = self.kcm.kcm_set_theta_batch(chains, part, self.stream)
            _, reps = self.kcm.kcm_step(chains, 1, self.stream, report="array", check=False)
            del held  # kcm_step with reports has synchronised the stream
            bad = np.nonzero(reps["status"] != 0)[0]
            if bad.size:
                k = int(bad[0])
                raise self.kcm.KcmError(int(reps["status"][k]), f"grid point {g0 + k}: numeric status {reps['status'][k]}")
            out[g0:g0 + len(chains)] = np.stack([reps["e_elec"], reps["e_vdw"], reps["e_cav"]], axis=1)
        return out

    def free(self):
        for c in self.pool:
            c.free()
        self.pool = []


def grid_thetas(theta0, joints, values) -> np.ndarray:
    """Every combination of ``values`` (one sequence per joint) at ``joints``, the
    other dihedrals at ``theta0``: [prod(len(v)), len(theta0)], the last joint fastest."""
    base = np.asarray(theta0, dtype=np.float64)
    joints = list(joints)
    if len(joints) != len(values):
        raise ValueError("one value sequence per joint")
    if any(j < 0 or j >= base.size for j in joints):
        raise ValueError("joint index out of range")
    combos = list(itertools.product(*[np.asarray(v, dtype=np.float64) for v in values]))
    out = np.repeat(base[None, :], len(combos), axis=0)
    for k, c in enumerate(combos):
        out[k, joints] = c
    return out


def ramachandran(res_type, residue_types, residue: int, step_deg: float = 10.0, theta0=None, params=None,
                 batch: int = 256, stream=None):
    """Energy map over (phi, psi) of one residue: returns (phi, psi, E[n_phi, n_psi, 3])."""
    m = len(res_type)
    if not 0 <= residue < m:
        raise ValueError("residue out of range")
    vals = np.radians(np.arange(-180.0, 180.0, step_deg))
    th0 = np.full(2 * m, np.pi) if theta0 is None else np.asarray(theta0, dtype=np.float64)
    grid = grid_thetas(th0, [2 * residue, 2 * residue + 1], [vals, vals])
    sc = EnergyScanner(res_type, residue_types, params, batch=min(batch, len(grid)), stream=stream)
    try:
        E = sc.energies(grid)
    finally:
        sc.free()
    return vals, vals, E.reshape(len(vals), len(vals), 3)
