"""Polyalanine folding experiments (Sec. 5, alpha-helix formation, Table of
final helix angles, and the Ramachandran statistics of many short chains),
run through the batched KCM path.

* Helix coiling: a 15-residue chain started from the slightly pre-coiled
  phi = psi = +10 degrees or -10 degrees, in vacuum (Coulomb + Lennard-Jones)
  and in water (with the solvation term).  The four runs advance together in
  one batch; their energies are recorded along the way.
* Statistics: many chains of 10-20 residues from random phi, psi in
  [-90, 90] degrees, folded together by ``kcm_fold``; the folded (phi, psi) of
  every residue but the first are collected and sorted into Ramachandran
  regions.

The residue is Ala-shaped with element-typical constants
(``synth.alanine_like_types``), so the outcomes are qualitative: the hand each
start coils into, which hand ends lower in energy, where the folded angles
concentrate.  Everything runs through the C ABI; this module sets up chains
and reads their results back (the analysis of positions and angles is host
post-processing of finished runs).
"""
from __future__ import annotations

import numpy as np

CA_SLOT = 2
ATOMS_PER_RES = 10


def experiment_params(solvation: bool, precision=None, max_step: float = 1e-2, kappa: float = 1e-3):
    """Capped steps of at most max_step rad per joint; all three terms in water."""
    from . import kcm

    terms = kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW | (kcm.KCM_TERM_CAV if solvation else 0)
    return kcm.kcm_default_params(precision=kcm.KCM_FP64 if precision is None else precision,
                                  terms=terms, max_step=max_step, kappa=kappa,
                                  step_rule=kcm.KCM_STEP_CAPPED)


def ca_torsions(xyz) -> np.ndarray:
    """Virtual torsions (degrees) of consecutive C-alpha quadruples of a chain
    with 10 atom slots per residue: about +50 in a right-handed alpha-helix,
    about -50 in a left-handed one, near +-180 in an extended strand."""
    ca = np.asarray(xyz, dtype=np.float64).reshape(-1, ATOMS_PER_RES, 3)[:, CA_SLOT]
    if ca.shape[0] < 4:
        return np.zeros(0)
    b1 = ca[1:-2] - ca[:-3]
    b2 = ca[2:-1] - ca[1:-2]
    b3 = ca[3:] - ca[2:-1]
    # IUPAC sign: atan2(|b2| b1 . (b2 x b3), (b1 x b2) . (b2 x b3))
    y = np.linalg.norm(b2, axis=1) * np.einsum("ij,ij->i", b1, np.cross(b2, b3))
    x = np.einsum("ij,ij->i", np.cross(b1, b2), np.cross(b2, b3))
    return np.degrees(np.arctan2(y, x))


def handedness(xyz) -> str:
    """'right' or 'left' when the median C-alpha torsion lies in (0, 120) or
    (-120, 0) degrees, else 'extended'."""
    t = ca_torsions(xyz)
    if t.size == 0:
        return "extended"
    med = float(np.median(t))
    if 0.0 < med < 120.0:
        return "right"
    if -120.0 < med < 0.0:
        return "left"
    return "extended"


REGIONS = ("alpha_R", "alpha_L", "beta", "other")


def regions(phi_deg, psi_deg) -> np.ndarray:
    """Ramachandran region of each (phi, psi) in degrees, as indices into REGIONS:
    alpha_R phi in (-160, -20), psi in (-120, 50); alpha_L phi in (20, 160),
    psi in (-50, 120); beta phi in (-180, -45], psi >= 90 or psi <= -150."""
    phi = np.asarray(phi_deg, dtype=np.float64)
    psi = np.asarray(psi_deg, dtype=np.float64)
    out = np.full(phi.shape, 3, dtype=np.int32)
    beta = (phi > -180.0) & (phi <= -45.0) & ((psi >= 90.0) | (psi <= -150.0))
    out[beta] = 2
    al = (phi > 20.0) & (phi < 160.0) & (psi > -50.0) & (psi < 120.0)
    out[al] = 1
    ar = (phi > -160.0) & (phi < -20.0) & (psi > -120.0) & (psi < 50.0)
    out[ar] = 0
    return out


def _wrap_deg(x):
    return (np.asarray(x) + 180.0) % 360.0 - 180.0


def helix_runs(n_res: int = 15, starts_deg=(10.0, -10.0), n_iter: int = 1500, trace_every: int = 10,
               precision=None, max_step: float = 1e-2, stream=None):
    """The helix-coiling runs: every start in vacuum and in water, one batch.

    Returns a list of dicts (start_deg, solvation, theta, phi, psi in degrees,
    xyz, handedness, mean phi/psi over residues 2..n, energies [k, 3] and
    iterations [k] of the trace, final total energy, status)."""
    import synth

    from . import kcm

    T = synth.alanine_like_types()
    seq = np.zeros(n_res, np.int32)
    runs = []
    chains = []
    for start in starts_deg:
        for solv in (False, True):
            p = experiment_params(solv, precision, max_step)
            th = np.full(2 * n_res, np.radians(start))
            chains.append(kcm.Chain(seq, T, p, theta0=th, stream=stream))
            runs.append({"start_deg": float(start), "solvation": solv})
    trace = [[] for _ in chains]
    its = []
    done = 0
    try:
        while done < n_iter:
            k = min(trace_every, n_iter - done)
            _, reps = kcm.kcm_step(chains, k, stream, report=True, check=False)
            done += k
            its.append(done)
            for t, r in zip(trace, reps):
                t.append((r.e_elec, r.e_vdw, r.e_cav))
        for run, c, t, r in zip(runs, chains, trace, reps):
            st = c.state(stream)
            th = st["theta"]
            # one more force evaluation would be needed for the energies of the
            # final angles; the trace's last entry is the conformation before
            # the last step
            phi = _wrap_deg(np.degrees(th[0::2]))
            psi = _wrap_deg(np.degrees(th[1::2]))
            run.update({
                "theta": th, "phi": phi, "psi": psi, "xyz": st["xyz"],
                "handedness": handedness(st["xyz"]),
                "mean_phi_psi": (float(phi[1:].mean()), float(psi[1:].mean())),
                "energies": np.array(t), "iterations": np.array(its),
                "status": int(r.status),
            })
            e = run["energies"][-1]
            run["energy"] = float(e[0] + e[1] + (e[2] if run["solvation"] else 0.0))
    finally:
        for c in chains:
            c.free()
    return runs


def ramachandran_statistics(n_chains: int = 2000, seed: int = 1712, lo: int = 10, hi: int = 20,
                            solvation: bool = False, max_iter: int = 2000, tol: float = 1e-4,
                            precision=None, max_step: float = 1e-2, check_every: int = 20,
                            batch: int | None = None, stream=None):
    """Fold n_chains random polyalanine chains (lengths in [lo, hi], phi, psi
    uniform in [-90, 90] degrees) through the batched path and collect the
    folded (phi, psi) of every residue except the first of each chain.

    Returns a dict with phi, psi (degrees), the region counts over REGIONS,
    per-chain iterations and converged flags, the atom-steps done and the
    seconds spent in ``kcm_fold``."""
    import synth

    from . import kcm

    T = synth.alanine_like_types()
    lengths, thetas = synth.polyala_starts(n_chains, seed, lo, hi)
    p = experiment_params(solvation, precision, max_step)
    B = n_chains if batch is None else max(1, int(batch))
    phis, psis, iters, conv, status = [], [], [], [], []
    atom_steps = 0
    fold_s = 0.0
    for b0 in range(0, n_chains, B):
        chains = [kcm.Chain(np.zeros(m, np.int32), T, p, theta0=th, stream=stream)
                  for m, th in zip(lengths[b0:b0 + B], thetas[b0:b0 + B])]
        try:
            _, res = kcm.kcm_fold(chains, tol, max_iter, check_every, stream, check=False)
            fold_s += max(r.seconds for r in res)
            for c, r in zip(chains, res):
                th = c.theta(stream)
                phis.append(_wrap_deg(np.degrees(th[2::2])))
                psis.append(_wrap_deg(np.degrees(th[3::2])))
                iters.append(int(r.iterations))
                conv.append(bool(r.converged))
                status.append(int(r.status))
                atom_steps += int(r.iterations) * c.n_atoms
        finally:
            for c in chains:
                c.free()
    phi = np.concatenate(phis)
    psi = np.concatenate(psis)
    reg = regions(phi, psi)
    return {
        "phi": phi, "psi": psi,
        "region_counts": {name: int((reg == k).sum()) for k, name in enumerate(REGIONS)},
        "iterations": np.array(iters), "converged": np.array(conv), "status": np.array(status),
        "lengths": lengths, "atom_steps": atom_steps, "fold_seconds": fold_s,
    }


def mc_versus_descent(n_chains: int = 2000, seed: int = 1712, lo: int = 10, hi: int = 20, n_trials: int = 20,
                      n_descent: int = 50, kT: float = 1.0, n_moved: int = 2, max_rad: float = 0.5,
                      solvation: bool = False, precision=None, max_step: float = 1e-2, stream=None):
    """Monte Carlo minimization (``kcm_mc_minimize``) against plain KCM descent
    with the same number of force evaluations, on the statistics' chains.

    Both start from the same random conformations.  The descent runs
    1 + n_trials (n_descent + 1) iterations; the search makes n_trials trials
    of n_moved joints perturbed by up to max_rad, each descended n_descent
    iterations.  Returns per-chain final descent energies, lowest search
    energies, acceptance counts and the two calls' seconds."""
    import time

    import synth

    from . import kcm

    T = synth.alanine_like_types()
    lengths, thetas = synth.polyala_starts(n_chains, seed, lo, hi)
    p = experiment_params(solvation, precision, max_step)
    evals = 1 + n_trials * (n_descent + 1)
    out = {"n_chains": n_chains, "evaluations": evals, "n_trials": n_trials, "n_descent": n_descent, "kT": kT}
    chains = [kcm.Chain(np.zeros(m, np.int32), T, p, theta0=th, stream=stream) for m, th in zip(lengths, thetas)]
    try:
        kcm.kcm_step(chains, 1, stream)  # first launches and graph capture outside the timing
        held = kcm.kcm_set_theta_batch(chains, thetas, stream)
        t0 = time.perf_counter()
        _, reps = kcm.kcm_step(chains, evals, stream, report=True, check=False)
        out["descent_seconds"] = time.perf_counter() - t0
        e_desc = np.array([r.e_elec + r.e_vdw + (r.e_cav if solvation else 0.0) for r in reps])
        held = kcm.kcm_set_theta_batch(chains, thetas, stream)
        moves = [synth.mc_moves(n_trials, 2 * int(m), seed * 7919 + k, n_moved, max_rad)
                 for k, m in enumerate(lengths)]
        t0 = time.perf_counter()
        _, res = kcm.kcm_mc_minimize(chains, [mv[0] for mv in moves], np.stack([mv[1] for mv in moves]),
                                     n_descent, kT, stream, check=False)
        out["search_seconds"] = time.perf_counter() - t0
        del held
    finally:
        for c in chains:
            c.free()
    out["atoms"] = int(10 * lengths.sum())
    out["e_descent"] = e_desc
    out["e_search_best"] = np.array([r.e_best for r in res])
    out["accepted"] = np.array([r.accepted for r in res])
    out["status"] = np.array([r.status for r in res])
    return out
