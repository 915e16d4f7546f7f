"""Shared helpers of the GPU tests: build a chain on both sides from the same
seeded inputs and compare the HIP path with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import synth
from paper_1712_05012_amd import kcm

TYPES = synth.residue_types()

# Tolerances stated for the method: per-atom force error relative to the
# largest force, and per-step joint-angle error in each precision form.
F_TOL = 1e-5
DTHETA_TOL = {kcm.KCM_FP64: 1e-7, kcm.KCM_MIXED: 1e-5}
# Joint torques, relative to the largest one: FP64 sums of FP64 forces differ
# from the oracle's by rounding order only; the mixed form's FP32 pair forces
# carry a relative error of about 1e-6 each, summed in FP64 along the chain.
TAU_TOL = {kcm.KCM_FP64: 1e-9, kcm.KCM_MIXED: 1e-5}
# Solvation forces are sums of integer event counts times a per-atom quantum
# held in 2^-32 fixed point: equal decisions leave a rounding of at most 2^-33
# per event, far below this bound for any atom of the tested chains.
F_CAV_ABS = 1e-8


def params(precision=kcm.KCM_FP64, **kw):
    return kcm.kcm_default_params(precision=precision, **kw)


def oracle_params(p):
    pp = oracle.PairParams(cutoff=p.cutoff, diel_k=p.diel_k, w13=p.w13, w14_elec=p.w14_elec, w14_vdw=p.w14_vdw)
    sp = oracle.SasaParams(delta_r=p.delta_r, r_probe=p.r_probe, n_orbits=p.n_orbits)
    return pp, sp


def terms_str(t):
    parts = []
    if t & (kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW):
        parts.append("elec+vdw")
    if t & kcm.KCM_TERM_CAV:
        parts.append("cav")
    return "+".join(parts)


def build_pair(m, seed, p, theta=None, mask=None, side_chains=False):
    seq = synth.sequence(m, seed)
    if theta is not None:
        th = np.asarray(theta, dtype=np.float64)
    elif side_chains:
        th = np.concatenate([synth.random_dihedrals(m, seed), synth.random_chi(m, seed)])
    else:
        th = synth.random_dihedrals(m, seed)
    gpu = kcm.Chain(seq, TYPES, p, theta0=th, joint_mask=mask, side_chains=side_chains)
    ref = oracle.OracleChain(seq, TYPES, g_hydro=p.g_hydro)
    return gpu, ref, th


def oracle_step(ref, th, p, mask=None):
    pp, sp = oracle_params(p)
    return oracle.iterate(ref, th, pp, sp, terms=terms_str(p.terms), mask=mask,
                          rule=oracle.StepRule(p.step_rule), kappa=p.kappa, s=p.max_step)


def compare_step(gpu, ref, th, p, mask=None, want_margin=1e-10):
    """One iteration on both sides from the same theta; returns (gpu state, oracle dict, errors)."""
    gpu.set_theta(th)
    rep = gpu.step(1)
    st = gpu.state()
    fp, fc = gpu.forces()
    o = oracle_step(ref, th, p, mask)
    fmax = max(np.abs(o["F"]).max(), 1e-300)
    err = {
        "xyz": float(np.abs(st["xyz"] - o["r"]).max()),
        "F": float(np.abs(st["force"] - o["F"]).max() / fmax),
        "F_pair": float(np.abs(fp - o["F_pair"]).max() / fmax),
        "F_cav": float(np.abs(fc - o["F_cav"]).max() / fmax),
        "tau": float(np.abs(st["tau"] - o["tau"]).max() / max(np.abs(o["tau"]).max(), 1e-300)),
        "dtheta": float(np.abs(st["dtheta"] - o["dtheta"]).max()),
        "theta": float(np.abs(np.angle(np.exp(1j * (st["theta"] - o["theta"])))).max()),
        "E_elec": abs(rep.e_elec - o["E_elec"]) / max(abs(o["E_elec"]), 1.0),
        "E_vdw": abs(rep.e_vdw - o["E_vdw"]) / max(abs(o["E_vdw"]), 1.0),
        "E_cav": abs(rep.e_cav - o["E_cav"]) / max(abs(o["E_cav"]), 1.0),
        "margin": o["margin"],
        "status": rep.status,
    }
    return st, o, err
