#!/usr/bin/env python3
"""Throughput of KCM iterations (atom-steps/s) on one MI355X.

Headline workload: the ragged batch of 256 chains with lengths uniform in
[50, 600] residues (818,020 atoms), random-coil starts from per-chain seeds,
10 A cutoff, 250 samples per offset sphere, mixed precision (FP32 pair forces
and sample tests, FP64 kinematics, torques and step), the cell edge and the
iterations per replayed HIP graph picked by the autotuner on the same batch
before timing.  One step is one KCM iteration of every chain of the batch
(forward kinematics, cell list, Coulomb + LJ + SASA solvation forces,
torques, compliance step).  Inputs are built and every graph is captured
before the timed region, which covers exactly --steps iterations between two
device synchronisations.  Prints one JSON line.

Sub-legs (each with its own roofline): the 1000-residue compact globule
(10,000 atoms, 1,000 iterations) in mixed precision and in FP64, the
10,000-residue globule (100,000 atoms, 200 iterations), the batch run for its
500 iterations, the serving loop, energy scans and the polyalanine runs.

Roofline of the dominant kernel (the force kernel): algorithmic FP work per
launch = 40 flops per unordered pair within the cutoff + 9 flops per
(sample, solvation neighbour) coverage test + 9 flops per (exposed sample,
neighbour) pair for the three displaced tests, summed over the chains of the
launch, divided by the kernel's mean launch time from HIP events recorded on
its launch stream on sampled iterations of the timed region (at least five).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}  # MI355X vector FP32 / FP64
MIN_SAMPLES = 5    # HIP-event samples of the force kernel in a timed region, at least
MAX_EVERY = 50     # and at least one every 50 timed iterations
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kernel_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1712_05012_amd", "csrc", "kcm_kernels.hip")


# Single-chain workloads: residues and the sequence-seed config number.  Both
# start from a stored compact globule (radius of gyration 2.2 m^0.38 A).
WORKLOADS = {
    "globule1000": (1000, 2, 1000),    # (residues, seed config, default steps)
    "globule10000": (10000, 4, 200),
}


def workload(m: int = 1000):
    import synth

    T = synth.residue_types()
    cfg = {res: c for res, c, _ in WORKLOADS.values()}.get(m, 2)
    seq = synth.sequence(m, synth.config_seed(cfg))
    th = synth.load_globule(m)
    return T, seq, th


def algorithmic_units(xyz, T, seq, p, n_exposed, n_samples):
    """Unit counts of one force evaluation at positions xyz."""
    import numpy as np
    from scipy.spatial import cKDTree

    tree = cKDTree(xyz)
    n_pairs = len(tree.query_pairs(p.cutoff, output_type="ndarray"))
    sig = np.asarray(T.sigma)[seq].reshape(-1)
    roff = 0.5 * 2.0 ** (1.0 / 6.0) * sig + p.r_probe
    cand = tree.query_pairs(2 * roff.max() + p.delta_r, output_type="ndarray")
    d = np.linalg.norm(xyz[cand[:, 0]] - xyz[cand[:, 1]], axis=1)
    keep = cand[d <= roff[cand[:, 0]] + roff[cand[:, 1]] + p.delta_r]
    nbr = np.bincount(keep.reshape(-1), minlength=xyz.shape[0])
    tests1 = int(n_samples) * int(nbr.sum())
    tests2 = int((np.asarray(n_exposed, dtype=np.int64) * nbr).sum())
    flops = 40.0 * n_pairs + 9.0 * tests1 + 9.0 * tests2
    return {"pairs_within_cutoff": int(n_pairs), "sasa_neighbours_mean": float(nbr.mean()),
            "coverage_tests": tests1, "exposed_sample_neighbour_pairs": tests2,
            "exposed_fraction": float(np.mean(n_exposed) / n_samples), "flops": flops}


def timing_every(steps: int) -> int:
    """Sample interval of the HIP events over a timed region of `steps`
    iterations: at least MIN_SAMPLES samples, and one per MAX_EVERY."""
    return max(1, min(MAX_EVERY, steps // MIN_SAMPLES))


def timed_steps(kcm, chains, steps, stream):
    """Exactly `steps` iterations of `chains` between two device
    synchronisations, with the force kernel bracketed by HIP events on sampled
    iterations; returns (seconds, force-kernel ms per launch, iteration ms,
    number of samples)."""
    import torch

    kcm.kcm_get_timing(reset=True)
    kcm.kcm_set_timing(timing_every(steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kcm.kcm_step(chains, steps, stream, report=False)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    kcm.kcm_set_timing(0)
    tm = kcm.kcm_get_timing(reset=True)
    n = max(tm["force_launches"], 1)
    return secs, tm["force_ms"] / n, tm["iter_ms"] / max(tm["iterations"], 1), int(tm["force_launches"])


def run_gpu(precision: str, steps: int, warmup: int, m: int, side_chains: bool = False, depth: int = 8):
    """A single globule chain; warm-up of at least one graph depth so that
    every graph is captured before the timed region."""
    import numpy as np
    import torch

    from paper_1712_05012_amd import kcm

    T, seq, th = workload(m)
    if side_chains:
        # chi at its zero position: the same conformation, with m more joints
        th = np.concatenate([th, np.full(m, np.pi / 3)])
    prec = kcm.KCM_MIXED if precision == "mixed" else kcm.KCM_FP64
    p = kcm.kcm_default_params(precision=prec)
    chain = kcm.Chain(seq, T, p, theta0=th, side_chains=side_chains)
    stream = torch.cuda.current_stream()
    kcm.kcm_step([chain], max(warmup, 1) + depth, stream, report=False)
    torch.cuda.synchronize()
    secs, force_ms, iter_ms, samples = timed_steps(kcm, [chain], steps, stream)
    _, reps = kcm.kcm_step([chain], 0, stream, report=True, check=False)
    st = chain.state()
    terms = chain.atom_terms()
    units = algorithmic_units(st["xyz"], T, seq, p, terms["n_exposed"], chain.n_samples)
    out = {
        "n_atoms": chain.n_atoms,
        "steps": steps,
        "seconds": secs,
        "ms_per_step": 1e3 * secs / steps,
        "value": chain.n_atoms * steps / secs,
        "force_ms_mean": force_ms,
        "iter_ms_mean": iter_ms,
        "force_samples": samples,
        "units": units,
        "status": reps[0].status,
        "energies": [reps[0].e_elec, reps[0].e_vdw, reps[0].e_cav],
        "n_samples": chain.n_samples,
    }
    chain.free()
    return out


def roofline(units, force_ms, precision, traffic=None):
    achieved = units["flops"] / (force_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic}


def sum_units(per_chain):
    tot = {"pairs_within_cutoff": 0, "coverage_tests": 0, "exposed_sample_neighbour_pairs": 0, "flops": 0.0}
    nbr = atoms = exp = 0.0
    for u, n, ns in per_chain:
        for k in tot:
            tot[k] += u[k]
        nbr += u["sasa_neighbours_mean"] * n
        exp += u["exposed_fraction"] * n
        atoms += n
    tot["sasa_neighbours_mean"] = nbr / atoms
    tot["exposed_fraction"] = exp / atoms
    return tot


def batch_workload(n_chains: int = 256):
    """256 chains, lengths uniform in [50, 600] residues, per-chain seeds, random dihedrals."""
    import synth

    T = synth.residue_types()
    lens = synth.batch_lengths(n_chains, synth.config_seed(3))
    chains = []
    for b, m in enumerate(lens):
        seed = synth.config_seed(3, b)
        chains.append((synth.sequence(int(m), seed), synth.random_dihedrals(int(m), seed)))
    return T, chains


def run_batch(steps: int, warmup: int, n_chains: int = 256, tune: bool = True, direct: bool = False,
              full_steps: int = 500, setting=None):
    """Ragged batch in mixed precision: all chains advanced together by replayed
    HIP graphs, with the cell edge and the iterations per graph picked by the
    autotuner on the same batch first.  Times `steps` iterations (events on
    sampled ones), then, on fresh chains, the workload's full `full_steps`
    iterations without event samples."""
    import torch

    from paper_1712_05012_amd import autotune, kcm

    T, items = batch_workload(n_chains)
    stream = torch.cuda.current_stream()
    if setting is not None:
        # a fixed (cell edge, force variant, graph depth), e.g. the tuner's
        # choice taken again under a profiler
        tuned = autotune.TuneResult(cell_size=setting[0], force_variant=setting[1], graph_depth=setting[2],
                                    atom_steps_per_s=0.0)
        kcm.kcm_set_force_variant(tuned.force_variant)
    else:
        tuned = autotune.tune(T, items, kcm.KCM_MIXED, stream=stream) if tune and not direct else None
    p = kcm.kcm_default_params(precision=kcm.KCM_MIXED, cell_size=tuned.cell_size if tuned else 0.0)
    depth = 0 if direct else (tuned.graph_depth if tuned else 1)
    chains = [kcm.Chain(seq, T, p, theta0=th) for seq, th in items]
    atoms = sum(c.n_atoms for c in chains)
    n_samples = chains[0].n_samples
    kcm.kcm_set_graphs(depth)
    full = None
    try:
        # warm-up: captures the one-iteration and the depth-iteration graphs
        kcm.kcm_step(chains, max(warmup, 1) + depth, stream, report=False)
        torch.cuda.synchronize()
        secs, force_ms, iter_ms, samples = timed_steps(kcm, chains, steps, stream)
        _, reps = kcm.kcm_step(chains, 0, stream, report=True, check=False)
        bad = sum(r.status != 0 for r in reps)
        per_chain = []
        for c, (seq, _) in zip(chains, items):
            st = c.state()
            terms = c.atom_terms()
            per_chain.append((algorithmic_units(st["xyz"], T, seq, p, terms["n_exposed"], c.n_samples),
                              c.n_atoms, c.n_samples))
        units = sum_units(per_chain)
        if full_steps > 0:
            fresh = [kcm.Chain(seq, T, p, theta0=th) for seq, th in items]
            try:
                kcm.kcm_step(fresh, depth + 1, stream, report=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                kcm.kcm_step(fresh, full_steps, stream, report=False)
                torch.cuda.synchronize()
                fs = time.perf_counter() - t0
                _, freps = kcm.kcm_step(fresh, 0, stream, report=True, check=False)
                full = {"steps": full_steps, "seconds": fs, "ms_per_step": 1e3 * fs / full_steps,
                        "value": atoms * full_steps / fs,
                        "failed_chains": int(sum(r.status != 0 for r in freps)),
                        "note": "fresh chains from the same starts, depth+1 warm-up iterations, no event samples"}
            finally:
                for c in fresh:
                    c.free()
    finally:
        kcm.kcm_set_graphs(0 if direct else 1)
        kcm.kcm_set_force_variant(0)
        for c in chains:
            c.free()
    out = {"chains": len(items), "atoms": atoms, "steps": steps, "seconds": secs, "ms_per_step": 1e3 * secs / steps,
           "value": atoms * steps / secs, "failed_chains": int(bad), "cell_size": p.cell_size, "graph_depth": depth,
           "force_variant": tuned.force_variant if tuned else 0,
           "force_ms_mean": force_ms, "iter_ms_mean": iter_ms, "force_samples": samples, "units": units,
           "n_samples": n_samples}
    if full:
        out["full_run"] = full
    if tuned:
        out["autotune"] = tuned.as_dict()
    return out


def run_per_chain_fp64(steps: int, n_sample: int = 16, n_chains: int = 256):
    """The plain FP64 path run one chain at a time, on a sample of the batch's chains."""
    import torch

    from paper_1712_05012_amd import kcm

    T, items = batch_workload(n_chains)
    p = kcm.kcm_default_params(precision=kcm.KCM_FP64)
    pick = items[:n_sample]
    atom_steps, secs = 0, 0.0
    for seq, th in pick:
        c = kcm.Chain(seq, T, p, theta0=th)
        kcm.kcm_step([c], 2, report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kcm.kcm_step([c], steps, report=False)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        atom_steps += c.n_atoms * steps
        c.free()
    return {"value": atom_steps / secs, "sample": f"{n_sample} of the {n_chains} chains, {steps} iterations each, "
            "one chain per call"}


def run_serving(n_jobs: int, max_iter: int, budget_gib: float, skip: int, setting=(0.0, 0)):
    """Poisson arrivals at 50 jobs/s, lognormal lengths; continuous batching by HBM budget.

    Latency percentiles leave out the first ``skip`` jobs (warm-up); the queue
    growth rate says whether one GPU keeps up with the offered load.  The jobs
    run with ``setting`` = (cell edge, force-kernel shape), by default the
    automatic cell edge and shape 0; the full run passes the setting the batch
    leg tuned on random coils of the same kind."""
    import numpy as np

    import synth
    from paper_1712_05012_amd import kcm
    from paper_1712_05012_amd.serve import FoldService, Job, KcmEngine

    T = synth.residue_types()
    seed = synth.config_seed(5)
    arrivals, lengths = synth.serving_jobs(n_jobs, seed)
    jobs = []
    for k, (a, m) in enumerate(zip(arrivals, lengths)):
        js = seed + 1000 * (k + 1)
        jobs.append(Job(job_id=k, res_type=synth.sequence(int(m), js), theta0=synth.random_dihedrals(int(m), js),
                        arrival=float(a), tol=1e-4, max_iter=max_iter))
    eng = KcmEngine(T, kcm.kcm_default_params(precision=kcm.KCM_MIXED, cell_size=setting[0]))
    svc = FoldService(eng, hbm_budget=int(budget_gib * (1 << 30)), max_slots=1024, check_every=20)
    def progress(job, n_done):
        if n_done % 250 == 0 or n_done == n_jobs:
            print(f"serving: {n_done} of {n_jobs} jobs done", file=sys.stderr, flush=True)

    kcm.kcm_set_force_variant(setting[1])
    try:
        st = svc.run(jobs, on_retire=progress)
    finally:
        kcm.kcm_set_force_variant(0)
    out = st.summary(skip=min(skip, max(0, n_jobs - 1)))
    offered = 50.0 * 10.0 * float(np.mean(lengths)) * max_iter
    out.update({"arrival_rate_per_s": 50.0, "max_iter": max_iter, "tol_dtheta": 1e-4,
                "hbm_budget_gib": budget_gib, "cell_size": setting[0], "force_variant": setting[1],
                "offered_atom_steps_per_s_at_iteration_cap": offered,
                "note": "latency is finish minus arrival and includes queueing; a positive queue "
                        "growth means the offered load exceeds what one GPU serves"})
    return out


def run_landscape(step_deg: float = 5.0, batch: int = 1024):
    """Ramachandran energy map of a residue pair (one residue type), every joint
    fixed: grid points evaluated per second, host marshalling included."""
    import numpy as np
    import torch

    import synth
    from paper_1712_05012_amd import kcm
    from paper_1712_05012_amd.landscape import EnergyScanner, grid_thetas

    T = synth.residue_types()
    res = np.zeros(2, np.int32)
    vals = np.radians(np.arange(-180.0, 180.0, step_deg))
    grid = grid_thetas(np.full(4, np.pi), [2, 3], [vals, vals])
    sc = EnergyScanner(res, T, kcm.kcm_default_params(precision=kcm.KCM_MIXED), batch=batch)
    sc.energies(grid[:batch])  # warm-up: graphs and first launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = sc.energies(grid)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sc.free()
    return {"grid_points": int(len(grid)), "step_deg": step_deg, "batch": batch, "seconds": dt,
            "points_per_s": len(grid) / dt, "atom_steps_per_s": 20 * len(grid) / dt,
            "e_min": float(E.sum(axis=1).min()),
            "note": "residue pair of type 0 (20 atoms), (phi, psi) of the second residue, mixed precision; "
                    "per point: set the dihedrals, rebuild the grid, one iteration with every joint fixed"}


def run_polyala(n_chains: int = 2000):
    """The polyalanine experiments through the batched path: the four helix
    runs (15 residues, starts +-10 degrees, vacuum and water) and the folding
    statistics of n_chains chains of 10-20 residues from random starts, in
    vacuum (converged below 1e-4 rad or 2,000 iterations) and in water
    (500 iterations: the piecewise-constant solvation forces keep the steps at
    their cap)."""
    import numpy as np

    from paper_1712_05012_amd import kcm, polyala

    out = {}
    t0 = time.perf_counter()
    runs = polyala.helix_runs(n_iter=1500, trace_every=100, precision=kcm.KCM_MIXED)
    out["helix"] = {
        "seconds": time.perf_counter() - t0,
        "runs": [{"start_deg": r["start_deg"], "water": r["solvation"], "hand": r["handedness"],
                  "mean_phi_psi": [round(x, 1) for x in r["mean_phi_psi"]], "energy": r["energy"]}
                 for r in runs],
    }
    for water, max_iter in ((False, 2000), (True, 500)):
        t0 = time.perf_counter()
        st = polyala.ramachandran_statistics(n_chains=n_chains, solvation=water, max_iter=max_iter, tol=1e-4,
                                             precision=kcm.KCM_MIXED, check_every=50)
        wall = time.perf_counter() - t0
        n_res = int(st["phi"].size)
        out["statistics_water" if water else "statistics_vacuum"] = {
            "chains": n_chains, "residues_counted": n_res, "max_iter": max_iter,
            "fold_seconds": st["fold_seconds"], "wall_seconds_with_build": wall,
            "atom_steps_per_s": st["atom_steps"] / st["fold_seconds"],
            "mean_iterations": float(np.mean(st["iterations"])),
            "converged_fraction": float(np.mean(st["converged"])),
            "failed_chains": int((st["status"] != 0).sum()),
            "region_fractions": {k: v / n_res for k, v in st["region_counts"].items()},
        }
    mc = polyala.mc_versus_descent(n_chains=n_chains, precision=kcm.KCM_MIXED)
    ok = mc["status"] == 0
    out["mc_versus_descent"] = {
        "chains": n_chains, "evaluations_each": mc["evaluations"], "trials": mc["n_trials"],
        "descent_per_trial": mc["n_descent"], "kT": mc["kT"],
        "descent_seconds": mc["descent_seconds"], "search_seconds": mc["search_seconds"],
        "search_atom_evaluations_per_s": mc["atoms"] * mc["evaluations"] / mc["search_seconds"],
        "mean_energy_descent": float(np.mean(mc["e_descent"][ok])),
        "mean_energy_search_best": float(np.mean(mc["e_search_best"][ok])),
        "median_energy_descent": float(np.median(mc["e_descent"][ok])),
        "median_energy_search_best": float(np.median(mc["e_search_best"][ok])),
        "search_lower_fraction": float(np.mean(mc["e_search_best"][ok] < mc["e_descent"][ok])),
        "mean_accepted": float(np.mean(mc["accepted"])),
        "failed_chains": int((~ok).sum()),
    }
    out["note"] = ("Ala-like residue type with element-typical constants, mixed precision, capped steps "
                   "of at most 0.01 rad; statistics leave out the first residue of every chain; the Monte "
                   "Carlo search and the plain descent make the same number of force evaluations")
    return out


def traffic_for(precision: str, workload_name: str):
    """HBM bytes per force launch from committed rocprofv3 counters of this
    workload, while the kernel source is the one they were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if rec.get("kernel_sha256") != sha:
            return None
        entry = rec.get("workloads", {}).get(workload_name, {}).get(precision)
        return float(entry["bytes_per_launch"]) if entry else None
    except Exception:
        return None


CPU_SUBSAMPLE = 16  # chains of the batch the oracle is timed on


def cpu_baseline(seconds: float):
    """The FP64 oracle as it stands, on the host cores, over a bounded sample
    of the headline workload: whole KCM iterations of the batch's first
    CPU_SUBSAMPLE chains, repeated (each chain from its own last angles) until
    `seconds` have passed; the rate is the sample's atom-steps per second,
    taken as the batch's."""
    import oracle

    T, items = batch_workload(256)
    pick = items[:CPU_SUBSAMPLE]
    refs = [oracle.OracleChain(seq, T) for seq, _ in pick]
    ths = [th.copy() for _, th in pick]
    atom_steps = passes = 0
    t0 = time.perf_counter()
    while True:
        for k, ch in enumerate(refs):
            ths[k] = oracle.iterate(ch, ths[k])["theta"]
            atom_steps += ch.n
        passes += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    n_atoms = sum(ch.n for ch in refs)
    out = {"value": atom_steps / dt, "unit": "atom-steps/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{passes} FP64 KCM iterations of each of the first {CPU_SUBSAMPLE} of the 256 batch chains "
                     f"({n_atoms} atoms), {dt:.1f} s; the subsample's rate stands for the batch's"}
    single = cpu_single_core(max(2.0, seconds / 3))
    if single is not None:
        out["single_core_value"] = single
    return out


def cpu_single_core(seconds: float):
    """The same oracle sample on one host core (a child process with one
    OpenMP thread); atom-steps/s, or None if the child fails."""
    import subprocess

    code = (
        "import json, sys, time\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.abspath(__file__))!r})\n"
        "import bench, oracle\n"
        "T, items = bench.batch_workload(256)\n"
        f"pick = items[:{CPU_SUBSAMPLE}]\n"
        "refs = [oracle.OracleChain(seq, T) for seq, _ in pick]\n"
        "ths = [th.copy() for _, th in pick]\n"
        "n = 0\n"
        "t0 = time.perf_counter()\n"
        f"while n == 0 or time.perf_counter() - t0 < {float(seconds)}:\n"
        "    for k, ch in enumerate(refs):\n"
        "        ths[k] = oracle.iterate(ch, ths[k])['theta']\n"
        "        n += ch.n\n"
        "print(json.dumps({'v': n / (time.perf_counter() - t0), 't': oracle.threads()}))\n"
    )
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=seconds * 10 + 120)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        return d["v"] if d["t"] == 1 else None
    except Exception:
        return None


def globule_leg(name: str, precision: str, warmup: int, steps: int | None = None):
    residues, _, default_steps = WORKLOADS[name]
    r = run_gpu(precision, steps or default_steps, warmup, residues)
    return {"workload": f"single chain, {residues} residues ({10 * residues:,} atoms), compact random globule, "
                        f"{precision} precision", "value": r["value"], "steps": r["steps"],
            "ms_per_step": r["ms_per_step"], "status": r["status"],
            "kernel_ms": {"force": r["force_ms_mean"], "iteration": r["iter_ms_mean"],
                          "chain_kernels": r["iter_ms_mean"] - r["force_ms_mean"]},
            "force_samples": r["force_samples"], "units_per_step": r["units"],
            "roofline": roofline(r["units"], r["force_ms_mean"], precision, traffic_for(precision, name))}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed iterations of the batch (the workload's 500)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full-steps", type=int, default=500,
                    help="iterations of the batch's full run on fresh chains (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="jobs of the serving run (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=100,
                    help="earliest jobs left out of the serving latency percentiles")
    ap.add_argument("--serve-max-iter", type=int, default=2000)
    ap.add_argument("--legs", default="batch,globule1000,globule1000_fp64,globule10000,chi,serving,landscape,"
                                      "polyala,cpu",
                    help="comma-separated legs (batch is the headline; globule1000, globule1000_fp64, "
                         "globule10000, chi, serving, landscape, polyala, cpu); profiling runs use a subset")
    ap.add_argument("--globule-steps", type=int, default=None,
                    help="timed iterations of the globule legs (default: the workload's, 1,000 and 200)")
    ap.add_argument("--graph-depth", type=int, default=8,
                    help="iterations per replayed HIP graph in the single-chain legs")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch each iteration's kernels directly instead of replaying a HIP graph")
    ap.add_argument("--no-tune", action="store_true", help="batch leg with the default cell edge, one-deep graphs")
    ap.add_argument("--batch-setting", default=None, metavar="CELL,VARIANT,DEPTH",
                    help="batch leg at this cell edge, force variant and graph depth instead of tuning")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs its chains on a single MI355X "
              "(how chains would shard over several GPUs is described in the design notes); "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_1712_05012_amd import kcm

    depth = 0 if args.no_graphs else args.graph_depth
    kcm.kcm_set_graphs(depth)
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    legs = set(args.legs.split(","))
    if args.serve_jobs <= 0:
        legs.discard("serving")
    if args.no_cpu_baseline:
        legs.discard("cpu")

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    line = {}
    serve_setting = (0.0, 0)
    if "batch" in legs:
        setting = None
        if args.batch_setting:
            cs, v, d = args.batch_setting.split(",")
            setting = (float(cs), int(v), 0 if args.no_graphs else int(d))
        b = run_batch(args.steps, args.warmup, tune=not args.no_tune, direct=args.no_graphs,
                      full_steps=args.full_steps, setting=setting)
        progress(f"batch done: {b['value']:.4g} atom-steps/s")
        u = b.pop("units")
        line = {
            "metric": "atom-steps/s per KCM iteration",
            "value": b["value"],
            "unit": "atom-steps/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": b["ms_per_step"],
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32+f64",
            "data": "synthetic",
            "config": {
                "workload": f"ragged batch of {b['chains']} chains, lengths uniform in [50, 600] residues "
                            f"({b['atoms']:,} atoms), random-coil starts, 10 A cutoff, 250 samples per offset "
                            "sphere, mixed precision, one KCM iteration of every chain per step",
                "name": "batch256",
                "precision": "mixed",
                "n_atoms": b["atoms"],
                "n_chains": b["chains"],
                "cell_size": b["cell_size"],
                "force_variant": b["force_variant"],
                "graph_depth": b["graph_depth"],
            },
            "roofline": roofline(u, b["force_ms_mean"], "mixed", traffic_for("mixed", "batch256")),
            "kernel_ms": {"force": b["force_ms_mean"], "iteration": b["iter_ms_mean"],
                          "chain_kernels": b["iter_ms_mean"] - b["force_ms_mean"]},
            "force_samples": b["force_samples"],
            "units_per_step": u,
            "failed_chains": b["failed_chains"],
        }
        if "full_run" in b:
            line["full_run"] = b["full_run"]
        if "autotune" in b:
            line["autotune"] = b["autotune"]
        serve_setting = (b["cell_size"], b["force_variant"])
        fp64 = run_per_chain_fp64(10)
        line["plain_fp64_per_chain"] = fp64
        line["speedup_vs_plain_fp64_per_chain"] = b["value"] / fp64["value"]
    sub = {}
    for name, prec in (("globule1000", "mixed"), ("globule1000_fp64", "fp64"), ("globule10000", "mixed")):
        if name in legs:
            sub[name] = globule_leg(name.replace("_fp64", ""), prec, args.warmup, args.globule_steps)
            progress(f"{name} done: {sub[name]['value']:.4g} atom-steps/s")
    if "chi" in legs:
        # the 1000-residue globule with one side-chain joint per residue
        residues, _, st = WORKLOADS["globule1000"]
        ch = run_gpu("mixed", args.globule_steps or st, args.warmup, residues, side_chains=True)
        sub["globule1000_side_chains"] = {"value": ch["value"], "ms_per_step": ch["ms_per_step"],
                                          "force_ms": ch["force_ms_mean"], "joints": 3 * residues}
    if sub:
        line["legs"] = sub
    if "serving" in legs:
        line["serving"] = run_serving(args.serve_jobs, args.serve_max_iter, 64.0, args.serve_warmup, serve_setting)
        progress("serving done")
    if "landscape" in legs:
        line["landscape"] = run_landscape()
    if "polyala" in legs:
        line["polyala"] = run_polyala()
    if "cpu" in legs:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
