#!/usr/bin/env python3
"""Throughput of KCM iterations (atom-steps/s) on one MI355X.

One step is one full KCM iteration of the chain (forward kinematics, cell
list, Coulomb + LJ + SASA solvation forces, torques, compliance step) on the
single 1000-residue chain (10,000 atoms) in a compact-globule start, 10 A
cutoff, 250 samples per offset sphere (--workload globule10000: the
10,000-residue chain, 100,000 atoms, 200 steps).  Inputs are built once and stay in
HBM; the timed region covers exactly --steps iterations between two device
synchronisations.  Prints one JSON line.

Roofline of the dominant kernel (the force kernel): algorithmic FP work per
launch = 40 flops per unordered pair within the cutoff + 9 flops per
(sample, solvation neighbour) coverage test + 9 flops per (exposed sample,
neighbour) pair for the three displaced tests, divided by the kernel's mean
launch time from HIP events recorded on its launch stream (on every 50th
timed iteration, so that the events barely perturb the timeline).
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
TIMING_EVERY = 50  # HIP events bracket the force kernel on every 50th timed iteration
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


def run_gpu(precision: str, steps: int, warmup: int, m: int, side_chains: bool = False):
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
    kcm.kcm_step([chain], warmup, stream, report=False)
    torch.cuda.synchronize()
    kcm.kcm_get_timing(reset=True)
    kcm.kcm_set_timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kcm.kcm_step([chain], steps, stream, report=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kcm.kcm_set_timing(0)
    tm = kcm.kcm_get_timing(reset=True)
    _, reps = kcm.kcm_step([chain], 0, stream, report=True, check=False)
    st = chain.state()
    terms = chain.atom_terms()
    units = algorithmic_units(st["xyz"], T, seq, p, terms["n_exposed"], chain.n_samples)
    secs = t1 - t0
    out = {
        "n_atoms": chain.n_atoms,
        "seconds": secs,
        "ms_per_step": 1e3 * secs / steps,
        "value": chain.n_atoms * steps / secs,
        "force_ms_mean": tm["force_ms"] / max(tm["force_launches"], 1),
        "iter_ms_mean": tm["iter_ms"] / max(tm["iterations"], 1),
        "units": units,
        "status": reps[0].status,
        "energies": [reps[0].e_elec, reps[0].e_vdw, reps[0].e_cav],
        "n_samples": chain.n_samples,
    }
    chain.free()
    return out


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


def run_batch(steps: int, warmup: int, n_chains: int = 256, tune: bool = True, direct: bool = False):
    """Ragged batch in mixed precision: all chains advanced together by replayed
    HIP graphs, with the cell edge and the iterations per graph picked by the
    autotuner on the same batch first."""
    import torch

    from paper_1712_05012_amd import autotune, kcm

    T, items = batch_workload(n_chains)
    stream = torch.cuda.current_stream()
    tuned = autotune.tune(T, items, kcm.KCM_MIXED, stream=stream) if tune and not direct else None
    p = kcm.kcm_default_params(precision=kcm.KCM_MIXED, cell_size=tuned.cell_size if tuned else 0.0)
    depth = 0 if direct else (tuned.graph_depth if tuned else 1)
    chains = [kcm.Chain(seq, T, p, theta0=th) for seq, th in items]
    atoms = sum(c.n_atoms for c in chains)
    kcm.kcm_set_graphs(depth)
    try:
        kcm.kcm_step(chains, warmup + depth, stream, report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kcm.kcm_step(chains, steps, stream, report=False)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
    finally:
        kcm.kcm_set_graphs(0 if direct else 1)
    _, reps = kcm.kcm_step(chains, 0, stream, report=True, check=False)
    bad = sum(r.status != 0 for r in reps)
    for c in chains:
        c.free()
    out = {"chains": len(items), "atoms": atoms, "steps": steps, "ms_per_step": 1e3 * secs / steps,
           "value": atoms * steps / secs, "failed_chains": int(bad), "cell_size": p.cell_size, "graph_depth": depth}
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


def run_serving(n_jobs: int, max_iter: int, budget_gib: float, skip: int):
    """Poisson arrivals at 50 jobs/s, lognormal lengths; continuous batching by HBM budget.

    Latency percentiles leave out the first ``skip`` jobs (warm-up); the queue
    growth rate says whether one GPU keeps up with the offered load."""
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
    eng = KcmEngine(T, kcm.kcm_default_params(precision=kcm.KCM_MIXED))
    svc = FoldService(eng, hbm_budget=int(budget_gib * (1 << 30)), max_slots=1024, check_every=20)
    def progress(job, n_done):
        if n_done % 250 == 0 or n_done == n_jobs:
            print(f"serving: {n_done} of {n_jobs} jobs done", file=sys.stderr, flush=True)

    st = svc.run(jobs, on_retire=progress)
    out = st.summary(skip=min(skip, max(0, n_jobs - 1)))
    offered = 50.0 * 10.0 * float(np.mean(lengths)) * max_iter
    out.update({"arrival_rate_per_s": 50.0, "max_iter": max_iter, "tol_dtheta": 1e-4,
                "hbm_budget_gib": budget_gib,
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


def traffic_for(precision: str, workload_name: str = "globule1000"):
    """HBM bytes per force launch from committed rocprofv3 counters, if still current."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if rec.get("workload", "globule1000") != workload_name:
            return None
        entry = rec.get(precision)
        if not entry or rec.get("kernel_sha256") != sha:
            return None
        return float(entry["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(seconds: float, m: int):
    """The FP64 oracle as it stands, on the host cores, over a bounded sample."""
    import oracle

    T, seq, th = workload(m)
    ch = oracle.OracleChain(seq, T)
    iters = 0
    t0 = time.perf_counter()
    while True:
        o = oracle.iterate(ch, th)
        th = o["theta"]
        iters += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    out = {"value": ch.n * iters / dt, "unit": "atom-steps/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{iters} FP64 KCM iterations of the {m}-residue globule ({ch.n} atoms), {dt:.1f} s"}
    single = cpu_single_core(max(2.0, seconds / 3), m)
    if single is not None:
        out["single_core_value"] = single
    return out


def cpu_single_core(seconds: float, m: int):
    """The same oracle sample on one host core (a child process with one
    OpenMP thread); atom-steps/s, or None if the child fails."""
    import subprocess

    code = (
        "import json, sys, time\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.abspath(__file__))!r})\n"
        "import bench, oracle\n"
        f"T, seq, th = bench.workload({int(m)})\n"
        "ch = oracle.OracleChain(seq, T)\n"
        "it = 0\n"
        "t0 = time.perf_counter()\n"
        f"while it == 0 or time.perf_counter() - t0 < {float(seconds)}:\n"
        "    th = oracle.iterate(ch, th)['theta']\n"
        "    it += 1\n"
        "print(json.dumps({'v': ch.n * it / (time.perf_counter() - t0), 't': oracle.threads()}))\n"
    )
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=seconds * 10 + 120)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        return d["v"] if d["t"] == 1 else None
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="globule1000",
                    help="single-chain workload: 1,000 residues (10,000 atoms) or 10,000 residues (100,000 atoms)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companion", action="store_true", help="skip the other precision's measurement")
    ap.add_argument("--batch-steps", type=int, default=100, help="iterations of the 256-chain batch (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="jobs of the serving run (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=100,
                    help="earliest jobs left out of the serving latency percentiles")
    ap.add_argument("--serve-max-iter", type=int, default=2000)
    ap.add_argument("--legs", default="main,companion,chi,batch,serving,landscape,polyala,cpu",
                    help="comma-separated legs to run (main, companion, chi, batch, serving, landscape, "
                         "polyala, cpu); "
                         "profiling runs use a subset, the benchmark line needs main")
    ap.add_argument("--graph-depth", type=int, default=8,
                    help="iterations per replayed HIP graph in the single-chain legs")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch each iteration's kernels directly instead of replaying a HIP graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs a chain on a single MI355X "
              "(how chains would shard over several GPUs is described in the design notes); "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    residues, _, default_steps = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = default_steps

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_1712_05012_amd import kcm

    kcm.kcm_set_graphs(0 if args.no_graphs else args.graph_depth)
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    legs = set(args.legs.split(","))
    if args.no_companion:
        legs.discard("companion")
    if args.batch_steps <= 0:
        legs.discard("batch")
    if args.serve_jobs <= 0:
        legs.discard("serving")
    if args.no_cpu_baseline:
        legs.discard("cpu")
    if "main" not in legs:
        # a profiling run of the other legs only
        line = {"legs": sorted(legs)}
        if "batch" in legs:
            line["batched"] = run_batch(args.batch_steps, 5, direct=args.no_graphs)
        if "serving" in legs:
            line["serving"] = run_serving(args.serve_jobs, args.serve_max_iter, 64.0, args.serve_warmup)
        if "landscape" in legs:
            line["landscape"] = run_landscape()
        if "polyala" in legs:
            line["polyala"] = run_polyala()
        print(json.dumps(line), flush=True)
        return

    main_run = run_gpu(args.precision, args.steps, args.warmup, residues)
    other = "fp64" if args.precision == "mixed" else "mixed"
    companion = run_gpu(other, args.steps, args.warmup, residues) if "companion" in legs else None

    u = main_run["units"]
    achieved = u["flops"] / (main_run["force_ms_mean"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    line = {
        "metric": "atom-steps/s per KCM iteration",
        "value": main_run["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"single chain, {residues} residues ({10 * residues:,} atoms), compact random globule, "
                        "10 A cutoff, 250 samples per offset sphere, 1 KCM iteration per step",
            "name": args.workload,
            "precision": args.precision,
            "n_atoms": main_run["n_atoms"],
            "n_samples": main_run["n_samples"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic_for(args.precision, args.workload),
        },
        "graph_depth": 0 if args.no_graphs else args.graph_depth,
        "kernel_ms": {"force": main_run["force_ms_mean"],
                      "iteration": main_run["iter_ms_mean"],
                      "chain_kernels": main_run["iter_ms_mean"] - main_run["force_ms_mean"]},
        "units_per_step": u,
        "status": main_run["status"],
    }
    if companion is not None:
        line[other] = {"value": companion["value"], "ms_per_step": companion["ms_per_step"],
                       "force_ms": companion["force_ms_mean"],
                       "frac": companion["units"]["flops"] / (companion["force_ms_mean"] * 1e-3) / 1e12
                       / PEAK_TFLOPS[other]}
    if "chi" in legs:
        # the same workload with one side-chain joint per residue
        ch = run_gpu(args.precision, args.steps, args.warmup, residues, side_chains=True)
        line["side_chains"] = {"value": ch["value"], "ms_per_step": ch["ms_per_step"],
                               "force_ms": ch["force_ms_mean"], "joints": 3 * residues,
                               "relative_to_main": ch["value"] / main_run["value"]}
    if "batch" in legs:
        b = run_batch(args.batch_steps, 5, direct=args.no_graphs)
        fp64 = run_per_chain_fp64(max(5, args.batch_steps // 10))
        b["plain_fp64_per_chain"] = fp64
        b["speedup_vs_plain_fp64_per_chain"] = b["value"] / fp64["value"]
        line["batched"] = b
    if "serving" in legs:
        line["serving"] = run_serving(args.serve_jobs, args.serve_max_iter, 64.0, args.serve_warmup)
    if "landscape" in legs:
        line["landscape"] = run_landscape()
    if "polyala" in legs:
        line["polyala"] = run_polyala()
    if "cpu" in legs:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, residues)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
