"""Host-side logic of bench.py: the algorithmic unit counts behind the
roofline (checked against brute force), the event sampling interval, the
roofline arithmetic, the traffic record lookup and the one-GPU guard.  No GPU."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1712_05012_amd import kcm  # noqa: E402


def _brute_units(xyz, T, seq, p, n_exposed, n_samples):
    """The same counts by their definitions, over every pair."""
    n = xyz.shape[0]
    d = np.sqrt(((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(-1))
    iu = np.triu_indices(n, 1)
    pairs = int((d[iu] <= p.cutoff).sum())
    # offset radius: half the LJ minimum distance of the slot's type plus the probe
    sig = np.asarray(T.sigma)[seq].reshape(-1)
    roff = 2.0 ** (1.0 / 6.0) * sig / 2.0 + p.r_probe
    nb = (d <= roff[:, None] + roff[None, :] + p.delta_r)
    np.fill_diagonal(nb, False)
    nbr = nb.sum(axis=1)
    tests1 = n_samples * int(nbr.sum())
    tests2 = int((n_exposed * nbr).sum())
    return pairs, nbr, tests1, tests2


def test_algorithmic_units_match_brute_force():
    T = synth.residue_types()
    m = 12
    seq = synth.sequence(m, 4242)
    rng = np.random.default_rng(7)
    xyz = rng.uniform(0.0, 14.0, size=(10 * m, 3))
    p = kcm.kcm_default_params(precision=kcm.KCM_MIXED)
    n_samples = 250
    n_exposed = rng.integers(0, n_samples + 1, size=10 * m)
    u = bench.algorithmic_units(xyz, T, seq, p, n_exposed, n_samples)
    pairs, nbr, tests1, tests2 = _brute_units(xyz, T, seq, p, n_exposed, n_samples)
    assert pairs > 0 and tests2 > 0
    assert u["pairs_within_cutoff"] == pairs
    assert u["coverage_tests"] == tests1
    assert u["exposed_sample_neighbour_pairs"] == tests2
    assert u["sasa_neighbours_mean"] == pytest.approx(nbr.mean(), rel=1e-15)
    assert u["exposed_fraction"] == pytest.approx(n_exposed.mean() / n_samples, rel=1e-15)
    # 40 flops per unordered pair, 9 per coverage test and per displaced triple
    assert u["flops"] == 40.0 * pairs + 9.0 * tests1 + 9.0 * tests2


def test_timing_interval_gives_enough_samples():
    for steps in (1, 4, 5, 20, 100, 249, 250, 251, 500, 5000):
        every = bench.timing_every(steps)
        assert 1 <= every <= bench.MAX_EVERY
        if steps >= bench.MIN_SAMPLES:
            # iterations 0, every, 2 every, ... inside the timed region
            assert (steps + every - 1) // every >= bench.MIN_SAMPLES


def test_roofline_arithmetic():
    units = {"flops": 3.0e11}
    r = bench.roofline(units, 2.5, "mixed", traffic=1.0e8)
    assert r["achieved"] == pytest.approx(3.0e11 / 2.5e-3 / 1e12)
    assert r["peak"] == 157.3 and r["unit"] == "TFLOP/s" and r["bound"] == "alu"
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["traffic"] == 1.0e8
    assert bench.roofline(units, 2.5, "fp64")["peak"] == 78.6


def test_sum_units_weights_means_by_atoms():
    a = {"pairs_within_cutoff": 10, "coverage_tests": 100, "exposed_sample_neighbour_pairs": 7, "flops": 1.0,
         "sasa_neighbours_mean": 40.0, "exposed_fraction": 0.1}
    b = {"pairs_within_cutoff": 5, "coverage_tests": 50, "exposed_sample_neighbour_pairs": 3, "flops": 2.0,
         "sasa_neighbours_mean": 70.0, "exposed_fraction": 0.4}
    t = bench.sum_units([(a, 100, 250), (b, 300, 250)])
    assert (t["pairs_within_cutoff"], t["coverage_tests"], t["exposed_sample_neighbour_pairs"], t["flops"]) == \
        (15, 150, 10, 3.0)
    assert t["sasa_neighbours_mean"] == pytest.approx((40.0 * 100 + 70.0 * 300) / 400)
    assert t["exposed_fraction"] == pytest.approx((0.1 * 100 + 0.4 * 300) / 400)


def test_traffic_record_only_for_the_kernel_it_was_taken_on(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    rec = tmp_path / "traffic.json"
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    rec.write_text(json.dumps({"kernel_sha256": sha,
                               "workloads": {"batch256": {"mixed": {"bytes_per_launch": 1.25e8}}}}))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.traffic_for("mixed", "batch256") == 1.25e8
    assert bench.traffic_for("fp64", "batch256") is None
    assert bench.traffic_for("mixed", "globule1000") is None
    src.write_text("// kernel source, changed\n")
    assert bench.traffic_for("mixed", "batch256") is None


def test_batch_workload_shape():
    T, items = bench.batch_workload(256)
    lens = [len(seq) for seq, _ in items]
    assert len(items) == 256 and min(lens) >= 50 and max(lens) <= 600
    assert 10 * sum(lens) == 818020
    assert all(th.shape == (2 * len(seq),) for seq, th in items)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
