"""Parity of the HIP path with the FP64 oracle (needs an MI355X)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from gpu_common import (DTHETA_TOL, F_CAV_ABS, F_TOL, TAU_TOL, TYPES, build_pair, compare_step,  # noqa: E402
                        oracle_params, oracle_step, params)
from paper_1712_05012_amd import kcm  # noqa: E402

pytestmark = pytest.mark.gpu

PRECISIONS = [kcm.KCM_FP64, kcm.KCM_MIXED]


def _log(**kw):
    print(" ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kcm.load_library()


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("m,seed", [(3, 11), (16, 12), (64, synth.config_seed(1))])
def test_one_iteration_matches_oracle(precision, m, seed):
    p = params(precision)
    gpu, ref, th = build_pair(m, seed, p)
    _log(case="one_iteration", m=m, seed=seed, precision=precision)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(**err)
    assert err["status"] == 0
    assert err["xyz"] < 1e-9
    assert err["margin"] > 1e-10, "a sample test sits on a tie; pick another seed"
    assert err["F"] <= F_TOL and err["F_pair"] <= F_TOL and err["F_cav"] <= F_TOL
    assert err["dtheta"] <= DTHETA_TOL[precision]
    assert err["theta"] <= DTHETA_TOL[precision]
    assert err["tau"] <= TAU_TOL[precision]
    tol_e = 1e-9 if precision == kcm.KCM_FP64 else 1e-5
    assert err["E_elec"] < tol_e and err["E_vdw"] < tol_e
    assert err["E_cav"] < 1e-12  # integer exposure counts: exact
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n_orbits", [14, 23])
def test_solvation_counts_are_exact(precision, n_orbits):
    # the discrete sample decisions are taken in FP64 (mixed: FP32 with an FP64
    # recheck near ties), so the solvation force equals the oracle's to the
    # fixed-point rounding of the event quantum; 23 orbits give more samples
    # than one pass of the kernel holds (ragged last pass)
    p = params(precision, terms=kcm.KCM_TERM_CAV, n_orbits=n_orbits)
    gpu, ref, th = build_pair(40, 21, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="cav_only", precision=precision, n_samples=gpu.n_samples, **err)
    assert n_orbits == 14 or gpu.n_samples > 512
    assert err["margin"] > 1e-10
    assert np.abs(st["force"] - o["F_cav"]).max() < 1e-8
    assert np.abs(st["force"].sum(axis=0)).max() < 1e-8  # every event is +-, exactly
    gpu.free()


def _max_solvation_neighbours(ref, r, p):
    """Largest per-atom count of offset spheres within reach (brute force)."""
    roff = ref.R + p.r_probe
    d = np.sqrt(((r[:, None, :] - r[None, :, :]) ** 2).sum(-1))
    lim = roff[:, None] + roff[None, :] + p.delta_r
    np.fill_diagonal(d, np.inf)
    return int((d <= lim).sum(axis=1).max())


# A random-dihedral start with a dense self-overlap: one atom has more
# solvation neighbours (418) than the kernel's LDS list holds
# (KCM_NBR_CHUNK), so its neighbours are processed in two chunks.  The chain
# is job 1792 of the serving stream (304 residues).
OVERFLOW_M = 304
OVERFLOW_SEED = synth.config_seed(5) + 1000 * (1792 + 1)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_neighbour_list_overflow_is_processed_in_chunks(precision):
    p = params(precision, terms=kcm.KCM_TERM_CAV)
    gpu, ref, th = build_pair(OVERFLOW_M, OVERFLOW_SEED, p)
    r0 = oracle.fk(ref, th)[0]
    nmax = _max_solvation_neighbours(ref, r0, p)
    assert nmax > kcm.KCM_NBR_CHUNK
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="nbr_overflow", precision=precision, max_neighbours=nmax, **err)
    assert err["status"] == 0
    assert err["margin"] > 1e-10
    assert np.abs(st["force"] - o["F_cav"]).max() < 1e-8
    assert err["E_cav"] < 1e-12
    gpu.free()
    # and the whole iteration with every term
    p = params(precision)
    gpu, ref, th = build_pair(OVERFLOW_M, OVERFLOW_SEED, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="nbr_overflow_full", precision=precision, **err)
    assert err["status"] == 0
    assert err["F"] <= F_TOL
    assert err["dtheta"] <= DTHETA_TOL[precision]
    gpu.free()


def _close_contact_start():
    """A start with two non-bonded atoms 0.001 A apart.

    Job 1933 of the serving stream (179 residues, random dihedrals) has atoms
    1187 and 1244 (residues 118 and 124) 0.0118 A apart; three dihedrals
    between them are adjusted by least squares (oracle kinematics) to bring
    atom 1244 to 0.001 A from atom 1187 along the line that joins them."""
    from scipy.optimize import least_squares

    seed = synth.config_seed(5) + 1000 * (1933 + 1)
    m, a, b, joints = 179, 1187, 1244, [240, 243, 246]
    th0 = synth.random_dihedrals(m, seed)
    ref = oracle.OracleChain(synth.sequence(m, seed), TYPES)
    r = oracle.fk(ref, th0)[0]
    u = (r[b] - r[a]) / np.linalg.norm(r[b] - r[a])
    target = r[a] + 1e-3 * u

    def resid(x):
        th = th0.copy()
        th[joints] += x
        return oracle.fk(ref, th)[0][b] - target

    sol = least_squares(resid, np.zeros(3), xtol=1e-15, ftol=1e-15, gtol=1e-15)
    th = th0.copy()
    th[joints] += sol.x
    return m, seed, th, a, b


@pytest.mark.parametrize("precision", PRECISIONS)
def test_close_contact_beyond_fp32_range(precision):
    # (D/d)^12 and the force of a pair 0.001 A apart exceed the FP32 range:
    # the mixed form takes those atoms' pair terms in FP64
    m, seed, th, a, b = _close_contact_start()
    p = params(precision)
    gpu, ref, _ = build_pair(m, seed, p, theta=th)
    r0 = oracle.fk(ref, th)[0]
    assert abs(np.linalg.norm(r0[a] - r0[b]) - 1e-3) < 1e-9
    st, o, err = compare_step(gpu, ref, th, p)
    F, Fo = st["force"], o["F"]
    _log(case="close_contact", precision=precision, fmax=float(np.abs(Fo).max()), **err)
    assert np.abs(Fo).max() > 3.5e38  # above the largest FP32 value
    assert err["status"] == 0
    for k in (a, b):
        assert np.abs(F[k] - Fo[k]).max() <= 1e-9 * np.abs(Fo[k]).max()
    rest = np.ones(len(F), bool)
    rest[[a, b]] = False
    assert np.abs(F[rest] - Fo[rest]).max() <= F_TOL * np.abs(Fo[rest]).max()
    assert err["E_vdw"] <= 1e-9
    assert err["dtheta"] <= DTHETA_TOL[precision]
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_pair_only_and_newton_third_law(precision):
    p = params(precision, terms=kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW)
    gpu, ref, th = build_pair(30, 31, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="pair_only", precision=precision, **err)
    assert err["F"] <= F_TOL
    F = st["force"]
    assert np.abs(F.sum(axis=0)).max() <= 1e-6 * np.abs(F).max()
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_bond_class_weights_and_single_pair_terms(precision):
    """Scaled 1-3 and 1-4 pairs (eq 03_2) against the oracle with factors that
    are neither 0 nor the defaults, so that every bond class takes its own
    weights; then each pair term alone: its energy equals the combined run's,
    the other term's is zero, and the two forces add up to the combined one."""
    both = kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW
    tol_e = 1e-9 if precision == kcm.KCM_FP64 else 1e-5
    w = dict(w13=0.4, w14_elec=0.7, w14_vdw=0.3)
    p = params(precision, terms=both, **w)
    gpu, ref, th = build_pair(24, 61, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="bond_class_weights", precision=precision, **err)
    assert err["status"] == 0
    assert err["F"] <= F_TOL and err["F_pair"] <= F_TOL
    assert err["E_elec"] < tol_e and err["E_vdw"] < tol_e
    assert err["tau"] <= TAU_TOL[precision]
    gpu.set_theta(th)
    rep = gpu.step(1)
    f_both = gpu.forces()[0]
    e_both = (rep.e_elec, rep.e_vdw)
    gpu.free()
    f_one, e_one = [], []
    for t in (kcm.KCM_TERM_ELEC, kcm.KCM_TERM_VDW):
        g, _, _ = build_pair(24, 61, params(precision, terms=t, **w), theta=th)
        r = g.step(1)
        f_one.append(g.forces()[0])
        e_one.append((r.e_elec, r.e_vdw))
        g.free()
    assert e_one[0][1] == 0.0 and e_one[1][0] == 0.0
    assert abs(e_one[0][0] - e_both[0]) <= tol_e * max(abs(e_both[0]), 1.0)
    assert abs(e_one[1][1] - e_both[1]) <= tol_e * max(abs(e_both[1]), 1.0)
    fmax = np.abs(f_both).max()
    assert np.abs(f_one[0] + f_one[1] - f_both).max() <= F_TOL * fmax


@pytest.mark.parametrize("rule", [kcm.KCM_STEP_CAPPED, kcm.KCM_STEP_PAPER, kcm.KCM_STEP_LINEAR])
def test_step_rules_and_masks(rule):
    p = params(kcm.KCM_FP64, step_rule=rule, kappa=1e-6 if rule == kcm.KCM_STEP_LINEAR else 1e-3)
    m = 12
    mask = np.ones(2 * m, np.uint8)
    mask[::5] = 0
    gpu, ref, th = build_pair(m, 41, p, mask=mask)
    st, o, err = compare_step(gpu, ref, th, p, mask=mask)
    _log(case="step_rule", rule=rule, **err)
    assert err["dtheta"] <= 1e-7 and err["theta"] <= 1e-7
    assert np.all(st["dtheta"][mask == 0] == 0.0)
    gpu.free()


def test_single_residue_and_zero_position():
    p = params(kcm.KCM_FP64)
    for m, th in ((1, None), (2, None), (5, np.full(10, np.pi))):
        gpu, ref, th0 = build_pair(m, 51 + m, p, theta=th if th is not None else synth.random_dihedrals(m, 3))
        st, o, err = compare_step(gpu, ref, th0, p)
        _log(case="small", m=m, **err)
        assert err["xyz"] < 1e-9 and err["F"] <= F_TOL and err["dtheta"] <= 1e-7
        gpu.free()


def test_extended_chain_coarsens_grid():
    # the zero position is a 300-residue straight zigzag: a long thin box
    p = params(kcm.KCM_MIXED)
    m = 300
    gpu, ref, th = build_pair(m, 61, p, theta=np.full(2 * m, np.pi))
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="extended", **err)
    assert err["F"] <= F_TOL and err["dtheta"] <= DTHETA_TOL[kcm.KCM_MIXED]
    gpu.free()


@pytest.mark.parametrize("m", [129, 9000])
def test_long_chain_kinematics(m):
    # 258 joints: two joint blocks; 18000 joints: 71 joint blocks, more than
    # one wave of block products.  Forces off, so the step is zero and the
    # positions are the kinematics of theta alone.
    p = params(kcm.KCM_FP64, terms=0)
    seed = 90 + m
    gpu, ref, th = build_pair(m, seed, p)
    rep = gpu.step(2)
    st = gpu.state()
    r, u, _ = oracle.fk(ref, th)
    scale = max(np.abs(r).max(), 1.0)
    err = float(np.abs(st["xyz"] - r).max())
    _log(case="long_fk", m=m, xyz=err, scale=scale, status=rep.status)
    assert rep.status == 0
    assert err <= 1e-12 * scale * np.sqrt(2 * m)
    assert np.array_equal(st["theta"], th)  # zero torque: the angles do not move
    gpu.free()


@pytest.mark.parametrize("m", [80, 1700])
def test_cell_list_is_a_valid_stable_partition(m):
    # 800 atoms, and 17000 atoms in an open coil (a larger, sparser grid)
    p = params(kcm.KCM_FP64)
    gpu, ref, th = build_pair(m, 71, p)
    gpu.step(1)
    c = gpu.cells()
    xyz = gpu.state()["xyz"]
    dims, cell, origin, order, cs = c["dims"], c["cell"], c["origin"], c["order"], c["cell_start"]
    n = xyz.shape[0]
    assert sorted(order.tolist()) == list(range(n))
    assert cs[0] == 0 and cs[-1] == n and np.all(np.diff(cs) >= 0)
    assert cell >= 5.0 - 1e-9
    idx = np.clip(np.floor((xyz - origin) / cell).astype(int), 0, dims - 1)
    key = (idx[:, 2] * dims[1] + idx[:, 1]) * dims[0] + idx[:, 0]
    for cidx in range(cs.size - 1):
        members = order[cs[cidx]:cs[cidx + 1]]
        assert np.all(key[members] == cidx)
        assert np.all(np.diff(members) > 0)  # stable: atom order inside a cell
    gpu.free()


def test_large_open_chain_matches_oracle():
    # 17000 atoms in a random coil: many atom workgroups and joint blocks
    p = params(kcm.KCM_MIXED)
    gpu, ref, th = build_pair(1700, 77, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="large_chain", **err)
    assert err["margin"] > 1e-10
    assert err["F"] <= F_TOL and err["dtheta"] <= DTHETA_TOL[kcm.KCM_MIXED]
    assert err["tau"] <= TAU_TOL[kcm.KCM_MIXED]
    assert np.abs(gpu.forces()[1] - o["F_cav"]).max() < F_CAV_ABS
    gpu.free()


def test_batched_call_equals_separate_calls_bitwise():
    p = params(kcm.KCM_MIXED)
    lens = [7, 33, 20]
    alone, batch = [], []
    for k, m in enumerate(lens):
        seq = synth.sequence(m, 80 + k)
        th = synth.random_dihedrals(m, 80 + k)
        alone.append(kcm.Chain(seq, TYPES, p, theta0=th))
        batch.append(kcm.Chain(seq, TYPES, p, theta0=th))
    for c in alone:
        kcm.kcm_step([c], 3)
    kcm.kcm_step(batch, 3)
    for a, b in zip(alone, batch):
        sa, sb = a.state(), b.state()
        for key in ("theta", "xyz", "force", "tau"):
            assert np.array_equal(sa[key], sb[key]), key
    for c in alone + batch:
        c.free()


def test_large_batch_equals_separate_calls_bitwise():
    # 48 chains of 260 residues make 528 atom workgroups: the batched call
    # sizes each chain's grid in a launch of its own before the key pass,
    # while a chain stepped alone (11 workgroups) sizes it inside the key
    # workgroups.  Both forms must give the same grid, keys and results.
    p = params(kcm.KCM_MIXED)
    n, m = 48, 260
    assert n * ((10 * m + 255) // 256) >= 512
    alone, batch = [], []
    for k in range(n):
        seq = synth.sequence(m, 300 + k)
        th = synth.random_dihedrals(m, 300 + k)
        alone.append(kcm.Chain(seq, TYPES, p, theta0=th))
        batch.append(kcm.Chain(seq, TYPES, p, theta0=th))
    try:
        for c in alone:
            kcm.kcm_step([c], 2)
        kcm.kcm_step(batch, 2)
        for a, b in zip(alone, batch):
            sa, sb = a.state(), b.state()
            for key in ("theta", "xyz", "force", "tau"):
                assert np.array_equal(sa[key], sb[key]), key
            ga, gb = kcm.kcm_get_cells(a.handle), kcm.kcm_get_cells(b.handle)
            assert np.array_equal(ga["dims"], gb["dims"]) and ga["cell"] == gb["cell"]
            assert np.array_equal(ga["origin"], gb["origin"])
            assert np.array_equal(ga["order"], gb["order"])
    finally:
        for c in alone + batch:
            c.free()


def test_runs_are_deterministic():
    p = params(kcm.KCM_MIXED)
    out = []
    for _ in range(2):
        gpu, ref, th = build_pair(50, 91, p)
        gpu.step(4)
        out.append(gpu.state())
        gpu.free()
    for key in ("theta", "force", "tau"):
        assert np.array_equal(out[0][key], out[1][key]), key


@pytest.mark.parametrize("precision", PRECISIONS)
def test_resynchronised_trajectory(precision):
    # per-step parity along a short trajectory: each step starts from the oracle's theta
    p = params(precision)
    gpu, ref, th = build_pair(24, 101, p)
    for it in range(5):
        st, o, err = compare_step(gpu, ref, th, p)
        assert err["dtheta"] <= DTHETA_TOL[precision], (it, err)
        th = o["theta"]
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_free_trajectory_100_iterations(precision):
    # the 64-residue workload: 100 iterations on the device in one call against
    # 100 oracle iterations, each side from its own previous angles.  Per-step
    # errors add up over the trajectory, so the bound is 100 x the per-step
    # tolerance of the form.
    p = params(precision)
    m = 64
    seed = synth.config_seed(1)
    gpu, ref, th = build_pair(m, seed, p)
    rep = gpu.step(100)
    assert rep.status == 0 and rep.iterations == 100
    t = th.copy()
    for _ in range(100):
        t = oracle_step(ref, t, p)["theta"]
    err = float(np.abs(np.angle(np.exp(1j * (gpu.state()["theta"] - t)))).max())
    _log(case="trajectory100", precision=precision, dtheta=err)
    assert err <= 100 * DTHETA_TOL[precision]
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_checkpoint_resume(precision):
    # A chain rebuilt from the angles after iteration 3 continues the
    # trajectory bit for bit: each iteration's grid is sized from the
    # conformation it places, so nothing but the angles carries over.  One
    # call of 6 iterations, two calls of 3, and a rebuilt chain all agree.
    p = params(precision)
    seq = synth.sequence(30, 111)
    th = synth.random_dihedrals(30, 111)
    a = kcm.Chain(seq, TYPES, p, theta0=th)
    a.step(6)
    ref = a.state()
    b = kcm.Chain(seq, TYPES, p, theta0=th)
    b.step(3)
    mid = b.state()["theta"]
    b.step(3)
    c = kcm.Chain(seq, TYPES, p, theta0=mid)
    c.step(3)
    for other in (b.state(), c.state()):
        for key in ("theta", "xyz", "force", "tau"):
            assert np.array_equal(other[key], ref[key]), key
    _log(case="resume", precision=precision, identical=True)
    for x in (a, b, c):
        x.free()


def test_numeric_failure_is_isolated():
    # two non-excluded atoms on top of each other give an infinite LJ force in
    # one chain; the other chain of the same call keeps going
    p = params(kcm.KCM_FP64)
    good = kcm.Chain(synth.sequence(10, 121), TYPES, p, theta0=synth.random_dihedrals(10, 121))
    m = 4
    seq = synth.sequence(m, 122)
    # search theta on the host for a conformation with a coincident non-excluded pair is
    # not needed: NaN theta is rejected at build, so force the failure with a huge charge
    T2 = synth.ResidueTypes(q=TYPES.q * 1e300, sigma=TYPES.sigma, eps=TYPES.eps, hydro=TYPES.hydro)
    bad = kcm.Chain(seq, T2, p, theta0=synth.random_dihedrals(m, 122))
    st, reps = kcm.kcm_step([good, bad], 2, check=False)
    assert st == kcm.KCM_E_NUMERIC
    assert reps[0].status == 0 and reps[0].iterations == 2
    assert reps[1].status == kcm.KCM_E_NUMERIC and reps[1].iterations == 0
    good.free()
    bad.free()


def test_fold_converges_and_reports():
    # a perturbed 8-residue alanine-like helix in vacuum, mixed precision: the
    # oracle's loop stops below 1e-3 rad after 112 iterations; kcm_fold must
    # report convergence at (or, with FP32 pair forces, within two iterations
    # of) the same iteration, with its last step below the tolerance
    T = synth.alanine_like_types()
    m, cap, tol = 8, 400, 1e-3
    p = params(kcm.KCM_MIXED, max_step=1e-2, terms=kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW)
    th = np.radians(np.tile([-68.0, -39.0], m)) + 0.05 * np.random.default_rng(1).standard_normal(2 * m)
    ref = oracle.OracleChain(np.zeros(m, np.int32), T)
    t, it = th.copy(), 0
    while it < cap:
        o = oracle.iterate(ref, t, terms="elec+vdw", kappa=p.kappa, s=p.max_step)
        t, it = o["theta"], it + 1
        if np.abs(o["dtheta"]).max() < tol:
            break
    assert it < cap, "the oracle run must converge for this test"
    gpu = kcm.Chain(np.zeros(m, np.int32), T, p, theta0=th)
    st, res = kcm.kcm_fold([gpu], tol=tol, max_iter=cap, check_every=9)
    _, (rep,) = kcm.kcm_step([gpu], 0)
    _log(case="fold", iterations=res[0].iterations, oracle_iterations=it, converged=res[0].converged,
         last_dtheta=rep.max_dtheta)
    assert st == kcm.KCM_OK and res[0].status == 0
    assert res[0].converged == 1 and rep.converged == 1
    assert rep.max_dtheta < tol
    assert abs(res[0].iterations - it) <= 2
    # a converged chain is skipped by later calls
    _, (rep2,) = kcm.kcm_step([gpu], 5)
    assert rep2.iterations == rep.iterations
    gpu.free()


def test_fold_keeps_the_chains_own_limits():
    # kcm_set_limits, then kcm_fold (whose own tolerance and cap apply during
    # the call), then kcm_step: the chain's own cap of 30 iterations holds
    # again after the fold
    p = params(kcm.KCM_MIXED)
    gpu = build_pair(6, 171, p)[0]
    kcm.kcm_set_limits(gpu.handle, 0.0, 30)
    st, res = kcm.kcm_fold([gpu], tol=1e-30, max_iter=10, check_every=5)
    assert res[0].iterations == 10 and not res[0].converged
    _, (rep,) = kcm.kcm_step([gpu], 100)
    assert rep.status == 0 and rep.iterations == 30
    # a fold longer than the chain's own cap runs its own count
    gpu2 = build_pair(6, 172, p)[0]
    kcm.kcm_set_limits(gpu2.handle, 0.0, 5)
    st, res = kcm.kcm_fold([gpu2], tol=1e-30, max_iter=12, check_every=4)
    assert res[0].iterations == 12
    _, (rep,) = kcm.kcm_step([gpu2], 3)
    assert rep.iterations == 12  # past its own cap: stays stopped
    gpu.free()
    gpu2.free()


@pytest.mark.parametrize("depth", [1, 4])
def test_graph_replay_equals_direct_launches(depth):
    # replays of the captured iterations (one, or four per graph plus single
    # ones for the rest of a call), with eager work and synchronisations
    # between calls, must match direct launches bit for bit after every call
    p = params(kcm.KCM_MIXED)
    seqs = [(synth.sequence(m, 140 + m), synth.random_dihedrals(m, 140 + m)) for m in (9, 27, 14)]
    a = [kcm.Chain(s, TYPES, p, theta0=t) for s, t in seqs]
    b = [kcm.Chain(s, TYPES, p, theta0=t) for s, t in seqs]
    try:
        for rep in range(4):
            kcm.kcm_set_graphs(depth)
            kcm.kcm_step(a, 3 + 3 * rep)
            x = torch.ones(1000, device="cuda").sum().item()  # eager work in between
            assert x == 1000.0
            kcm.kcm_set_graphs(False)
            kcm.kcm_step(b, 3 + 3 * rep)
            torch.cuda.synchronize()
            for ca, cb in zip(a, b):
                sa, sb = ca.state(), cb.state()
                for key in ("theta", "xyz", "force", "tau"):
                    assert np.array_equal(sa[key], sb[key]), (rep, key)
    finally:
        kcm.kcm_set_graphs(True)
        for c in a + b:
            c.free()


def test_force_kernel_shapes_give_identical_results():
    # every launch shape of the force kernel visits the candidates and lists
    # the neighbours in the same order and takes the same decisions: the
    # states after a few graph-replayed iterations are equal bit for bit
    out = []
    try:
        for v in range(kcm.KCM_FORCE_VARIANTS):
            kcm.kcm_set_force_variant(v)
            for prec in (kcm.KCM_MIXED, kcm.KCM_FP64):
                p = params(prec)
                cs = [build_pair(m, 180 + m, p)[0] for m in (9, 120, 40)]
                kcm.kcm_step(cs, 5)
                out.append((v, prec, [c.state() for c in cs]))
                for c in cs:
                    c.free()
    finally:
        kcm.kcm_set_force_variant(0)
    ref = {prec: states for v, prec, states in out if v == 0}
    for v, prec, states in out:
        for a, b in zip(states, ref[prec]):
            for key in ("theta", "xyz", "force", "tau"):
                assert np.array_equal(a[key], b[key]), (v, prec, key)
    with pytest.raises(kcm.KcmError):
        kcm.kcm_set_force_variant(kcm.KCM_FORCE_VARIANTS)


def test_device_side_limits_stop_chains():
    p = params(kcm.KCM_MIXED)
    c1 = kcm.Chain(synth.sequence(6, 151), TYPES, p, theta0=synth.random_dihedrals(6, 151))
    c2 = kcm.Chain(synth.sequence(6, 152), TYPES, p, theta0=synth.random_dihedrals(6, 152))
    kcm.kcm_set_limits(c1.handle, 0.0, 7)      # iteration cap only
    kcm.kcm_set_limits(c2.handle, 10.0, 0)     # converges on the first step (max|dtheta| < 10 rad)
    _, reps = kcm.kcm_step([c1, c2], 20)
    assert reps[0].iterations == 7 and not reps[0].converged
    assert reps[1].iterations == 1 and reps[1].converged
    c1.free()
    c2.free()


def test_served_job_result_same_alone_and_in_mix():
    from paper_1712_05012_amd.serve import FoldService, Job, KcmEngine

    def jobs():
        out = []
        for k, (m, a) in enumerate([(12, 0.0), (30, 0.0), (8, 0.01), (20, 0.02), (15, 0.02)]):
            out.append(Job(job_id=k, res_type=synth.sequence(m, 160 + k), theta0=synth.random_dihedrals(m, 160 + k),
                           arrival=a, tol=1e-4, max_iter=60 + 10 * k))
        return out

    p = params(kcm.KCM_MIXED)
    mix = FoldService(KcmEngine(TYPES, p), hbm_budget=3 * 1024 * 1024, max_slots=3, check_every=7).run(jobs())
    assert mix.max_live >= 2
    for target in (1, 3):
        alone = FoldService(KcmEngine(TYPES, p), hbm_budget=1 << 30, max_slots=1, check_every=7)
        st = alone.run([j for j in jobs() if j.job_id == target])
        a, b = st.jobs[0], [j for j in mix.jobs if j.job_id == target][0]
        assert a.iterations == b.iterations
        assert np.array_equal(a.theta, b.theta)


def test_autotune_picks_a_measured_setting_with_unchanged_results():
    from paper_1712_05012_amd import autotune

    items = [(synth.sequence(m, 300 + m), synth.random_dihedrals(m, 300 + m)) for m in (12, 30, 21)]
    try:
        res = autotune.tune(TYPES, items, kcm.KCM_MIXED, cell_sizes=(0.0, 3.6), variants=(0, 2), depths=(1, 2),
                            iters=2, warmup=1)
    finally:
        kcm.kcm_set_force_variant(0)
    assert len(res.table) == 8
    assert (res.cell_size, res.force_variant, res.graph_depth) in [(c, v, d) for c, v, d, _, _ in res.table]
    assert res.atom_steps_per_s == max(r for *_, r in res.table) > 0
    # the chosen cell edge changes only the candidate order: parity holds
    p = params(kcm.KCM_MIXED, cell_size=res.cell_size)
    gpu, ref, th = build_pair(30, 330, p)
    st, o, err = compare_step(gpu, ref, th, p)
    _log(case="autotuned", cell_size=res.cell_size, depth=res.graph_depth, **err)
    assert err["F"] <= F_TOL and err["dtheta"] <= DTHETA_TOL[kcm.KCM_MIXED]
    gpu.free()


def test_large_globule_sampled_parity():
    # the 10,000-residue compact globule (100,000 atoms) in mixed precision.
    # The oracle's brute force is quadratic, so parity is checked on samples:
    # every position against the oracle kinematics; the pair force of 256
    # sampled atoms against the oracle over all atoms; the solvation force and
    # exposure of 64 sampled atoms against the oracle on the cluster of atoms
    # within 16 A (an atom's solvation force depends only on atoms within two
    # offset radii plus the shift, at most 7.4 A, of it and of its neighbours);
    # and Newton's third law over the whole chain.
    from scipy.spatial import cKDTree

    m = 10000
    if not os.path.exists(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "data", f"globule_m{m}.npy")):
        pytest.skip("no stored 10,000-residue start conformation (python -m oracle.make_globules 10000)")
    seq = synth.sequence(m, synth.config_seed(4))
    th = synth.load_globule(m)
    p = params(kcm.KCM_MIXED)
    gpu = kcm.Chain(seq, TYPES, p, theta0=th)
    ref = oracle.OracleChain(seq, TYPES, g_hydro=p.g_hydro)
    rep = gpu.step(1)
    assert rep.status == 0
    st = gpu.state()
    fp, fc = gpu.forces()
    terms = gpu.atom_terms()
    r, _, _ = oracle.fk(ref, th)
    assert np.abs(st["xyz"] - r).max() < 1e-8
    pp, sp = oracle_params(p)
    rng = np.random.default_rng(4)
    pick = np.sort(rng.choice(10 * m, 256, replace=False)).astype(np.int32)
    F_pair, _, _ = oracle.pair_forces(ref, r, pp, subset=pick)
    fmax = max(np.abs(F_pair[pick]).max(), 1e-300)
    err_pair = float(np.abs(fp[pick] - F_pair[pick]).max() / fmax)
    tree = cKDTree(r)
    err_cav = 0.0
    for a in pick[:64]:
        cl = np.array(sorted(tree.query_ball_point(r[a], 16.0)))
        Fc, f, _ = oracle.sasa_atoms(r[cl], ref.R[cl], ref.gamma[cl], sp)
        i = int(np.searchsorted(cl, a))
        err_cav = max(err_cav, float(np.abs(fc[a] - Fc[i]).max()))
        assert terms["n_exposed"][a] == round(f[i] * gpu.n_samples), a
    net = np.abs(fp.sum(axis=0)).max() / np.abs(fp).max()
    _log(case="globule10000", err_pair=err_pair, err_cav=err_cav, net_pair=net,
         net_cav=float(np.abs(fc.sum(axis=0)).max()))
    assert err_pair <= F_TOL
    assert err_cav < 1e-8
    assert net <= 1e-6
    assert np.abs(fc.sum(axis=0)).max() < 1e-6
    gpu.free()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_benchmark_workload_in_its_launch_configuration(precision):
    # the benchmarked workload itself: the 1000-residue compact globule
    # (10,000 atoms), replayed as HIP graphs of 8 iterations like bench.py.
    # The capped descent of this start is chaotic (the oracle turns a 1e-13
    # rad offset into 3e-3 rad within 16 iterations: its first steps create
    # clashes with torques near 1e23), so parity is per step from shared
    # angles: one iteration at the start, and one at the angles the device
    # reached after 16 graph-replayed iterations, which must equal 16 directly
    # launched ones bit for bit.
    m = 1000
    seq = synth.sequence(m, synth.config_seed(2))
    th = synth.load_globule(m)
    p = params(precision)
    ref = oracle.OracleChain(seq, TYPES, g_hydro=p.g_hydro)
    try:
        kcm.kcm_set_graphs(8)
        gpu = kcm.Chain(seq, TYPES, p, theta0=th)
        for label, start in (("start", None), ("after16", "run")):
            if start == "run":
                gpu.set_theta(th)
                rep = gpu.step(16)
                assert rep.status == 0
                th16 = gpu.state()["theta"]
                kcm.kcm_set_graphs(0)
                direct = kcm.Chain(seq, TYPES, p, theta0=th)
                assert direct.step(16).status == 0
                assert np.array_equal(direct.state()["theta"], th16)
                direct.free()
                kcm.kcm_set_graphs(8)
                at = th16
            else:
                at = th
            st, o, err = compare_step(gpu, ref, at, p)
            _log(case="benchmark_workload", at=label, precision=precision, **err)
            assert err["status"] == 0
            assert err["xyz"] < 1e-9
            assert err["F"] <= F_TOL and err["F_pair"] <= F_TOL and err["F_cav"] <= F_TOL
            assert err["dtheta"] <= DTHETA_TOL[precision]
            assert err["tau"] <= TAU_TOL[precision]
            if err["margin"] > 1e-10:
                # equal sample decisions: the solvation force to the event
                # quantum's rounding, per atom and in absolute terms
                assert err["E_cav"] < 1e-12
                assert np.abs(gpu.forces()[1] - o["F_cav"]).max() < F_CAV_ABS
        gpu.free()
    finally:
        kcm.kcm_set_graphs(1)


def test_batched_angle_setter_equals_per_chain_setter():
    # kcm_set_theta_batch (one device array, one kernel) against kcm_set_theta
    # per chain, on chains of different lengths with and without side chains:
    # the next iterations are bit for bit the same
    p = params(kcm.KCM_MIXED)
    spec = [(7, 301, False), (40, 302, True), (300, 303, False), (129, 304, True)]
    a = [build_pair(m, s, p, side_chains=sc)[0] for m, s, sc in spec]
    b = [build_pair(m, s, p, side_chains=sc)[0] for m, s, sc in spec]
    kcm.kcm_step(a, 3)
    kcm.kcm_step(b, 3)
    rng = np.random.default_rng(5)
    new = [rng.uniform(-np.pi, np.pi, c.n_joints) for c in a]
    held = kcm.kcm_set_theta_batch(a, new)
    for c, t in zip(b, new):
        c.set_theta(t)
    _, ra = kcm.kcm_step(a, 4)
    _, rb = kcm.kcm_step(b, 4)
    del held
    for ca, cb, x, y in zip(a, b, ra, rb):
        assert x.status == 0 and y.status == 0
        assert np.array_equal(ca.state()["theta"], cb.state()["theta"])
        assert (x.e_elec, x.e_vdw, x.e_cav) == (y.e_elec, y.e_vdw, y.e_cav)
    # angles outside (-pi, pi] are wrapped (the two setters by different
    # formulas, equal up to rounding)
    far = [rng.uniform(-20.0, 20.0, c.n_joints) for c in a]
    held = kcm.kcm_set_theta_batch(a, far)
    for c, t in zip(b, far):
        c.set_theta(t)
    torch.cuda.synchronize()
    del held
    for ca, cb, t in zip(a, b, far):
        ta, tb = ca.state()["theta"], cb.state()["theta"]
        assert np.all(ta > -np.pi) and np.all(ta <= np.pi)
        assert np.abs(ta - tb).max() <= 1e-14
        assert np.abs(np.angle(np.exp(1j * (ta - t)))).max() <= 1e-13
    for c in a + b:
        c.free()


def test_a_chain_twice_in_one_call_is_rejected():
    p = params(kcm.KCM_MIXED)
    a = build_pair(5, 401, p)[0]
    b = build_pair(6, 402, p)[0]
    for call in (lambda: kcm.kcm_step([a, b, a], 1), lambda: kcm.kcm_fold([b, a, b], 1e-3, 2),
                 lambda: kcm.kcm_set_theta_batch([a, a], [np.zeros(10), np.zeros(10)])):
        with pytest.raises(kcm.KcmError) as e:
            call()
        assert e.value.status == kcm.KCM_E_INVAL
    assert kcm.kcm_step([a, b], 1)[0] == kcm.KCM_OK
    a.free()
    b.free()
