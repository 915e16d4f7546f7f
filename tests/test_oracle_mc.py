"""Pins of the oracle's Monte Carlo minimization (oracle/mc.py): special cases
with a known outcome, and the Metropolis rule reproducing the Boltzmann
distribution of one dihedral (closed form by quadrature).  No GPU."""
import numpy as np

import oracle
import synth

T = synth.alanine_like_types()


def _chain(m):
    return oracle.OracleChain(np.zeros(m, np.int32), T)


def test_zero_moves_keep_the_state():
    # no perturbation and no descent: every trial ties (dE = 0) and is accepted
    c = _chain(4)
    th = synth.random_dihedrals(4, 3)
    r = oracle.mc_minimize(c, th, np.zeros((5, 8)), np.full(5, 0.5), 0, 1.0, terms="elec+vdw")
    assert r["accepted"] == 5 and np.array_equal(r["theta"], th) and r["E"] == r["E_start"] == r["E_best"]


def test_infinite_temperature_accepts_every_trial():
    # kT -> inf: the accepted state is the plain composition of perturb-then-descend
    c = _chain(4)
    rng = np.random.default_rng(7)
    th = synth.random_dihedrals(4, 4)
    d = rng.uniform(-0.3, 0.3, (4, 8))
    r = oracle.mc_minimize(c, th, d, rng.uniform(0, 1, 4), 3, 1e300, terms="elec+vdw", s=1e-2)
    want = th.copy()
    for t in range(4):
        want = np.angle(np.exp(1j * (want + d[t])))
        for _ in range(3):
            want = oracle.iterate(c, want, terms="elec+vdw", s=1e-2)["theta"]
    assert r["accepted"] == 4
    assert np.abs(np.angle(np.exp(1j * (r["theta"] - want)))).max() < 1e-12


def test_zero_temperature_only_goes_downhill():
    c = _chain(5)
    rng = np.random.default_rng(11)
    th = synth.random_dihedrals(5, 5)
    d = rng.uniform(-0.6, 0.6, (12, 10))
    r = oracle.mc_minimize(c, th, d, rng.uniform(0, 1, 12), 4, 0.0, terms="elec+vdw", s=1e-2)
    assert r["E"] <= r["E_start"] and r["E_best"] == r["E"]
    assert 0 < r["accepted"] < 12


def test_masked_joints_are_not_perturbed():
    c = _chain(3)
    th = synth.random_dihedrals(3, 6)
    mask = np.array([1, 0, 1, 1, 0, 1], np.uint8)
    d = np.full((2, 6), 0.2)
    r = oracle.mc_minimize(c, th, d, np.zeros(2), 0, 1e300, terms="elec+vdw", mask=mask)
    assert np.array_equal(r["theta"][mask == 0], th[mask == 0])
    assert np.allclose(r["theta"][mask == 1], np.angle(np.exp(1j * (th[mask == 1] + 0.4))))


def test_metropolis_samples_the_boltzmann_distribution():
    # one free dihedral (psi_1 of a dipeptide), no descent: the chain of
    # accepted states samples p(psi) ~ exp(-E(psi)/kT) for symmetric proposals
    c = _chain(2)
    th0 = np.radians(np.array([-60.0, 140.0, -70.0, 150.0]))
    mask = np.array([0, 1, 0, 0], np.uint8)
    kT = 2.0
    n = 12000
    rng = np.random.default_rng(2024)
    d = np.zeros((n, 4))
    d[:, 1] = rng.uniform(-1.0, 1.0, n)
    u = rng.uniform(0.0, 1.0, n)
    # the accepted psi after each trial, from successive one-trial calls
    psi = np.empty(n)
    th = th0.copy()
    E = None
    for t in range(n):
        r = oracle.mc_minimize(c, th, d[t:t + 1], u[t:t + 1], 0, kT, terms="elec+vdw", mask=mask)
        th = r["theta"]
        psi[t] = th[1]
    grid = np.linspace(-np.pi, np.pi, 721)[:-1] + np.pi / 720
    E = np.array([(lambda o: o["E_elec"] + o["E_vdw"])(
        oracle.iterate(c, np.array([th0[0], g, th0[2], th0[3]]), terms="elec+vdw", mask=mask)) for g in grid])
    w = np.exp(-(E - E.min()) / kT)
    bins = np.linspace(-np.pi, np.pi, 25)
    p_want = np.histogram(grid, bins, weights=w)[0]
    p_want /= p_want.sum()
    p_got = np.histogram(psi[1000:], bins)[0].astype(float)
    p_got /= p_got.sum()
    tv = 0.5 * np.abs(p_got - p_want).sum()
    assert tv < 0.06, (tv, p_got, p_want)
