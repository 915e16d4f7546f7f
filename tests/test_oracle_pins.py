"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these retypes an oracle formula: each checks a closed form, an
invariant, a limit, a brute-force recount or a value printed in the paper.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TYPES = synth.residue_types()


def chain(m, seed=1):
    return oracle.OracleChain(synth.sequence(m, synth.config_seed(seed)), TYPES)


def dihedral(p0, p1, p2, p3):
    b1, b2, b3 = p1 - p0, p2 - p1, p3 - p2
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    return np.arctan2(np.linalg.norm(b2) * np.dot(b1, n2), np.dot(n1, n2))


def angle(a, b, c):
    u, v = a - b, c - b
    return np.degrees(np.arccos(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v)))


def wrap(x):
    return (x + np.pi) % (2 * np.pi) - np.pi


# --------------------------------------------------------------------------
# synthetic inputs
# --------------------------------------------------------------------------
def test_synth_recipe_ranges_and_determinism():
    t = synth.residue_types()
    assert t.q.shape == (20, 10)
    assert np.all(np.abs(t.q) <= 0.5 + 1e-15)
    net = t.q.sum(axis=1)
    assert np.all(np.isin(np.round(net), [-1, 0, 1]))
    assert np.allclose(net, np.round(net), atol=1e-12)
    assert t.sigma.min() >= 1.8 and t.sigma.max() <= 4.0
    assert t.eps.min() >= 0.02 and t.eps.max() <= 0.2
    assert np.abs(t.hydro).max() <= 4.5
    t2 = synth.residue_types()
    assert np.array_equal(t.q, t2.q) and np.array_equal(t.sigma, t2.sigma)
    th = synth.random_dihedrals(100, 7)
    assert th.min() > -np.pi and th.max() <= np.pi
    assert np.array_equal(th, synth.random_dihedrals(100, 7))
    a, L = synth.serving_jobs(500, 3)
    assert np.all(np.diff(a) >= 0) and L.min() >= 30 and L.max() <= 2000
    assert 150 < np.median(L) < 260


# --------------------------------------------------------------------------
# zero position and forward kinematics (Sec. 2.1, eqs kin_02-kin_04, r1)
# --------------------------------------------------------------------------
def test_zp_bond_lengths_and_angles():
    ch = chain(5)
    r = ch.r0
    for i in range(5):
        N, CA, C, O = r[10 * i], r[10 * i + 2], r[10 * i + 8], r[10 * i + 9]
        assert abs(np.linalg.norm(CA - N) - 1.458) < 1e-12
        assert abs(np.linalg.norm(C - CA) - 1.525) < 1e-12
        assert abs(np.linalg.norm(O - C) - 1.231) < 1e-12
        assert abs(angle(N, CA, C) - 111.2) < 1e-9
        assert abs(angle(CA, C, O) - 120.8) < 1e-9
        for s in (3, 4):  # HA, CB: tetrahedral at CA
            assert abs(angle(N, CA, r[10 * i + s]) - 109.5) < 1e-9
        if i + 1 < 5:
            Nn, CAn = r[10 * (i + 1)], r[10 * (i + 1) + 2]
            assert abs(np.linalg.norm(Nn - C) - 1.329) < 1e-12
            assert abs(angle(CA, C, Nn) - 116.2) < 1e-9
            assert abs(angle(C, Nn, CAn) - 121.7) < 1e-9
            # ZP: all peptide planes coplanar, phi = psi = omega = 180 deg
            assert abs(abs(dihedral(N, CA, C, Nn)) - np.pi) < 1e-9
            assert abs(abs(dihedral(CA, C, Nn, CAn)) - np.pi) < 1e-9
    # N of the first residue anchored at the origin
    assert np.all(r[0] == 0.0)


def test_zp_l_chirality():
    # L-amino acids: improper C-N-CA-CB is about -120 degrees
    r = chain(3).r0
    for i in range(3):
        d = np.degrees(dihedral(r[10 * i + 8], r[10 * i], r[10 * i + 2], r[10 * i + 4]))
        assert -130 < d < -110


def test_table1_peptide_plane_structure():
    """Table 1: sign pattern of (C1, C2) and CaC + CN = 1*b_{2i} + 0*b_{2i+1}."""
    rows = {}
    for line in open(os.path.join(GOLDEN, "table1_peptide_plane.txt")):
        if line.strip() and not line.startswith("#"):
            k, c1, c2 = line.split()
            rows[k] = (float(c1), float(c2))
    assert np.allclose(np.add(rows["CaC"], rows["CN"]), (1.0, 0.0), atol=1e-12)
    r = chain(3).r0
    i = 0
    CA, C, O, Nn, Hn, CAn = r[2], r[8], r[9], r[10], r[11], r[12]
    b2i, b2i1 = Nn - CA, CAn - Nn
    B = np.stack([b2i, b2i1], axis=1)
    ours = {}
    for k, v in {"CaC": C - CA, "CN": Nn - C, "CO": O - C, "NH": Hn - Nn}.items():
        c, res, *_ = np.linalg.lstsq(B, v, rcond=None)
        assert np.linalg.norm(B @ c - v) < 1e-12  # the vector lies in the rigid peptide plane
        ours[k] = c
    assert np.allclose(ours["CaC"] + ours["CN"], (1.0, 0.0), atol=1e-12)
    for k in rows:
        assert np.all(np.sign(ours[k]) == np.sign(rows[k])), k
    del i


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fk_preserves_geometry_and_sets_dihedrals(seed):
    m = 7
    ch = chain(m, seed)
    th = synth.random_dihedrals(m, 100 + seed)
    r, u, p = oracle.fk(ch, th)
    b = ch.bonds()
    d0 = np.linalg.norm(ch.r0[b[:, 0]] - ch.r0[b[:, 1]], axis=1)
    d1 = np.linalg.norm(r[b[:, 0]] - r[b[:, 1]], axis=1)
    assert np.abs(d1 - d0).max() < 1e-12
    # all bond angles preserved (every pair of bonds sharing an atom)
    for x in range(ch.n):
        nb = [int(y) for e in b for y in e if x in e and y != x]
        for k1 in range(len(nb)):
            for k2 in range(k1 + 1, len(nb)):
                a0 = angle(ch.r0[nb[k1]], ch.r0[x], ch.r0[nb[k2]])
                a1 = angle(r[nb[k1]], r[x], r[nb[k2]])
                assert abs(a0 - a1) < 1e-8
    # IUPAC phi_i = C_{i-1}-N-CA-C, psi_i = N-CA-C-N_{i+1}; omega stays trans
    for i in range(m):
        if i > 0:
            phi = dihedral(r[10 * (i - 1) + 8], r[10 * i], r[10 * i + 2], r[10 * i + 8])
            assert abs(wrap(phi - th[2 * i])) < 1e-10
            om = dihedral(r[10 * (i - 1) + 2], r[10 * (i - 1) + 8], r[10 * i], r[10 * i + 2])
            assert abs(abs(om) - np.pi) < 1e-10
        if i + 1 < m:
            psi = dihedral(r[10 * i], r[10 * i + 2], r[10 * i + 8], r[10 * (i + 1)])
            assert abs(wrap(psi - th[2 * i + 1])) < 1e-10
    # joint axes are unit vectors along N->CA and CA->C through N and CA
    for j in range(2 * m):
        i = j // 2
        a, c = (r[10 * i], r[10 * i + 2]) if j % 2 == 0 else (r[10 * i + 2], r[10 * i + 8])
        assert np.allclose(u[j], (c - a) / np.linalg.norm(c - a), atol=1e-12)
        assert np.allclose(p[j], a, atol=1e-12)


def test_fk_zero_position_identity():
    ch = chain(4)
    r, _, _ = oracle.fk(ch, np.full(8, np.pi))
    assert np.abs(r - ch.r0).max() < 1e-13


def test_fk_first_joint_rotates_everything_downstream_rigidly():
    # turning only phi_1 is a rigid rotation of all atoms past link 0 about N1->CA1
    ch = chain(4)
    th = np.full(8, np.pi)
    th[0] = np.pi - 0.7
    r, _, _ = oracle.fk(ch, th)
    moved = np.arange(2, ch.n)
    d0 = np.linalg.norm(ch.r0[moved][:, None] - ch.r0[moved][None], axis=-1)
    d1 = np.linalg.norm(r[moved][:, None] - r[moved][None], axis=-1)
    assert np.abs(d0 - d1).max() < 1e-12
    assert np.allclose(r[:3], ch.r0[:3], atol=1e-14)  # N1, H1 fixed, CA1 on the axis


# --------------------------------------------------------------------------
# interaction classes (Sec. 3.3)
# --------------------------------------------------------------------------
def test_bond_path_classes():
    ch = chain(4)
    # slots: 0 N, 1 H, 2 CA, 3 HA, 4 CB, 5-7 HB, 8 C, 9 O
    assert ch.bond_path(0, 2) == 1          # N-CA (1-2)
    assert ch.bond_path(0, 8) == 2          # N-C across CA (1-3)
    assert ch.bond_path(1, 3) == 3          # H-N-CA-HA (1-4)
    assert ch.bond_path(5, 6) == 2          # two H on CB (siblings, 1-3)
    assert ch.bond_path(9, 11) == 3         # O_i-C_i-N_{i+1}-H_{i+1}
    assert ch.bond_path(2, 12) == 3         # CA_i-C_i-N_{i+1}-CA_{i+1}
    assert ch.bond_path(8, 20) == 4         # C_i .. N_{i+2}: four bonds
    assert ch.bond_path(5, 9) == 4          # HB-CB-CA-C-O
    assert ch.bond_path(0, 0) == 0


# --------------------------------------------------------------------------
# Coulomb and Lennard-Jones (eqs 02-03_9)
# --------------------------------------------------------------------------
def spread_positions(n, spacing=100.0):
    r = np.zeros((n, 3))
    r[:, 0] = np.arange(n) * spacing
    return r


def test_lj_minimum_depth_and_coulomb_value():
    ch = chain(4)
    i, j = 4, 34  # CB of residue 0 and CB of residue 3: w = 1
    r = spread_positions(ch.n)
    D = ch.R[i] + ch.R[j]
    r[j] = r[i] + np.array([0.0, D, 0.0])
    pp = oracle.PairParams(cutoff=10.0)
    F, Ee, Ev = oracle.pair_forces(ch, r, pp)
    # at d = D the LJ term sits at its minimum: zero force and depth -eps_ij
    assert abs(Ev + np.sqrt(ch.eps[i] * ch.eps[j])) < 1e-12
    # the remaining force is pure Coulomb: |F| = 2 E_elec / d, along the line of centres
    assert abs(np.linalg.norm(F[j]) - 2 * abs(Ee) / D) < 1e-9 * max(1, abs(Ee))
    assert np.allclose(F[i], -F[j], atol=1e-12)
    # distance-dependent dielectric: E scales as 1/d^2
    r2 = r.copy()
    r2[j] = r[i] + np.array([0.0, 2 * D, 0.0])
    _, Ee2, _ = oracle.pair_forces(ch, r2, pp)
    assert abs(Ee2 * 4 - Ee) < 1e-12 * max(1, abs(Ee))


def test_cutoff_is_inclusive_and_hard():
    ch = chain(4)
    i, j = 4, 34
    r = spread_positions(ch.n)
    r[j] = r[i] + np.array([0.0, 0.0, 10.0])
    _, Ee, Ev = oracle.pair_forces(ch, r, oracle.PairParams(cutoff=10.0))
    assert Ee != 0.0 and Ev != 0.0
    r[j] = r[i] + np.array([0.0, 0.0, 10.0 + 1e-9])
    F, Ee, Ev = oracle.pair_forces(ch, r, oracle.PairParams(cutoff=10.0))
    assert Ee == 0.0 and Ev == 0.0 and not F.any()


def test_weights_exclusions_and_one_four():
    ch = chain(3)
    r = spread_positions(ch.n)
    # 1-2 pair N-CA placed 3 A apart: weight 0, no force
    r[2] = r[0] + np.array([3.0, 0, 0])
    F, Ee, Ev = oracle.pair_forces(ch, r, oracle.PairParams())
    assert Ee == 0.0 and Ev == 0.0
    # 1-4 pair H-HA: scaled by w14 relative to the same geometry at w14 = 1
    r = spread_positions(ch.n)
    r[3] = r[1] + np.array([0, 3.0, 0])
    _, Ee, Ev = oracle.pair_forces(ch, r, oracle.PairParams())
    _, Ee1, Ev1 = oracle.pair_forces(ch, r, oracle.PairParams(w14_elec=1.0, w14_vdw=1.0))
    assert abs(Ee - Ee1 / 1.2) < 1e-12 * abs(Ee1) and abs(Ev - 0.5 * Ev1) < 1e-12 * abs(Ev1)


@pytest.mark.parametrize("seed", [3, 4])
def test_pair_newton_third_law_and_rigid_invariance(seed):
    m = 12
    ch = chain(m, seed)
    r, _, _ = oracle.fk(ch, synth.random_dihedrals(m, seed))
    F, Ee, Ev = oracle.pair_forces(ch, r)
    assert np.abs(F.sum(axis=0)).max() < 1e-11 * np.abs(F).max()
    # net torque about the origin vanishes too (central forces)
    assert np.abs(np.cross(r, F).sum(axis=0)).max() < 1e-10 * np.abs(F).max() * np.abs(r).max()
    rng = np.random.default_rng(seed)
    A, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    r2 = r @ A.T + rng.normal(size=3) * 20
    F2, Ee2, Ev2 = oracle.pair_forces(ch, r2)
    assert abs(Ee2 - Ee) < 1e-10 * max(1, abs(Ee)) and abs(Ev2 - Ev) < 1e-10 * max(1, abs(Ev))
    assert np.abs(F2 - F @ A.T).max() < 1e-9 * np.abs(F).max()


def test_pair_force_is_minus_energy_gradient():
    m = 5
    ch = chain(m, 9)
    r, _, _ = oracle.fk(ch, synth.random_dihedrals(m, 9))
    pp = oracle.PairParams(cutoff=1e6)
    F, _, _ = oracle.pair_forces(ch, r, pp)
    h = 1e-6
    for a in (0, 7, 23, 41):
        for s in range(3):
            rp, rm = r.copy(), r.copy()
            rp[a, s] += h
            rm[a, s] -= h
            _, e1, v1 = oracle.pair_forces(ch, rp, pp)
            _, e0, v0 = oracle.pair_forces(ch, rm, pp)
            fd = -((e1 + v1) - (e0 + v0)) / (2 * h)
            assert abs(fd - F[a, s]) < 1e-5 * max(1.0, np.abs(F).max())


# --------------------------------------------------------------------------
# torques: tau = -dE/dtheta (eqs KCM_01-KCM_06), no cutoff, small chains
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,seed", [(4, 1), (8, 2), (12, 5)])
def test_torque_is_minus_energy_gradient_in_theta(m, seed):
    ch = chain(m, seed)
    th = synth.random_dihedrals(m, 40 + seed)
    pp = oracle.PairParams(cutoff=1e6)

    def E(t):
        r, _, _ = oracle.fk(ch, t)
        _, a, b = oracle.pair_forces(ch, r, pp)
        return a + b

    r, u, p = oracle.fk(ch, th)
    F, _, _ = oracle.pair_forces(ch, r, pp)
    tau = oracle.torques(ch, r, F, u, p)
    h = 1e-6
    fd = np.array([-(E(th + h * e) - E(th - h * e)) / (2 * h) for e in np.eye(2 * m)])
    assert np.abs(tau - fd).max() < 1e-6 * max(1.0, np.abs(tau).max())


def test_torque_of_uniform_force_field():
    # a uniform force c on every atom: the moment about joint k is
    # (sum of downstream r_a - n_k p_k) x c, projected on u_k
    m = 5
    ch = chain(m, 2)
    r, u, p = oracle.fk(ch, synth.random_dihedrals(m, 2))
    c = np.array([0.3, -1.1, 0.7])
    F = np.tile(c, (ch.n, 1))
    tau = oracle.torques(ch, r, F, u, p)
    link = ch.link_of_atom()
    for k in range(2 * m):
        down = link > k
        want = np.dot(u[k], np.cross(r[down].sum(0) - down.sum() * p[k], c))
        assert abs(tau[k] - want) < 1e-10 * max(1, abs(want))


# --------------------------------------------------------------------------
# SASA enumeration (eqs 04-finitediff, Algorithm 1)
# --------------------------------------------------------------------------
def test_sample_set_rule():
    for n_orb, N in ((10, 128), (14, 250), (20, 508), (28, 998)):
        Q = oracle.samples(n_orb)
        assert Q.shape == (N, 3)
        assert np.allclose(np.linalg.norm(Q, axis=1), 1.0, atol=1e-15)
        assert np.abs(Q.mean(axis=0)).max() < 1e-12  # orbits symmetric about the equator
    assert len(np.unique(np.round(oracle.samples(14), 12), axis=0)) == 250


def test_isolated_atom_fully_exposed():
    r = np.array([[0.0, 0, 0], [50.0, 0, 0]])
    R = np.array([1.7, 1.2])
    g = np.array([0.05, -0.1])
    F, f, E = oracle.sasa_atoms(r, R, g)
    assert np.all(f == 1.0) and not F.any()
    want = sum(4 * np.pi * g[k] * (R[k] + 1.4) ** 2 for k in range(2))
    assert abs(E - want) < 1e-12


def test_buried_atom_fully_covered():
    # a small sphere strictly inside a large one: every sample covered
    r = np.array([[0.0, 0, 0], [0.3, 0.1, 0]])
    R = np.array([1.0, 3.5])
    F, f, E = oracle.sasa_atoms(r, R, np.array([0.1, 0.1]))
    assert f[0] == 0.0


@pytest.mark.parametrize("d", [3.0, 4.5, 6.0])
def test_two_sphere_exposed_fraction_closed_form(d):
    Ri, Rj = 1.6, 2.1
    a, b = Ri + 1.4, Rj + 1.4
    sp = oracle.SasaParams(n_orbits=300)
    r = np.array([[0.0, 0, 0], [d * 0.6, d * 0.48, d * 0.64]])
    F, f, E = oracle.sasa_atoms(r, np.array([Ri, Rj]), np.array([0.1, 0.1]), sp)
    hi = (b * b - (d - a) ** 2) / (2 * d)
    hj = (a * a - (d - b) ** 2) / (2 * d)
    assert abs(f[0] - (1 - hi / (2 * a))) < 2e-3
    assert abs(f[1] - (1 - hj / (2 * b))) < 2e-3


def test_two_sphere_force_approaches_area_gradient():
    # F_j = -F_i = -(g_i dA_i/dd + g_j dA_j/dd) e_ij with A = 4 pi R^2 - 2 pi R h
    Ri, Rj, gi, gj, d = 1.6, 2.1, 0.1, 0.05, 4.5
    a, b = Ri + 1.4, Rj + 1.4
    e = np.array([0.6, 0.48, 0.64])
    r = np.array([[0.0, 0, 0], d * e])
    sp = oracle.SasaParams(n_orbits=400, delta_r=0.02)
    F, f, E = oracle.sasa_atoms(r, np.array([Ri, Rj]), np.array([gi, gj]), sp)

    def area(dd):
        hi = (b * b - (dd - a) ** 2) / (2 * dd)
        hj = (a * a - (dd - b) ** 2) / (2 * dd)
        return gi * (4 * np.pi * a * a - 2 * np.pi * a * hi) + gj * (4 * np.pi * b * b - 2 * np.pi * b * hj)

    dGdd = (area(d + 1e-6) - area(d - 1e-6)) / 2e-6
    want_j = -dGdd * e
    assert np.allclose(F[0], -F[1], atol=1e-12)
    assert np.linalg.norm(F[1] - want_j) < 0.06 * np.linalg.norm(want_j)


@pytest.mark.parametrize("seed", range(6))
def test_c_state_rules_equal_definitional_recount(seed):
    rng = np.random.default_rng(seed)
    n = 9
    r = rng.uniform(0, 6.0, size=(n, 3))
    R = rng.uniform(1.0, 2.2, size=n)
    sp = oracle.SasaParams(n_orbits=10)
    D1, e1 = oracle.sasa_definitional(r, R, sp)
    D2, e2 = oracle.sasa_events(r, R, sp)
    assert np.array_equal(e1, e2)
    assert np.array_equal(D1, D2)
    assert np.abs(D1).sum() > 0


def test_sasa_chain_matches_free_atom_form_and_conserves_momentum():
    m = 6
    ch = chain(m, 3)
    r, _, _ = oracle.fk(ch, synth.random_dihedrals(m, 11))
    F, f, E, margin = oracle.sasa_forces(ch, r)
    F2, f2, E2 = oracle.sasa_atoms(r, ch.R, ch.gamma)
    assert np.array_equal(f, f2)
    assert np.abs(F - F2).max() < 1e-12 * max(1, np.abs(F).max())
    assert abs(E - E2) < 1e-12 * max(1, abs(E))
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * max(1, np.abs(F).max())
    assert margin > 0


def test_sasa_translation_invariance():
    m = 5
    ch = chain(m, 4)
    r, _, _ = oracle.fk(ch, synth.random_dihedrals(m, 12))
    _, f, E, mg = oracle.sasa_forces(ch, r)
    _, f2, E2, _ = oracle.sasa_forces(ch, r + np.array([16.0, -8.0, 4.0]))
    if mg > 1e-9:
        assert np.array_equal(f, f2)


# --------------------------------------------------------------------------
# compliance step (eq KCM_07)
# --------------------------------------------------------------------------
def test_step_rules():
    rng = np.random.default_rng(0)
    tau = rng.normal(size=20) * 50
    th = synth.random_dihedrals(10, 1)
    s, kappa = 1e-3, 1e-3
    t1, d1, mx1 = oracle.step(tau, th, rule=oracle.StepRule.PAPER, kappa=kappa, s=s)
    assert abs(mx1 - s) < 1e-18 and abs(np.abs(d1).max() - s) < 1e-18
    assert np.allclose(d1 / tau, s / np.abs(tau).max(), rtol=1e-14)
    t2, d2, _ = oracle.step(tau, th, rule=oracle.StepRule.LINEAR, kappa=kappa, s=s)
    assert np.allclose(d2, kappa * tau, rtol=1e-15)
    t3, d3, mx3 = oracle.step(tau, th, rule=oracle.StepRule.CAPPED, kappa=kappa, s=s)
    assert abs(mx3 - min(kappa * np.abs(tau).max(), s)) < 1e-18
    small = tau * 1e-3
    _, d4, _ = oracle.step(small, th, rule=oracle.StepRule.CAPPED, kappa=kappa, s=s)
    assert np.allclose(d4, kappa * small, rtol=1e-15)
    mask = np.ones(20, np.uint8)
    mask[::3] = 0
    t5, d5, _ = oracle.step(tau, th, mask=mask, rule=oracle.StepRule.PAPER, kappa=kappa, s=s)
    assert np.all(d5[mask == 0] == 0) and np.all(t5[mask == 0] == th[mask == 0])
    assert abs(np.abs(d5).max() - s) < 1e-18
    # wrapping to (-pi, pi]
    t6, _, _ = oracle.step(np.array([1.0]), np.array([np.pi - 1e-4]), rule=oracle.StepRule.PAPER, s=1e-3)
    assert -np.pi < t6[0] < 0


def test_one_iteration_lowers_energy_for_small_step():
    # eq (KCM_07) is a steepest-descent step: for a small step E must drop
    m = 8
    ch = chain(m, 6)
    th = synth.random_dihedrals(m, 66)
    pp = oracle.PairParams(cutoff=1e6)
    out = oracle.iterate(ch, th, pp=pp, terms="elec+vdw", rule=oracle.StepRule.PAPER, s=1e-5)
    r2, _, _ = oracle.fk(ch, out["theta"])
    _, e2, v2 = oracle.pair_forces(ch, r2, pp)
    assert e2 + v2 < out["E_elec"] + out["E_vdw"]


def test_coulomb_constant_from_si_units():
    # 1/(4 pi eps0) in kcal A / (mol e^2) from CODATA constants, with the
    # distance-dependent dielectric eps = 4 d eps0: E = C q_i q_j / (4 d^2)
    e, eps0, NA = 1.602176634e-19, 8.8541878128e-12, 6.02214076e23
    C = e * e / (4 * np.pi * eps0 * 1e-10) * NA / 4184.0
    ch = chain(4)
    i, j = 4, 34
    r = spread_positions(ch.n)
    d = 6.0
    r[j] = r[i] + np.array([d, 0.0, 0.0])
    _, Ee, _ = oracle.pair_forces(ch, r, oracle.PairParams())
    assert abs(Ee - C * ch.q[i] * ch.q[j] / (4.0 * d * d)) < 1e-5 * abs(Ee)


def _coulomb_constant():
    e, eps0, NA = 1.602176634e-19, 8.8541878128e-12, 6.02214076e23
    return e * e / (4 * np.pi * eps0 * 1e-10) * NA / 4184.0


# (slot of an atom of residue 0, slot of an atom of residue 3): every pair is
# three residues apart, so its weight is 1 (Sec. 3.3)
_TABLE_PAIRS = [(4, 4), (0, 9), (2, 7), (9, 1), (5, 8)]


@pytest.mark.parametrize("seed", [1, 6])
def test_atom_parameters_follow_the_type_table(seed):
    # The per-atom inputs are read from the residue-type table, never from the
    # oracle's own per-atom arrays.  Sec. 2.2 gives the LJ well distance as
    # D_ij = R_i + R_j (eq 03, 03_1) with eps_ij = sqrt(eps_i eps_j); with the
    # reading R = 2^(1/6) sigma / 2 the LJ energy of a pair placed at
    # D = 2^(1/6) (sigma_i + sigma_j) / 2 is exactly -sqrt(eps_i eps_j) and its
    # force is zero, so what is left of the force is the Coulomb closed form
    # with the table's charges of (residue type, slot).
    m = 4
    seq = synth.sequence(m, synth.config_seed(seed))
    assert len({int(seq[0]), int(seq[3])}) == 2, "the two residues must have different types"
    ch = oracle.OracleChain(seq, TYPES)
    C = _coulomb_constant()
    k6 = 2.0 ** (1.0 / 6.0)
    for si, sj in _TABLE_PAIRS:
        i, j = si, 30 + sj
        ti, tj = int(seq[0]), int(seq[3])
        D = k6 * (TYPES.sigma[ti, si] + TYPES.sigma[tj, sj]) / 2.0
        r = spread_positions(ch.n)
        e = np.array([0.36, -0.48, 0.8])
        r[j] = r[i] + D * e
        F, Ee, Ev = oracle.pair_forces(ch, r, oracle.PairParams(cutoff=10.0))
        depth = np.sqrt(TYPES.eps[ti, si] * TYPES.eps[tj, sj])
        assert abs(Ev + depth) < 1e-12 * max(1.0, depth), (si, sj)
        qi, qj = TYPES.q[ti, si], TYPES.q[tj, sj]
        E_want = C * qi * qj / (4.0 * D * D)
        assert abs(Ee - E_want) < 2e-6 * abs(E_want) + 1e-15, (si, sj)
        # -dE/dd of C q q / (4 d^2) is 2E/d, repulsive for like charges; F_j
        # points along +e (from i to j) when E > 0
        Fj_want = (2.0 * E_want / D) * e
        assert np.abs(F[j] - Fj_want).max() < 2e-6 * np.abs(Fj_want).max() + 1e-15, (si, sj)
        assert np.allclose(F[i], -F[j], rtol=0, atol=1e-12 * max(1.0, np.abs(F[j]).max()))


@pytest.mark.parametrize("g_hydro", [0.025, 0.05])
def test_isolated_atoms_solvation_energy_from_the_type_table(g_hydro):
    # Every atom of a chain spread 100 A apart is isolated: all its samples are
    # exposed (f = 1), and its solvation energy is 4 pi gamma R_off^2 (eq
    # G_cav_patch) with gamma = g_h * hydrophobicity of its residue type
    # (reading of Table 3) and R_off = 2^(1/6) sigma / 2 + r_probe.
    m = 3
    seq = synth.sequence(m, synth.config_seed(2))
    ch = oracle.OracleChain(seq, TYPES, g_hydro=g_hydro)
    r = spread_positions(ch.n)
    sp = oracle.SasaParams(r_probe=1.4)
    F, f, E = oracle.sasa_forces(ch, r, sp)[:3]
    assert np.all(f == 1.0) and not F.any()
    want = 0.0
    for a in range(ch.n):
        t, s = int(seq[a // 10]), a % 10
        R_off = 2.0 ** (1.0 / 6.0) * TYPES.sigma[t, s] / 2.0 + 1.4
        want += 4.0 * np.pi * g_hydro * TYPES.hydro[t] * R_off ** 2
    assert abs(E - want) < 1e-12 * max(1.0, abs(want))
    # one atom at a time: the free-atom form gives the same per-atom value
    a = 17
    t, s = int(seq[a // 10]), a % 10
    R = 2.0 ** (1.0 / 6.0) * TYPES.sigma[t, s] / 2.0
    _, fa, Ea = oracle.sasa_atoms(r[[a]], np.array([R]), np.array([g_hydro * TYPES.hydro[t]]), sp)
    assert fa[0] == 1.0
    assert abs(Ea - 4.0 * np.pi * g_hydro * TYPES.hydro[t] * (R + 1.4) ** 2) < 1e-12


def test_fk_extend_grows_the_same_chain_as_fk():
    # the residue-by-residue kinematics used to grow start conformations is the
    # same sequence of operations as the whole-chain kinematics: equal bit for bit
    m = 30
    ch = oracle.OracleChain(synth.sequence(m, 5), synth.residue_types())
    th = synth.random_dihedrals(m, 5)
    r, _, _ = oracle.fk(ch, th)
    grown = np.zeros_like(r)
    grown[0:2] = ch.r0.reshape(-1, 3)[0:2]
    M, p = np.eye(3), ch.r0.reshape(-1, 3)[0].copy()
    for k in range(m):
        pos, M, p = oracle.fk_extend(ch, k, M, p, th[2 * k], th[2 * k + 1])
        grown[10 * k + 2: 10 * k + 2 + len(pos)] = pos
    assert np.array_equal(grown, r)


# --------------------------------------------------------------------------
# side-chain joints (Sec. 2.1): chi_i = dihedral N-CA-CB-HB1 turns HB1..HB3
# --------------------------------------------------------------------------
def _chi_thetas(m, seed):
    rng = np.random.default_rng(500 + seed)
    return np.concatenate([synth.random_dihedrals(m, 300 + seed), rng.uniform(-np.pi, np.pi, m)])


@pytest.mark.parametrize("seed", [1, 2])
def test_chi_kinematics_geometry_dihedrals_and_branch(seed):
    m = 6
    ch = chain(m, seed)
    th = _chi_thetas(m, seed)
    r, u, p = oracle.fk(ch, th)
    rb, _, _ = oracle.fk(ch, th[: 2 * m])
    assert u.shape == (3 * m, 3) and p.shape == (3 * m, 3)
    # only the branch atoms HB1..HB3 differ from the backbone-only kinematics
    branch = np.zeros(ch.n, bool)
    for i in range(m):
        branch[10 * i + 5: 10 * i + 8] = True
    assert np.array_equal(r[~branch], rb[~branch])
    # every bond length and bond angle of the zero position is kept
    b = ch.bonds()
    d0 = np.linalg.norm(ch.r0[b[:, 0]] - ch.r0[b[:, 1]], axis=1)
    assert np.abs(np.linalg.norm(r[b[:, 0]] - r[b[:, 1]], axis=1) - d0).max() < 1e-12
    for i in range(m):
        CA, CB = 10 * i + 2, 10 * i + 4
        for h in (5, 6, 7):
            a0 = angle(ch.r0[CA], ch.r0[CB], ch.r0[10 * i + h])
            assert abs(angle(r[CA], r[CB], r[10 * i + h]) - a0) < 1e-8
        # chi is the dihedral N-CA-CB-HB1; HB2 and HB3 keep their 120 degree offsets
        N = 10 * i
        chi = dihedral(r[N], r[CA], r[CB], r[10 * i + 5])
        assert abs(wrap(chi - th[2 * m + i])) < 1e-10
        assert abs(wrap(dihedral(r[N], r[CA], r[CB], r[10 * i + 6]) - chi - 2 * np.pi / 3)) < 1e-10
        assert abs(wrap(dihedral(r[N], r[CA], r[CB], r[10 * i + 7]) - chi + 2 * np.pi / 3)) < 1e-10
        # axis along CA->CB through CA
        assert np.allclose(u[2 * m + i], (r[CB] - r[CA]) / np.linalg.norm(r[CB] - r[CA]), atol=1e-12)
        assert np.allclose(p[2 * m + i], r[CA], atol=1e-12)


def test_chi_at_zero_position_leaves_the_template():
    m = 3
    ch = chain(m)
    th = np.concatenate([np.full(2 * m, np.pi), np.full(m, np.radians(60.0))])
    r, _, _ = oracle.fk(ch, th)
    assert np.abs(r - ch.r0).max() < 1e-13


@pytest.mark.parametrize("m,seed", [(4, 1), (7, 3)])
def test_chi_torque_is_minus_energy_gradient(m, seed):
    # all 3m torques against central differences of the pair energy
    ch = chain(m, seed)
    th = _chi_thetas(m, seed)
    pp = oracle.PairParams(cutoff=1e6)

    def E(t):
        r, _, _ = oracle.fk(ch, t)
        _, a, b = oracle.pair_forces(ch, r, pp)
        return a + b

    r, u, p = oracle.fk(ch, th)
    F, _, _ = oracle.pair_forces(ch, r, pp)
    tau = oracle.torques(ch, r, F, u, p)
    h = 1e-6
    fd = np.array([-(E(th + h * e) - E(th - h * e)) / (2 * h) for e in np.eye(3 * m)])
    assert np.abs(tau - fd).max() < 1e-6 * max(1.0, np.abs(tau).max())
    assert np.abs(tau[2 * m:]).max() > 0.0  # the branch feels the field


def test_chi_step_moves_only_free_joints():
    m = 5
    ch = chain(m, 4)
    th = _chi_thetas(m, 4)
    mask = np.ones(3 * m, np.uint8)
    mask[2 * m + 1] = 0
    o = oracle.iterate(ch, th, terms="elec+vdw", mask=mask)
    assert o["dtheta"].shape == (3 * m,)
    assert o["dtheta"][2 * m + 1] == 0.0
    assert np.abs(o["dtheta"][2 * m:]).max() > 0.0
