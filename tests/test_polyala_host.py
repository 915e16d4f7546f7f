"""Polyalanine experiments (Sec. 5): host analysis (C-alpha torsions, handedness,
Ramachandran regions), the start generator, and the oracle's own helix runs
against the hand and helical region the paper reports.  No GPU."""
import os

import numpy as np
import pytest

import oracle
import synth
from paper_1712_05012_amd import polyala

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "polyala_helix_averages.txt")


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        start, medium, phi, psi = line.split()
        rows[(float(start), medium)] = (float(phi), float(psi))
    return rows


def _ideal(phi, psi, m=15):
    ref = oracle.OracleChain(np.zeros(m, np.int32), synth.alanine_like_types())
    r, _, _ = oracle.fk(ref, np.radians(np.tile([phi, psi], m).astype(float)))
    return r


def test_ca_torsion_sign_and_handedness():
    # ideal right-handed alpha-helix: C-alpha torsion near +50 degrees; its
    # mirror (phi, psi negated) near -50; a beta strand near -170
    t = polyala.ca_torsions(_ideal(-57.0, -47.0))
    assert t.size == 12 and np.all(np.abs(t - t[0]) < 1e-9) and 40.0 < t[0] < 60.0
    assert polyala.handedness(_ideal(-57.0, -47.0)) == "right"
    tl = polyala.ca_torsions(_ideal(57.0, 47.0))
    assert abs(tl[0] + t[0]) < 1.0  # the template is chiral (L), so not an exact mirror
    assert polyala.handedness(_ideal(57.0, 47.0)) == "left"
    assert polyala.handedness(_ideal(-120.0, 130.0)) == "extended"
    assert polyala.ca_torsions(_ideal(-57.0, -47.0, m=3)).size == 0


def test_ca_torsion_matches_rotated_copy():
    # a rigid rotation and translation leaves every torsion unchanged
    r = _ideal(-80.0, -30.0)
    a = np.radians(37.0)
    R = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])
    assert np.allclose(polyala.ca_torsions(r @ R.T + 5.0), polyala.ca_torsions(r), atol=1e-9)


def test_regions():
    phi = np.array([-60.0, 60.0, -120.0, -60.0, 90.0, -170.0, 0.0])
    psi = np.array([-45.0, 45.0, 130.0, 140.0, -90.0, -160.0, 0.0])
    names = [polyala.REGIONS[k] for k in polyala.regions(phi, psi)]
    assert names == ["alpha_R", "alpha_L", "beta", "beta", "other", "beta", "other"]


def test_polyala_starts_and_type():
    T = synth.alanine_like_types()
    assert T.q.shape == (1, 10) and abs(T.q.sum()) < 1e-12
    lengths, thetas = synth.polyala_starts(500, 3)
    assert lengths.min() >= 10 and lengths.max() <= 20 and set(np.unique(lengths)) == set(range(10, 21))
    assert all(t.shape == (2 * m,) for m, t in zip(lengths, thetas))
    allt = np.concatenate(thetas)
    assert np.abs(allt).max() <= np.radians(90.0) and np.abs(allt).max() > np.radians(89.0)
    l2, t2 = synth.polyala_starts(500, 3)
    assert np.array_equal(lengths, l2) and all(np.array_equal(a, b) for a, b in zip(thetas, t2))


def _oracle_helix(start, terms, n_iter=1500):
    ref = oracle.OracleChain(np.zeros(15, np.int32), synth.alanine_like_types())
    th = np.full(30, np.radians(start))
    for _ in range(n_iter):
        o = oracle.iterate(ref, th, terms=terms, kappa=1e-3, s=1e-2)
        th = o["theta"]
    r, _, _ = oracle.fk(ref, th)
    deg = (np.degrees(th) + 180.0) % 360.0 - 180.0
    return deg[2::2].mean(), deg[3::2].mean(), polyala.handedness(r), o


@pytest.mark.parametrize("start", [10.0, -10.0])
def test_oracle_helix_in_vacuum_follows_the_paper(start):
    # the start's hand decides the helix's hand, and the mean folded angles of
    # residues 2..15 lie within 10 degrees of the paper's averages
    phi, psi, hand, _ = _oracle_helix(start, "elec+vdw")
    want = _golden()[(start, "vacuum")]
    assert hand == ("left" if start > 0 else "right")
    assert abs(phi - want[0]) < 10.0 and abs(psi - want[1]) < 10.0, (phi, psi, want)


def test_oracle_right_handed_helix_is_lower_in_energy():
    el = _oracle_helix(10.0, "elec+vdw")[3]
    er = _oracle_helix(-10.0, "elec+vdw")[3]
    assert er["E_elec"] + er["E_vdw"] < el["E_elec"] + el["E_vdw"] - 10.0
