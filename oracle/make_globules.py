"""Write compact-globule starting dihedrals to ``data/globule_m<m>.npy``.

Input preparation only (never timed).  The chain is grown one residue at a
time inside a sphere of radius sqrt(5/3) * Rg_target (a filled ball of that
radius has radius of gyration Rg_target), with Rg_target = 2.2 m^0.38 A.  For
each residue K (phi, psi) candidates are drawn around the Ramachandran basins;
the candidate with the fewest contacts closer than ``clash`` A to earlier
non-excluded atoms (then the least excursion beyond the sphere) is kept.
Positions come from the oracle's kinematics: one residue at a time while
growing (``fk_extend``, the same operations as the whole-chain form), and the
finished chain is measured with the whole-chain ``fk``.  The radius is
rescaled until the final Rg is within 5 % of the target.

Usage: python -m oracle.make_globules 1000 10000 [--seed S] [--out-dir DIR]

Both stored files (1000 and 10,000 residues) were written with the default
seed.
"""
from __future__ import annotations

import os
import sys

import numpy as np
from scipy.spatial import cKDTree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

BASINS = np.radians(np.array([  # (phi, psi, spread) of the broad Ramachandran regions
    [-63.0, -43.0, 15.0],
    [-120.0, 130.0, 20.0],
    [-75.0, 145.0, 15.0],
    [60.0, 45.0, 15.0],
]))


def _excluded_pairs(ch):
    """(slot_prev, slot_cur) pairs of adjacent residues within three bonds."""
    ex = np.zeros((10, 10), dtype=bool)
    for a in range(10):
        for b in range(10):
            ex[a, b] = ch.bond_path(10 + a, 20 + b) <= 3
    return ex


def grow(m: int, radius: float, seed: int, K: int = 24, clash: float = 2.0):
    types = synth.residue_types()
    ch = oracle.OracleChain(np.zeros(m, np.int32), types)
    ex_prev = _excluded_pairs(oracle.OracleChain(np.zeros(4, np.int32), types))
    rng = np.random.default_rng(seed)
    theta = np.full(2 * m, np.pi)
    cell = clash
    span = int(np.ceil(2 * (radius + 20.0) / cell)) + 4
    off = span // 2
    grid = np.full((span, span, span, 8), -1, dtype=np.int32)
    slot_of = np.full((10 * m, 4), -1, dtype=np.int32)  # cell (3) + slot of each placed atom
    pos = np.zeros((10 * m, 3))
    nbr = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])

    def cells(p):
        return np.clip(np.floor(p / cell).astype(int) + off, 1, span - 2)

    def insert(a):
        g = cells(pos[a][None])[0]
        free = np.nonzero(grid[g[0], g[1], g[2]] < 0)[0]
        if free.size == 0:
            raise RuntimeError("grid cell overflow")
        grid[g[0], g[1], g[2], free[0]] = a
        slot_of[a] = (g[0], g[1], g[2], free[0])

    def remove(a):
        g = slot_of[a]
        if g[0] >= 0:
            grid[g[0], g[1], g[2], g[3]] = -1
            slot_of[a] = -1

    def clashes(k, new):
        cc = cells(new)[:, None, :] + nbr[None]
        ids = grid[cc[..., 0], cc[..., 1], cc[..., 2]].reshape(10, -1)
        bad = 0
        for a in range(10):
            js = ids[a][ids[a] >= 0]
            if js.size == 0:
                continue
            close = np.linalg.norm(pos[js] - new[a], axis=1) < clash
            if k > 0:
                close &= ~((js // 10 == k - 1) & ex_prev[js % 10, a])
            bad += int(close.sum())
        return bad

    fails = np.zeros(m, dtype=np.int64)
    # kinematic state before residue k: rotation of link 2k, point of joint 2k
    # (atom N of residue k), and the already placed atoms N, H of residue k
    rot = np.zeros((m + 1, 3, 3))
    pnt = np.zeros((m + 1, 3))
    nh = np.zeros((m + 1, 2, 3))
    rot[0] = np.eye(3)
    pnt[0] = ch.r0[0]
    nh[0] = ch.r0[0:2]
    k = 0
    while k < m:
        best, best_key, best_state = None, None, None
        # a residue that has failed more than 50 times (only ever in long
        # chains) also gets a wider draw and deeper backtracking
        widths = (K, 4 * K) if fails[k] <= 50 else (K, 4 * K, 16 * K)
        for width in widths:
            b = BASINS[rng.integers(0, len(BASINS), width)]
            cand = b[:, :2] + rng.normal(size=(width, 2)) * b[:, 2:3]
            for c in range(width):
                ext, Mn, pn = oracle.fk_extend(ch, k, rot[k], pnt[k], cand[c][0], cand[c][1])
                new = np.concatenate([nh[k], ext[:8]])
                tip = ext[8] if k + 1 < m else ext[6]  # N_{k+1} moves with phi_k and psi_k
                key = (clashes(k, new), max(0.0, np.linalg.norm(tip) - radius))
                if best_key is None or key < best_key:
                    best, best_key, best_state = cand[c].copy(), key, (new, Mn, pn, ext[8:10])
            if best_key[0] == 0:
                break
        if best_key[0] > 0:
            fails[k] += 1
            if fails[k] > 400:
                raise RuntimeError(f"stuck at residue {k}")
            back = min(k, 1 + int(fails[k]) // (3 if fails[k] <= 50 else 2))
            for kk in range(k - back, k):
                for a in range(10 * kk, 10 * kk + 10):
                    remove(a)
            k -= back
            continue
        theta[2 * k: 2 * k + 2] = best
        new, Mn, pn, nh_next = best_state
        pos[10 * k: 10 * k + 10] = new
        for a in range(10 * k, 10 * k + 10):
            insert(a)
        rot[k + 1], pnt[k + 1] = Mn, pn
        if k + 1 < m:
            nh[k + 1] = nh_next
        k += 1
        if k % 1000 == 0:
            print(f"  grown {k} of {m} residues", flush=True)
    # the whole-chain kinematics reproduces the grown chain
    r, _, _ = oracle.fk(ch, theta)
    assert np.array_equal(r, pos)
    return theta, pos, ch


def min_nonexcluded_distance(ch, pos, limit=2.5):
    tree = cKDTree(pos)
    pairs = tree.query_pairs(limit, output_type="ndarray")
    best = np.inf
    for a, b in pairs:
        if abs(a // 10 - b // 10) <= 1 and ch.bond_path(int(a), int(b)) <= 3:
            continue
        best = min(best, float(np.linalg.norm(pos[a] - pos[b])))
    return best


def make(m: int, seed: int = 0, out_dir: str | None = None):
    target = 2.2 * m ** 0.38
    radius = np.sqrt(5.0 / 3.0) * target
    # long chains pack with a smaller contact distance while growing: at 2 A
    # the tip of a 10,000-residue chain gets trapped deep inside the ball;
    # the acceptance test below still asks for 1.5 A between any two atoms
    clash = 2.0 if m <= 2000 else 1.6
    for attempt in range(6):
        theta, pos, ch = grow(m, radius, seed + attempt, clash=clash)
        rg = float(np.sqrt(((pos - pos.mean(0)) ** 2).sum(1).mean()))
        dmin = min_nonexcluded_distance(ch, pos)
        print(f"m={m} radius={radius:.2f} Rg={rg:.2f} target={target:.2f} min_d={dmin:.3f}", flush=True)
        if abs(rg / target - 1.0) < 0.05 and dmin > 1.5:
            break
        radius *= target / rg
    else:
        raise RuntimeError(f"no acceptable globule for m={m}")
    theta = (theta + np.pi) % (2 * np.pi) - np.pi
    theta[theta <= -np.pi] += 2 * np.pi
    out = os.path.join(out_dir or os.path.join(ROOT, "data"), f"globule_m{m}.npy")
    np.save(out, theta)
    print("wrote", out, f"(seed {seed + attempt})", flush=True)


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="write compact-globule start conformations")
    ap.add_argument("m", type=int, nargs="*", default=[1000], help="residue counts")
    ap.add_argument("--seed", type=int, default=0, help="growth seed of the first attempt")
    ap.add_argument("--out-dir", default=None, help="directory of the .npy files (default: data/)")
    a = ap.parse_args()
    for m in a.m:
        make(m, a.seed, a.out_dir)
