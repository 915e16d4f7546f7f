"""Randomised one-iteration parity sweep over the method's options: chain
length (1-48 residues), side-chain joints, joint masks, cutoff, sample-set
size, terms, capped or normalised step and precision, each case against the
FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import DTHETA_TOL, F_TOL, TAU_TOL, build_pair, compare_step, params  # noqa: E402
from paper_1712_05012_amd import kcm  # noqa: E402

pytestmark = pytest.mark.gpu

N_CASES = 64


def _cases():
    rng = np.random.default_rng(0x5EED)
    out = []
    for k in range(N_CASES):
        m = int(rng.integers(1, 49))
        out.append({
            "m": m,
            "seed": 9000 + k,
            "side_chains": bool(rng.integers(0, 2)),
            "masked": bool(rng.integers(0, 2)),
            "precision": int(rng.choice([kcm.KCM_FP64, kcm.KCM_MIXED])),
            "cutoff": float(rng.choice([6.0, 8.0, 10.0, 14.0])),
            "n_orbits": int(rng.choice([8, 14, 20])),
            "terms": int(rng.choice([kcm.KCM_TERM_ALL, kcm.KCM_TERM_ELEC | kcm.KCM_TERM_VDW, kcm.KCM_TERM_CAV])),
            # the linear rule has its own test: with the random starts' torques
            # (up to 1e13) it makes steps of millions of radians
            "step_rule": int(rng.choice([kcm.KCM_STEP_CAPPED, kcm.KCM_STEP_PAPER])),
        })
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kcm.load_library()


def test_randomised_option_sweep():
    ties = 0
    for c in _cases():
        p = params(c["precision"], cutoff=c["cutoff"], n_orbits=c["n_orbits"], terms=c["terms"],
                   step_rule=c["step_rule"])
        m = c["m"]
        J = (3 if c["side_chains"] else 2) * m
        mask = None
        if c["masked"]:
            mask = (np.random.default_rng(c["seed"]).uniform(0, 1, J) < 0.7).astype(np.uint8)
        print("case=sweep " + " ".join(f"{k}={v}" for k, v in c.items()), flush=True)
        gpu, ref, th = build_pair(m, c["seed"], p, mask=mask, side_chains=c["side_chains"])
        st, o, err = compare_step(gpu, ref, th, p, mask=mask)
        gpu.free()
        print("  " + " ".join(f"{k}={v:.3g}" for k, v in err.items()), flush=True)
        assert err["status"] == 0
        if err["margin"] <= 1e-10:
            ties += 1  # a sample test on its threshold: either count is right
            continue
        assert err["xyz"] < 1e-9
        assert err["F"] <= F_TOL and err["F_pair"] <= F_TOL and err["F_cav"] <= F_TOL
        assert err["dtheta"] <= DTHETA_TOL[c["precision"]] and err["theta"] <= DTHETA_TOL[c["precision"]]
        assert err["tau"] <= TAU_TOL[c["precision"]]
        if c["terms"] & kcm.KCM_TERM_CAV:
            assert err["E_cav"] < 1e-12
        if mask is not None:
            assert np.all(st["dtheta"][mask == 0] == 0.0)
    assert ties <= N_CASES // 10
