"""kcm_step_noalloc, the entry point that allocates nothing, against kcm_step:
the same chains stepped through either entry point give the same reports
and states bit for bit, on two calls in a row, the second with a smaller
input (fewer, shorter chains and fewer iterations) (needs an MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from gpu_common import TYPES, params  # noqa: E402
from paper_1712_05012_amd import kcm  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("e_elec", "e_vdw", "e_cav", "max_tau", "max_dtheta", "iterations", "status", "converged")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kcm.load_library()


def _chains(spec, p):
    return [kcm.Chain(synth.sequence(m, s), TYPES, p, theta0=synth.random_dihedrals(m, s)) for m, s in spec]


@pytest.mark.parametrize("precision", [kcm.KCM_FP64, kcm.KCM_MIXED])
def test_noalloc_step_equals_kcm_step(precision):
    p = params(precision)
    spec = [(7, 501), (40, 502), (120, 503), (15, 504), (64, 505)]
    a, b = _chains(spec, p), _chains(spec, p)
    try:
        # a call with five chains, then a smaller one with two of them
        for idx, n_iter in (([0, 1, 2, 3, 4], 3), ([1, 3], 2)):
            print(f"case=noalloc precision={precision} chains={idx} n_iter={n_iter}", flush=True)
            sa, ra = kcm.kcm_step([a[i] for i in idx], n_iter)
            sb, rb = kcm.kcm_step_noalloc([b[i] for i in idx], n_iter)
            assert sa == sb == kcm.KCM_OK
            for i, x, y in zip(idx, ra, rb):
                for f in FIELDS:
                    assert getattr(x, f) == getattr(y, f), (i, f)
                xa, xb = a[i].state(), b[i].state()
                for key in ("theta", "xyz", "force", "tau", "dtheta"):
                    assert np.array_equal(xa[key], xb[key]), (i, key)
        # without reports the call only queues work; the next report agrees
        kcm.kcm_step([a[0], a[2]], 2, report=False)
        kcm.kcm_step_noalloc([b[0], b[2]], 2, report=False)
        _, ra = kcm.kcm_step([a[0], a[2]], 0)
        _, rb = kcm.kcm_step_noalloc([b[0], b[2]], 0)
        for x, y in zip(ra, rb):
            assert x.iterations == y.iterations == 5 and x.e_cav == y.e_cav
        assert np.array_equal(a[2].state()["theta"], b[2].state()["theta"])
    finally:
        for c in a + b:
            c.free()


def test_noalloc_rejects_more_chains_than_its_table_holds():
    p = params(kcm.KCM_MIXED)
    (c,) = _chains([(5, 510)], p)
    try:
        with pytest.raises(kcm.KcmError) as e:
            kcm.kcm_step_noalloc([c] * (kcm.KCM_NOALLOC_MAX_CHAINS + 1), 1)
        assert e.value.status == kcm.KCM_E_INVAL
        assert "1024" in str(e.value)
        with pytest.raises(kcm.KcmError) as e:
            kcm.kcm_step_noalloc([c, c], 1)
        assert e.value.status == kcm.KCM_E_INVAL
        assert kcm.kcm_step_noalloc([c], 1)[0] == kcm.KCM_OK
    finally:
        c.free()
