"""The C-ABI library loads and exports every symbol include/kcm.h declares;
host-side argument checks work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_1712_05012_amd import kcm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kcm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kcm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = kcm.load_library()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(kcm.EXPORTED)


def test_header_constants_are_mirrored():
    src = open(os.path.join(ROOT, "include", "kcm.h")).read()
    defines = dict(re.findall(r"^#define (KCM_[A-Z0-9_]+) (\d+)\s*$", src, flags=re.M))
    assert {"KCM_NBR_CHUNK", "KCM_FORCE_VARIANTS", "KCM_NOALLOC_MAX_CHAINS"} <= set(defines)
    for name, value in defines.items():
        assert getattr(kcm, name) == int(value), name


def test_default_params_match_header():
    p = kcm.kcm_default_params()
    assert (p.cutoff, p.kappa, p.max_step, p.n_orbits) == (10.0, 1e-3, 1e-3, 14)
    assert p.step_rule == kcm.KCM_STEP_CAPPED and p.precision == kcm.KCM_FP64 and p.terms == kcm.KCM_TERM_ALL
    assert abs(p.w14_elec - 1 / 1.2) < 1e-16 and p.w14_vdw == 0.5 and p.w13 == 0.0
    assert (p.delta_r, p.r_probe, p.g_hydro, p.diel_k, p.cell_size) == (0.05, 1.4, 0.025, 4.0, 0.0)


def test_chain_bytes_scale_and_validation():
    T = synth.residue_types()
    p = kcm.kcm_default_params()
    b64 = kcm.kcm_chain_bytes(kcm.make_desc(synth.sequence(64, 1), T), p)
    b1k = kcm.kcm_chain_bytes(kcm.make_desc(synth.sequence(1000, 1), T), p)
    assert b64 % 256 == 0 and b1k > 10 * b64 // 2
    bad = kcm.make_desc(np.array([0, 25], np.int32), T)
    with pytest.raises(kcm.KcmError) as e:
        kcm.kcm_chain_bytes(bad, p)
    assert e.value.status == kcm.KCM_E_INVAL
    with pytest.raises(kcm.KcmError):
        kcm.kcm_chain_bytes(kcm.make_desc(synth.sequence(4, 1), T), kcm.kcm_default_params(n_orbits=0))
    with pytest.raises(kcm.KcmError):
        kcm.kcm_chain_bytes(kcm.make_desc(synth.sequence(4, 1), T), kcm.kcm_default_params(precision=7))
    assert "precision" in kcm.load_library().kcm_last_error().decode()


def test_build_rejects_bad_arguments_before_touching_the_device():
    T = synth.residue_types()
    p = kcm.kcm_default_params()
    inp = kcm.make_desc(synth.sequence(4, 1), T)
    lib = kcm.load_library()
    h = C.c_void_p()
    # misaligned block
    st = lib.kcm_build_chain(C.byref(inp.desc), C.byref(p), C.c_void_p(0x1001), C.c_size_t(1 << 20), None, C.byref(h))
    assert st == kcm.KCM_E_INVAL
    # block too small
    st = lib.kcm_build_chain(C.byref(inp.desc), C.byref(p), C.c_void_p(0x1000), C.c_size_t(256), None, C.byref(h))
    assert st == kcm.KCM_E_NOMEM
    # null handle array
    assert lib.kcm_step(None, 0, 1, None, None) == kcm.KCM_E_INVAL


def test_binding_fails_loudly_without_the_library(tmp_path):
    with pytest.raises(ImportError):
        kcm.load_library.__wrapped__(str(tmp_path / "missing.so")) if hasattr(kcm.load_library, "__wrapped__") \
            else _load_missing(str(tmp_path / "missing.so"))


def _load_missing(path):
    saved = kcm._lib
    kcm._lib = None
    try:
        kcm.load_library(path)
    finally:
        kcm._lib = saved


def test_launch_mode_settings_are_validated():
    lib = kcm.load_library()
    assert lib.kcm_set_graphs(-1) == kcm.KCM_E_INVAL
    assert lib.kcm_set_graphs(65) == kcm.KCM_E_INVAL
    for depth in (0, 8, 1):
        assert lib.kcm_set_graphs(depth) == kcm.KCM_OK
    assert lib.kcm_set_timing(-1) == kcm.KCM_E_INVAL
    assert lib.kcm_set_timing(0) == kcm.KCM_OK


def test_side_chain_layout_and_validation():
    T = synth.residue_types()
    p = kcm.kcm_default_params()
    seq = synth.sequence(100, 1)
    b = kcm.kcm_chain_bytes(kcm.make_desc(seq, T), p)
    bs = kcm.kcm_chain_bytes(kcm.make_desc(seq, T, side_chains=True), p)
    assert bs > b and bs % 256 == 0
    with pytest.raises(ValueError):
        kcm.make_desc(seq, T, theta0=np.zeros(200), side_chains=True)
    bad = kcm.make_desc(seq, T)
    bad.desc.side_chains = 2
    with pytest.raises(kcm.KcmError) as e:
        kcm.kcm_chain_bytes(bad, p)
    assert e.value.status == kcm.KCM_E_INVAL
