"""ctypes binding of ``include/kcm.h`` (argument marshalling only).

Device memory and streams come from PyTorch: a chain's device block is a
``torch.uint8`` CUDA tensor and the stream is ``torch.cuda.current_stream()``
unless one is given.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KCM_LIB", os.path.join(_HERE, "libkcm.so"))
_lib = None

KCM_OK, KCM_E_INVAL, KCM_E_NOMEM, KCM_E_DEVICE, KCM_E_NUMERIC, KCM_E_STATE, KCM_E_CAPACITY = 0, -1, -2, -3, -4, -5, -6
KCM_STEP_CAPPED, KCM_STEP_PAPER, KCM_STEP_LINEAR = 0, 1, 2
KCM_FP64, KCM_MIXED = 0, 1
KCM_TERM_ELEC, KCM_TERM_VDW, KCM_TERM_CAV, KCM_TERM_ALL = 1, 2, 4, 7

EXPORTED = ("kcm_default_params", "kcm_chain_bytes", "kcm_build_chain", "kcm_step", "kcm_fold",
            "kcm_get_state", "kcm_get_forces", "kcm_set_theta", "kcm_get_cells", "kcm_chain_info",
            "kcm_set_timing", "kcm_get_timing", "kcm_chain_free", "kcm_last_error", "kcm_get_atom_terms",
            "kcm_set_limits", "kcm_set_graphs", "kcm_mc_minimize", "kcm_mc_best_theta", "kcm_set_theta_batch",
            "kcm_step_noalloc", "kcm_set_force_variant")
KCM_FORCE_VARIANTS = 4
KCM_NBR_CHUNK = 240
KCM_NOALLOC_MAX_CHAINS = 1024
KCM_NOALLOC_SCRATCH_BYTES = 262144


class KcmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kcm status {status}: {msg}")
        self.status = status


class kcm_residue_type(C.Structure):
    _fields_ = [("q", C.c_double * 10), ("sigma", C.c_double * 10), ("eps", C.c_double * 10),
                ("hydrophobicity", C.c_double)]


class kcm_chain_desc(C.Structure):
    _fields_ = [("n_res", C.c_int32), ("res_type", C.POINTER(C.c_int32)),
                ("types", C.POINTER(kcm_residue_type)), ("n_types", C.c_int32),
                ("theta0", C.POINTER(C.c_double)), ("joint_mask", C.POINTER(C.c_uint8)),
                ("side_chains", C.c_int32)]


class kcm_params(C.Structure):
    _fields_ = [("cutoff", C.c_double), ("kappa", C.c_double), ("max_step", C.c_double),
                ("step_rule", C.c_int32), ("precision", C.c_int32), ("terms", C.c_int32),
                ("n_orbits", C.c_int32), ("diel_k", C.c_double), ("w13", C.c_double),
                ("w14_elec", C.c_double), ("w14_vdw", C.c_double), ("delta_r", C.c_double),
                ("r_probe", C.c_double), ("g_hydro", C.c_double), ("cell_size", C.c_double)]


class kcm_step_report(C.Structure):
    _fields_ = [("e_elec", C.c_double), ("e_vdw", C.c_double), ("e_cav", C.c_double),
                ("max_tau", C.c_double), ("max_dtheta", C.c_double), ("iterations", C.c_int64),
                ("status", C.c_int32), ("converged", C.c_int32)]


class kcm_fold_result(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("converged", C.c_int32), ("status", C.c_int32),
                ("seconds", C.c_double)]


class kcm_mc_result(C.Structure):
    _fields_ = [("e_start", C.c_double), ("e_accepted", C.c_double), ("e_best", C.c_double),
                ("trials", C.c_int64), ("accepted", C.c_int64), ("status", C.c_int32), ("pad", C.c_int32)]


def load_library(path: str = LIB_PATH):
    """Load libkcm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libkcm.so not built: {path} (run paper_1712_05012_amd/build.py)")
    lib = C.CDLL(path)
    vp, st = C.c_void_p, C.c_int
    lib.kcm_default_params.argtypes = [C.POINTER(kcm_params)]
    lib.kcm_default_params.restype = None
    lib.kcm_chain_bytes.argtypes = [C.POINTER(kcm_chain_desc), C.POINTER(kcm_params), C.POINTER(C.c_size_t)]
    lib.kcm_build_chain.argtypes = [C.POINTER(kcm_chain_desc), C.POINTER(kcm_params), vp, C.c_size_t, vp,
                                    C.POINTER(vp)]
    lib.kcm_step.argtypes = [C.POINTER(vp), C.c_int, C.c_int, vp, C.POINTER(kcm_step_report)]
    lib.kcm_step_noalloc.argtypes = [C.POINTER(vp), C.c_int, C.c_int, vp, C.POINTER(kcm_step_report)]
    lib.kcm_fold.argtypes = [C.POINTER(vp), C.c_int, C.c_double, C.c_int, C.c_int, vp,
                             C.POINTER(kcm_fold_result)]
    lib.kcm_get_state.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.kcm_get_forces.argtypes = [vp, vp, vp, vp]
    lib.kcm_set_theta.argtypes = [vp, vp, vp]
    lib.kcm_get_atom_terms.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.kcm_set_limits.argtypes = [vp, C.c_double, C.c_int64, vp]
    lib.kcm_set_graphs.argtypes = [C.c_int]
    lib.kcm_set_force_variant.argtypes = [C.c_int]
    lib.kcm_get_cells.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32]
    lib.kcm_chain_info.argtypes = [vp, vp, vp, vp, vp]
    lib.kcm_set_timing.argtypes = [C.c_int]
    lib.kcm_get_timing.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.kcm_chain_free.argtypes = [vp]
    lib.kcm_mc_minimize.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int32, C.c_double, vp, vp, vp,
                                    C.POINTER(kcm_mc_result)]
    lib.kcm_mc_best_theta.argtypes = [vp, vp, vp]
    lib.kcm_set_theta_batch.argtypes = [C.POINTER(vp), C.c_int32, vp, vp]
    lib.kcm_last_error.argtypes = []
    lib.kcm_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("kcm_default_params", "kcm_last_error"):
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def _check(status):
    if status != KCM_OK:
        raise KcmError(status, load_library().kcm_last_error().decode())
    return status


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# C-ABI names
# ---------------------------------------------------------------------------
def kcm_default_params(**overrides) -> kcm_params:
    p = kcm_params()
    load_library().kcm_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


@dataclass
class ChainInputs:
    """Host arrays describing one chain (kept alive while the C call reads them)."""

    res_type: np.ndarray
    types: object          # ctypes array of kcm_residue_type
    theta0: np.ndarray | None
    mask: np.ndarray | None
    desc: kcm_chain_desc = field(default=None)


def make_desc(res_type, residue_types, theta0=None, joint_mask=None, side_chains: bool = False) -> ChainInputs:
    """residue_types: object with q, sigma, eps (n_types, 10) and hydro (n_types,) arrays.

    theta0 and joint_mask hold 2 n_res backbone entries, followed by n_res
    side-chain angles chi when ``side_chains`` is set."""
    rt = np.ascontiguousarray(res_type, dtype=np.int32)
    nt = len(residue_types.hydro)
    types = (kcm_residue_type * nt)()
    for t in range(nt):
        types[t].q[:] = [float(x) for x in residue_types.q[t]]
        types[t].sigma[:] = [float(x) for x in residue_types.sigma[t]]
        types[t].eps[:] = [float(x) for x in residue_types.eps[t]]
        types[t].hydrophobicity = float(residue_types.hydro[t])
    th = None if theta0 is None else np.ascontiguousarray(theta0, dtype=np.float64)
    mk = None if joint_mask is None else np.ascontiguousarray(joint_mask, dtype=np.uint8)
    J = (3 if side_chains else 2) * rt.size
    if th is not None and th.shape != (J,):
        raise ValueError(f"theta0 must have {J} entries")
    if mk is not None and mk.shape != (J,):
        raise ValueError(f"joint_mask must have {J} entries")
    d = kcm_chain_desc()
    d.n_res = rt.size
    d.res_type = rt.ctypes.data_as(C.POINTER(C.c_int32))
    d.types = C.cast(types, C.POINTER(kcm_residue_type))
    d.n_types = nt
    d.theta0 = th.ctypes.data_as(C.POINTER(C.c_double)) if th is not None else None
    d.joint_mask = mk.ctypes.data_as(C.POINTER(C.c_uint8)) if mk is not None else None
    d.side_chains = 1 if side_chains else 0
    return ChainInputs(rt, types, th, mk, d)


def kcm_chain_bytes(inputs: ChainInputs, params: kcm_params) -> int:
    n = C.c_size_t(0)
    _check(load_library().kcm_chain_bytes(C.byref(inputs.desc), C.byref(params), C.byref(n)))
    return int(n.value)


def kcm_build_chain(inputs: ChainInputs, params: kcm_params, dev_ptr: int, nbytes: int, stream=None):
    h = C.c_void_p()
    _check(load_library().kcm_build_chain(C.byref(inputs.desc), C.byref(params), C.c_void_p(dev_ptr),
                                          C.c_size_t(nbytes), _stream_handle(stream), C.byref(h)))
    return h


def _handles(chains):
    arr = (C.c_void_p * len(chains))()
    for i, c in enumerate(chains):
        arr[i] = c.handle.value if isinstance(c, Chain) else c.value
    return arr


def kcm_step(chains, n_iter: int = 1, stream=None, report=True, check: bool = True):
    """report: True for a list of kcm_step_report, "array" for one numpy
    structured array with the same fields, False for none."""
    arr = _handles(chains)
    reps = (kcm_step_report * len(chains))() if report else None
    st = load_library().kcm_step(arr, len(chains), int(n_iter), _stream_handle(stream),
                                 reps if report else None)
    if check:
        _check(st)
    if not report:
        return st, None
    if isinstance(report, str) and report == "array":
        return st, np.ctypeslib.as_array(reps)
    return st, list(reps)


def kcm_step_noalloc(chains, n_iter: int = 1, stream=None, report=True, check: bool = True):
    """kcm_step through the entry point that allocates nothing (at most
    KCM_NOALLOC_MAX_CHAINS chains, direct launches); same return values."""
    arr = _handles(chains)
    reps = (kcm_step_report * len(chains))() if report else None
    st = load_library().kcm_step_noalloc(arr, len(chains), int(n_iter), _stream_handle(stream),
                                         reps if report else None)
    if check:
        _check(st)
    if not report:
        return st, None
    return st, list(reps)


def kcm_fold(chains, tol: float, max_iter: int, check_every: int = 10, stream=None, check: bool = True):
    arr = _handles(chains)
    res = (kcm_fold_result * len(chains))()
    st = load_library().kcm_fold(arr, len(chains), float(tol), int(max_iter), int(check_every),
                                 _stream_handle(stream), res)
    if check:
        _check(st)
    return st, list(res)


def kcm_mc_minimize(chains, delta, u, n_descent: int, kT: float, stream=None, check: bool = True):
    """Monte Carlo minimization of every chain on the device.

    delta: one host array [n_trials, J_c] per chain (radians); u: host array
    [n_chains, n_trials] uniform in [0, 1).  Both are copied to the device
    here.  Returns (status, [kcm_mc_result])."""
    import torch

    n = len(chains)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 2 or u.shape[0] != n:
        raise ValueError("u must have shape [n_chains, n_trials]")
    n_trials = u.shape[1]
    if len(delta) != n:
        raise ValueError("one delta array per chain")
    parts = []
    for c, d in zip(chains, delta):
        d = np.ascontiguousarray(d, dtype=np.float64)
        J = kcm_chain_info(c.handle if isinstance(c, Chain) else c)[1]
        if d.shape != (n_trials, J):
            raise ValueError(f"delta of a chain must have shape [{n_trials}, {J}]")
        parts.append(d.reshape(-1))
    dev = torch.device("cuda")
    d_dev = torch.from_numpy(np.concatenate(parts) if parts else np.zeros(0)).to(dev)
    u_dev = torch.from_numpy(u.reshape(-1)).to(dev)
    res = (kcm_mc_result * n)()
    st = load_library().kcm_mc_minimize(_handles(chains), n, n_trials, int(n_descent), float(kT),
                                        C.c_void_p(d_dev.data_ptr()), C.c_void_p(u_dev.data_ptr()),
                                        _stream_handle(stream), res)
    if check:
        _check(st)
    return st, list(res)


def kcm_set_theta_batch(chains, thetas, stream=None):
    """New angles for every chain in one device copy and one kernel.

    thetas: one host array [J_c] per chain (a 2-D array works when all chains
    have the same J).  Returns the device tensor holding them, which the
    caller keeps until work queued after this call on the stream has run."""
    import torch

    if len(thetas) != len(chains):
        raise ValueError("one theta array per chain")
    Js = [c.n_joints if isinstance(c, Chain) else kcm_chain_info(c)[1] for c in chains]
    if isinstance(thetas, np.ndarray) and thetas.ndim == 2 and all(J == thetas.shape[1] for J in Js):
        flat = np.ascontiguousarray(thetas, dtype=np.float64).reshape(-1)
    else:
        parts = []
        for J, t in zip(Js, thetas):
            t = np.ascontiguousarray(t, dtype=np.float64)
            if t.shape != (J,):
                raise ValueError(f"theta of a chain must have {J} entries")
            parts.append(t)
        flat = np.concatenate(parts)
    dev = torch.from_numpy(flat).to(torch.device("cuda"))
    torch.cuda.current_stream().synchronize()
    _check(load_library().kcm_set_theta_batch(_handles(chains), len(chains), C.c_void_p(dev.data_ptr()),
                                              _stream_handle(stream)))
    return dev


def kcm_mc_best_theta(handle, stream=None):
    _, J, _, _ = kcm_chain_info(handle)
    th = np.zeros(J)
    _check(load_library().kcm_mc_best_theta(handle, _stream_handle(stream), _p(th)))
    return th


def kcm_chain_info(handle):
    v = [C.c_int32() for _ in range(4)]
    _check(load_library().kcm_chain_info(handle, *[C.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def kcm_get_state(handle, stream=None):
    n, J, _, _ = kcm_chain_info(handle)
    theta, tau, dth = np.zeros(J), np.zeros(J), np.zeros(J)
    xyz, F = np.zeros((n, 3)), np.zeros((n, 3))
    _check(load_library().kcm_get_state(handle, _stream_handle(stream), _p(theta), _p(xyz), _p(F), _p(tau),
                                        _p(dth)))
    return {"theta": theta, "xyz": xyz, "force": F, "tau": tau, "dtheta": dth}


def kcm_get_theta(handle, stream=None):
    """The angles alone (one copy instead of the whole state)."""
    _, J, _, _ = kcm_chain_info(handle)
    theta = np.zeros(J)
    _check(load_library().kcm_get_state(handle, _stream_handle(stream), _p(theta), None, None, None, None))
    return theta


def kcm_get_forces(handle, stream=None):
    n, _, _, _ = kcm_chain_info(handle)
    fp, fc = np.zeros((n, 3)), np.zeros((n, 3))
    _check(load_library().kcm_get_forces(handle, _stream_handle(stream), _p(fp), _p(fc)))
    return fp, fc


def kcm_get_atom_terms(handle, stream=None):
    n, _, _, _ = kcm_chain_info(handle)
    ee, ev, ec = np.zeros(n), np.zeros(n), np.zeros(n)
    nx = np.zeros(n, np.int32)
    _check(load_library().kcm_get_atom_terms(handle, _stream_handle(stream), _p(ee), _p(ev), _p(ec), _p(nx)))
    return {"e_elec": ee, "e_vdw": ev, "e_cav": ec, "n_exposed": nx}


def kcm_set_limits(handle, tol: float, max_iterations: int, stream=None):
    _check(load_library().kcm_set_limits(handle, float(tol), int(max_iterations), _stream_handle(stream)))


def kcm_set_theta(handle, theta, stream=None):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    _, J, _, _ = kcm_chain_info(handle)
    if th.shape != (J,):
        raise ValueError(f"theta must have {J} entries")
    _check(load_library().kcm_set_theta(handle, _p(th), _stream_handle(stream)))


def kcm_get_cells(handle, stream=None):
    n, _, _, _ = kcm_chain_info(handle)
    dims = np.zeros(3, np.int32)
    cell = C.c_double()
    origin = np.zeros(3)
    nc = C.c_int32()
    lib = load_library()
    _check(lib.kcm_get_cells(handle, _stream_handle(stream), _p(dims), C.byref(cell), _p(origin), C.byref(nc),
                             None, None, 0))
    order = np.zeros(n, np.int32)
    cs = np.zeros(nc.value + 1, np.int32)
    _check(lib.kcm_get_cells(handle, _stream_handle(stream), None, None, None, None, _p(order), _p(cs),
                             cs.size))
    return {"dims": dims, "cell": cell.value, "origin": origin, "order": order, "cell_start": cs}


def kcm_set_graphs(iterations):
    """Iterations per replayed HIP graph (True = 1, False = 0: direct launches)."""
    if isinstance(iterations, bool):
        iterations = 1 if iterations else 0
    _check(load_library().kcm_set_graphs(int(iterations)))


def kcm_set_force_variant(variant: int):
    """Launch shape of the force kernel (0 .. KCM_FORCE_VARIANTS-1), process-wide."""
    _check(load_library().kcm_set_force_variant(int(variant)))


def kcm_set_timing(every: int):
    """Sample HIP events on every `every`-th iteration (0 = off)."""
    _check(load_library().kcm_set_timing(int(every)))


def kcm_get_timing(reset: bool = False):
    fm, fl, im, it = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
    _check(load_library().kcm_get_timing(C.byref(fm), C.byref(fl), C.byref(im), C.byref(it), 1 if reset else 0))
    return {"force_ms": fm.value, "force_launches": fl.value, "iter_ms": im.value, "iterations": it.value}


def kcm_chain_free(handle):
    _check(load_library().kcm_chain_free(handle))


# ---------------------------------------------------------------------------
# convenience: a chain whose device block is a torch tensor
# ---------------------------------------------------------------------------
class Chain:
    """Builds one chain in a torch-allocated device block on the current device."""

    def __init__(self, res_type, residue_types, params: kcm_params | None = None, theta0=None,
                 joint_mask=None, stream=None, device=None, side_chains: bool = False):
        import torch
        self.params = params if params is not None else kcm_default_params()
        self.inputs = make_desc(res_type, residue_types, theta0, joint_mask, side_chains)
        self.nbytes = kcm_chain_bytes(self.inputs, self.params)
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.block = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = self.block.data_ptr()
        self.offset = (-ptr) % 256
        self.handle = kcm_build_chain(self.inputs, self.params, ptr + self.offset, self.nbytes, stream)
        self.n_atoms, self.n_joints, self.n_samples, self.precision = kcm_chain_info(self.handle)

    def step(self, n_iter=1, stream=None):
        return kcm_step([self], n_iter, stream)[1][0]

    def state(self, stream=None):
        return kcm_get_state(self.handle, stream)

    def theta(self, stream=None):
        return kcm_get_theta(self.handle, stream)

    def forces(self, stream=None):
        return kcm_get_forces(self.handle, stream)

    def atom_terms(self, stream=None):
        return kcm_get_atom_terms(self.handle, stream)

    def set_theta(self, theta, stream=None):
        kcm_set_theta(self.handle, theta, stream)

    def mc_best_theta(self, stream=None):
        return kcm_mc_best_theta(self.handle, stream)

    def cells(self, stream=None):
        return kcm_get_cells(self.handle, stream)

    def free(self):
        if self.handle is not None:
            kcm_chain_free(self.handle)
            self.handle = None
            self.block = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
