"""ctypes wrapper around the C oracle (``kcm_oracle.c``).

Each wrapper states the passage of the paper that the C routine follows; the
arithmetic itself lives in the C file only.
"""
from __future__ import annotations

import ctypes as C
import enum
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kcm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

APR = 10


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (OpenMP over atoms, FP64 throughout)."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class _PairP(C.Structure):
    _fields_ = [("cutoff", C.c_double), ("diel_k", C.c_double), ("w13", C.c_double),
                ("w14_elec", C.c_double), ("w14_vdw", C.c_double)]


class _SasaP(C.Structure):
    _fields_ = [("delta_r", C.c_double), ("r_probe", C.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    lib.or_build_zp.argtypes = [C.c_int, _dp]
    lib.or_bonds.argtypes = [C.c_int, vp]
    lib.or_bond_path.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.or_link_of_atom.argtypes = [C.c_int]
    lib.or_atom_params.argtypes = [C.c_int, _ip, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp, _dp]
    lib.or_fk.argtypes = [C.c_int, _dp, _dp, _dp, vp, vp]
    lib.or_fk_extend.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
    lib.or_pair_forces.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.POINTER(_PairP), vp, C.c_int, _dp, vp]
    lib.or_samples.argtypes = [C.c_int, vp]
    lib.or_sasa_forces.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(_SasaP), _dp, vp, vp, vp]
    lib.or_sasa_definitional.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, C.POINTER(_SasaP), _ip, vp]
    lib.or_sasa_events.argtypes = [C.c_int, _dp, _dp, _dp, C.c_int, C.POINTER(_SasaP), _ip, vp]
    lib.or_sasa_atoms.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, C.POINTER(_SasaP), _dp, vp, vp]
    lib.or_torques.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.or_fk_chi.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
    lib.or_torques_chi.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.or_step.argtypes = [C.c_int, _dp, vp, C.c_int, C.c_double, C.c_double, _dp, vp, vp]
    lib.or_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class StepRule(enum.IntEnum):
    CAPPED = 0
    PAPER = 1
    LINEAR = 2


@dataclass
class PairParams:
    cutoff: float = 10.0
    diel_k: float = 4.0
    w13: float = 0.0
    w14_elec: float = 1.0 / 1.2
    w14_vdw: float = 0.5

    def c(self):
        return _PairP(self.cutoff, self.diel_k, self.w13, self.w14_elec, self.w14_vdw)


@dataclass
class SasaParams:
    delta_r: float = 0.05
    r_probe: float = 1.4
    n_orbits: int = 14

    def c(self):
        return _SasaP(self.delta_r, self.r_probe)


class OracleChain:
    """ZP geometry, bonds and per-atom parameters of one chain (Sec. 2.1-2.2).

    ``types`` is a ``synth.ResidueTypes``; ``res_type`` an int array of length m.
    """

    def __init__(self, res_type, types, g_hydro: float = 0.025):
        lib = _load()
        self.res_type = np.ascontiguousarray(res_type, dtype=np.int32)
        self.m = int(self.res_type.size)
        self.n = APR * self.m
        self.J = 2 * self.m
        self.r0 = np.zeros((self.n, 3))
        lib.or_build_zp(self.m, self.r0)
        self.q = np.zeros(self.n)
        self.R = np.zeros(self.n)
        self.eps = np.zeros(self.n)
        self.gamma = np.zeros(self.n)
        lib.or_atom_params(self.m, self.res_type,
                           np.ascontiguousarray(types.q, dtype=np.float64),
                           np.ascontiguousarray(types.sigma, dtype=np.float64),
                           np.ascontiguousarray(types.eps, dtype=np.float64),
                           np.ascontiguousarray(types.hydro, dtype=np.float64),
                           float(g_hydro), self.q, self.R, self.eps, self.gamma)

    def bonds(self) -> np.ndarray:
        lib = _load()
        nb = lib.or_bonds(self.m, None)
        out = np.zeros(2 * nb, dtype=np.int32)
        lib.or_bonds(self.m, out.ctypes.data_as(C.c_void_p))
        return out.reshape(nb, 2)

    def bond_path(self, a: int, b: int) -> int:
        return int(_load().or_bond_path(self.m, int(a), int(b)))

    def link_of_atom(self) -> np.ndarray:
        lib = _load()
        return np.array([lib.or_link_of_atom(a) for a in range(self.n)], dtype=np.int32)


def fk(chain: OracleChain, theta):
    """Eqs (kin_02)-(kin_04), (r1): positions r[n,3], joint axes u[J,3], joint points p[J,3].

    theta holds the 2m backbone angles (phi_1, psi_1, ...), optionally
    followed by the m side-chain angles chi_1..chi_m (Sec. 2.1); their axes
    and points then follow the backbone joints' in u and p."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    J = th.size
    assert J in (chain.J, chain.J + chain.m)
    r = np.zeros((chain.n, 3))
    u = np.zeros((J, 3))
    p = np.zeros((J, 3))
    _load().or_fk(chain.m, chain.r0, np.ascontiguousarray(th[: chain.J]), r, _ptr(u), _ptr(p))
    if J > chain.J:
        uc = np.zeros((chain.m, 3))
        pc = np.zeros((chain.m, 3))
        _load().or_fk_chi(chain.m, np.ascontiguousarray(th[chain.J:]), r, uc, pc)
        u[chain.J:] = uc
        p[chain.J:] = pc
    return r, u, p


def pair_forces(chain: OracleChain, r, pp: PairParams = PairParams(), subset=None):
    """Eqs (02)-(03_9) by brute force: F[n,3] and (E_elec, E_vdw)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    F = np.zeros((chain.n, 3))
    e = np.zeros(2)
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    _load().or_pair_forces(chain.m, r, chain.q, chain.R, chain.eps, C.byref(pp.c()),
                           _ptr(sub), 0 if sub is None else int(sub.size), F, _ptr(e))
    return F, float(e[0]), float(e[1])


def samples(n_orbits: int = 14) -> np.ndarray:
    """Polar geodesic unit-sphere samples Q[N,3] (Sec. 3.4)."""
    lib = _load()
    N = lib.or_samples(int(n_orbits), None)
    Q = np.zeros((N, 3))
    lib.or_samples(int(n_orbits), Q.ctypes.data_as(C.c_void_p))
    return Q


def sasa_forces(chain: OracleChain, r, sp: SasaParams = SasaParams(), Q=None):
    """Algorithm 1 (C-state rules): F[n,3], f_exp[n], E_cav, smallest |d^2-R^2| of any test."""
    if Q is None:
        Q = samples(sp.n_orbits)
    r = np.ascontiguousarray(r, dtype=np.float64)
    F = np.zeros((chain.n, 3))
    f = np.zeros(chain.n)
    e = np.zeros(1)
    mg = np.zeros(1)
    _load().or_sasa_forces(chain.m, r, chain.R, chain.gamma, np.ascontiguousarray(Q), Q.shape[0],
                           C.byref(sp.c()), F, _ptr(f), _ptr(e), _ptr(mg))
    return F, f, float(e[0]), float(mg[0])


def sasa_atoms(r, R, gamma, sp: SasaParams = SasaParams(), Q=None):
    """Algorithm 1 on a free atom set: F[n,3], f_exp[n], E_cav."""
    if Q is None:
        Q = samples(sp.n_orbits)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    F = np.zeros((n, 3))
    f = np.zeros(n)
    e = np.zeros(1)
    _load().or_sasa_atoms(n, r, np.ascontiguousarray(R, dtype=np.float64),
                          np.ascontiguousarray(gamma, dtype=np.float64), np.ascontiguousarray(Q),
                          Q.shape[0], C.byref(sp.c()), F, _ptr(f), _ptr(e))
    return F, f, float(e[0])


def sasa_events(r, R, sp: SasaParams = SasaParams(), Q=None):
    """C-state event counts D[i,j,s] = N (f_{i,j,s} - f_i) and exposed counts, free atom set."""
    if Q is None:
        Q = samples(sp.n_orbits)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    D = np.zeros((n, n, 3), dtype=np.int32)
    ex = np.zeros(n, dtype=np.int32)
    _load().or_sasa_events(n, r, np.ascontiguousarray(R, dtype=np.float64), np.ascontiguousarray(Q),
                           Q.shape[0], C.byref(sp.c()), D, _ptr(ex))
    return D, ex


def sasa_definitional(r, R, sp: SasaParams = SasaParams(), Q=None):
    """Eq (finitediff) by full recount: D[i,j,s] = N (f_{i,j,s} - f_i), exposed counts."""
    if Q is None:
        Q = samples(sp.n_orbits)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    D = np.zeros((n, n, 3), dtype=np.int32)
    ex = np.zeros(n, dtype=np.int32)
    _load().or_sasa_definitional(n, 1, r, np.ascontiguousarray(R, dtype=np.float64),
                                 np.ascontiguousarray(Q), Q.shape[0], C.byref(sp.c()), D, _ptr(ex))
    return D, ex


def torques(chain: OracleChain, r, F, u, p):
    """Eqs (KCM_01)-(KCM_06): tau_j = u_j . sum_{a downstream of j} (r_a - p_j) x F_a.

    With side-chain joints (u, p of 3m rows) the chi torques follow, each over
    its residue's branch HB1..HB3."""
    J = len(u)
    tau = np.zeros(J)
    r = np.ascontiguousarray(r, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    tb = np.zeros(chain.J)
    _load().or_torques(chain.m, r, F, np.ascontiguousarray(u[: chain.J]), np.ascontiguousarray(p[: chain.J]), tb)
    tau[: chain.J] = tb
    if J > chain.J:
        tc = np.zeros(chain.m)
        _load().or_torques_chi(chain.m, r, F, np.ascontiguousarray(u[chain.J:]), np.ascontiguousarray(p[chain.J:]), tc)
        tau[chain.J:] = tc
    return tau


def step(tau, theta, mask=None, rule: StepRule = StepRule.CAPPED, kappa: float = 1e-3, s: float = 1e-3):
    """Eq (KCM_07) + angle update: returns (theta_new, dtheta, max|dtheta|)."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    th = np.array(theta, dtype=np.float64, copy=True)
    d = np.zeros_like(th)
    mx = np.zeros(1)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    _load().or_step(th.size, tau, _ptr(mk), int(rule), float(kappa), float(s), th, _ptr(d), _ptr(mx))
    return th, d, float(mx[0])


def iterate(chain: OracleChain, theta, pp: PairParams = PairParams(), sp: SasaParams = SasaParams(),
            terms: str = "elec+vdw+cav", mask=None, rule: StepRule = StepRule.CAPPED,
            kappa: float = 1e-3, s: float = 1e-3, Q=None):
    """One KCM iteration (Fig. 5 steps 4-8): FK, forces, torques, step.

    Returns a dict with r, F (total), F_pair, F_cav, tau, dtheta, theta (new),
    energies and the SASA decision margin.
    """
    r, u, p = fk(chain, theta)
    F = np.zeros((chain.n, 3))
    out = {"r": r, "u": u, "p": p}
    Fp = np.zeros((chain.n, 3))
    Ee = Ev = Ec = 0.0
    mg = np.inf
    if "elec" in terms or "vdw" in terms:
        pp2 = pp
        if "elec" not in terms or "vdw" not in terms:
            raise ValueError("the oracle evaluates elec and vdw together")
        Fp, Ee, Ev = pair_forces(chain, r, pp2)
    Fc = np.zeros((chain.n, 3))
    if "cav" in terms:
        Fc, fexp, Ec, mg = sasa_forces(chain, r, sp, Q)
        out["f_exp"] = fexp
    F = Fp + Fc
    tau = torques(chain, r, F, u, p)
    th_new, d, mx = step(tau, theta, mask, rule, kappa, s)
    out.update(F=F, F_pair=Fp, F_cav=Fc, tau=tau, dtheta=d, theta=th_new, max_dtheta=mx,
               E_elec=Ee, E_vdw=Ev, E_cav=Ec, margin=mg)
    return out


def threads() -> int:
    return int(_load().or_threads())


def fk_extend(chain: OracleChain, k: int, M, p, phi: float, psi: float):
    """One residue of the kinematics (for growing start conformations): atoms of
    links 2k+1 and 2k+2 (slots 2..9 of residue k, then slots 0..1 of residue
    k+1) from the rotation M of link 2k and the point p of joint 2k; returns
    (positions, rotation of link 2k+2, point of joint 2k+2)."""
    pos = np.zeros((10, 3))
    Mn = np.zeros(9)
    pn = np.zeros(3)
    w = _load().or_fk_extend(chain.m, chain.r0, int(k), np.ascontiguousarray(M, dtype=np.float64).reshape(9),
                             np.ascontiguousarray(p, dtype=np.float64), float(phi), float(psi), pos, Mn, pn)
    return pos[:w], Mn.reshape(3, 3), pn


def fk_prefix(chain: OracleChain, theta, k: int):
    """Positions of the first k residues (they depend on theta[:2k] only)."""
    th = np.ascontiguousarray(theta[: 2 * k], dtype=np.float64)
    r = np.zeros((APR * k, 3))
    _load().or_fk(int(k), np.ascontiguousarray(chain.r0[: APR * k]), th, r, None, None)
    return r
