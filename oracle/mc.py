"""Monte Carlo minimization over the KCM descent (test infrastructure only).

The paper's list of improvements to the search names a hybrid of Monte Carlo
sampling and steepest descent (Sec. 4, the implementation notes on the
search phase).  The form written here is Monte Carlo minimization (Li and
Scheraga, 1987): every trial perturbs the accepted dihedrals, descends from
there with KCM steps (eq KCM_07), and keeps the descended state by the
Metropolis rule on its energy (Metropolis et al., 1953).  Plain Python loops
over ``oracle.iterate``; the random numbers are inputs.
"""
from __future__ import annotations

import math

import numpy as np

from .oracle import PairParams, SasaParams, StepRule, iterate


def _wrap(t):
    """Angles into (-pi, pi]; an angle already inside comes back unchanged."""
    t = np.asarray(t, dtype=np.float64)
    t = t - 2.0 * np.pi * np.floor((t + np.pi) / (2.0 * np.pi))
    return np.where(t <= -np.pi, t + 2.0 * np.pi, t)


def _energy(o, terms):
    e = 0.0
    if "elec" in terms:
        e += o["E_elec"] + o["E_vdw"]
    if "cav" in terms:
        e += o["E_cav"]
    return e


def mc_minimize(chain, theta, delta, u, n_descent: int, kT: float, pp: PairParams = PairParams(),
                sp: SasaParams = SasaParams(), terms: str = "elec+vdw+cav", mask=None,
                rule: StepRule = StepRule.CAPPED, kappa: float = 1e-3, s: float = 1e-3):
    """Monte Carlo minimization from theta.

    delta[t, j]: perturbation of joint j in trial t (masked joints ignore it);
    u[t]: uniform [0, 1) number of trial t's Metropolis test.  The starting
    state is theta itself with its energy.  Trial t: theta' = wrap(accepted +
    delta[t]); n_descent KCM iterations from theta'; E' = energy at the
    result.  Accepted when E' <= E or u[t] < exp(-(E' - E)/kT) (kT = 0: only
    downhill).  Returns the accepted and the lowest state with energies, the
    starting energy, the number of accepted trials, and per trial the
    smallest distance of the decision from its threshold."""
    th0 = _wrap(theta)
    J = th0.size
    mk = np.ones(J, np.uint8) if mask is None else np.asarray(mask, dtype=np.uint8)
    d = np.asarray(delta, dtype=np.float64).reshape(-1, J)
    u = np.asarray(u, dtype=np.float64)

    def run(th, k):
        # k descent iterations, then the energy of the reached angles
        for _ in range(k):
            th = iterate(chain, th, pp, sp, terms, mask, rule, kappa, s)["theta"]
        return th, _energy(iterate(chain, th, pp, sp, terms, mask, rule, kappa, s), terms)

    _, e0 = run(th0, 0)
    acc_th, acc_e = th0, e0
    best_th, best_e = th0, e0
    accepted = 0
    margins = []
    for t in range(d.shape[0]):
        prop = np.where(mk != 0, _wrap(acc_th + d[t]), acc_th)
        th, e = run(prop, n_descent)
        de = e - acc_e
        if de <= 0.0:
            ok = True
            margins.append(abs(de))
        elif kT > 0.0:
            p = math.exp(-de / kT)
            ok = u[t] < p
            margins.append(min(abs(de), abs(u[t] - p)))
        else:
            ok = False
            margins.append(abs(de))
        if e < best_e:
            best_th, best_e = th, e
        if ok:
            acc_th, acc_e = th, e
            accepted += 1
    return {"theta": acc_th, "E": acc_e, "theta_best": best_th, "E_best": best_e, "E_start": e0,
            "accepted": accepted, "margins": np.array(margins)}
