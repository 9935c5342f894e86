"""Shifted, fused and optimistic time stepping (Sec. 5, Techniques 3-5;
Alg. 2), composed from the oracle's predictor and corrector.

Oracle (test infrastructure only).  A step is split at the hull: ``stp`` is
the STP task (predict, extrapolate and integrateVolume brought forward,
Technique 1) and ``corrector`` the Riemann solves, integrateFace and update.
``run_fused`` takes the steps of Alg. 2 in the paper's order: the STP of a
step runs with Delta T_new right after the corrector of the step before
(Delta T_old) and before Delta T_adm of the new state is known; if the
admissible step then turns out smaller, the STP is rerun with
C_dT * Delta T_adm.  Delta T_new then creeps towards C_dT * Delta T_adm.
"""

import torch

from . import step as ostep


def stp(Q, par, dt, s):
    """STP task: (Q~ = Q + dt V, face hull) of every cell (Eq. (3), Table 1)."""
    u = ostep._spatial(Q, s)
    q = ostep.predictor(u, par, dt, s)
    qbar, Fbar = ostep.time_average(q, par, s)
    return ostep.integrate_volume(u, Fbar, dt, s), ostep.extrapolate(qbar, Fbar, s)


def corrector(Qt, tr, par, dt, s):
    """Riemann + Corrector: Q(T + dt) from Q~ and the hull (Eq. (2), (4))."""
    C = Qt.shape[0]
    plus, minus = ostep.neighbor_index(s.n_cells)
    Fp, Fm = [], []
    for i in range(s.dim):
        pi = torch.as_tensor(plus[i])
        mi = torch.as_tensor(minus[i])
        tr_plus = tuple(t[pi] for t in tr[i])
        par_plus = None if par is None else par[pi]
        F = ostep.face_fluxes(tr[i], tr_plus, par, par_plus, i, s)
        Fp.append(F)
        Fm.append(F[mi])
    return ostep.integrate_face(Qt, Fp, Fm, dt, s).reshape(C, -1, s.m)


def admissible_dt(Q, par, cfl, s):
    """Delta T_adm of a state (calcTimeStep, Sec. 3)."""
    return ostep.cfl_dt(ostep.max_wave_speed(Q, par, s), cfl, s)


def run_fused(Q, par, s, steps, cfl, c_dt, creeping=True):
    """Alg. 2 over ``steps`` steps.  Returns (Q, dts used, number of reruns).

    The first STP uses C_dT * Delta T_adm(Q(T)).  Each sweep corrects with
    Delta T_old and predicts with Delta T_new; after the sweep, if
    Delta T_adm < Delta T_new the STP is rerun with Delta T_old = Delta T_new
    = C_dT Delta T_adm.  Then Delta T_old <- Delta T_new and Delta T_new <-
    (Delta T_old + C_dT Delta T_adm) / 2 (creeping average) or C_dT Delta T_adm.
    """
    dt_new = c_dt * admissible_dt(Q, par, cfl, s)
    dt_old = dt_new
    pending = stp(Q, par, dt_new, s)
    used, reruns = [], 0
    for k in range(1, steps + 1):
        Q = corrector(*pending, par, dt_old, s)
        used.append(dt_old)
        if k == steps:
            break
        pending = stp(Q, par, dt_new, s)
        adm = admissible_dt(Q, par, cfl, s)
        if adm < dt_new:                      # the optimistic guess was wrong
            reruns += 1
            dt_new = c_dt * adm
            pending = stp(Q, par, dt_new, s)
        dt_old = dt_new
        dt_new = 0.5 * (dt_old + c_dt * adm) if creeping else c_dt * adm
    return Q, used, reruns
