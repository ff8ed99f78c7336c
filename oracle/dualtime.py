"""Plain FP64 reference of dual time stepping (test infrastructure only: imported by tests/,
never by the library).

The paper's Concluding Remarks find its explicit time step a hundred times smaller than the
literature's and ask for a preconditioned dual-time procedure. This reference takes the
standard dual-time construction on the paper's own residual and stage scheme (the low-Mach
preconditioning of the pseudo-time term is not part of it):

* physical time by the second-order backward difference, or backward Euler for a first step
  without history: (a0 Q^{n+1} + a1 Q^n + a2 Q^{n-1}) / dt + J RHS(Q^{n+1}) = 0, with
  (a0, a1, a2) = (3/2, -2, 1/2), respectively (1, -1, 0);
* each physical step solved by `subiters` pseudo-time iterations of the five-stage scheme
  (alpha = 1/4, 1/6, 3/8, 1/2, 1), with the local pseudo-time step
  dtau_i = cfl_tau J^-1 / (Lam_xi + Lam_eta + Lam_zeta) at each updated node, from the state at
  the start of the iteration;
* the physical-time term point-implicit in every stage:
  Q^(l) = [Q^(0) - alpha_l dtau (J RHS(Q^(l-1)) + (a1 Q^n + a2 Q^{n-1})/dt)]
          / (1 + alpha_l dtau a0 / dt),
  at updated nodes, then the boundary conditions;
* monitor: the root mean square over updated nodes of the mass component of the unsteady
  residual (a0 Q + a1 Q^n + a2 Q^{n-1})/dt + J RHS(Q) at the start of every iteration.

At convergence of the pseudo-time iterations the stage details drop out and the step is the
backward-difference step of the paper's semi-discrete system.
"""
from __future__ import annotations

import numpy as np

from . import primitives

ALPHA = (0.25, 1.0 / 6.0, 0.375, 0.5, 1.0)
BDF2 = (1.5, -2.0, 0.5)
BDF1 = (1.0, -1.0, 0.0)


def updated_mask(p):
    """Nodes the time integration updates (those not on a non-periodic face)."""
    m = np.ones(p.shape, dtype=bool)
    per = (p.bc[0] == 0, p.bc[2] == 0, p.bc[4] == 0)
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        if not per[d]:
            sl = [slice(None)] * 3
            sl[ax] = 0
            m[tuple(sl)] = False
            sl[ax] = p.shape[ax] - 1
            m[tuple(sl)] = False
    return m


def local_pseudo_step(o, q, cfl_tau):
    """cfl_tau J^-1 / sum_d (|S_d . u| + a |S_d|) at updated nodes, 0 elsewhere."""
    p = o.p
    x = primitives(q, p.gamma)
    a = np.sqrt(p.gamma * x[4] / x[0])
    lam = np.zeros(p.shape)
    for d in range(3):
        sx, sy, sz = o.S[3 * d], o.S[3 * d + 1], o.S[3 * d + 2]
        lam += np.abs(sx * x[1] + sy * x[2] + sz * x[3]) + a * np.sqrt(sx * sx + sy * sy + sz * sz)
    upd = updated_mask(p)
    return np.where(upd, cfl_tau * o.jinv / np.where(upd, lam, 1.0), 0.0)


def dual_step(o, q, q_prev, nsteps, dt, subiters, cfl_tau):
    """nsteps physical steps of size dt of the oracle `o` from q (Q^n) with history q_prev
    (Q^{n-1}, or None: the first step is backward Euler). Returns (q, q_prev, residuals
    [nsteps][subiters])."""
    p = o.p
    upd = updated_mask(p)
    J = np.where(upd, 1.0 / np.where(upd, o.jinv, 1.0), 0.0)
    q = np.array(q, dtype=np.float64, copy=True)
    prev = None if q_prev is None else np.array(q_prev, dtype=np.float64, copy=True)
    res = np.zeros((nsteps, subiters))
    nupd = np.count_nonzero(upd)
    for n in range(nsteps):
        a0, a1, a2 = BDF1 if prev is None else BDF2
        qn = q.copy()
        hist = a1 * qn + (0.0 if prev is None else a2 * prev)
        for s in range(subiters):
            q0 = q.copy()
            dtau = local_pseudo_step(o, q0, cfl_tau)
            for l, al in enumerate(ALPHA):
                rhs = o.residual(q)
                jr = J[None] * rhs
                if l == 0:
                    rstar = (a0 * q0[0] + hist[0]) / dt + jr[0]
                    res[n, s] = np.sqrt(np.sum(np.where(upd, rstar, 0.0) ** 2) / nupd)
                new = (q0 - al * dtau[None] * (jr + hist / dt)) / (1.0 + al * dtau[None] * a0 / dt)
                q = np.where(upd[None], new, q)
                q = o.apply_bc(q)
        prev = qn
    return q, prev, res
