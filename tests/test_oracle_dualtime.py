"""Pins of the dual-time reference (oracle/dualtime.py).

On a uniform Cartesian periodic grid of spacing h, the entropy wave rho = 1 + A sin(kx) with
uniform velocity (U, 0, 0) and pressure, no viscosity, no subgrid model and k4 = 0, is an exact
discrete solution whose density mode exp(ikx) obeys d rho_hat/dt = L rho_hat with the
central-difference symbol L = -(i U / h) sin(kh) (pressure uniform, so the sensor and eps2
vanish). Once the pseudo-time iterations have converged, a physical step is therefore the
backward-difference recurrence of that mode:

* first step, backward Euler: (1 - dt L) rho_hat^1 = rho_hat^0;
* then the second-order backward difference:
  (3/2 - dt L) rho_hat^{n+1} = 2 rho_hat^n - 1/2 rho_hat^{n-1},

here at a physical time step five times the explicit CFL limit. The pins check that
recurrence to 1e-10 of the amplitude after three steps (a wrong backward-difference
coefficient, a dropped point-implicit denominator or a wrong history term each breaks it by
orders of magnitude more), and that the unsteady residual falls geometrically with the
pseudo-time iterations.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
from oracle import dualtime
import synthetic as sy
from synthetic.grids import cartesian_grid


def _wave_case(nx=16, h=0.2, U=0.3, mode=2, A=1e-3):
    xyz, sh = cartesian_grid((nx, 4, 4), (h, h, h))
    p = sy.box_params((nx, 4, 4), sh, re_acoustic=0.0, cs=0.0, k2=0.25, k4=0.0)
    o = oracle.Oracle(p, xyz)
    x = xyz[0]
    kx = 2 * math.pi * mode / (nx * h)
    q = sy.conserved_from_primitive(1.0 + A * np.sin(kx * x), np.full_like(x, U), 0 * x, 0 * x,
                                    np.full_like(x, 1.0 / p.gamma), p.gamma)
    L = -(1j * U / h) * math.sin(kx * h)
    return o, p, q, x, kx, L, A


def test_converged_dual_time_is_the_backward_difference_recurrence():
    o, p, q, x, kx, L, A = _wave_case()
    dt_explicit = o.dt(q, 1.0)
    dt = 5.0 * dt_explicit
    got, prev, res = dualtime.dual_step(o, q, None, 3, dt, 80, 2.5)
    rh = [1.0 + 0j]
    rh.append(rh[0] / (1.0 - dt * L))
    for _ in range(2):
        rh.append((2.0 * rh[-1] - 0.5 * rh[-2]) / (1.5 - dt * L))
    want = 1.0 + A * np.imag(rh[-1] * np.exp(1j * kx * x))
    err = np.abs(got[0] - want).max()
    print("dual-time recurrence error / A", err / A, "residual", res[:, [0, -1]])
    assert err <= 1e-10 * A
    # the history passed back is Q^n of the last step
    want_prev = 1.0 + A * np.imag(rh[-2] * np.exp(1j * kx * x))
    assert np.abs(prev[0] - want_prev).max() <= 1e-10 * A
    # velocity and pressure stay uniform
    xp = oracle.primitives(got, p.gamma)
    assert np.abs(xp[1] - 0.3).max() < 1e-12 and np.abs(xp[4] - 1 / p.gamma).max() < 1e-12


def test_pseudo_time_residual_falls_geometrically():
    o, p, q, x, kx, L, A = _wave_case()
    dt = 5.0 * o.dt(q, 1.0)
    _, _, res = dualtime.dual_step(o, q, None, 2, dt, 20, 2.5)
    for n in range(2):
        r = res[n]
        print("residual history", r)
        # a steady contraction (about 2/3 per iteration at this pseudo-time step), above the
        # round-off floor, which 20 iterations do not reach
        ratios = r[1:] / r[:-1]
        assert np.all(ratios < 0.75) and r[-1] < 1e-3 * r[0]


def test_history_argument_takes_the_second_order_step_at_once():
    o, p, q, x, kx, L, A = _wave_case()
    dt = 5.0 * o.dt(q, 1.0)
    q1, prev, _ = dualtime.dual_step(o, q, None, 1, dt, 80, 2.5)
    # two steps in one call equal one step then one more with the history passed back
    a, _, _ = dualtime.dual_step(o, q, None, 2, dt, 80, 2.5)
    b, _, _ = dualtime.dual_step(o, q1, prev, 1, dt, 80, 2.5)
    assert np.array_equal(a, b)


def test_one_pseudo_time_iteration_follows_the_point_implicit_stages():
    """One pseudo-time iteration of the first (backward Euler) step: with J RHS = -L rho_hat for
    the mode and the pseudo-time step dtau = cfl_tau h / (|U| + 3a) of the uniform base state
    (the density perturbation changes it at second order in A), the stages are the scalar
    recursion q_l = [q_0 + alpha_l dtau (L q_{l-1} + q^n / dt)] / (1 + alpha_l dtau / dt)."""
    o, p, q, x, kx, L, A = _wave_case(A=1e-7)
    dt = 5.0 * o.dt(q, 1.0)
    cfl_tau = 2.5
    got, _, _ = dualtime.dual_step(o, q, None, 1, dt, 1, cfl_tau)
    h, U, a = 0.2, 0.3, 1.0
    dtau = cfl_tau * h / (abs(U) + 3 * a)
    q0 = qn = 1.0 + 0j
    ql = q0
    for al in dualtime.ALPHA:
        ql = (q0 + al * dtau * (L * ql + qn / dt)) / (1.0 + al * dtau / dt)
    want = 1.0 + A * np.imag(ql * np.exp(1j * kx * x))
    assert np.abs(got[0] - want).max() <= 1e-6 * A
    # the point-implicit denominators matter here: the explicit form is far off
    qe = q0
    for al in dualtime.ALPHA:
        qe = q0 + al * dtau * (L * qe - (qe - qn) / dt)
    assert abs(qe - ql) > 1e-2
