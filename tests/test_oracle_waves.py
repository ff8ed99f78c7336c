"""Closed-form pins of the oracle's central flux, fourth-difference dissipation, scaled
spectral radius, compact viscous flux and five-stage Runge-Kutta scheme.

On a uniform Cartesian periodic grid of spacing h, a small-amplitude wave exp(i k x)
evolves, to first order in its amplitude A, by the amplification factor P(dt L) per step:

* entropy wave (rho = 1 + A sin kx, uniform u = (U,0,0) and p, inviscid, no SGS):
  L = -(1/h) [i U sin(theta) + 16 k4 Lb sin^4(theta/2)], Lb = (|U|+a) + 2 sqrt((|U|+a) a),
* shear wave (v = A sin kx, rho = 1, p = 1/gamma, no SGS):
  L = -(mu(1)/Re)(4/h^2) sin^2(theta/2) - (48 a k4 / h) sin^4(theta/2),

with theta = k h, a = 1 and P(z) the stability polynomial of the five-stage scheme with
alpha = (1/4, 1/6, 3/8, 1/2, 1): P(z) = 1 + z + z^2/2 + 3 z^3/16 + z^4/32 + z^5/128.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import synthetic as sy
from golden_data import paper_constants
from synthetic.grids import cartesian_grid


# The five stage coefficients as the paper states them (Time Marching Method).
ALPHAS = tuple(paper_constants()["rk_alpha"])


def P5(z):
    # Nested form of the five-stage scheme applied to dq/dt = (L) q:
    # q1 = 1 + a1 z, q2 = 1 + a2 z q1, ... ; independent of the oracle's C code.
    q = 1.0
    for a in ALPHAS:
        q = 1.0 + a * z * q
    return q


def test_stability_polynomial_coefficients_and_imaginary_axis_limit():
    # Expand the nested form at a few points and compare with the closed polynomial.
    for z in (0.3, -1.2 + 0.4j, 2.5j):
        poly = 1 + z + z ** 2 / 2 + 3 * z ** 3 / 16 + z ** 4 / 32 + z ** 5 / 128
        assert abs(P5(z) - poly) < 1e-14
    # On the imaginary axis |P(iy)|^2 - 1 = y^4 (y^2 - 8)^2 (y^2 - 16) / 16384, so the
    # scheme is stable for |y| <= 4, with neutral points at y = 2 sqrt(2) (the bound the
    # paper quotes, which holds but is not sharp) and y = 4.
    for y in np.linspace(0.01, 4.0, 400):
        lhs = abs(P5(1j * y)) ** 2 - 1.0
        rhs = y ** 4 * (y * y - 8) ** 2 * (y * y - 16) / 16384.0
        assert abs(lhs - rhs) < 1e-12
        assert abs(P5(1j * y)) <= 1.0 + 1e-14
    assert abs(abs(P5(2 * math.sqrt(2) * 1j)) - 1.0) < 1e-14
    assert abs(abs(P5(4j)) - 1.0) < 1e-14
    assert abs(P5(4.001j)) > 1.0
    assert abs(P5(3.9j)) < 1.0


def _periodic_line(nx, h, ny=4):
    xyz, sh = cartesian_grid((nx, ny, ny), (h, h, h))
    return xyz, sh


@pytest.mark.parametrize("k4", [0.0, 0.016])
@pytest.mark.parametrize("mode", [1, 3, 5])
def test_entropy_wave_amplification(k4, mode):
    nx, h, U = 16, 0.2, 0.3
    xyz, sh = _periodic_line(nx, h)
    p = sy.box_params((nx, 4, 4), sh, re_acoustic=0.0, cs=0.0, k2=0.25, k4=k4)
    o = oracle.Oracle(p, xyz)
    x = xyz[0]
    A = 1e-7
    kx = 2 * math.pi * mode / (nx * h)
    theta = kx * h
    rho = 1.0 + A * np.sin(kx * x)
    q = sy.conserved_from_primitive(rho, np.full_like(x, U), 0 * x, 0 * x,
                                    np.full_like(x, 1.0 / p.gamma), p.gamma)
    a = 1.0
    lb = (abs(U) + a) + 2.0 * math.sqrt((abs(U) + a) * a)
    L = -(1.0 / h) * (1j * U * math.sin(theta) + 16.0 * k4 * lb * math.sin(theta / 2) ** 4)
    dt = 0.6 * h / (U + a)
    nsteps = 4
    q2, _ = o.step(q, nsteps, cfl=0.0, dt_fixed=dt)
    g = P5(dt * L) ** nsteps
    expect = A * np.imag(g * np.exp(1j * kx * x))
    got = q2[0] - 1.0
    err = np.abs(got - expect).max() / A
    assert err < 2e-6, err
    # The prediction is not trivially satisfied: the wave moved and (k4 > 0) decayed.
    assert np.abs(got - (rho - 1.0)).max() / A > 1e-2


def test_entropy_wave_detects_wrong_dissipation_constant():
    """The tolerance above is tight enough to tell k4 = 0.016 from k4 = 1/64."""
    nx, h, U, mode = 16, 0.2, 0.3, 5
    kx = 2 * math.pi * mode / (nx * h)
    theta = kx * h
    a = 1.0
    lb = (abs(U) + a) + 2.0 * math.sqrt((abs(U) + a) * a)
    dt = 0.6 * h / (U + a)
    g1 = P5(dt * -(1.0 / h) * (1j * U * math.sin(theta) + 16 * 0.016 * lb * math.sin(theta / 2) ** 4)) ** 4
    g2 = P5(dt * -(1.0 / h) * (1j * U * math.sin(theta) + 16 / 64 * lb * math.sin(theta / 2) ** 4)) ** 4
    assert abs(g1 - g2) > 1e-3


@pytest.mark.parametrize("mode", [1, 2, 6])
def test_shear_wave_amplification(mode):
    nx, h = 16, 0.25
    xyz, sh = _periodic_line(nx, h)
    re = 2.0
    k4 = 0.016
    p = sy.box_params((nx, 4, 4), sh, re_acoustic=re, cs=0.0, k2=0.25, k4=k4)
    o = oracle.Oracle(p, xyz)
    x = xyz[0]
    A = 1e-7
    kx = 2 * math.pi * mode / (nx * h)
    theta = kx * h
    v = A * np.sin(kx * x)
    q = sy.conserved_from_primitive(np.ones_like(x), 0 * x, v, 0 * x,
                                    np.full_like(x, 1.0 / p.gamma), p.gamma)
    a = 1.0
    L = -(1.0 / re) * (4.0 / h ** 2) * math.sin(theta / 2) ** 2 \
        - (48.0 * a * k4 / h) * math.sin(theta / 2) ** 4
    dt = 0.3 * min(h / a, re * h * h / 4)
    nsteps = 5
    q2, _ = o.step(q, nsteps, cfl=0.0, dt_fixed=dt)
    expect = A * np.imag(P5(dt * L) ** nsteps * np.exp(1j * kx * x))
    got = q2[2]
    err = np.abs(got - expect).max() / A
    assert err < 2e-6, err
    assert np.abs(got - v).max() / A > 1e-2


def test_tgv_initial_kinetic_energy_decay_rate():
    """dK/dt(0) = -6 nu K(0) for the Taylor-Green vortex (K = V0^2/8), nu = 1/Re_a in
    acoustic units, with dissipation and SGS switched off. Compressibility (M = 0.1) and
    the grid (theta = 2 pi / 32) perturb it by about 1 %."""
    n = 32
    p, xyz, q = sy.make_case("tgv", n)
    re = 400.0
    p = p.replace(k2=0.0, k4=0.0, cs=0.0, re_acoustic=re)
    o = oracle.Oracle(p, xyz)
    k0 = o.diagnostics(q)[0]
    assert k0 == pytest.approx(0.1 ** 2 / 8, rel=1e-4)
    dt = 0.02
    qa, _ = o.step(q, 1, cfl=0.0, dt_fixed=dt)
    qb, _ = o.step(qa, 1, cfl=0.0, dt_fixed=dt)
    k1 = o.diagnostics(qa)[0]
    k2 = o.diagnostics(qb)[0]
    # Second-order one-sided estimate of dK/dt at t = 0.
    dkdt = (-3 * k0 + 4 * k1 - k2) / (2 * dt)
    expect = -6.0 / re * k0
    assert dkdt == pytest.approx(expect, rel=0.03)
