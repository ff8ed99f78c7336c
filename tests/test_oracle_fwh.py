"""Pins of the Ffowcs Williams-Hawkings reference (oracle/fwh.py) against exact solutions.

* Monopole: the velocity potential phi = -f(t - R/c0)/(4 pi R) of a point source, with
  u = grad phi and p' = -rho0 d phi/dt = rho0 f'(t - R/c0)/(4 pi R), sampled on a sphere around
  the source at small amplitude (the loading's rho u u is second order): the surface integral
  must give the exact far-field p' at an outside observer, converging at second order when the
  surface and the sampling are refined together (midpoint quadrature, central differences,
  linear interpolation in time).
* Gauss: a uniform pressure offset c with the fluid at rest gives L = c n, whose integral
  sum n . r_hat dS / r^2 is 0 for an outside observer and -4 pi at the centre, so p' = 0
  outside and -c at the centre.
* A fluid at rest at p0 gives exactly 0.
* The control surface on a polar jet grid: the lateral cylinder's area 2 pi r L and normal
  r_hat, the caps' areas pi r^2 and normals -/+ x_hat.
* Retarded times outside the samples are counted.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fwh
import synthetic as sy
from synthetic.grids import jet_grid

RHO0, C0, GAMMA = 1.2, 1.3, 1.4   # non-unit, so a misplaced factor shows
P0 = 1.0 / GAMMA


def sphere(a, nth, nph):
    th = (np.arange(nth) + 0.5) * math.pi / nth
    ph = np.arange(nph) * 2 * math.pi / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    n = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1).reshape(-1, 3)
    dS = (a * a * np.sin(T) * (math.pi / nth) * (2 * math.pi / nph)).reshape(-1)
    return a * n, n, dS


def monopole_samples(y, A, omega, taus):
    R = np.sqrt(np.sum(y * y, axis=1))
    Rh = y / R[:, None]
    tr = taus[:, None] - R[None, :] / C0
    f = A * np.sin(omega * tr)
    fd = A * omega * np.cos(omega * tr)
    ur = f / (4 * math.pi * R * R) + fd / (4 * math.pi * R * C0)
    pp = RHO0 * fd / (4 * math.pi * R)
    u = ur[..., None] * Rh[None]
    return RHO0 + pp / C0 ** 2, u, P0 + pp


def monopole_error(nth, nph, per_period):
    A, omega = 1e-6, 2 * math.pi
    y, n, dS = sphere(1.0, nth, nph)
    dtau = 1.0 / per_period
    taus = np.arange(0, int(4.0 / dtau) + 1) * dtau
    rho, u, p = monopole_samples(y, A, omega, taus)
    D = 10.0
    x = np.array([[2.0, 2.0, 1.0]]) / 3.0 * D
    times = D / C0 + np.linspace(1.3, 2.3, 17)
    got, scale, skipped = fwh.fwh_pressure(y, n, dS, rho, u, p, 0.0, dtau, RHO0, C0, P0, x, times)
    exact = RHO0 * A * omega * np.cos(omega * (times - D / C0)) / (4 * math.pi * D)
    assert skipped == 0
    return np.max(np.abs(got[0] - exact)) / np.max(np.abs(exact))


def test_monopole_far_field_second_order():
    e1 = monopole_error(24, 48, 32)
    e2 = monopole_error(48, 96, 64)
    print("monopole errors", e1, e2)
    assert e2 < 5e-3
    assert e1 / e2 > 3.0


def test_gauss_uniform_pressure_offset():
    y, n, dS = sphere(1.0, 40, 80)
    M = 8
    c = 0.01
    rho = np.full((M, len(dS)), RHO0)
    u = np.zeros((M, len(dS), 3))
    p = np.full((M, len(dS)), P0 + c)
    obs = np.array([[5.0, 0.0, 0.0], [0.0, -3.0, 4.0], [0.0, 0.0, 0.0]])
    times = np.array([6.5])   # retarded times inside the samples for every node
    got, _, skipped = fwh.fwh_pressure(y, n, dS, rho, u, p, 0.0, 1.0, RHO0, C0, P0, obs, times)
    assert skipped == 0
    assert abs(got[0, 0]) < 1e-3 * c and abs(got[1, 0]) < 1e-3 * c
    assert got[2, 0] == pytest.approx(-c, rel=1e-3)


def test_fluid_at_rest_is_silent():
    y, n, dS = sphere(1.0, 8, 16)
    M = 6
    rho = np.full((M, len(dS)), RHO0)
    u = np.zeros((M, len(dS), 3))
    p = np.full((M, len(dS)), P0)
    got, _, _ = fwh.fwh_pressure(y, n, dS, rho, u, p, 0.0, 1.0, RHO0, C0, P0,
                                 np.array([[7.0, 1.0, 0.0]]), np.array([9.0]))
    assert got[0, 0] == 0.0


def test_time_derivative_exact_on_quadratics():
    t = np.arange(7) * 0.3
    f = 2.0 - 1.5 * t + 0.7 * t * t
    np.testing.assert_allclose(fwh.time_derivative(f, 0.3), -1.5 + 1.4 * t, rtol=0, atol=1e-13)


def test_jet_surface_geometry():
    n = (48, 40, 64)
    xyz, _ = jet_grid(n)
    p = sy.jet_params(n)
    o = oracle.Oracle(p, xyz)
    i1, i2, js = 4, 40, 24
    ids, y, nrm, dS = fwh.jet_surface(o.S, xyz, i1, i2, js)
    nlat = (i2 - i1 + 1) * n[2]
    ncap = (js + 1) * n[2]
    assert len(ids) == nlat + 2 * ncap
    r = math.hypot(xyz[1, 0, js, 0], xyz[2, 0, js, 0])
    L = xyz[0, 0, 0, i2] - xyz[0, 0, 0, i1]
    lat = dS[:nlat].sum()
    assert lat == pytest.approx(2 * math.pi * r * L, rel=2e-3)
    for cap in (slice(nlat, nlat + ncap), slice(nlat + ncap, None)):
        assert dS[cap].sum() == pytest.approx(math.pi * r * r, rel=1e-2)
    radial = y[:nlat, 1:] / np.sqrt(np.sum(y[:nlat, 1:] ** 2, axis=1))[:, None]
    assert np.max(np.abs(nrm[:nlat, 1:] - radial)) < 1e-2 and np.max(np.abs(nrm[:nlat, 0])) < 2e-2
    # (the axis nodes, j = 0, carry a round-off area in an arbitrary direction)
    big = dS > 1e-9 * dS.max()
    up = nrm[nlat:nlat + ncap][big[nlat:nlat + ncap]]
    dn = nrm[nlat + ncap:][big[nlat + ncap:]]
    assert np.allclose(up[:, 0], -1.0, atol=1e-3) and np.allclose(dn[:, 0], 1.0, atol=1e-3)


def test_retarded_times_outside_the_samples_are_counted():
    y, n, dS = sphere(1.0, 6, 12)
    M = 5
    rho = np.full((M, len(dS)), RHO0)
    u = np.zeros((M, len(dS), 3))
    p = np.full((M, len(dS)), P0)
    # observer 10 away: retarded times t - r/c0 with r in [9, 11], r/c0 in [6.9, 8.5];
    # the samples cover [0, 4]
    _, _, skipped = fwh.fwh_pressure(y, n, dS, rho, u, p, 0.0, 1.0, RHO0, C0, P0,
                                     np.array([[10.0, 0.0, 0.0]]), np.array([5.0, 10.0, 16.0]))
    assert skipped == 2 * len(dS)   # t = 5 (all before the first sample) and 16 (all after)
