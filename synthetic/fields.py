"""Initial conserved fields (inputs only).

Units follow the paper's dimensionless formulation: density by the reference density,
velocity by the reference speed of sound, pressure and energy by rho_ref a_ref^2, so the
reference state has p = 1/gamma and T = gamma p / rho = 1. Every field is returned as a
float64 array ``q`` of shape ``(5, nk, nj, ni)`` holding
(rho, rho u, rho v, rho w, e) with e = p/(gamma-1) + rho |u|^2 / 2 (the System-I total
energy per unit volume).
"""
from __future__ import annotations

import math

import numpy as np


def conserved_from_primitive(rho, u, v, w, p, gamma):
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, e]).astype(np.float64))


def uniform_field(shape, rho, vel, p, gamma):
    nk, nj, ni = shape
    one = np.ones((nk, nj, ni))
    return conserved_from_primitive(rho * one, vel[0] * one, vel[1] * one, vel[2] * one,
                                    p * one, gamma)


def tgv_field(xyz, gamma=1.4, v0=0.1, seed=0, noise=1e-6):
    """Taylor-Green vortex on the (2 pi)^3 box.

    u = V0 sin x cos y cos z, v = -V0 cos x sin y cos z, w = 0,
    p = 1/gamma + V0^2/16 (cos 2x + cos 2y)(cos 2z + 2), T = 1 (so rho = gamma p).
    Tiny seeded noise V0*noise*U(-1, 1) is added to u, v, w in that order, each drawn as
    one i-fastest flat array from numpy's default_rng(seed)."""
    x, y, z = xyz
    u = v0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -v0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = 1.0 / gamma + (v0 * v0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = gamma * p
    if noise:
        rng = np.random.default_rng(seed)
        amp = noise * v0
        u = u + amp * rng.uniform(-1.0, 1.0, size=u.size).reshape(u.shape)
        v = v + amp * rng.uniform(-1.0, 1.0, size=v.size).reshape(v.shape)
        w = w + amp * rng.uniform(-1.0, 1.0, size=w.size).reshape(w.shape)
    return conserved_from_primitive(rho, u, v, w, p, gamma)


def jet_field(xyz, gamma=1.4, mach_jet=1.4, u_inf=0.05, seed=0, n_rings=8,
              amplitude=0.01, shear_theta=0.025, ring_sigma=0.1):
    """Perfectly expanded round jet (pressure and temperature ratios 1) with seeded
    axisymmetric vortex-ring perturbations.

    Mean axial velocity U(r) = U_inf + (U_j - U_inf) (1 + tanh((0.5 - r)/(2 theta)))/2 with
    momentum thickness theta = shear_theta, extended along the whole domain. rho = 1,
    p = 1/gamma. Each ring n has centre x_n ~ U(0.5, 10), radius 0.5, random sign s_n, and
    Stokes stream function psi_n = s_n r^2 exp(-((x-x_n)^2 + (r-0.5)^2)/sigma^2), giving
    the divergence-free perturbation u_x = (1/r) dpsi/dr, u_r = -(1/r) dpsi/dx. The summed
    perturbation is scaled so that its largest magnitude equals amplitude * U_j."""
    x, y, z = xyz
    r = np.sqrt(y * y + z * z)
    uj = mach_jet
    ubar = u_inf + (uj - u_inf) * 0.5 * (1.0 + np.tanh((0.5 - r) / (2.0 * shear_theta)))
    rng = np.random.default_rng(seed)
    xc = rng.uniform(0.5, 10.0, size=n_rings)
    sign = np.where(rng.uniform(0.0, 1.0, size=n_rings) < 0.5, -1.0, 1.0)
    ux = np.zeros_like(r)
    ur = np.zeros_like(r)
    s2 = ring_sigma * ring_sigma
    for n in range(n_rings):
        g = np.exp(-((x - xc[n]) ** 2 + (r - 0.5) ** 2) / s2)
        # (1/r) d/dr [r^2 g] = g (2 - 2 r (r - 0.5)/s2);  -(1/r) d/dx [r^2 g] = 2 r (x-xc) g / s2
        ux += sign[n] * g * (2.0 - 2.0 * r * (r - 0.5) / s2)
        ur += sign[n] * 2.0 * r * (x - xc[n]) * g / s2
    mag = np.sqrt(ux * ux + ur * ur).max()
    if mag > 0:
        scale = amplitude * uj / mag
        ux *= scale
        ur *= scale
    with np.errstate(invalid="ignore", divide="ignore"):
        cth = np.where(r > 0, y / np.where(r > 0, r, 1.0), 0.0)
        sth = np.where(r > 0, z / np.where(r > 0, r, 1.0), 0.0)
    u = ubar + ux
    v = ur * cth
    w = ur * sth
    rho = np.ones_like(r)
    p = np.full_like(r, 1.0 / gamma)
    return conserved_from_primitive(rho, u, v, w, p, gamma)
