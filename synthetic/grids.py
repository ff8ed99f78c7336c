"""Structured grid generators (inputs only; no solver arithmetic).

Every grid is returned as a float64 array ``xyz`` of shape ``(3, nk, nj, ni)``: the x, y
and z coordinates of node (i, j, k), i fastest in memory. Periodic directions store
distinct nodes only; the translation that maps the first node onto the one past the last
is returned separately as ``period_shift[direction][component]``.

The jet grids follow the paper's mesh-generation section: a 2-D (x, r) mesh rotated
about the x axis, refined axially near the entrance and radially at the lip line
r = D/2, with x the axial direction (xi), r radial (eta) and theta azimuthal (zeta).
All jet grids, whatever their point counts, sample the same two continuous maps, so a
coarse grid is nested in a fine one of twice the resolution.
"""
from __future__ import annotations

import math

import numpy as np

# Axial map x(s) = Lx (exp(beta s) - 1) / (exp(beta) - 1), s in [0, 1]. With 256 points the
# cell growth is 1.5 % per cell and the first cell is 0.0126 D long, the smallest axial
# spacing quoted for the paper's production grid.
AXIAL_BETA = 255.0 * math.log(1.015)
AXIAL_LENGTH = 36.58

# Radial map: spacing proportional to eps + tanh^2((s - s_lip)/w), which is smallest on the
# lip line r = 0.5. At 128 points the smallest radial cell is 0.005 D. The far boundary
# sits at r = 6 D.
RADIAL_RMAX = 6.0
RADIAL_LIP = 0.5
RADIAL_WIDTH = 0.1
RADIAL_DRMIN_128 = 0.005


def cartesian_periodic_grid(n, length=2.0 * math.pi):
    """Uniform triply periodic box with n[d] nodes per direction and side ``length``.

    Returns (xyz, period_shift)."""
    ni, nj, nk = n
    xs = [length * np.arange(m, dtype=np.float64) / m for m in (ni, nj, nk)]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    xyz = np.stack([x, y, z]).astype(np.float64)
    shift = np.diag([length, length, length]).astype(np.float64)
    return np.ascontiguousarray(xyz), shift


def cartesian_grid(n, spacing, periodic=(True, True, True)):
    """Uniform box with spacing h[d]; a periodic direction wraps after n[d] cells.

    Returns (xyz, period_shift). period_shift rows of non-periodic directions are zero."""
    ni, nj, nk = n
    hs = spacing
    xs = [hs[d] * np.arange(m, dtype=np.float64) for d, m in enumerate((ni, nj, nk))]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    xyz = np.stack([x, y, z]).astype(np.float64)
    shift = np.zeros((3, 3))
    for d, m in enumerate((ni, nj, nk)):
        if periodic[d]:
            shift[d, d] = hs[d] * m
    return np.ascontiguousarray(xyz), shift


def skewed_periodic_grid(n, amplitude=0.3):
    """Smooth, skewed, triply periodic curvilinear grid on a (2 pi)^3 box.

    x = s1 + A sin(s2) sin(s3), y = s2 + A sin(s3) sin(s1), z = s3 + A sin(s1) sin(s2),
    with s_d = 2 pi index_d / n_d. The map is periodic up to a 2 pi translation in each
    direction. Returns (xyz, period_shift)."""
    ni, nj, nk = n
    s = [2.0 * math.pi * np.arange(m, dtype=np.float64) / m for m in (ni, nj, nk)]
    s3, s2, s1 = np.meshgrid(s[2], s[1], s[0], indexing="ij")
    a = amplitude
    x = s1 + a * np.sin(s2) * np.sin(s3)
    y = s2 + a * np.sin(s3) * np.sin(s1)
    z = s3 + a * np.sin(s1) * np.sin(s2)
    xyz = np.ascontiguousarray(np.stack([x, y, z]))
    shift = np.diag([2.0 * math.pi] * 3)
    return xyz, shift


def jet_axial_map(ni):
    s = np.arange(ni, dtype=np.float64) / (ni - 1)
    return AXIAL_LENGTH * np.expm1(AXIAL_BETA * s) / math.expm1(AXIAL_BETA)


def _radial_coefficients():
    """Solve for (A, eps, s_lip) of r(s) = A[(1+eps) s - w tanh((s-s0)/w) - w tanh(s0/w)].

    Conditions: r(s_lip) = RADIAL_LIP, r(1) = RADIAL_RMAX, and the spacing at the lip with
    128 points, A eps / 127, equals RADIAL_DRMIN_128. Solved by Newton's method on s0."""
    w = RADIAL_WIDTH
    aeps = RADIAL_DRMIN_128 * 127.0

    def residual(s0):
        # From r(1) = RMAX: A (1 + eps) = B; with A eps = aeps, A = B - aeps.
        # r(1): B - A w [tanh((1-s0)/w) + tanh(s0/w)] = RMAX
        t = math.tanh((1.0 - s0) / w) + math.tanh(s0 / w)
        b = (RADIAL_RMAX - aeps * w * t) / (1.0 - w * t)
        a = b - aeps
        return b * s0 - a * w * math.tanh(s0 / w) - RADIAL_LIP, a, b

    s0 = 0.15
    for _ in range(100):
        f, _, _ = residual(s0)
        df = (residual(s0 + 1e-7)[0] - residual(s0 - 1e-7)[0]) / 2e-7
        step = f / df
        s0 -= step
        if abs(step) < 1e-15:
            break
    _, a, b = residual(s0)
    eps = aeps / a
    return a, eps, s0


_RADIAL = None


def jet_radial_map(nj):
    global _RADIAL
    if _RADIAL is None:
        _RADIAL = _radial_coefficients()
    a, eps, s0 = _RADIAL
    w = RADIAL_WIDTH
    s = np.arange(nj, dtype=np.float64) / (nj - 1)
    r = a * ((1.0 + eps) * s - w * np.tanh((s - s0) / w) - w * math.tanh(s0 / w))
    r[0] = 0.0
    return r


def jet_grid(n):
    """Polar jet grid of n = (n_axial, n_radial, n_azimuthal) nodes.

    Node (i, j, k) sits at x = x(i), y = r(j) cos(theta_k), z = r(j) sin(theta_k), with
    theta_k = 2 pi k / n_k (distinct azimuthal nodes; the direction is periodic with zero
    translation). j = 0 is the jet axis r = 0. Returns (xyz, period_shift)."""
    ni, nj, nk = n
    x1 = jet_axial_map(ni)
    r1 = jet_radial_map(nj)
    th = 2.0 * math.pi * np.arange(nk, dtype=np.float64) / nk
    T, R, X = np.meshgrid(th, r1, x1, indexing="ij")
    xyz = np.stack([X, R * np.cos(T), R * np.sin(T)])
    shift = np.zeros((3, 3))
    return np.ascontiguousarray(xyz), shift
