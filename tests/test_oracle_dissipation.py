"""Pins of the oracle's pressure sensor, Turkel-Vatsa coefficient switch and CFL time step.

Residual pins (paper, Spatial Discretization: the pressure sensor, eps2 = k2 max(nu_i,
nu_i+1) and eps4 = max(0, k4 - eps2), and D = Lam_f (eps2 dW - eps4 d3W)). On a uniform
Cartesian grid the field varies along x only, the fluid is at rest and there is no viscous or
subgrid flux (1/Re = 0, C_s = 0). The mass and energy residuals are then pure
dissipation-flux differences along xi, and the x-momentum residual is the centred pressure
difference. The expected values are evaluated here on the 1-D line, node by node, from the
paper's formulas and the metric identities of a Cartesian grid (S_d = h^2 e_d, J^-1 = h^3,
so Lam_d = a h^2 and the anisotropic scaling gives Lambar = 3 a h^2):

* periodic line: a pressure profile with a face where eps2 > k4 (eps4 clipped to 0), faces
  with 0 < eps2 < k4, and faces where nu_i != nu_i+1;
* the jet boundary set (xi non-periodic): the sensor of a boundary node is its interior
  neighbour's, and the fourth difference at the first and last face uses the mirrored
  difference (Delta W)_outside = -(Delta W)_inside. The pressure is linear near the
  entrance, so the sensor there vanishes, while a mirrored-ghost or wrapped boundary sensor
  would not.

A denominator p+ + p + p-, a mean in place of max(nu_i, nu_i+1), a dropped max(0, .) clip or a
different boundary-sensor rule each changes one of these residuals by far more than
round-off.

Time-step pins (paper, Time Marching Method; the reading dt = CFL min over updated nodes of
J^-1 / sum_d (|S_d . u| + a |S_d|)):

* uniform flow on a uniform Cartesian box: dt = CFL / (|u|/hx + |v|/hy + |w|/hz +
  a (1/hx + 1/hy + 1/hz)), the textbook multidimensional CFL limit;
* a box stretched along x with a node-dependent velocity: the same expression with the
  local spacing dx_i = (x_i+1 - x_i-1)/2, minimised over the nodes;
* the jet boundary set: boundary nodes do not enter the minimum.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy
from synthetic.grids import cartesian_grid

H = 0.1
K2, K4, GAMMA = 0.25, 0.016, 1.4


def _line_params(n, periodic):
    if periodic:
        xyz, sh = cartesian_grid(n, (H, H, H))
        p = sy.box_params(n, sh, re_acoustic=0.0, cs=0.0, k2=K2, k4=K4, gamma=GAMMA)
    else:
        xyz, sh = cartesian_grid(n, (H, H, H), periodic=(False, False, True))
        # Lift the grid off the y = 0 plane (nothing in the residual depends on it).
        xyz = xyz.copy()
        xyz[1] += 1.0
        p = sy.jet_params(n, re_acoustic=0.0, cs=0.0, k2=K2, k4=K4, gamma=GAMMA)
        p = p.replace(period_shift=sh)
    return p, xyz


def _field_along_x(p, rho1, p1):
    nk, nj, ni = p.shape
    rho = np.broadcast_to(np.asarray(rho1)[None, None, :], (nk, nj, ni)).copy()
    pr = np.broadcast_to(np.asarray(p1)[None, None, :], (nk, nj, ni)).copy()
    z = np.zeros_like(rho)
    return sy.conserved_from_primitive(rho, z, z, z, pr, GAMMA)


def _expected_line(rho1, p1, periodic):
    """Mass, x-momentum and energy residuals on the line from the paper's formulas."""
    n = len(p1)
    rho1, p1 = np.asarray(rho1, float), np.asarray(p1, float)
    a = np.sqrt(GAMMA * p1 / rho1)
    lam = a * H * H                  # |S_d . u| + a |S_d| with u = 0, |S_d| = h^2
    lbar = lam + 2.0 * np.sqrt(lam * lam)
    W = {0: rho1, 4: p1 / (GAMMA - 1.0) + p1}

    def sensor_at(c):
        pm, p0, pp = p1[(c - 1) % n], p1[c], p1[(c + 1) % n]
        return abs(pp - 2.0 * p0 + pm) / (pp + 2.0 * p0 + pm)

    nu = np.empty(n)
    for m in range(n):
        c = m
        if not periodic:
            c = min(max(m, 1), n - 2)   # a boundary node takes its interior neighbour's
        nu[m] = sensor_at(c)
    faces = range(n) if periodic else range(n - 1)
    D = {0: {}, 4: {}}
    eps = {}
    for f in faces:
        A, B = f, (f + 1) % n
        eps2 = K2 * max(nu[A], nu[B])
        eps4 = max(0.0, K4 - eps2)
        eps[f] = (eps2, eps4, nu[A], nu[B])
        lf = 0.5 * (lbar[A] + lbar[B])
        for c in (0, 4):
            w = W[c]
            dW = w[B] - w[A]
            if periodic or (0 < f < n - 2):
                d3 = w[(f + 2) % n] - 3.0 * w[B] + 3.0 * w[A] - w[(f - 1) % n]
            elif f == 0:
                d3 = (w[2] - w[1]) - 3.0 * dW
            else:
                d3 = -3.0 * dW + (w[A] - w[A - 1])
            D[c][f] = lf * (eps2 * dW - eps4 * d3)
    nodes = range(n) if periodic else range(1, n - 1)
    out = {0: {}, 1: {}, 4: {}}
    for m in nodes:
        for c in (0, 4):
            out[c][m] = -(D[c][m] - D[c][(m - 1) % n])
        out[1][m] = 0.5 * (p1[(m + 1) % n] - p1[(m - 1) % n]) * H * H
    return out, eps


PERIODIC_P = [1.0, 1.01, 1.0, 2.0, 2.05, 2.0, 1.5, 1.02]
PERIODIC_RHO = [1.0, 1.02, 0.98, 1.3, 1.35, 1.31, 1.1, 1.0]


def test_sensor_switch_on_a_periodic_line():
    n = (8, 4, 4)
    p, xyz = _line_params(n, True)
    o = oracle.Oracle(p, xyz)
    rhs = o.residual(_field_along_x(p, PERIODIC_RHO, PERIODIC_P))
    exp, eps = _expected_line(PERIODIC_RHO, PERIODIC_P, True)
    # the regimes the pin has to cover
    assert any(e2 > K4 for e2, _, _, _ in eps.values())
    assert any(0.0 < e2 < K4 for e2, _, _, _ in eps.values())
    assert any(e2 > 0.0 and abs(na - nb) > 0.05 for e2, _, na, nb in eps.values())
    for c in (0, 1, 4):
        want = np.array([exp[c][m] for m in range(8)])
        scale = np.abs(want).max()
        for k in range(4):
            for j in range(4):
                np.testing.assert_allclose(rhs[c, k, j, :], want, rtol=0, atol=1e-13 * scale)
    # the other momentum components and directions carry nothing
    assert np.abs(rhs[2:4]).max() <= 1e-15


def test_clipped_eps4_changes_the_residual():
    """The clip matters on this field: without max(0, .) the clipped face would add a
    negative fourth-difference term (the pin above would then fail)."""
    _, eps = _expected_line(PERIODIC_RHO, PERIODIC_P, True)
    w = np.asarray(PERIODIC_RHO)
    clipped = [f for f, (e2, _, _, _) in eps.items() if e2 > K4]
    d3 = [w[(f + 2) % 8] - 3 * w[(f + 1) % 8] + 3 * w[f] - w[(f - 1) % 8] for f in clipped]
    assert max(abs(x) for x in d3) > 0.05


JET_P = [1.0, 1.5, 2.0, 2.1, 1.4, 1.3, 1.9, 1.0]
JET_RHO = [1.0, 1.2, 1.4, 1.45, 1.1, 1.05, 1.35, 1.0]


def test_boundary_sensor_and_mirrored_difference_on_the_jet_set():
    n = (8, 5, 4)
    p, xyz = _line_params(n, False)
    o = oracle.Oracle(p, xyz)
    assert o.grid_rc == 0
    rhs = o.residual(_field_along_x(p, JET_RHO, JET_P))
    exp, eps = _expected_line(JET_RHO, JET_P, False)
    # The entrance pressure is linear: the copied sensor vanishes there, a mirrored ghost
    # (|p1 - p0|/(p1 + p0)) or a wrapped one would not.
    assert eps[0][2] == 0.0 and eps[0][3] == 0.0
    mirrored = abs(2 * JET_P[1] - 2 * JET_P[0]) / (2 * JET_P[1] + 2 * JET_P[0])
    assert K2 * mirrored > K4
    for c in (0, 1, 4):
        want = np.array([exp[c][m] for m in range(1, 7)])
        scale = np.abs(want).max()
        for k in range(4):
            for j in range(1, 4):   # updated rows
                np.testing.assert_allclose(rhs[c, k, j, 1:7], want, rtol=0,
                                           atol=1e-13 * scale)
    # boundary nodes carry a zero residual
    assert np.all(rhs[:, :, :, 0] == 0.0) and np.all(rhs[:, :, :, 7] == 0.0)


def _box(n, spacing):
    xyz, sh = cartesian_grid(n, spacing)
    return sy.box_params(n, sh, re_acoustic=100.0, cs=0.18), xyz


@pytest.mark.parametrize("vel", [(0.3, -0.2, 0.1), (0.0, 0.0, 0.0), (-1.7, 0.4, 2.2)])
def test_dt_uniform_flow_cartesian_closed_form(vel):
    hx, hy, hz = 0.1, 0.07, 0.13
    p, xyz = _box((6, 5, 4), (hx, hy, hz))
    o = oracle.Oracle(p, xyz)
    rho, pr = 1.2, 0.9
    q = sy.uniform_field(p.shape, rho, vel, pr, p.gamma)
    a = math.sqrt(p.gamma * pr / rho)
    cfl = 0.5
    want = cfl / (abs(vel[0]) / hx + abs(vel[1]) / hy + abs(vel[2]) / hz +
                  a * (1 / hx + 1 / hy + 1 / hz))
    assert o.dt(q, cfl) == pytest.approx(want, rel=1e-14)
    if vel == (0.0, 0.0, 0.0):   # at rest: the acoustic limit CFL h / (3a) on a cube
        pc, xc = _box((5, 5, 5), (0.2, 0.2, 0.2))
        oc = oracle.Oracle(pc, xc)
        qc = sy.uniform_field(pc.shape, rho, vel, pr, pc.gamma)
        assert oc.dt(qc, cfl) == pytest.approx(cfl * 0.2 / (3 * a), rel=1e-14)


def test_dt_stretched_grid_minimum_over_nodes():
    ni, nj, nk = 12, 5, 4
    hy, hz = 0.08, 0.11
    L = 1.2
    s = np.arange(ni) / ni
    x1 = L * s + 0.25 * (L / ni) * np.sin(2 * math.pi * s) * 3.0   # periodic stretching
    z, y, x = np.meshgrid(hz * np.arange(nk), hy * np.arange(nj), x1, indexing="ij")
    xyz = np.ascontiguousarray(np.stack([x, y, z]))
    sh = np.diag([L, hy * nj, hz * nk])
    p = sy.box_params((ni, nj, nk), sh, re_acoustic=100.0, cs=0.18)
    o = oracle.Oracle(p, xyz)
    assert o.grid_rc == 0
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.2 * rng.random(p.shape)
    u = 0.6 * rng.standard_normal(p.shape)
    v = 0.3 * rng.standard_normal(p.shape)
    w = 0.3 * rng.standard_normal(p.shape)
    pr = 0.7 + 0.1 * rng.random(p.shape)
    q = sy.conserved_from_primitive(rho, u, v, w, pr, p.gamma)
    xp = np.concatenate([x1[-1:] - L, x1, x1[:1] + L])
    dx = 0.5 * (xp[2:] - xp[:-2])                       # local spacing at node i
    a = np.sqrt(p.gamma * pr / rho)
    inv = (np.abs(u) / dx[None, None, :] + np.abs(v) / hy + np.abs(w) / hz +
           a * (1.0 / dx[None, None, :] + 1.0 / hy + 1.0 / hz))
    cfl = 0.7
    want = cfl * (1.0 / inv).min()
    assert o.dt(q, cfl) == pytest.approx(want, rel=1e-13)
    # The minimising node is not in the column of the smallest cell: the node-dependent
    # velocity decides it, so the pin is on the node-wise minimum, not on the grid alone.
    assert np.unravel_index(np.argmax(inv), inv.shape)[2] != int(np.argmin(dx))


def test_dt_excludes_boundary_nodes():
    n = (7, 6, 4)
    xyz, sh = cartesian_grid(n, (0.1, 0.1, 0.1), periodic=(False, False, True))
    xyz = xyz.copy()
    xyz[1] += 1.0
    p = sy.jet_params(n).replace(period_shift=sh)
    o = oracle.Oracle(p, xyz)
    rho = np.ones(p.shape)
    u = 0.2 * np.ones(p.shape)
    # a fast boundary layer of nodes (entrance, exit, centreline and far-field rows)
    u[:, :, 0] = u[:, :, -1] = 50.0
    u[:, 0, :] = u[:, -1, :] = 50.0
    z = np.zeros(p.shape)
    pr = np.full(p.shape, 1.0 / p.gamma)
    q = sy.conserved_from_primitive(rho, u, z, z, pr, p.gamma)
    a = 1.0
    want = 0.5 / ((0.2 / 0.1) + 3 * a / 0.1)
    assert o.dt(q, 0.5) == pytest.approx(want, rel=1e-14)
