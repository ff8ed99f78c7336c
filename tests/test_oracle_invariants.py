"""Pins of the CPU oracle against properties the discretisation must have.

* free-stream preservation on a skewed curvilinear periodic grid (the conservative metric
  form satisfies the discrete geometric conservation law; the paper's plain product form
  only to O(h^2)),
* discrete conservation on a periodic grid (the residual is a difference of face fluxes),
* the Smagorinsky viscosity vanishes for uniform flow and solid-body rotation and takes
  its closed-form value for pure shear,
* Sutherland's law at the reference temperature and against the dimensional law.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as sy
from synthetic.grids import cartesian_grid, skewed_periodic_grid


def _oracle_skewed(n, metric_form=0, **kw):
    xyz, sh = skewed_periodic_grid((n, n, n))
    p = sy.box_params((n, n, n), sh, **kw)
    return oracle.Oracle(p, xyz, metric_form=metric_form), p


def _smooth_field(o, p, amp=0.05):
    x, y, z = o.xyz
    rho = 1.0 + amp * np.sin(x) * np.cos(y + z)
    u = 0.3 + amp * np.cos(x + y) * np.sin(z)
    v = -0.2 + amp * np.sin(y) * np.cos(x - z)
    w = 0.1 + amp * np.cos(z + 2 * x) * np.sin(y)
    pr = 1.0 / p.gamma + amp * np.cos(x - y) * np.sin(z)
    return sy.conserved_from_primitive(rho, u, v, w, pr, p.gamma)


@pytest.mark.parametrize("n", [12, 20])
def test_free_stream_preserved_on_skewed_grid(n):
    o, p = _oracle_skewed(n, re_acoustic=50.0, cs=0.18)
    assert o.grid_rc == 0
    q = sy.uniform_field(p.shape, 1.0, (0.4, -0.25, 0.15), 1.0 / p.gamma, p.gamma)
    rhs = o.residual(q)
    # Scale: the size of one node flux |F||S|.
    scale = np.abs(o.S).max() * 1.0
    assert np.abs(rhs).max() <= 1e-13 * scale


def test_plain_metric_form_is_not_free_stream_preserving_and_converges_second_order():
    errs = []
    for n in (16, 32):
        o, p = _oracle_skewed(n, metric_form=1, re_acoustic=0.0, cs=0.0)
        q = sy.uniform_field(p.shape, 1.0, (0.4, -0.25, 0.15), 1.0 / p.gamma, p.gamma)
        rhs = o.residual(q)
        # J * RHS approximates -dQ/dt, which is zero exactly for a uniform flow.
        errs.append(np.abs(rhs[1] / o.jinv).max())
    assert errs[0] > 1e-6
    order = math.log(errs[0] / errs[1], 2)
    assert 1.7 < order < 2.5, (errs, order)


def test_residual_sums_to_zero_on_periodic_grid():
    o, p = _oracle_skewed(16, re_acoustic=30.0, cs=0.18)
    q = _smooth_field(o, p, amp=0.1)
    rhs = o.residual(q).reshape(5, -1)
    total = rhs.sum(axis=1)
    scale = np.abs(rhs).sum(axis=1)
    assert np.all(np.abs(total) <= 1e-13 * scale), (total, scale)


def test_totals_conserved_over_steps():
    o, p = _oracle_skewed(12, re_acoustic=30.0, cs=0.18)
    q = _smooth_field(o, p, amp=0.1)
    d0 = o.diagnostics(q)
    q2, dt = o.step(q, 10, cfl=0.5)
    d1 = o.diagnostics(q2)
    assert dt > 0
    # Totals sum J^-1 Q over all nodes; scale each by sum J^-1 |Q|.
    scale = np.array([np.sum(o.jinv * np.abs(q[c])) for c in range(5)])
    drift = np.abs(d1[1:] - d0[1:]) / scale
    assert np.all(drift < 1e-13), drift
    # The flow did change.
    assert np.abs(q2 - q).max() > 1e-4


def test_smagorinsky_zero_for_uniform_flow_on_curvilinear_grid():
    o, p = _oracle_skewed(12, re_acoustic=30.0, cs=0.18)
    q = sy.uniform_field(p.shape, 1.3, (0.4, -0.25, 0.15), 0.9, p.gamma)
    mut = o.sgs_viscosity(q)
    assert np.abs(mut).max() < 1e-13


def _cartesian_jet_box(n, h):
    """Cartesian grid with the jet's boundary set (i and j non-periodic, k periodic)."""
    xyz, sh = cartesian_grid(n, h, periodic=(False, False, True))
    p = sy.jet_params(n)
    p = p.replace(period_shift=sh)
    return xyz, p


def test_smagorinsky_zero_for_solid_body_rotation():
    xyz, p = _cartesian_jet_box((10, 9, 6), (0.3, 0.2, 0.25))
    o = oracle.Oracle(p, xyz)
    x, y, z = xyz
    om = 0.7
    q = sy.conserved_from_primitive(np.ones_like(x), -om * (y - 0.5), om * (x - 1.0),
                                    np.zeros_like(x), np.full_like(x, 0.7), p.gamma)
    mut = o.sgs_viscosity(q)
    assert np.abs(mut).max() < 1e-15


def test_smagorinsky_pure_shear_closed_form():
    h = (0.3, 0.3, 0.3)
    xyz, p = _cartesian_jet_box((10, 9, 6), h)
    p = p.replace(cs=0.17)
    o = oracle.Oracle(p, xyz)
    x, y, z = xyz
    G = 0.9
    rho = 1.2
    q = sy.conserved_from_primitive(np.full_like(x, rho), G * y, np.zeros_like(x),
                                    np.zeros_like(x), np.full_like(x, 0.7), p.gamma)
    mut = o.sgs_viscosity(q)
    # |S| = (2 S_ij S_ij)^(1/2) = |G| for u = G y; Delta = (h^3)^(1/3) = h.
    expect = rho * (0.17 * 0.3) ** 2 * G
    assert np.allclose(mut, expect, rtol=1e-13, atol=0)


def test_sutherland_reference_and_dimensional_law():
    o, p = _oracle_skewed(4)
    assert o.sutherland(np.array([1.0]))[0] == 1.0
    # Dimensional Sutherland law with S1 = 110.4 K, T_ref = 288.15 K:
    # mu(T)/mu(T_ref) = (T/T_ref)^(3/2) (T_ref + S1)/(T + S1).
    for T in (200.0, 288.15, 400.0, 700.0):
        expect = (T / 288.15) ** 1.5 * (288.15 + 110.4) / (T + 110.4)
        got = o.sutherland(np.array([T / 288.15]))[0]
        assert got == pytest.approx(expect, rel=1e-14)


def test_bad_grid_reported():
    n = 8
    xyz, sh = skewed_periodic_grid((n, n, n))
    xyz = xyz.copy()
    xyz[0] = -xyz[0]               # mirror x: left-handed grid, J^-1 < 0
    sh = sh.copy()
    sh[0, 0] = -sh[0, 0]
    p = sy.box_params((n, n, n), sh)
    o = oracle.Oracle(p, xyz)
    assert o.grid_rc == -3


def test_invalid_parameters_rejected():
    n = 8
    xyz, sh = skewed_periodic_grid((n, n, n))
    p = sy.box_params((n, n, n), sh).replace(bc=(0, 0, 0, 0, 1, 3))
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(p, xyz)
