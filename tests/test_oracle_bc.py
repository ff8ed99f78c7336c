"""Pins of the oracle's boundary conditions and near-boundary dissipation by the properties
that define them (paper, Boundary Conditions):

* far field: the boundary state carries the interior Riemann invariant
  R+ = q_n + 2a/(gamma-1) and the free-stream one R- = q_n - 2a/(gamma-1); the entropy
  p/rho^gamma and the tangential velocity come from the interior (outflow) or the free
  stream (inflow); supersonic cases copy the interior or the free stream;
* centreline: every axis node holds the azimuthal mean of the first ring;
* entrance: jet state inside r <= D/2, far-field procedure with the xi normal outside;
* exit: subsonic -> p = p_inf with velocity and p/rho of the interior; supersonic -> copy;
* the fourth difference at a non-periodic face equals the interior formula applied with a
  mirrored ghost node W_{-1} = W_1, which is what (Delta W)_{-1/2} = -(Delta W)_{1/2}
  (centreline section) states.
"""
import numpy as np
import pytest

import oracle
import synthetic as sy
from synthetic.grids import cartesian_grid, jet_grid

G = 1.4


def prim(q):
    rho = q[0]
    u = q[1:4] / rho
    p = (G - 1) * (q[4] - 0.5 * rho * (u * u).sum(axis=0))
    return rho, u, p


def _jet_case(n=(12, 10, 8), seed=3, u_scale=1.0):
    xyz, _ = jet_grid(n)
    p = sy.jet_params(n)
    o = oracle.Oracle(p, xyz)
    rng = np.random.default_rng(seed)
    shape = p.shape
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, shape)
    u = u_scale * rng.uniform(-1.5, 1.5, (3,) + shape)
    pr = (1.0 / G) * (1.0 + 0.3 * rng.uniform(-1, 1, shape))
    q = sy.conserved_from_primitive(rho, u[0], u[1], u[2], pr, G)
    return o, p, q


def _normals(o, d, sign):
    s = o.S[3 * d:3 * d + 3]
    with np.errstate(invalid="ignore", divide="ignore"):
        return sign * s / np.sqrt((s * s).sum(axis=0))


def _check_farfield_node(qb, qe, n, pinf, rhoinf, uinf):
    rb, ub, pb = qb
    re_, ue, pe = qe
    ab, ae = np.sqrt(G * pb / rb), np.sqrt(G * pe / re_)
    ainf = np.sqrt(G * pinf / rhoinf)
    qnb, qne, qninf = ub @ n, ue @ n, np.asarray(uinf) @ n
    mn = qne / ae
    if mn >= 1.0:
        assert np.allclose([rb, pb], [re_, pe], rtol=1e-14) and np.allclose(ub, ue, rtol=1e-14)
        return "supersonic-out"
    if mn <= -1.0:
        assert np.allclose([rb, pb], [rhoinf, pinf], rtol=1e-14)
        assert np.allclose(ub, uinf, atol=1e-14)
        return "supersonic-in"
    assert qnb + 2 * ab / (G - 1) == pytest.approx(qne + 2 * ae / (G - 1), rel=1e-12)
    assert qnb - 2 * ab / (G - 1) == pytest.approx(qninf - 2 * ainf / (G - 1), rel=1e-12, abs=1e-12)
    if mn >= 0.0:
        assert pb / rb ** G == pytest.approx(pe / re_ ** G, rel=1e-12)
        assert np.allclose(ub - qnb * n, ue - qne * n, atol=1e-12)
        return "subsonic-out"
    assert pb / rb ** G == pytest.approx(pinf / rhoinf ** G, rel=1e-12)
    assert np.allclose(ub - qnb * n, np.asarray(uinf) - qninf * n, atol=1e-12)
    return "subsonic-in"


def test_farfield_riemann_invariants_entropy_and_tangential_velocity():
    seen = set()
    for seed in range(4):
        o, p, q = _jet_case(seed=seed, u_scale=1.0)
        qb = o.apply_bc(q)
        n = _normals(o, 1, 1.0)
        ni, nj, nk = p.ni, p.nj, p.nk
        rb, ub, pb = prim(qb)
        rq, uq, pq = prim(q)
        for k in range(nk):
            for i in range(1, ni - 1):
                b = (k, nj - 1, i)
                e = (k, nj - 2, i)
                case = _check_farfield_node((rb[b], ub[(slice(None),) + b], pb[b]),
                                            (rq[e], uq[(slice(None),) + e], pq[e]),
                                            n[(slice(None),) + b], p.p_inf, p.rho_inf, p.u_inf)
                seen.add(case)
    assert seen == {"supersonic-out", "supersonic-in", "subsonic-out", "subsonic-in"}


def test_centreline_is_azimuthal_mean_of_first_ring():
    o, p, q = _jet_case()
    qb = o.apply_bc(q)
    for i in range(1, p.ni - 1):
        mean = q[:, :, 1, i].mean(axis=1)
        for k in range(p.nk):
            assert np.allclose(qb[:, k, 0, i], mean, rtol=1e-14, atol=1e-15)


def test_entrance_jet_state_and_riemann_outside():
    o, p, q = _jet_case(seed=5)
    qb = o.apply_bc(q)
    r = np.sqrt(o.xyz[1] ** 2 + o.xyz[2] ** 2)
    rb, ub, pb = prim(qb)
    n = _normals(o, 0, -1.0)
    # The entrance reads node i = 1 after the far field and the centreline were set.
    after_j = q.copy()
    jet_inner = 0
    for k in range(p.nk):
        for j in range(p.nj):
            if r[k, j, 0] <= p.jet_radius:
                jet_inner += 1
                assert rb[k, j, 0] == 1.0 and pb[k, j, 0] == pytest.approx(1.0 / G, rel=1e-15)
                assert np.allclose(ub[:, k, j, 0], [p.mach_jet, 0, 0], atol=1e-15)
    assert jet_inner > 0
    # Outside the jet, check the invariants against node i = 1 of the updated field.
    qe_all = qb  # node i = 1 is untouched by the entrance and exit conditions
    re_, ue, pe = prim(qe_all)
    for k in range(p.nk):
        for j in range(p.nj):
            if r[k, j, 0] > p.jet_radius:
                _check_farfield_node((rb[k, j, 0], ub[:, k, j, 0], pb[k, j, 0]),
                                     (re_[k, j, 1], ue[:, k, j, 1], pe[k, j, 1]),
                                     n[:, k, j, 0], p.p_inf, p.rho_inf, p.u_inf)
    del after_j


@pytest.mark.parametrize("supersonic", [False, True])
def test_exit_condition(supersonic):
    o, p, q = _jet_case(seed=7, u_scale=0.2)
    if supersonic:
        q = q.copy()
        q[1] += 2.0 * q[0]          # u += 2 > a: supersonic through the exit plane
        q[4] += 2.0 * q[0] + 2.0 * (q[1] - 2.0 * q[0])   # e += rho(|u+2|^2 - |u|^2)/2: p kept
    qb = o.apply_bc(q)
    rb, ub, pb = prim(qb)
    i = p.ni - 1
    n = _normals(o, 0, 1.0)
    counts = {"copy": 0, "pressure": 0}
    for k in range(p.nk):
        for j in range(p.nj):
            # The exit reads node i-1 after the far field and centreline were applied; on
            # the axis the normal is that of j = 1 (the xi metric vanishes there).
            nn = n[:, k, max(j, 1), i]
            mach = ub[:, k, j, i - 1] @ nn / np.sqrt(G * pb[k, j, i - 1] / rb[k, j, i - 1])
            if mach >= 1.0:
                counts["copy"] += 1
                assert np.allclose(qb[:, k, j, i], qb[:, k, j, i - 1], rtol=1e-14)
            else:
                counts["pressure"] += 1
                assert pb[k, j, i] == pytest.approx(p.p_inf, rel=1e-12)
                assert np.allclose(ub[:, k, j, i], ub[:, k, j, i - 1], rtol=1e-13)
                assert pb[k, j, i] / rb[k, j, i] == pytest.approx(
                    pb[k, j, i - 1] / rb[k, j, i - 1], rel=1e-12)
    if supersonic:
        assert counts["copy"] >= (p.nj - 1) * p.nk
    else:
        assert counts["pressure"] == p.nj * p.nk


def test_periodic_box_has_no_boundary_nodes():
    p, xyz, q = sy.make_case("tgv", 8)
    o = oracle.Oracle(p, xyz)
    assert np.array_equal(o.apply_bc(q), q)


def _line_state(x, seed):
    rng = np.random.default_rng(seed)
    n = x.shape[-1]
    rho1 = 1.0 + 0.1 * rng.uniform(-1, 1, n)
    e1 = 1.8 + 0.2 * rng.uniform(-1, 1, n)
    return rho1, e1


def test_boundary_fourth_difference_equals_ghost_extrapolation():
    """Residual at the first and last interior nodes of a non-periodic direction with the
    boundary rule equals the interior formula on a grid one node longer at each end whose
    extra nodes mirror the first interior node, W_{-1} = W_1 (so W_0 - W_{-1} =
    -(W_1 - W_0))."""
    n = 9
    h = 0.3
    shape_j = 5
    xyz, sh = cartesian_grid((n, shape_j, 4), (h, h, h), periodic=(False, False, True))
    p = sy.jet_params((n, shape_j, 4)).replace(period_shift=sh, re_acoustic=0.0, cs=0.0,
                                                 k2=0.0, k4=0.016)
    o = oracle.Oracle(p, xyz)
    rho1, e1 = _line_state(xyz[0], 1)
    # u = 0 so that W = (rho, 0, 0, 0, e + p) is linear in the conserved variables.
    ones = np.ones(p.shape)
    q = np.stack([ones * rho1, 0 * ones, 0 * ones, 0 * ones, ones * e1])
    rhs = o.residual(q)

    xyz2, sh2 = cartesian_grid((n + 2, shape_j, 4), (h, h, h), periodic=(False, False, True))
    p2 = p.replace(ni=n + 2)
    o2 = oracle.Oracle(p2, xyz2)
    rho2 = np.concatenate([[rho1[1]], rho1, [rho1[-2]]])
    e2 = np.concatenate([[e1[1]], e1, [e1[-2]]])
    ones2 = np.ones(p2.shape)
    q2 = np.stack([ones2 * rho2, 0 * ones2, 0 * ones2, 0 * ones2, ones2 * e2])
    rhs2 = o2.residual(q2)
    # Nodes i = 1 and i = n-2 of the short grid are nodes 2 and n-1 of the long one.
    for i_short, i_long in ((1, 2), (n - 2, n - 1)):
        a = rhs[:, :, 1:-1, i_short]
        b = rhs2[:, :, 1:-1, i_long]
        assert np.abs(a).max() > 1e-6
        assert np.allclose(a, b, rtol=1e-12, atol=1e-18)
