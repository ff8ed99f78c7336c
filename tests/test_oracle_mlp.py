"""Pins of the learned-closure reference (oracle/mlp.py) against values fixed by the
mathematics: closed-form invariants of simple velocity gradients, rotation and scale
invariance, the exact GELU and softplus at known points, central finite differences of the
loss, Adam's first step, and the box-filter target of a linear velocity field."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
import synthetic as sy


def _one(A):
    f, smag = mlp.invariants(np.asarray(A, dtype=float).reshape(3, 3, 1))
    return f[:, 0], smag[0]


def test_invariants_pure_shear():
    a = 0.7
    f, smag = _one([[0, a, 0], [0, 0, 0], [0, 0, 0]])
    assert smag == pytest.approx(a)
    assert np.allclose(f, [0.0, 0.5, -0.5, 0.0, 0.0, -0.125], atol=1e-15)


def test_invariants_dilatation_and_axisymmetric_strain():
    f, smag = _one(np.eye(3) * 0.3)
    assert smag == pytest.approx(0.3 * math.sqrt(6))
    assert np.allclose(f, [3 / math.sqrt(6), 0, 0, 0, 0, 0], atol=1e-15)
    a = 0.2
    f, smag = _one(np.diag([-2 * a, a, a]))
    # S:S = 6a^2, |S| = a sqrt(12); tr(S^3) = -6a^3.
    assert smag == pytest.approx(a * math.sqrt(12))
    assert f[1] == pytest.approx(0.5)
    assert f[3] == pytest.approx(-6 / 12 ** 1.5)


def test_invariants_rotation_and_scale_invariant():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    f0, s0 = _one(A)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    f1, s1 = _one(Q @ A @ Q.T)
    f2, s2 = _one(2.5 * A)
    assert np.allclose(f1, f0, rtol=1e-12, atol=1e-14)
    assert np.allclose(f2, f0, rtol=1e-12, atol=1e-14)
    assert s1 == pytest.approx(s0) and s2 == pytest.approx(2.5 * s0)


def test_solid_rotation_has_no_inputs():
    f, smag = _one([[0, 1, 0], [-1, 0, 0], [0, 0, 0]])
    assert smag == 0 and np.all(np.isnan(f))


def test_activations():
    assert mlp.gelu(np.array(0.0)) == 0.0
    xs = np.linspace(-4, 4, 81)
    exact = 0.5 * xs * (1 + np.vectorize(math.erf)(xs / math.sqrt(2)))
    assert np.max(np.abs(mlp.gelu(xs) - exact)) < 1e-3  # tanh form vs erf form
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(xs), (mlp.gelu(xs + h) - mlp.gelu(xs - h)) / (2 * h),
                       atol=1e-8)
    assert mlp.softplus(np.array(0.0)) == pytest.approx(math.log(2))
    assert mlp.softplus(np.array(50.0)) == pytest.approx(50.0)
    assert mlp.sigmoid(np.array(0.0)) == 0.5


def test_forward_constant_network():
    th = np.zeros(mlp.NPARAMS)
    th[mlp.OFF_B1:mlp.OFF_W2] = 0.3
    th[mlp.OFF_W2:mlp.OFF_B2] = 0.01
    th[mlp.OFF_W3:mlp.OFF_B3] = 0.5
    th[mlp.OFF_B3] = -1.0
    x = np.random.default_rng(0).normal(size=(5, 6))
    c, _ = mlp.forward(th, x)
    h1 = mlp.gelu(0.3)
    h2 = mlp.gelu(64 * 0.01 * h1)
    z = 64 * 0.5 * h2 - 1.0
    assert np.allclose(c, math.log1p(math.exp(z)), rtol=1e-14)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(1)
    th = rng.normal(scale=0.3, size=mlp.NPARAMS)
    x = rng.normal(size=(40, 6))
    y = rng.uniform(0, 0.1, size=40)
    w = rng.uniform(0.5, 1.5, size=40)
    loss, g = mlp.loss_grad(th, x, y, w)
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 60, replace=False),
                          [mlp.OFF_B3, mlp.OFF_W3, mlp.OFF_B2, mlp.OFF_B1, mlp.OFF_W1]])
    h = 1e-6
    for i in idx:
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (mlp.loss_grad(tp, x, y, w)[0] - mlp.loss_grad(tm, x, y, w)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10), i


def test_adam_first_step_is_signed_lr():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 2.0])
    t, m, v = mlp.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(t, th - 0.01 * np.sign(g))


def test_coefficient_fallback():
    th = np.zeros(mlp.NPARAMS)
    f = np.array([[0.0, 0.0, np.nan, 5.0],
                  [0.5, 0.5, 0.5, 0.5], [-0.5] * 4, [0.0] * 4, [0.0] * 4, [-0.1] * 4])
    smag = np.array([1.0, 0.0, 1.0, 1.0])
    lo, hi = -np.ones(6), np.ones(6)
    c, fb = mlp.coefficient(th, np.zeros(6), np.ones(6), lo, hi, f, smag, 0.0324)
    assert list(fb) == [False, True, True, True]
    assert c[0] == pytest.approx(math.log(2)) and np.all(c[1:] == 0.0324)


def test_filter_target_linear_field():
    # Fine Cartesian grid, spacing h, u = G x with G an axisymmetric strain diag(-2a, a, a)
    # (a > 0, for which the projection is positive). Over a 2x2x2 block
    # sigma = rho (h^2/4) G G^T exactly, the coarse gradient of u~ is G, and
    # c* = (6 |a|^3 h^2/4) / (2 (2h)^2 |a| sqrt(12) 6 a^2) = 1 / (32 sqrt(12)).
    nf = 16
    h = 2 * math.pi / nf
    a = 0.05
    G = np.diag([-2 * a, a, a])
    xyz_f, _ = sy.cartesian_periodic_grid((nf, nf, nf))
    x = xyz_f
    u = np.einsum("mn,n...->m...", G, x)
    rho = np.full(x.shape[1:], 1.2)
    p = np.full(x.shape[1:], 1 / 1.4)
    qf = sy.conserved_from_primitive(rho, u[0], u[1], u[2], p, 1.4)
    qb, sig = mlp.filtered_state(qf)
    assert np.allclose(sig, 1.2 * h * h / 4 * np.einsum("mk,nk->mn", G, G)[..., None, None, None],
                       rtol=1e-10, atol=1e-16)
    nc = nf // 2
    xyz_c = mlp.box_filter(xyz_f)
    pc = sy.box_params((nc, nc, nc), np.eye(3) * 2 * math.pi)
    o = oracle.Oracle(pc, np.ascontiguousarray(xyz_c))
    grad = o.velocity_gradient(qb)
    inner = (slice(None), slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(grad[inner], G[..., None, None, None], atol=1e-12)
    c = mlp.target(sig, grad, qb[0], o.jinv)
    assert np.allclose(c[1:-1, 1:-1, 1:-1], 1 / (32 * math.sqrt(12)), rtol=1e-10)
    c = mlp.target(sig, -grad, qb[0], o.jinv)  # the opposite strain projects negative: 0
    assert np.all(c[1:-1, 1:-1, 1:-1] == 0.0)


def test_closure_step_with_constant_network_is_the_smagorinsky_step():
    """The learned-closure step (Python stages around the C oracle's residual) with a network
    whose output is the constant C_s^2 (zero output weights, b3 = softplus^-1(C_s^2)) must be
    the C oracle's own Smagorinsky Runge-Kutta step: two independent implementations of the
    stage loop, the time step and the boundary conditions."""
    from synthetic.grids import jet_grid
    n = (20, 12, 8)
    xyz, _ = jet_grid(n)
    p = sy.jet_params(n)
    q = sy.jet_field(xyz, gamma=p.gamma, mach_jet=p.mach_jet, u_inf=p.u_inf[0], seed=2)
    o = oracle.Oracle(p, xyz)
    q = o.apply_bc(q)
    cs2 = p.cs ** 2
    th = np.zeros(mlp.NPARAMS)
    th[mlp.OFF_B3] = math.log(math.expm1(cs2))
    norm = (np.zeros(6), np.ones(6), np.full(6, -np.inf), np.full(6, np.inf))
    got, dt = mlp.closure_step(o, th, norm, cs2, q, 3, cfl=0.5)
    ref, dtref = o.step(q, 3, cfl=0.5)
    assert dt == pytest.approx(dtref, rel=1e-15)
    err = np.abs(got - ref).reshape(5, -1).max(1) / np.abs(ref).reshape(5, -1).max(1)
    assert np.all(err <= 1e-13), err
    # and the closure acts: with c = 0 the state differs
    th0 = th.copy()
    th0[mlp.OFF_B3] = -50.0
    off, _ = mlp.closure_step(o, th0, norm, cs2, q, 3, cfl=0.5)
    assert np.abs(off - ref).max() > 1e3 * np.abs(got - ref).max()
