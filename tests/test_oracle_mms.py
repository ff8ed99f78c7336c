"""Method of manufactured solutions: the oracle's residual converges at second order to the
exact flux divergence of the filtered Navier-Stokes equations.

For a smooth periodic state Q_m, dQ/dt = -J RHS_h must approach -div(F - F_v)(Q_m), the
Cartesian divergence of the inviscid and viscous (molecular + Smagorinsky/Eidson) fluxes,
computed symbolically here with sympy from the continuous equations (paper: LES
formulation, subgrid-scale modelling). A wrong sign, factor, index or dropped term in
the metrics, fluxes or viscous terms breaks the second-order convergence.

* case "curvilinear": smooth skewed periodic grid, molecular viscosity, the paper's
  artificial dissipation on (it contributes O(h^3) to J RHS), no SGS model.
* case "sgs": affinely skewed periodic grid with C_s = c0 / h, so that the Smagorinsky
  viscosity rho (C_s Delta)^2 |S| stays O(1) as h -> 0 and its stress and Eidson heat flux
  are pinned too; dissipation off.
* case "euler": the curvilinear grid, inviscid, no dissipation.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
import synthetic as sy
from synthetic.grids import skewed_periodic_grid

GAMMA = 1.4
S1 = sy.configs.SUTHERLAND_S1
AFFINE = np.array([[1.0, 0.2, 0.1], [0.1, 1.0, 0.15], [0.05, 0.2, 1.0]])


def _exact_divergence(re, pr, pr_sgs, sgs_coef, affine):
    """Return a numpy function (x, y, z) -> div(F - F_v) for the 5 equations."""
    x, y, z = sp.symbols("x y z", real=True)
    X = [x, y, z]
    if affine:
        minv = sp.Matrix(AFFINE).inv()
        s = list(minv * sp.Matrix(X))
    else:
        s = X
    s1, s2, s3 = s
    rho = 1 + sp.Rational(1, 10) * sp.sin(s1) * sp.cos(s2 + s3)
    # The velocity is chosen so that |S| stays above 0.04 everywhere: the Smagorinsky
    # viscosity is not differentiable where the strain vanishes, which would spoil the
    # convergence order for reasons unrelated to the discretisation.
    u = sp.Rational(3, 10) + sp.Rational(1, 10) * sp.sin(s3) + sp.Rational(1, 4) * sp.cos(s2) \
        + sp.Rational(1, 20) * sp.cos(s1 + s2) * sp.sin(s3)
    v = -sp.Rational(1, 5) + sp.Rational(1, 10) * sp.sin(s1) + sp.Rational(1, 20) * sp.cos(s3)
    w = sp.Rational(1, 10) + sp.Rational(1, 10) * sp.sin(s2) \
        + sp.Rational(1, 20) * sp.cos(s3 + 2 * s1) * sp.sin(s2)
    p = 1 / sp.Float(GAMMA) + sp.Rational(1, 20) * sp.cos(s1 - s2) * sp.sin(s3)
    g = sp.Float(GAMMA)
    vel = [u, v, w]
    e = p / (g - 1) + rho * (u ** 2 + v ** 2 + w ** 2) / 2
    T = g * p / rho
    mu = T ** sp.Rational(3, 2) * (1 + sp.Float(S1)) / (T + sp.Float(S1))
    grad = [[sp.diff(vel[m], X[n]) for n in range(3)] for m in range(3)]
    div = grad[0][0] + grad[1][1] + grad[2][2]
    if sgs_coef:
        smag = sp.sqrt(2 * sum(((grad[m][n] + grad[n][m]) / 2) ** 2
                               for m in range(3) for n in range(3)))
        mut = rho * sp.Float(sgs_coef) * smag
    else:
        mut = 0
    inv_re = sp.Float(1.0 / re) if re > 0 else 0
    visc = mu * inv_re + mut
    kappa = (mu * inv_re / sp.Float(pr) + mut / sp.Float(pr_sgs)) / (g - 1)
    out = []
    for c in range(5):
        total = 0
        for j in range(3):
            if c == 0:
                F = rho * vel[j]
                Fv = 0
            elif c < 4:
                i = c - 1
                F = rho * vel[i] * vel[j] + (p if i == j else 0)
                Fv = visc * (grad[i][j] + grad[j][i] - (sp.Rational(2, 3) * div if i == j else 0))
            else:
                F = (e + p) * vel[j]
                tau_j = [visc * (grad[i][j] + grad[j][i] - (sp.Rational(2, 3) * div if i == j else 0))
                         for i in range(3)]
                heat = -kappa * sp.diff(T, X[j])
                Fv = sum(tau_j[i] * vel[i] for i in range(3)) - heat
            total += sp.diff(F - Fv, X[j])
        out.append(sp.lambdify((x, y, z), total, "numpy"))
    prim = sp.lambdify((x, y, z), [rho, u, v, w, p], "numpy")
    return out, prim


def _affine_grid(n):
    idx = [2.0 * math.pi * np.arange(m) / m for m in (n, n, n)]
    s3, s2, s1 = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    S = np.stack([s1, s2, s3])
    xyz = np.einsum("cd,d...->c...", AFFINE, S)
    shift = (2.0 * math.pi * AFFINE).T.copy()   # row d = translation across direction d
    return np.ascontiguousarray(xyz), shift


def _errors(case, ns):
    if case == "curvilinear":
        re, cs0, k2, k4, affine = 5.0, 0.0, 0.25, 0.016, False
    elif case == "sgs":
        re, cs0, k2, k4, affine = 20.0, 0.6, 0.0, 0.0, True
    else:
        re, cs0, k2, k4, affine = 0.0, 0.0, 0.0, 0.0, False
    sgs_coef = cs0 ** 2 * np.linalg.det(AFFINE) ** (2.0 / 3.0) if cs0 else 0.0
    fexact, prim = _exact_divergence(re, 0.72, 0.6, sgs_coef, affine)
    errs, errs2, scale = [], [], None
    for n in ns:
        if affine:
            xyz, sh = _affine_grid(n)
        else:
            xyz, sh = skewed_periodic_grid((n, n, n))
        h = 2.0 * math.pi / n
        p = sy.box_params((n, n, n), sh, re_acoustic=re, cs=cs0 / h if cs0 else 0.0,
                          k2=k2, k4=k4, gamma=GAMMA)
        o = oracle.Oracle(p, xyz)
        x, y, z = xyz
        rho, u, v, w, pr = [np.broadcast_to(a, x.shape) for a in prim(x, y, z)]
        q = sy.conserved_from_primitive(rho, u, v, w, pr, GAMMA)
        jrhs = o.residual(q) / o.jinv
        ex = np.stack([np.broadcast_to(f(x, y, z), x.shape) for f in fexact])
        diff = (jrhs - ex).reshape(5, -1)
        errs.append(np.abs(diff).max(axis=1))
        errs2.append(np.sqrt((diff * diff).mean(axis=1)))
        scale = np.abs(ex).reshape(5, -1).max(axis=1)
    return np.array(errs), np.array(errs2), scale


@pytest.mark.parametrize("case", ["curvilinear", "sgs", "euler"])
def test_manufactured_solution_second_order(case):
    ns = (16, 32, 64)
    errs, errs2, scale = _errors(case, ns)
    orders2 = np.log2(errs2[1] / errs2[2])
    assert np.all(orders2 > 1.9), (case, errs2, orders2)
    if case != "sgs":
        # With the Smagorinsky term the max norm is still pre-asymptotic at 64^3 near the
        # smallest strain rates (the square root in |S| has curvature ~ 1/|S| there); the
        # mean-square norm is not.
        orders = np.log2(errs[1] / errs[2])
        assert np.all(orders > 1.9), (case, errs, orders)
    # At the finest grid the error is small against the exact divergence itself.
    assert np.all(errs[2] < 0.05 * scale), (errs[2], scale)
