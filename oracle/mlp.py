"""FP64 CPU reference of the learned subgrid closure (test infrastructure only: imported by
tests/, the smoke check and the benchmark's CPU baseline, never by the library).

The paper closes the filtered equations with the Smagorinsky eddy viscosity
mu_t = rho (C_s Delta)^2 |S| (Subgrid Scale Modeling). The learned closure keeps that form
and replaces the constant C_s^2 by a coefficient c predicted per node by a small network
from scale-free invariants of the resolved velocity gradient:

* inputs: with A = grad u, S = sym A, O = skew A, S^d = S - tr(S)/3 I and
  |S| = (2 S:S)^(1/2):
  f = (tr S/|S|, tr(S^d S^d)/|S|^2, tr(O O)/|S|^2, tr(S^d S^d S^d)/|S|^3,
       tr(S^d O O)/|S|^3, tr(S^d S^d O O)/|S|^4);
* network: x = (f - mean) * inv_std, h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2),
  z = w3 . h2 + b3, c = softplus(z), with 64 hidden units per layer and GELU in its tanh
  form;
* closure: mu_t = rho c Delta^2 |S|, with c = C_s^2 (plain Smagorinsky) wherever |S| = 0,
  an input is not finite, or an input lies outside the trained range [lo, hi];
* training target (least-squares eddy-viscosity projection of a box-filtered finer
  solution): c* = max(0, -sigma^d : S~^d / (2 rho~ Delta^2 |S~| S~^d : S~^d)), with
  sigma_mn = mean(rho u_m u_n) - rho~ u~_m u~_n over 2 x 2 x 2 blocks of fine nodes,
  rho~ = mean(rho) and rho~ u~ = mean(rho u); loss = sum w (c - c*)^2 / sum w.

Parameter vector layout (NPARAMS = 4673 values): W1[64][6], b1[64], W2[64][64], b2[64],
w3[64], b3.
"""
from __future__ import annotations

import math

import numpy as np

NIN = 6
NH = 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + NH * NIN
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAMS = OFF_B3 + 1

_K0 = math.sqrt(2.0 / math.pi)
_K1 = 0.044715


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    return (t[OFF_W1:OFF_B1].reshape(NH, NIN), t[OFF_B1:OFF_W2], t[OFF_W2:OFF_B2].reshape(NH, NH),
            t[OFF_B2:OFF_W3], t[OFF_W3:OFF_B3], t[OFF_B3])


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_K0 * (x + _K1 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(_K0 * (x + _K1 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _K0 * (1.0 + 3.0 * _K1 * x * x)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def invariants(grad):
    """grad[m, n, ...] = d u_m / d x_n. Returns (f[6, ...], |S|[...]); f is NaN where
    |S| = 0."""
    A = np.moveaxis(np.asarray(grad, dtype=np.float64), (0, 1), (-2, -1))  # A[..., m, n]
    S = 0.5 * (A + np.swapaxes(A, -1, -2))
    O = 0.5 * (A - np.swapaxes(A, -1, -2))
    trS = np.trace(S, axis1=-2, axis2=-1)
    eye = np.eye(3)
    Sd = S - trS[..., None, None] / 3.0 * eye
    smag = np.sqrt(2.0 * np.einsum("...mn,...mn->...", S, S))
    Sd2 = Sd @ Sd
    O2 = O @ O
    tr = lambda M: np.trace(M, axis1=-2, axis2=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.stack([trS / smag, tr(Sd2) / smag ** 2, tr(O2) / smag ** 2,
                      tr(Sd2 @ Sd) / smag ** 3, tr(Sd @ O2) / smag ** 3,
                      tr(Sd2 @ O2) / smag ** 4])
    f[:, smag == 0] = np.nan
    return f, smag


def forward(theta, x):
    """x: normalised inputs (n, 6). Returns c (n,) and the cached activations."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a1 = x @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    z = h2 @ w3 + b3
    return softplus(z), (x, a1, h1, a2, h2, z)


def loss_grad(theta, x, y, w):
    """Weighted mean-square loss sum w (c - y)^2 / sum w and its gradient (NPARAMS,)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    c, (x, a1, h1, a2, h2, z) = forward(theta, x)
    wsum = np.sum(w)
    r = c - y
    loss = np.sum(w * r * r) / wsum
    dz = 2.0 * w * r * sigmoid(z) / wsum
    g = np.zeros(NPARAMS)
    g[OFF_W3:OFF_B3] = h2.T @ dz
    g[OFF_B3] = np.sum(dz)
    da2 = np.outer(dz, w3) * gelu_grad(a2)
    g[OFF_W2:OFF_B2] = (da2.T @ h1).reshape(-1)
    g[OFF_B2:OFF_W3] = np.sum(da2, axis=0)
    da1 = (da2 @ W2) * gelu_grad(a1)
    g[OFF_W1:OFF_B1] = (da1.T @ x).reshape(-1)
    g[OFF_B1:OFF_W2] = np.sum(da1, axis=0)
    return loss, g


def coefficient(theta, mean, inv_std, lo, hi, f, smag, cs2):
    """Closure coefficient c per node: the network where its inputs are finite, |S| > 0
    and every input lies in [lo, hi]; C_s^2 elsewhere. f: (6, n). Returns (c, fallback)."""
    f = np.asarray(f, dtype=np.float64)
    lo = np.asarray(lo)[:, None]
    hi = np.asarray(hi)[:, None]
    ok = np.all(np.isfinite(f), axis=0) & (smag > 0) & np.all((f >= lo) & (f <= hi), axis=0)
    x = ((np.where(np.isfinite(f), f, 0.0) - np.asarray(mean)[:, None])
         * np.asarray(inv_std)[:, None]).T
    c, _ = forward(theta, x)
    return np.where(ok, c, cs2), ~ok


def adam(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step counted from 1. Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def box_filter(q_fine):
    """Means over 2 x 2 x 2 blocks of a fine field (..., 2nk, 2nj, 2ni) -> (..., nk, nj, ni)."""
    a = np.asarray(q_fine, dtype=np.float64)
    s = a.shape
    a = a.reshape(s[:-3] + (s[-3] // 2, 2, s[-2] // 2, 2, s[-1] // 2, 2))
    return a.mean(axis=(-5, -3, -1))


def filtered_state(q_fine):
    """Box-filtered conserved state (rho~, rho~ u~, e~) and the subgrid stress
    sigma_mn = mean(rho u_m u_n) - rho~ u~_m u~_n, shaped (3, 3, ...)."""
    q = np.asarray(q_fine, dtype=np.float64)
    rho = q[0]
    u = q[1:4] / rho
    qb = box_filter(q)
    ub = qb[1:4] / qb[0]
    sig = np.empty((3, 3) + qb.shape[1:])
    for m in range(3):
        for n in range(3):
            sig[m, n] = box_filter(rho * u[m] * u[n]) - qb[0] * ub[m] * ub[n]
    return qb, sig


def target(sig, grad, rho, jinv):
    """Least-squares coefficient c* = max(0, -sigma^d : S^d / (2 rho Delta^2 |S| S^d : S^d))
    with Delta = (J^-1)^(1/3); 0 where |S| = 0 or J^-1 <= 0."""
    S = 0.5 * (grad + np.swapaxes(grad, 0, 1))
    trS = S[0, 0] + S[1, 1] + S[2, 2]
    trs = sig[0, 0] + sig[1, 1] + sig[2, 2]
    Sd = S.copy()
    sd = sig.copy()
    for m in range(3):
        Sd[m, m] = Sd[m, m] - trS / 3.0
        sd[m, m] = sd[m, m] - trs / 3.0
    smag = np.sqrt(2.0 * np.einsum("mn...,mn...->...", S, S))
    num = -np.einsum("mn...,mn...->...", sd, Sd)
    den = 2.0 * rho * np.cbrt(np.where(jinv > 0, jinv, 0.0)) ** 2 * smag * \
        np.einsum("mn...,mn...->...", Sd, Sd)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where((den > 0) & (jinv > 0), num / den, 0.0)
    return np.maximum(c, 0.0)


def closure_step(o, theta, norm, cs2, q, nsteps, cfl=0.5, dt_fixed=0.0):
    """Runge-Kutta steps of the oracle `o` (an oracle.Oracle) with the learned closure, as
    the oracle's own step takes them with Smagorinsky (paper, Time Marching Method: the
    five stages with alpha = 1/4, 1/6, 3/8, 1/2, 1 and the boundary conditions after every
    stage; dt = CFL min J^-1 / sum of the spectral radii from the state at the start of the
    step), except that at every stage the eddy viscosity is mu_t = rho c Delta^2 |S|, with
    c from the FP64 network on that stage's velocity gradient (`coefficient`, with the
    fallback to cs2) and Delta^3 = J^-1.

    norm: (mean, inv_std, lo, hi) arrays. Returns (q, dt of the last step)."""
    alpha = (0.25, 1.0 / 6.0, 0.375, 0.5, 1.0)
    p = o.p
    shape = p.shape
    per = (p.bc[0] == 0, p.bc[2] == 0, p.bc[4] == 0)
    upd = np.ones(shape, dtype=bool)
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        if not per[d]:
            sl = [slice(None)] * 3
            sl[ax] = 0
            upd[tuple(sl)] = False
            sl[ax] = shape[ax] - 1
            upd[tuple(sl)] = False
    jinv = o.jinv
    J = np.where(upd, 1.0 / np.where(upd, jinv, 1.0), 0.0)
    delta2 = np.cbrt(np.maximum(jinv, 0.0)) ** 2
    mean, inv_std, lo, hi = norm
    q = np.array(q, dtype=np.float64, copy=True)
    dt = dt_fixed
    for _ in range(nsteps):
        if cfl > 0.0:
            dt = o.dt(q, cfl)
        q0 = q.copy()
        for a in alpha:
            f, smag = invariants(o.velocity_gradient(q))
            c, _ = coefficient(theta, mean, inv_std, lo, hi, f.reshape(6, -1), smag.reshape(-1),
                               cs2)
            mut = q[0] * c.reshape(shape) * delta2 * smag
            rhs = o.residual_with_mut(q, mut)
            q = np.where(upd[None], q0 - a * dt * J[None] * rhs, q)
            q = o.apply_bc(q)
    return q, dt
