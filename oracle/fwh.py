"""Plain FP64 reference of far-field noise by the Ffowcs Williams-Hawkings analogy from a
permeable control surface (test infrastructure only: imported by tests/, never by the
library).

The paper's Introduction and Concluding Remarks name the Ffowcs Williams and Hawkings
approach as the way its jet solutions are to give far-field noise. It states no formulation,
so this reference takes the standard one for a stationary permeable surface in a medium at
rest (Farassat's formulation 1A with the surface velocity zero), with the viscous stresses
left out of the loading:

* sources at a surface node with unit outward normal n, from the flow's rho, u, p:
  Q_n = rho u . n (mass flux), L_i = (p - p0) n_i + rho u_i (u . n) (momentum flux);
* observer x, surface node y, r = |x - y|, r_hat = (x - y)/r, retarded time tau = t - r/c0:
  4 pi p'(x, t) = sum over nodes of dS [ dQ_n/dtau / r + (dL_i/dtau) r_hat_i / (c0 r)
                                         + L_i r_hat_i / r^2 ] at tau;
* samples at uniform source times tau_m = tau_0 + m dtau; time derivatives by central
  differences (second-order one-sided at the first and last sample); values at tau by linear
  interpolation between the two samples around it; a node whose retarded time falls outside
  [tau_0, tau_last] contributes nothing and is counted.

Surface quadrature on the jet grid: node-based, the area vector of a node's cell being its
metric vector (S_eta on a surface j = const, S_xi on i = const; unit index spacing), with
half weights on the edges of each patch.
"""
from __future__ import annotations

import numpy as np


def sources(rho, u, p, n, p0):
    """Q_n [..., ns] and L [..., ns, 3] from samples rho [..., ns], u [..., ns, 3], p [..., ns]
    and unit normals n [ns, 3]."""
    un = np.einsum("...sc,sc->...s", u, n)
    Q = rho * un
    L = (p - p0)[..., None] * n + rho[..., None] * u * un[..., None]
    return Q, L


def time_derivative(f, dtau):
    """d f / d tau along axis 0 of samples at uniform spacing dtau: central differences, and
    second-order one-sided differences at the first and last sample."""
    f = np.asarray(f, dtype=np.float64)
    d = np.empty_like(f)
    d[1:-1] = (f[2:] - f[:-2]) / (2.0 * dtau)
    d[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * dtau)
    d[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * dtau)
    return d


def fwh_pressure(y, n, dS, rho, u, p, tau0, dtau, rho0, c0, p0, observers, times):
    """Acoustic pressure p'[no, nt] at observers [no, 3] and times [nt] from surface samples
    rho [M, ns], u [M, ns, 3], p [M, ns] taken at tau_m = tau0 + m dtau on nodes at y [ns, 3]
    with unit normals n [ns, 3] and areas dS [ns]. Returns (p', scale, skipped): scale[no, nt]
    is the sum of the absolute contributions (the size the sum is rounded against) and skipped
    the number of (observer, time, node) triples whose retarded time was outside the samples.
    (rho0 enters only through Q_n = rho0 U_n = rho u . n; it is kept as an argument for the
    record.)"""
    del rho0
    y = np.asarray(y, dtype=np.float64)
    M = rho.shape[0]
    Q, L = sources(rho, u, p, n, p0)
    Qd = time_derivative(Q, dtau)
    Ld = time_derivative(L, dtau)
    obs = np.asarray(observers, dtype=np.float64)
    times = np.asarray(times, dtype=np.float64)
    out = np.zeros((obs.shape[0], times.size))
    scale = np.zeros_like(out)
    skipped = 0
    ns = y.shape[0]
    cols = np.arange(ns)
    for a, x in enumerate(obs):
        dx = x[None, :] - y
        r = np.sqrt(np.sum(dx * dx, axis=1))
        rh = dx / r[:, None]
        for b, t in enumerate(times):
            s = (t - r / c0 - tau0) / dtau
            m = np.floor(s).astype(np.int64)
            ok = (m >= 0) & (m + 1 <= M - 1)
            # a retarded time exactly on the last sample uses the last interval
            last = (m == M - 1) & (s == M - 1)
            m = np.where(last, M - 2, m)
            ok |= last
            skipped += int(np.count_nonzero(~ok))
            mm = np.where(ok, m, 0)
            w = np.where(ok, s - mm, 0.0)

            def at(f):
                return (1.0 - w) * f[mm, cols] + w * f[mm + 1, cols]

            qd = at(Qd)
            lr = np.sum(np.stack([at(L[..., c]) for c in range(3)], axis=1) * rh, axis=1)
            ldr = np.sum(np.stack([at(Ld[..., c]) for c in range(3)], axis=1) * rh, axis=1)
            term = dS * (qd / r + ldr / (c0 * r) + lr / (r * r))
            term = np.where(ok, term, 0.0)
            out[a, b] = np.sum(term) / (4.0 * np.pi)
            scale[a, b] = np.sum(np.abs(term)) / (4.0 * np.pi)
    return out, scale, skipped


def jet_surface(S, xyz, i1, i2, js, caps=(True, True)):
    """Control surface on a jet grid (arrays shaped [.., nk, nj, ni]): the lateral cylinder
    j = js over i1 <= i <= i2 and every k, and, if asked, the end caps i = i1 (normal -S_xi)
    and i = i2 (normal +S_xi) over 0 <= j <= js. Returns (node ids [ns] into the flat grid,
    positions [ns, 3], unit normals [ns, 3], areas [ns]), nodes in the order: lateral (k, then
    i), then the upstream cap (k, then j), then the downstream cap."""
    nk, nj, ni = xyz.shape[1:]
    ids, area_vec, wts = [], [], []

    def flat(i, j, k):
        return i + ni * (j + nj * k)

    for k in range(nk):
        for i in range(i1, i2 + 1):
            ids.append(flat(i, js, k))
            area_vec.append(S[3:6, k, js, i])
            wts.append(0.5 if i in (i1, i2) else 1.0)
    for cap, (i, sign) in zip(caps, ((i1, -1.0), (i2, 1.0))):
        if not cap:
            continue
        for k in range(nk):
            for j in range(0, js + 1):
                ids.append(flat(i, j, k))
                area_vec.append(sign * S[0:3, k, j, i])
                wts.append(0.5 if j == js else 1.0)
    ids = np.array(ids, dtype=np.int64)
    av = np.array(area_vec, dtype=np.float64)
    mag = np.sqrt(np.sum(av * av, axis=1))
    nrm = np.where(mag[:, None] > 0, av / np.where(mag > 0, mag, 1.0)[:, None], 0.0)
    y = np.stack([xyz[c].reshape(-1)[ids] for c in range(3)], axis=1)
    return ids, y, nrm, mag * np.array(wts)


def sample_state(q, ids, gamma):
    """(rho [ns], u [ns, 3], p [ns]) of a conserved state q [5, ...] at flat node ids."""
    qf = np.asarray(q, dtype=np.float64).reshape(5, -1)[:, ids]
    rho = qf[0]
    u = (qf[1:4] / rho).T
    p = (gamma - 1.0) * (qf[4] - 0.5 * rho * np.sum(u * u, axis=1))
    return rho, u, p
