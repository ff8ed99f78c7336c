"""Plain FP64 running statistics of a jet run (test infrastructure only: imported by tests/
and by the scripts under tests/golden/ that write stored expected values, never by the
library).

The paper's production run could not accumulate converged time averages (Numerical Results,
and the Concluding Remarks, which ask for longer runs): the statistics it needs are the time
mean and the r.m.s. fluctuation of the primitive variables, reduced over the azimuth of the
round jet to the centreline axial-velocity decay and to radial profiles at axial stations.
This module computes those products from a sequence of conserved states, one sample per
state, with every sum taken in a fixed order:

* per node: sum of x and of x^2 for x in (rho, u, v, w, p), over samples in the order given;
* mean = sum/n, rms = sqrt(max(sum2/n - mean^2, 0));
* azimuthal average of a field f[k][j][i]: (1/nk) sum over k = 0..nk-1 in increasing k.
"""
from __future__ import annotations

import numpy as np

from . import primitives


class RunningStats:
    """Sums of the primitive variables and of their squares, sample by sample."""

    def __init__(self, shape, gamma):
        self.gamma = gamma
        self.s1 = np.zeros((5,) + tuple(shape))
        self.s2 = np.zeros((5,) + tuple(shape))
        self.n = 0

    def add(self, q):
        x = primitives(q, self.gamma)
        self.s1 += x
        self.s2 += x * x
        self.n += 1

    def mean_rms(self):
        mean = self.s1 / self.n
        rms = np.sqrt(np.maximum(self.s2 / self.n - mean * mean, 0.0))
        return mean, rms


def azimuthal_average(f):
    """Average over the azimuthal (k) axis of f[..., k, j, i], summed in increasing k."""
    f = np.asarray(f, dtype=np.float64)
    acc = np.zeros(f.shape[:-3] + f.shape[-2:])
    nk = f.shape[-3]
    for k in range(nk):
        acc = acc + f[..., k, :, :]
    return acc / nk


def jet_products(mean, rms, stations):
    """Centreline and radial products of azimuthally averaged statistics.

    mean, rms: [5][nk][nj][ni] (rho, u, v, w, p). Returns a dict with the centreline mean and
    r.m.s. axial velocity (j = 0, every station i) and, at each axial station i in
    `stations`, the radial profiles (every j) of the mean and r.m.s. axial velocity and of
    the mean density and pressure."""
    am, ar = azimuthal_average(mean), azimuthal_average(rms)
    out = {"centreline_u_mean": am[1, 0, :], "centreline_u_rms": ar[1, 0, :]}
    for i in stations:
        out[f"radial_u_mean_i{i}"] = am[1, :, i]
        out[f"radial_u_rms_i{i}"] = ar[1, :, i]
        out[f"radial_rho_mean_i{i}"] = am[0, :, i]
        out[f"radial_p_mean_i{i}"] = am[4, :, i]
    return out
