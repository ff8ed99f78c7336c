"""Pins of the statistics reference (oracle/stats.py) against closed forms.

* Running mean and r.m.s.: states whose primitive variables follow x_m = x0 + a cos(2 pi m/M
  + phase) over M samples (a whole period) have the mean x0 and the r.m.s. fluctuation
  |a|/sqrt(2) exactly (sum of cos over a period is 0, of cos^2 is M/2, for M >= 3); a
  constant state has r.m.s. 0. A dropped 1/n, a square root left out, or the mean not
  subtracted each fails.
* Azimuthal average: c + sum_m b_m cos(2 pi m k/nk + phi_m) over the nk nodes averages to c
  for 0 < m < nk.
* Jet products: on fields built as functions of (i, j), the centreline is row j = 0 and the
  radial profile at station i is column i, for the named variables.
"""
import math

import numpy as np

from oracle import primitives
from oracle.stats import RunningStats, azimuthal_average, jet_products
import synthetic as sy

GAMMA = 1.4


def test_running_mean_and_rms_of_a_periodic_sequence():
    shape = (3, 4, 5)
    M = 12
    x0 = {"rho": 1.1, "u": 0.3, "v": -0.2, "w": 0.05, "p": 0.7}
    amp = {"rho": 0.05, "u": 0.02, "v": -0.03, "w": 0.01, "p": 0.04}
    ph = {"rho": 0.3, "u": 1.1, "v": 2.0, "w": -0.7, "p": 0.9}
    rs = RunningStats(shape, GAMMA)
    for m in range(M):
        vals = {k: np.full(shape, x0[k] + amp[k] * math.cos(2 * math.pi * m / M + ph[k]))
                for k in x0}
        q = sy.conserved_from_primitive(vals["rho"], vals["u"], vals["v"], vals["w"],
                                        vals["p"], GAMMA)
        rs.add(q)
    mean, rms = rs.mean_rms()
    for c, k in enumerate(("rho", "u", "v", "w", "p")):
        np.testing.assert_allclose(mean[c], x0[k], rtol=0, atol=1e-14)
        np.testing.assert_allclose(rms[c], abs(amp[k]) / math.sqrt(2), rtol=1e-9, atol=0)
    assert rs.n == M


def test_constant_state_has_zero_rms():
    shape = (2, 3, 4)
    q = sy.conserved_from_primitive(np.full(shape, 1.3), np.full(shape, 0.4),
                                    np.zeros(shape), np.zeros(shape), np.full(shape, 0.8), GAMMA)
    rs = RunningStats(shape, GAMMA)
    for _ in range(5):
        rs.add(q)
    mean, rms = rs.mean_rms()
    np.testing.assert_allclose(mean, primitives(q, GAMMA), rtol=1e-15, atol=0)
    assert np.all(rms <= 1e-7)  # sqrt of a cancelled difference of equal sums


def test_azimuthal_average_of_harmonics():
    nk, nj, ni = 16, 3, 4
    k = np.arange(nk)[:, None, None]
    f = 2.5 + np.zeros((nk, nj, ni))
    for m in range(1, nk):
        f = f + (0.3 / m) * np.cos(2 * math.pi * m * k / nk + 0.7 * m)
    np.testing.assert_allclose(azimuthal_average(f), 2.5, rtol=0, atol=1e-14)
    # leading axes are kept
    g = np.stack([f, 2 * f])
    np.testing.assert_allclose(azimuthal_average(g), [[[2.5] * ni] * nj, [[5.0] * ni] * nj],
                               rtol=0, atol=1e-14)


def test_jet_products_pick_rows_and_columns():
    nk, nj, ni = 4, 5, 6
    j = np.arange(nj)[None, :, None]
    i = np.arange(ni)[None, None, :]
    mean = np.zeros((5, nk, nj, ni))
    rms = np.zeros((5, nk, nj, ni))
    for c in range(5):
        mean[c] = (c + 1) * 100 + 10 * j + i + np.zeros((nk, 1, 1))
        rms[c] = (c + 1) * 1000 + 10 * j + i + np.zeros((nk, 1, 1))
    out = jet_products(mean, rms, stations=(2, 5))
    np.testing.assert_array_equal(out["centreline_u_mean"], 200 + np.arange(ni))
    np.testing.assert_array_equal(out["centreline_u_rms"], 2000 + np.arange(ni))
    for s in (2, 5):
        np.testing.assert_array_equal(out[f"radial_u_mean_i{s}"], 200 + 10 * np.arange(nj) + s)
        np.testing.assert_array_equal(out[f"radial_u_rms_i{s}"], 2000 + 10 * np.arange(nj) + s)
        np.testing.assert_array_equal(out[f"radial_rho_mean_i{s}"], 100 + 10 * np.arange(nj) + s)
        np.testing.assert_array_equal(out[f"radial_p_mean_i{s}"], 500 + 10 * np.arange(nj) + s)
