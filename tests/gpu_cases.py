"""Seeded parity cases shared by the GPU tests (inputs only; expected values always come
from the oracle)."""
import math

import numpy as np

import synthetic as sy
from synthetic.grids import jet_grid, skewed_periodic_grid


def smooth_field(xyz, gamma, amp=0.05, seed=0):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * math.pi, 5)
    x, y, z = xyz
    rho = 1.0 + amp * np.sin(x + ph[0]) * np.cos(y + z)
    u = 0.3 + amp * np.cos(x + y + ph[1]) * np.sin(z)
    v = -0.2 + amp * np.sin(y + ph[2]) * np.cos(x - z)
    w = 0.1 + amp * np.cos(z + 2 * x + ph[3]) * np.sin(y)
    p = 1.0 / gamma + amp * np.cos(x - y + ph[4]) * np.sin(z)
    return sy.conserved_from_primitive(rho, u, v, w, p, gamma)


def case(name):
    """Return (params, xyz, q) for a named parity case."""
    if name == "tgv32":
        return sy.make_case("tgv", 32)
    if name == "box4":  # smallest supported grid
        xyz, sh = skewed_periodic_grid((4, 4, 4))
        p = sy.box_params((4, 4, 4), sh, re_acoustic=100.0, cs=0.18)
        return p, xyz, smooth_field(xyz, p.gamma, seed=4)
    if name == "skew24":
        xyz, sh = skewed_periodic_grid((24, 20, 18))
        p = sy.box_params((24, 20, 18), sh, re_acoustic=200.0, cs=0.18)
        return p, xyz, smooth_field(xyz, p.gamma, seed=1)
    if name == "skew_odd":  # ragged tiles in every direction, wraps past the grid's end
        xyz, sh = skewed_periodic_grid((37, 22, 9))
        p = sy.box_params((37, 22, 9), sh, re_acoustic=150.0, cs=0.18)
        return p, xyz, smooth_field(xyz, p.gamma, seed=7)
    if name.startswith("jet"):
        # jet_mesh6 and jet_mesh10: meshes 6 and 10 of the paper's mesh table (a thin
        # azimuthal direction, and the table's smallest mesh); jet_wide: more azimuthal nodes
        # than one LDS chunk of the centreline mean (256) and the fewest axial stations.
        shapes = {"jet_small": (64, 48, 32), "jet_ragged": (37, 21, 12),
                  "jet_c2": (256, 128, 128), "jet_mesh6": (400, 150, 10),
                  "jet_mesh10": (200, 75, 20), "jet_wide": (5, 9, 300)}
        n = shapes[name]
        xyz, _ = jet_grid(n)
        p = sy.jet_params(n)
        q = sy.jet_field(xyz, gamma=p.gamma, mach_jet=p.mach_jet, u_inf=p.u_inf[0], seed=0)
        return p, xyz, q
    raise ValueError(name)


def rel_l2(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1) if a.ndim > 1 else np.asarray(a)[None]
    b = np.asarray(b).reshape(a.shape)
    num = np.sqrt(((a - b) ** 2).sum(axis=1))
    den = np.sqrt((b ** 2).sum(axis=1))
    return num / np.where(den > 0, den, 1.0)
