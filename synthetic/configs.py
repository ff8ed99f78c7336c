"""Parameter sets for the workloads (plain data; both the oracle's and the library's
bindings translate a :class:`Params` into their own C structs)."""
from __future__ import annotations

import dataclasses
import numpy as np

from .fields import jet_field, tgv_field
from .grids import cartesian_periodic_grid, jet_grid

BC_PERIODIC = 0
BC_AXIS = 1
BC_JET_INFLOW = 2
BC_FARFIELD = 3
BC_EXIT = 4

# Sutherland constant 110.4 K over an unheated reference temperature of 288.15 K.
SUTHERLAND_S1 = 110.4 / 288.15

# Uneven member grids of the batched ensemble (n_axial, n_radial, n_azimuthal), four each.
ENSEMBLE_SHAPES = [(64, 64, 64), (96, 64, 64), (128, 96, 96), (160, 96, 96)]


@dataclasses.dataclass
class Params:
    ni: int
    nj: int
    nk: int
    bc: tuple = (BC_PERIODIC,) * 6
    period_shift: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((3, 3)))
    gamma: float = 1.4
    prandtl: float = 0.72
    prandtl_sgs: float = 0.6
    re_acoustic: float = 0.0        # rho_ref a_ref L / mu_ref; 0 switches molecular viscosity off
    suth_s1: float = SUTHERLAND_S1
    cs: float = 0.18
    k2: float = 0.25
    k4: float = 0.016
    mach_jet: float = 1.4
    jet_radius: float = 0.5
    rho_inf: float = 1.0
    u_inf: tuple = (0.05, 0.0, 0.0)
    p_inf: float = 1.0 / 1.4
    precision: int = 0               # 0 FP64, 1 mixed
    closure: int = 0                 # 0 Smagorinsky, 1 learned MLP

    @property
    def shape(self):
        return (self.nk, self.nj, self.ni)

    @property
    def n(self):
        return self.ni * self.nj * self.nk

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def box_params(n, shift, **kw):
    """Triply periodic box."""
    return Params(ni=n[0], nj=n[1], nk=n[2], bc=(BC_PERIODIC,) * 6,
                  period_shift=np.asarray(shift, dtype=np.float64), **kw)


def tgv_params(n=32, **kw):
    """Taylor-Green vortex: Mach 0.1, Re 1600 on V0 and L, so the acoustic Reynolds number
    is 1600/0.1 = 16000; Smagorinsky C_s = 0.17."""
    kw.setdefault("re_acoustic", 1600.0 / 0.1)
    kw.setdefault("cs", 0.17)
    _, shift = cartesian_periodic_grid((n, n, n))
    return box_params((n, n, n), shift, **kw)


def jet_params(n, **kw):
    """Jet: entrance i-, exit i+, axis j-, far field j+, periodic azimuth.
    Re_D = 1e5 on U_j = 1.4 a_j, so the acoustic Reynolds number is 1e5/1.4."""
    kw.setdefault("re_acoustic", 1.0e5 / 1.4)
    kw.setdefault("cs", 0.18)
    gamma = kw.get("gamma", 1.4)
    kw.setdefault("p_inf", 1.0 / gamma)
    return Params(ni=n[0], nj=n[1], nk=n[2],
                  bc=(BC_JET_INFLOW, BC_EXIT, BC_AXIS, BC_FARFIELD, BC_PERIODIC, BC_PERIODIC),
                  period_shift=np.zeros((3, 3)), **kw)


def make_case(name, n=None, seed=0):
    """Return (params, xyz, q) for a named workload."""
    if name == "tgv":
        n = n or 32
        xyz, _ = cartesian_periodic_grid((n, n, n))
        p = tgv_params(n)
        q = tgv_field(xyz, gamma=p.gamma, seed=seed)
        return p, xyz, q
    if name == "jet":
        n = n or (256, 128, 128)
        xyz, _ = jet_grid(n)
        p = jet_params(n)
        q = jet_field(xyz, gamma=p.gamma, mach_jet=p.mach_jet, u_inf=p.u_inf[0], seed=seed)
        return p, xyz, q
    raise ValueError(name)


def make_ensemble(precision=1, shapes=None, copies=4):
    """The batched ensemble: `copies` seeded jet realisations of each grid shape (seeds
    0, 1, 2, ... in member order, shapes in the given order, each repeated `copies` times).
    Returns a list of (params, xyz, q)."""
    shapes = shapes or ENSEMBLE_SHAPES
    out, seed = [], 0
    grids = {}
    for n in shapes:
        for _ in range(copies):
            if n not in grids:
                grids[n] = jet_grid(n)[0]
            xyz = grids[n]
            p = jet_params(n, precision=precision)
            q = jet_field(xyz, gamma=p.gamma, mach_jet=p.mach_jet, u_inf=p.u_inf[0], seed=seed)
            out.append((p, xyz, q))
            seed += 1
    return out


__all__ = ["Params", "BC_PERIODIC", "BC_AXIS", "BC_JET_INFLOW", "BC_FARFIELD", "BC_EXIT",
           "tgv_params", "jet_params", "box_params", "make_case", "make_ensemble",
           "ENSEMBLE_SHAPES", "SUTHERLAND_S1"]
