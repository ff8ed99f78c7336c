"""ctypes binding of the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is what the GPU library is checked against. Only the
tests, the package smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_BC = {"periodic": 0, "axis": 1, "inflow": 2, "farfield": 3, "exit": 4}


def build(force=True):
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
           "-Wall", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def set_threads(n):
    """Number of OpenMP threads the oracle uses from now on (for timing it)."""
    _load().omp_set_num_threads(int(n))


class _Params(ctypes.Structure):
    _fields_ = [
        ("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
        ("bc", ctypes.c_int * 6),
        ("period_shift", ctypes.c_double * 9),
        ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("prandtl_sgs", ctypes.c_double), ("re_acoustic", ctypes.c_double),
        ("suth_s1", ctypes.c_double), ("cs", ctypes.c_double), ("k2", ctypes.c_double),
        ("k4", ctypes.c_double), ("mach_jet", ctypes.c_double),
        ("jet_radius", ctypes.c_double), ("rho_inf", ctypes.c_double),
        ("u_inf", ctypes.c_double * 3), ("p_inf", ctypes.c_double),
        ("metric_form", ctypes.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.or_metrics.argtypes = [pp, dp, dp, dp]
        lib.or_sutherland.argtypes = [pp, ctypes.c_int, dp, dp]
        lib.or_sgs_viscosity.argtypes = [pp, dp, dp, dp, dp]
        lib.or_velocity_gradient.argtypes = [pp, dp, dp, dp, dp]
        lib.or_residual_mut.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.or_residual.argtypes = [pp, dp, dp, dp, dp]
        lib.or_apply_bc.argtypes = [pp, dp, dp, dp, dp]
        lib.or_dt.argtypes = [pp, dp, dp, dp, ctypes.c_double, dp]
        lib.or_step.argtypes = [pp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, dp]
        lib.or_diagnostics.argtypes = [pp, dp, dp, dp]
        _lib = lib
    return _lib


def primitives(q, gamma):
    """(rho, u, v, w, p) of a conserved state (paper, LES formulation: equation of state
    with the System-I total energy), shaped (5, ...)."""
    q = np.asarray(q, dtype=np.float64)
    rho = q[0]
    u, v, w = q[1] / rho, q[2] / rho, q[3] / rho
    p = (gamma - 1.0) * (q[4] - 0.5 * rho * (u * u + v * v + w * w))
    return np.stack([rho, u, v, w, p])


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params_struct(p, metric_form=0):
    s = _Params()
    s.ni, s.nj, s.nk = p.ni, p.nj, p.nk
    for i in range(6):
        s.bc[i] = int(p.bc[i])
    shift = np.asarray(p.period_shift, dtype=np.float64).reshape(9)
    for i in range(9):
        s.period_shift[i] = float(shift[i])
    s.gamma, s.prandtl, s.prandtl_sgs = p.gamma, p.prandtl, p.prandtl_sgs
    s.re_acoustic, s.suth_s1, s.cs, s.k2, s.k4 = p.re_acoustic, p.suth_s1, p.cs, p.k2, p.k4
    s.mach_jet, s.jet_radius, s.rho_inf = p.mach_jet, p.jet_radius, p.rho_inf
    for i in range(3):
        s.u_inf[i] = float(p.u_inf[i])
    s.p_inf = p.p_inf
    s.metric_form = metric_form
    return s


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


class Oracle:
    """The oracle bound to one parameter set and grid. Arrays are numpy float64, C order,
    shaped like the grid: xyz (3, nk, nj, ni), q and rhs (5, nk, nj, ni)."""

    def __init__(self, params, xyz, metric_form=0):
        self.lib = _load()
        self.p = params
        self.s = params_struct(params, metric_form)
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        shape = params.shape
        self.S = np.zeros((9,) + shape)
        self.jinv = np.zeros(shape)
        self.grid_rc = self.lib.or_metrics(ctypes.byref(self.s), _ptr(self.xyz), _ptr(self.S),
                                           _ptr(self.jinv))
        if self.grid_rc not in (0, -3):
            _check(self.grid_rc, "metrics")

    def residual(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        rhs = np.zeros_like(q)
        _check(self.lib.or_residual(ctypes.byref(self.s), _ptr(self.S), _ptr(self.jinv), _ptr(q),
                                    _ptr(rhs)), "residual")
        return rhs

    def residual_with_mut(self, q, mu_t):
        """Residual with the eddy viscosity field mu_t given (shape of the grid)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        mu_t = np.ascontiguousarray(mu_t, dtype=np.float64)
        rhs = np.zeros_like(q)
        _check(self.lib.or_residual_mut(ctypes.byref(self.s), _ptr(self.S), _ptr(self.jinv),
                                        _ptr(q), _ptr(mu_t), _ptr(rhs)), "residual_mut")
        return rhs

    def sgs_viscosity(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        mut = np.zeros(self.p.shape)
        _check(self.lib.or_sgs_viscosity(ctypes.byref(self.s), _ptr(self.S), _ptr(self.jinv),
                                         _ptr(q), _ptr(mut)), "sgs_viscosity")
        return mut

    def velocity_gradient(self, q):
        """d u_m / d x_n at every node, shaped (3, 3, nk, nj, ni)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        g = np.zeros((9,) + self.p.shape)
        _check(self.lib.or_velocity_gradient(ctypes.byref(self.s), _ptr(self.S), _ptr(self.jinv),
                                             _ptr(q), _ptr(g)), "velocity_gradient")
        return g.reshape((3, 3) + self.p.shape)

    def apply_bc(self, q):
        q = np.array(q, dtype=np.float64, order="C", copy=True)
        _check(self.lib.or_apply_bc(ctypes.byref(self.s), _ptr(self.xyz), _ptr(self.S),
                                    _ptr(self.jinv), _ptr(q)), "apply_bc")
        return q

    def dt(self, q, cfl):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(1)
        _check(self.lib.or_dt(ctypes.byref(self.s), _ptr(self.S), _ptr(self.jinv), _ptr(q),
                              float(cfl), _ptr(out)), "dt")
        return float(out[0])

    def step(self, q, nsteps, cfl=0.5, dt_fixed=0.0):
        """Advance a copy of q by nsteps Runge-Kutta steps; returns (q_new, dt_last)."""
        q = np.array(q, dtype=np.float64, order="C", copy=True)
        dt = np.zeros(1)
        _check(self.lib.or_step(ctypes.byref(self.s), _ptr(self.xyz), _ptr(self.S),
                                _ptr(self.jinv), _ptr(q), int(nsteps), float(cfl),
                                float(dt_fixed), _ptr(dt)), "step")
        return q, float(dt[0])

    def diagnostics(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(6)
        _check(self.lib.or_diagnostics(ctypes.byref(self.s), _ptr(self.jinv), _ptr(q), _ptr(out)),
               "diagnostics")
        return out

    def sutherland(self, T):
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        mu = np.zeros_like(T)
        _check(self.lib.or_sutherland(ctypes.byref(self.s), T.size, _ptr(T), _ptr(mu)),
               "sutherland")
        return mu
