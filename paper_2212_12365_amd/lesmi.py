"""Python binding of liblesmi.so (C ABI in include/lesmi.h).

Argument marshalling only: every step of the residual, boundary conditions and time
stepping runs in the library's HIP kernels. Device arrays are torch float64 CUDA (ROCm)
tensors, used purely as device memory; the stream is torch's current stream unless one
is given. There is no CPU fallback: if the library is missing or the GPU is absent the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblesmi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lesmi.h")

LES_OK, LES_EINVAL, LES_ENOMEM, LES_EGRID, LES_EHIP, LES_ENONFINITE, LES_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "LES_OK", -1: "LES_EINVAL", -2: "LES_ENOMEM", -3: "LES_EGRID",
                -4: "LES_EHIP", -5: "LES_ENONFINITE", -6: "LES_ESTATE"}


class LesError(RuntimeError):
    def __init__(self, code, what, msg=""):
        super().__init__(f"{what}: {STATUS_NAMES.get(code, code)} {msg}")
        self.code = code


class les_params(ctypes.Structure):
    _fields_ = [
        ("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
        ("bc", ctypes.c_int * 6),
        ("period_shift", ctypes.c_double * 9),
        ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("prandtl_sgs", ctypes.c_double), ("re_acoustic", ctypes.c_double),
        ("suth_s1", ctypes.c_double), ("cs", ctypes.c_double),
        ("k2", ctypes.c_double), ("k4", ctypes.c_double),
        ("mach_jet", ctypes.c_double), ("jet_radius", ctypes.c_double),
        ("rho_inf", ctypes.c_double), ("u_inf", ctypes.c_double * 3),
        ("p_inf", ctypes.c_double),
        ("precision", ctypes.c_int), ("closure", ctypes.c_int),
    ]


class les_mlp_norm(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_float * 6), ("inv_std", ctypes.c_float * 6),
                ("lo", ctypes.c_float * 6), ("hi", ctypes.c_float * 6)]

    @classmethod
    def from_arrays(cls, mean, inv_std, lo, hi):
        n = cls()
        for i in range(6):
            n.mean[i], n.inv_std[i] = float(mean[i]), float(inv_std[i])
            n.lo[i], n.hi[i] = float(lo[i]), float(hi[i])
        return n

    def arrays(self):
        return tuple(np.array(list(a), dtype=np.float64)
                     for a in (self.mean, self.inv_std, self.lo, self.hi))


MLP_NPARAMS = 4673

_lib = None


def load():
    """Load liblesmi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python paper_2212_12365_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        lib.les_init_grid.argtypes = [ctypes.POINTER(les_params), dp, ctypes.POINTER(vp)]
        lib.les_residual.argtypes = [vp, vp, vp, vp]
        lib.les_step.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, vp]
        lib.les_sgs_viscosity.argtypes = [vp, vp, vp, vp]
        lib.les_apply_bc.argtypes = [vp, vp, vp]
        lib.les_diagnostics.argtypes = [vp, vp, dp, vp]
        lib.les_get_metrics.argtypes = [vp, vp, vp, vp]
        lib.les_updated_nodes.argtypes = [vp]
        lib.les_updated_nodes.restype = ctypes.c_longlong
        lib.les_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        lib.les_set_graph.argtypes = [vp, ctypes.c_int]
        lib.les_dual_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_double, dp, vp]
        lib.les_tuning_count.argtypes = []
        lib.les_tuning_name.argtypes = [ctypes.c_int]
        lib.les_tuning_name.restype = ctypes.c_char_p
        lib.les_profile.argtypes = [vp, ctypes.c_int]
        lib.les_profile_read.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_longlong)]
        ip = ctypes.POINTER(ctypes.c_int)
        lib.les_autotune.argtypes = [vp, vp, ip, ip, vp]
        lib.les_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp)]
        lib.les_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, dp, vp]
        lib.les_batch_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        lib.les_batch_get_tuning.argtypes = [vp, ip, ip]
        lib.les_batch_autotune.argtypes = [vp, ctypes.POINTER(vp), ip, ip, vp]
        lib.les_batch_set_graph.argtypes = [vp, ctypes.c_int]
        lib.les_batch_destroy.argtypes = [vp]
        lib.les_batch_destroy.restype = None
        lib.les_batch_last_error.argtypes = [vp]
        lib.les_batch_last_error.restype = ctypes.c_char_p
        lib.les_fwh_create.argtypes = [vp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(vp)]
        lib.les_fwh_nodes.argtypes = [vp]
        lib.les_fwh_samples.argtypes = [vp]
        lib.les_fwh_geometry.argtypes = [vp, vp, vp]
        lib.les_fwh_sample.argtypes = [vp, vp, vp]
        lib.les_fwh_reset.argtypes = [vp]
        lib.les_fwh_pressure.argtypes = [vp, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, vp, vp,
                                         ctypes.POINTER(ctypes.c_longlong), vp]
        lib.les_fwh_destroy.argtypes = [vp]
        lib.les_fwh_last_error.argtypes = [vp]
        lib.les_fwh_last_error.restype = ctypes.c_char_p
        fp = ctypes.c_void_p
        np_ = ctypes.POINTER(les_mlp_norm)
        lib.les_mlp_set_network.argtypes = [vp, fp, np_]
        lib.les_mlp_fallback_count.argtypes = [vp, ctypes.POINTER(ctypes.c_ulonglong)]
        lib.les_mlp_features.argtypes = [vp, vp, fp, fp, vp]
        lib.les_mlp_coefficient.argtypes = [fp, np_, ctypes.c_float, fp, fp, ctypes.c_longlong,
                                            fp, vp, vp]
        lib.les_mlp_work_size.argtypes = [ctypes.c_longlong]
        lib.les_mlp_work_size.restype = ctypes.c_longlong
        lib.les_mlp_loss_grad.argtypes = [fp, np_, fp, ctypes.c_longlong, fp, fp, vp,
                                          ctypes.c_longlong, ctypes.c_float, fp, fp, fp, vp]
        lib.les_mlp_loss_grad_noalloc.argtypes = [fp, np_, fp, ctypes.c_longlong, fp, fp, vp,
                                                  ctypes.c_longlong, ctypes.c_float, fp, fp, vp]
        lib.les_mlp_adam.argtypes = [fp, fp, fp, fp, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, vp]
        lib.les_mlp_fit_norm.argtypes = [fp, fp, ctypes.c_longlong, ctypes.c_float, np_, vp]
        lib.les_filter_target.argtypes = [vp, vp, vp, ctypes.c_float, vp, vp, fp, fp, fp, fp, vp]
        lib.les_residual_norms.argtypes = [vp, vp, dp, vp]
        lib.les_stats_reset.argtypes = [vp]
        lib.les_stats_accumulate.argtypes = [vp, vp, vp]
        lib.les_stats_read.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_longlong), vp]
        lib.les_stats_azimuthal.argtypes = [vp, vp, vp]
        lib.les_destroy.argtypes = [vp]
        lib.les_destroy.restype = None
        lib.les_last_error.argtypes = [vp]
        lib.les_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def header_functions():
    """Names of the functions include/lesmi.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(les_[a-z0-9_]+)\s*\(", text)))


def make_params(p):
    s = les_params()
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
    s.precision, s.closure = int(p.precision), int(p.closure)
    return s


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _dev(t, n_expected, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous() or t.numel() != n_expected:
        raise ValueError(f"{what}: expected a contiguous float64 GPU tensor of "
                         f"{n_expected} elements")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, n_expected, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
            or not t.is_contiguous() or t.numel() != n_expected:
        raise ValueError(f"{what}: expected a contiguous float32 GPU tensor of "
                         f"{n_expected} elements")
    return ctypes.c_void_p(t.data_ptr())


def _lib_check(rc, what):
    if rc != LES_OK:
        raise LesError(rc, what)


class Context:
    """One grid and parameter set on the current GPU (les_init_grid .. les_destroy)."""

    def __init__(self, params, xyz, allow_bad_grid=False):
        self.lib = load()
        self.params = params
        self.n = params.ni * params.nj * params.nk
        self.shape = params.shape
        self._s = make_params(params)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        if xyz.size != 3 * self.n:
            raise ValueError("xyz must hold 3 * ni * nj * nk values")
        h = ctypes.c_void_p()
        rc = self.lib.les_init_grid(ctypes.byref(self._s),
                                    xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.byref(h))
        self.handle = h
        self.init_status = rc
        if rc != LES_OK and not (rc == LES_EGRID and allow_bad_grid and h.value):
            msg = self.lib.les_last_error(h).decode() if h.value else ""
            if h.value:
                self.lib.les_destroy(h)
                self.handle = ctypes.c_void_p()
            raise LesError(rc, "les_init_grid", msg)

    def _check(self, rc, what):
        if rc != LES_OK:
            raise LesError(rc, what, self.lib.les_last_error(self.handle).decode())

    def residual(self, q, rhs=None, stream=None):
        import torch
        if rhs is None:
            rhs = torch.empty_like(q)
        self._check(self.lib.les_residual(self.handle, _dev(q, 5 * self.n, "q"),
                                          _dev(rhs, 5 * self.n, "rhs"), _stream(stream)),
                    "les_residual")
        return rhs

    def step(self, q, nsteps, cfl=0.5, dt_fixed=0.0, stream=None):
        dt = ctypes.c_double(0.0)
        self._check(self.lib.les_step(self.handle, _dev(q, 5 * self.n, "q"), int(nsteps),
                                      float(cfl), float(dt_fixed), ctypes.byref(dt),
                                      _stream(stream)), "les_step")
        return dt.value

    def dual_step(self, q, nsteps, dt, subiters, cfl_tau, q_prev=None, stream=None):
        """les_dual_step; returns the residual history [nsteps][subiters] (numpy)."""
        res = np.zeros(max(nsteps * subiters, 1))
        prev = _dev(q_prev, 5 * self.n, "q_prev") if q_prev is not None else None
        self._check(self.lib.les_dual_step(self.handle, _dev(q, 5 * self.n, "q"), prev,
                                           int(nsteps), float(dt), int(subiters), float(cfl_tau),
                                           res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           _stream(stream)), "les_dual_step")
        return res[:nsteps * subiters].reshape(nsteps, subiters)

    def sgs_viscosity(self, q, mu_t=None, stream=None):
        import torch
        if mu_t is None:
            mu_t = torch.empty(self.shape, dtype=torch.float64, device=q.device)
        self._check(self.lib.les_sgs_viscosity(self.handle, _dev(q, 5 * self.n, "q"),
                                               _dev(mu_t, self.n, "mu_t"), _stream(stream)),
                    "les_sgs_viscosity")
        return mu_t

    def apply_bc(self, q, stream=None):
        self._check(self.lib.les_apply_bc(self.handle, _dev(q, 5 * self.n, "q"),
                                          _stream(stream)), "les_apply_bc")
        return q

    def diagnostics(self, q, stream=None):
        out = np.zeros(6)
        self._check(self.lib.les_diagnostics(self.handle, _dev(q, 5 * self.n, "q"),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             _stream(stream)), "les_diagnostics")
        return out

    def residual_norms(self, q, stream=None):
        """(r.m.s., max) of the mass residual over updated nodes."""
        out = np.zeros(2)
        self._check(self.lib.les_residual_norms(self.handle, _dev(q, 5 * self.n, "q"),
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                _stream(stream)), "les_residual_norms")
        return out

    def stats_reset(self):
        self._check(self.lib.les_stats_reset(self.handle), "les_stats_reset")

    def stats_accumulate(self, q, stream=None):
        self._check(self.lib.les_stats_accumulate(self.handle, _dev(q, 5 * self.n, "q"),
                                                  _stream(stream)), "les_stats_accumulate")

    def stats_read(self, stream=None):
        """(mean [5][N], rms [5][N], samples) of (rho, u, v, w, p)."""
        import torch
        mean = torch.empty((5,) + self.shape, dtype=torch.float64, device="cuda")
        rms = torch.empty_like(mean)
        n = ctypes.c_longlong(0)
        self._check(self.lib.les_stats_read(self.handle, _dev(mean, 5 * self.n, "mean"),
                                            _dev(rms, 5 * self.n, "rms"), ctypes.byref(n),
                                            _stream(stream)), "les_stats_read")
        return mean, rms, n.value

    def stats_azimuthal(self, stream=None):
        """Azimuthal averages of the time mean and r.m.s. of (rho, u, v, w, p): a tensor
        [2][5][nj][ni] (les_stats_azimuthal)."""
        import torch
        nk, nj, ni = self.shape
        out = torch.empty((2, 5, nj, ni), dtype=torch.float64, device="cuda")
        self._check(self.lib.les_stats_azimuthal(self.handle, _dev(out, 10 * nj * ni, "out"),
                                                 _stream(stream)), "les_stats_azimuthal")
        return out

    def metrics(self, stream=None):
        import torch
        S = torch.empty((9,) + self.shape, dtype=torch.float64, device="cuda")
        jinv = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        self._check(self.lib.les_get_metrics(self.handle, _dev(S, 9 * self.n, "S"),
                                             _dev(jinv, self.n, "jinv"), _stream(stream)),
                    "les_get_metrics")
        return S, jinv

    def set_tuning(self, tile, kmin=8):
        self._check(self.lib.les_set_tuning(self.handle, int(tile), int(kmin)), "les_set_tuning")

    def set_graph(self, enable):
        self._check(self.lib.les_set_graph(self.handle, int(bool(enable))), "les_set_graph")

    def tuning_names(self):
        return [self.lib.les_tuning_name(t).decode() for t in range(self.lib.les_tuning_count())]

    def profile(self, enable=True):
        self._check(self.lib.les_profile(self.handle, int(bool(enable))), "les_profile")

    def profile_read(self):
        """(node-kernel ms, face-kernel ms, timed stages) summed since the last read."""
        tn = ctypes.c_double(0.0)
        tf = ctypes.c_double(0.0)
        n = ctypes.c_longlong(0)
        self._check(self.lib.les_profile_read(self.handle, ctypes.byref(tn), ctypes.byref(tf),
                                              ctypes.byref(n)), "les_profile_read")
        return tn.value, tf.value, n.value

    def autotune(self, q, stream=None):
        """Times every stage-kernel launch shape on residuals of q; keeps and returns the
        fastest (tile, kmin)."""
        t, k = ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.les_autotune(self.handle, _dev(q, 5 * self.n, "q"), ctypes.byref(t),
                                          ctypes.byref(k), _stream(stream)), "les_autotune")
        return t.value, k.value

    def updated_nodes(self):
        return int(self.lib.les_updated_nodes(self.handle))

    # Learned closure ------------------------------------------------------------------
    def mlp_set_network(self, theta, norm):
        self._check(self.lib.les_mlp_set_network(self.handle, _f32(theta, MLP_NPARAMS, "theta"),
                                                 ctypes.byref(norm)), "les_mlp_set_network")

    def mlp_fallback_count(self):
        n = ctypes.c_ulonglong(0)
        self._check(self.lib.les_mlp_fallback_count(self.handle, ctypes.byref(n)),
                    "les_mlp_fallback_count")
        return n.value

    def mlp_features(self, q, stream=None):
        """(inputs [6][N], |S| [N]) of a state, float32 GPU tensors."""
        import torch
        feat = torch.empty((6,) + self.shape, dtype=torch.float32, device="cuda")
        smag = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        self._check(self.lib.les_mlp_features(self.handle, _dev(q, 5 * self.n, "q"),
                                              _f32(feat, 6 * self.n, "feat"),
                                              _f32(smag, self.n, "smag"), _stream(stream)),
                    "les_mlp_features")
        return feat, smag

    def close(self):
        if self.handle and self.handle.value:
            self.lib.les_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several contexts advanced together (les_batch_create .. les_batch_destroy). The
    contexts must outlive the batch and are not stepped on their own meanwhile."""

    def __init__(self, contexts):
        self.lib = load()
        self.members = list(contexts)
        n = len(self.members)
        arr = (ctypes.c_void_p * n)(*[c.handle.value for c in self.members])
        h = ctypes.c_void_p()
        rc = self.lib.les_batch_create(arr, n, ctypes.byref(h))
        self.handle = h
        if rc != LES_OK:
            msg = self.lib.les_batch_last_error(h).decode() if h.value else ""
            self.close()
            raise LesError(rc, "les_batch_create", msg)

    def _check(self, rc, what):
        if rc != LES_OK:
            raise LesError(rc, what, self.lib.les_batch_last_error(self.handle).decode())

    def _states(self, qs):
        if len(qs) != len(self.members):
            raise ValueError("one state per member")
        return (ctypes.c_void_p * len(qs))(*[
            _dev(q, 5 * c.n, f"q[{i}]").value for i, (q, c) in enumerate(zip(qs, self.members))])

    def step(self, qs, nsteps, cfl=0.5, dt_fixed=0.0, stream=None):
        """Advances every member in place; returns the members' last time steps."""
        dts = np.zeros(len(self.members))
        self._check(self.lib.les_batch_step(self.handle, self._states(qs), int(nsteps),
                                            float(cfl), float(dt_fixed),
                                            dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _stream(stream)), "les_batch_step")
        return dts

    def autotune(self, qs, stream=None):
        t, k = ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.les_batch_autotune(self.handle, self._states(qs), ctypes.byref(t),
                                                ctypes.byref(k), _stream(stream)),
                    "les_batch_autotune")
        return t.value, k.value

    def set_tuning(self, tile, kmin=8):
        self._check(self.lib.les_batch_set_tuning(self.handle, int(tile), int(kmin)),
                    "les_batch_set_tuning")

    def get_tuning(self):
        t, k = ctypes.c_int(0), ctypes.c_int(0)
        self._check(self.lib.les_batch_get_tuning(self.handle, ctypes.byref(t), ctypes.byref(k)),
                    "les_batch_get_tuning")
        return t.value, k.value

    def set_graph(self, enable=True):
        self._check(self.lib.les_batch_set_graph(self.handle, int(bool(enable))),
                    "les_batch_set_graph")

    def close(self):
        if self.handle and self.handle.value:
            self.lib.les_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Learned-closure kernels that do not need a context --------------------------------------
def mlp_coefficient(theta, norm, cs2, feat, smag, stream=None):
    """c [n] (float32 GPU) and the number of fallback samples."""
    import torch
    lib = load()
    n = smag.numel()
    c = torch.empty(n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib_check(lib.les_mlp_coefficient(_f32(theta, MLP_NPARAMS, "theta"), ctypes.byref(norm),
                                       float(cs2), _f32(feat, 6 * n, "feat"),
                                       _f32(smag, n, "smag"), n, _f32(c, n, "c"),
                                       ctypes.c_void_p(fb.data_ptr()), _stream(stream)),
               "les_mlp_coefficient")
    return c, int(fb.item())


def mlp_work_size(n):
    return int(load().les_mlp_work_size(int(n)))


def mlp_loss_grad(theta, norm, feat, target, weight, idx, inv_wsum, work=None, stream=None):
    """(grad [NPARAMS], loss [1]) float32 GPU tensors for the samples idx (int32 GPU)."""
    import torch
    lib = load()
    nfeat = target.numel()
    n = idx.numel()
    if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
        raise ValueError("idx: expected a contiguous int32 GPU tensor")
    if work is None:
        work = torch.empty(mlp_work_size(n), dtype=torch.float32, device="cuda")
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _lib_check(lib.les_mlp_loss_grad(_f32(theta, MLP_NPARAMS, "theta"), ctypes.byref(norm),
                                     _f32(feat, 6 * nfeat, "feat"), nfeat,
                                     _f32(target, nfeat, "target"), _f32(weight, nfeat, "weight"),
                                     ctypes.c_void_p(idx.data_ptr()), n, float(inv_wsum),
                                     _f32(grad, MLP_NPARAMS, "grad"), _f32(loss, 1, "loss"),
                                     _f32(work, mlp_work_size(n), "work"), _stream(stream)),
               "les_mlp_loss_grad")
    return grad, loss


MLP_NOALLOC_MAX_SAMPLES = 8192


def mlp_loss_grad_noalloc(theta, norm, feat, target, weight, idx, inv_wsum, grad, loss,
                          stream=None):
    """les_mlp_loss_grad_noalloc into the given grad [NPARAMS] and loss [1] float32 GPU
    tensors (the library allocates nothing)."""
    import torch
    lib = load()
    nfeat = target.numel()
    n = idx.numel()
    if idx.dtype != torch.int32 or not idx.is_cuda or not idx.is_contiguous():
        raise ValueError("idx: expected a contiguous int32 GPU tensor")
    _lib_check(lib.les_mlp_loss_grad_noalloc(
        _f32(theta, MLP_NPARAMS, "theta"), ctypes.byref(norm), _f32(feat, 6 * nfeat, "feat"),
        nfeat, _f32(target, nfeat, "target"), _f32(weight, nfeat, "weight"),
        ctypes.c_void_p(idx.data_ptr()), n, float(inv_wsum), _f32(grad, MLP_NPARAMS, "grad"),
        _f32(loss, 1, "loss"), _stream(stream)), "les_mlp_loss_grad_noalloc")
    return grad, loss


def mlp_adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _lib_check(load().les_mlp_adam(_f32(theta, MLP_NPARAMS, "theta"),
                                   _f32(grad, MLP_NPARAMS, "grad"), _f32(m, MLP_NPARAMS, "m"),
                                   _f32(v, MLP_NPARAMS, "v"), int(step), float(lr), float(beta1),
                                   float(beta2), float(eps), _stream(stream)), "les_mlp_adam")


def mlp_fit_norm(feat, weight, widen=0.1, stream=None):
    n = weight.numel()
    out = les_mlp_norm()
    _lib_check(load().les_mlp_fit_norm(_f32(feat, 6 * n, "feat"), _f32(weight, n, "weight"), n,
                                       float(widen), ctypes.byref(out), _stream(stream)),
               "les_mlp_fit_norm")
    return out


def filter_target(fine, coarse, q_fine, smin, stream=None):
    """Box-filtered state, subgrid stress, inputs, |S~|, target and weight on the coarse
    grid (dict of GPU tensors)."""
    import torch
    nc = coarse.n
    sh = coarse.shape
    out = {"q": torch.empty((5,) + sh, dtype=torch.float64, device="cuda"),
           "sigma": torch.empty((6,) + sh, dtype=torch.float64, device="cuda"),
           "feat": torch.empty((6,) + sh, dtype=torch.float32, device="cuda"),
           "smag": torch.empty(sh, dtype=torch.float32, device="cuda"),
           "target": torch.empty(sh, dtype=torch.float32, device="cuda"),
           "weight": torch.empty(sh, dtype=torch.float32, device="cuda")}
    rc = load().les_filter_target(fine.handle, coarse.handle, _dev(q_fine, 5 * fine.n, "q_fine"),
                                  float(smin), _dev(out["q"], 5 * nc, "q_coarse"),
                                  _dev(out["sigma"], 6 * nc, "sigma"),
                                  _f32(out["feat"], 6 * nc, "feat"), _f32(out["smag"], nc, "smag"),
                                  _f32(out["target"], nc, "target"),
                                  _f32(out["weight"], nc, "weight"), _stream(stream))
    if rc != LES_OK:
        raise LesError(rc, "les_filter_target", load().les_last_error(coarse.handle).decode())
    return out


class FWH:
    """Ffowcs Williams-Hawkings control surface of a jet context (les_fwh_create ..
    les_fwh_destroy)."""

    def __init__(self, ctx, xyz, i1, i2, js, caps=3, capacity=256, dtau=1.0):
        self.lib = load()
        self.ctx = ctx
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        h = ctypes.c_void_p()
        rc = self.lib.les_fwh_create(ctx.handle,
                                     xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     int(i1), int(i2), int(js), int(caps), int(capacity),
                                     float(dtau), ctypes.byref(h))
        self.handle = h
        if rc != LES_OK:
            msg = self.lib.les_fwh_last_error(h).decode() if h.value else ""
            if h.value:
                self.lib.les_fwh_destroy(h)
            raise LesError(rc, "les_fwh_create", msg)
        self.ns = self.lib.les_fwh_nodes(h)

    def _check(self, rc, what):
        if rc != LES_OK:
            raise LesError(rc, what, self.lib.les_fwh_last_error(self.handle).decode())

    def geometry(self, stream=None):
        """[7][ns] float64 GPU tensor: positions (3), unit normals (3), areas."""
        import torch
        g = torch.empty((7, self.ns), dtype=torch.float64, device="cuda")
        self._check(self.lib.les_fwh_geometry(self.handle, _dev(g, 7 * self.ns, "geo"),
                                              _stream(stream)), "les_fwh_geometry")
        return g

    def sample(self, q, stream=None):
        self._check(self.lib.les_fwh_sample(self.handle, _dev(q, 5 * self.ctx.n, "q"),
                                            _stream(stream)), "les_fwh_sample")

    def samples(self):
        return self.lib.les_fwh_samples(self.handle)

    def reset(self):
        self._check(self.lib.les_fwh_reset(self.handle), "les_fwh_reset")

    def pressure(self, observers, times, c0, p0, tau0=0.0, stream=None):
        """(p' [no][nt], scale [no][nt]) float64 GPU tensors and the skipped count."""
        import torch
        obs = np.ascontiguousarray(observers, dtype=np.float64).reshape(-1, 3)
        tt = np.ascontiguousarray(times, dtype=np.float64).reshape(-1)
        no, nt = obs.shape[0], tt.size
        p = torch.empty((no, nt), dtype=torch.float64, device="cuda")
        sc = torch.empty_like(p)
        sk = ctypes.c_longlong(0)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.les_fwh_pressure(self.handle, obs.ctypes.data_as(dp), no,
                                              tt.ctypes.data_as(dp), nt, float(c0), float(p0),
                                              float(tau0), _dev(p, no * nt, "p"),
                                              _dev(sc, no * nt, "scale"), ctypes.byref(sk),
                                              _stream(stream)), "les_fwh_pressure")
        return p, sc, sk.value

    def close(self):
        if self.handle and self.handle.value:
            self.lib.les_fwh_destroy(self.handle)
            self.handle = ctypes.c_void_p()
