"""GPU parity of the rows beyond the explicit step at the benchmark's full size (the
256 x 128 x 128 jet), in the configurations `bench.py` times.

* Learned closure, FP64, evaluated inside the node kernel: the residual against the oracle's
  residual with the eddy viscosity the GPU's closure gives (les_sgs_viscosity, which runs
  the separate inference kernel), relative L2 <= 1e-12 per component, so the network
  evaluated inside the node kernel agrees with the separate one; a random network at
  initialisation scale, input range open.
* Dual time, FP64: one backward-Euler step of four times the explicit CFL-0.5 step, two
  pseudo-time iterations at cfl_tau 1, against the oracle's dual step: relative L2 <= 1e-12
  per component, and the residual monitor within 1e-9 of its first value.
* Far-field noise: the bench's surface (x from 2 to 6, r = 1.5, both caps; 20,224 nodes),
  256 samples of a monopole field, 64 observers x 256 times on the GPU; the oracle at a
  sample of 4 observers x 8 times, within the rounding bound of test_gpu_fwh, and the
  skipped counts equal.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dualtime, fwh
from oracle import mlp as omlp
import synthetic as sy
from gpu_cases import rel_l2

pytestmark = pytest.mark.gpu
GRID = (256, 128, 128)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def c2():
    p, xyz, q = sy.make_case("jet", GRID, seed=0)
    o = oracle.Oracle(p, xyz)
    q = o.apply_bc(q)
    return p, xyz, q, o


def _announce(what):
    print(f"[gpu] {what}", flush=True)


def test_c2_closure_residual_fullsize(torch, c2):
    _announce("full size jet 256x128x128 fp64 closure residual")
    from paper_2212_12365_amd.lesmi import Context, les_mlp_norm
    from test_gpu_closure_steps import OPEN, _random_net
    p, xyz, q, o = c2
    ctx = Context(p.replace(closure=1), xyz)
    ctx.mlp_set_network(torch.from_numpy(_random_net(7).astype(np.float32)).cuda(),
                        les_mlp_norm.from_arrays(*OPEN))
    g = torch.from_numpy(q).cuda()
    got = ctx.residual(g).cpu().numpy()
    mut = ctx.sgs_viscosity(g).cpu().numpy()
    assert np.all(np.isfinite(mut)) and mut.max() > 0
    ref = o.residual_with_mut(q, mut)
    err = rel_l2(got, ref)
    print("C2 closure residual rel-L2", err, "fallbacks", ctx.mlp_fallback_count())
    assert np.all(err <= 1e-12), err
    ctx.close()


def test_c2_dual_time_fullsize(torch, c2):
    _announce("full size jet 256x128x128 fp64 dual time step")
    from paper_2212_12365_amd.lesmi import Context
    p, xyz, q, o = c2
    dt = 4.0 * o.dt(q, 0.5)
    ref, _, rref = dualtime.dual_step(o, q, None, 1, dt, 2, 1.0)
    ctx = Context(p, xyz)
    g = torch.from_numpy(q).cuda()
    r = ctx.dual_step(g, 1, dt, 2, 1.0)
    err = rel_l2(g.cpu().numpy(), ref)
    print("C2 dual step rel-L2", err, "residuals", r, rref)
    assert np.all(err <= 1e-12), err
    assert np.all(np.abs(r - rref) <= 1e-9 * rref[:, :1])
    ctx.close()


def test_c2_fwh_fullsize_sampled(torch, c2):
    _announce("full size jet 256x128x128 far-field noise, sampled observer times")
    from paper_2212_12365_amd.lesmi import FWH, Context
    p, xyz, q, o = c2
    r_of_j = np.hypot(xyz[1, 0, :, 0], xyz[2, 0, :, 0])
    x_of_i = xyz[0, 0, 0, :]
    js = int(np.argmin(np.abs(r_of_j - 1.5)))
    i1, i2 = int(np.argmin(np.abs(x_of_i - 2.0))), int(np.argmin(np.abs(x_of_i - 6.0)))
    src = np.array([0.5 * (x_of_i[i1] + x_of_i[i2]), 0.0, 0.0])
    M, T, A = 256, 4.0, 1e-4
    omega, dtau = 2 * math.pi / T, T / 32
    rho0, c0, p0, gam = p.rho_inf, 1.0, p.p_inf, p.gamma
    ids, y, nrm, dS = fwh.jet_surface(o.S, xyz, i1, i2, js)
    ctx = Context(p, xyz)
    f = FWH(ctx, xyz, i1, i2, js, caps=3, capacity=M, dtau=dtau)
    assert f.ns == len(ids) == 20224
    X = torch.from_numpy(xyz).cuda()
    d = X - torch.tensor(src, dtype=torch.float64, device="cuda").view(3, 1, 1, 1)
    R = torch.sqrt((d * d).sum(0))
    gq = torch.empty((5,) + p.shape, dtype=torch.float64, device="cuda")
    idt = torch.from_numpy(ids).cuda()
    rho = np.empty((M, len(ids)))
    u = np.empty((M, len(ids), 3))
    pr = np.empty((M, len(ids)))
    for m in range(M):  # the bench's monopole samples, formed on the GPU
        tr = m * dtau - R / c0
        fv = A * torch.sin(omega * tr)
        fd = A * omega * torch.cos(omega * tr)
        ur = fv / (4 * math.pi * R * R) + fd / (4 * math.pi * R * c0)
        pp = rho0 * fd / (4 * math.pi * R)
        rr = rho0 + pp / c0 ** 2
        uu = ur * d / R
        gq[0] = rr
        gq[1:4] = rr * uu
        gq[4] = (p0 + pp) / (gam - 1.0) + 0.5 * rr * (uu * uu).sum(0)
        f.sample(gq)
        qs = gq.view(5, -1)[:, idt].cpu().numpy()
        rho[m], u[m], pr[m] = fwh.sample_state(qs, np.arange(len(ids)), gam)
    ang = np.linspace(0.0, math.pi, 64)
    obs = src[None, :] + 30.0 * np.stack([np.cos(ang), np.sin(ang), 0 * ang], axis=1)
    times = np.linspace(38.0, 54.0, 256)
    got, scale, skipped = f.pressure(obs, times, c0, p0)
    got = got.cpu().numpy()
    ia, ib = np.array([0, 21, 42, 63]), np.array([0, 37, 74, 111, 148, 185, 222, 255])
    ref, ref_scale, ref_skipped = fwh.fwh_pressure(y, nrm, dS, rho, u, pr, 0.0, dtau, rho0, c0,
                                                   p0, obs[ia], times[ib])
    assert skipped == 0 and ref_skipped == 0
    Q, L = fwh.sources(rho, u, pr, nrm, p0)
    qmax = np.abs(Q).max(axis=0)
    lmax = np.sqrt(np.sum(L * L, axis=2)).max(axis=0)
    worst = 0.0
    for a, x in enumerate(obs[ia]):
        r = np.sqrt(np.sum((x[None, :] - y) ** 2, axis=1))
        bound = 1e-14 * np.sum(dS * (qmax / (dtau * r) + lmax / (dtau * c0 * r) +
                                     lmax / (r * r))) / (4 * math.pi)
        diff = np.abs(got[ia[a]][ib] - ref[a])
        worst = max(worst, float((diff / bound).max()))
        assert np.all(diff <= bound)
    print("full-size FW-H max |gpu - oracle| / bound", worst)
    np.testing.assert_allclose(scale.cpu().numpy()[np.ix_(ia, ib)], ref_scale, rtol=1e-12)
    f.close()
    ctx.close()
