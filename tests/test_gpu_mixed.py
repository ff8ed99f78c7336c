"""GPU parity of the mixed-precision form (FP32 flux and stencil arithmetic; FP64 state,
Runge-Kutta accumulation, J^-1 and time-step reduction) against the FP64 oracle.

Bar: per-component relative L2 <= 2e-5 for the residual and for the state increment of
a few Runge-Kutta steps, on the jet grids (the mixed-precision workload is a jet) and on a
skewed periodic box. The Mach 0.1 Taylor-Green box is reported: its mass and energy
residuals are O(M^2)-small differences of O(M) fluxes, beyond FP32 at 2e-5, so only its
momentum components are held to the bar."""
import numpy as np
import pytest

import oracle
from gpu_cases import case, rel_l2

pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _mixed(p, xyz):
    from paper_2212_12365_amd.lesmi import Context
    return Context(p.replace(precision=1), xyz)


@pytest.mark.parametrize("name", ["skew24", "skew_odd", "jet_ragged", "jet_small", "jet_mesh6",
                                  "jet_mesh10", "tgv32"])
def test_mixed_residual(torch, name):
    print(f"[gpu] mixed residual {name}", flush=True)
    p, xyz, q = case(name)
    o = oracle.Oracle(p, xyz)
    if p.bc[0] != 0:
        q = o.apply_bc(q)
    ref = o.residual(q)
    ctx = _mixed(p, xyz)
    got = ctx.residual(torch.from_numpy(q).cuda()).cpu().numpy()
    err = rel_l2(got, ref)
    print(f"mixed residual rel-L2 {name}: {err}")
    comps = [1, 2, 3] if name == "tgv32" else range(5)
    assert all(err[c] <= TOL for c in comps), err
    ctx.close()


@pytest.mark.parametrize("name,nsteps", [("skew24", 4), ("jet_ragged", 6), ("jet_small", 4)])
def test_mixed_step_increment(torch, name, nsteps):
    print(f"[gpu] mixed step {name}", flush=True)
    p, xyz, q = case(name)
    o = oracle.Oracle(p, xyz)
    if p.bc[0] != 0:
        q = o.apply_bc(q)
    ref, dt_ref = o.step(q, nsteps, cfl=0.5)
    ctx = _mixed(p, xyz)
    g = torch.from_numpy(q).cuda()
    dt = ctx.step(g, nsteps, cfl=0.5)
    got = g.cpu().numpy()
    # The time step is reduced in FP64 from the FP64 state.
    assert dt == pytest.approx(dt_ref, rel=1e-7)
    err = rel_l2(got - q, ref - q)
    print(f"mixed {nsteps}-step increment rel-L2 {name}: {err}")
    assert np.all(err <= TOL), err
    ctx.close()


def test_mixed_sgs_viscosity(torch):
    print("[gpu] mixed sgs", flush=True)
    p, xyz, q = case("jet_small")
    o = oracle.Oracle(p, xyz)
    ref = o.sgs_viscosity(q)
    ctx = _mixed(p, xyz)
    got = ctx.sgs_viscosity(torch.from_numpy(q).cuda()).cpu().numpy()
    assert rel_l2(got[None], ref[None])[0] <= 1e-5
    ctx.close()
