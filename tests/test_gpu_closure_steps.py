"""The learned-closure time step on the GPU against the oracle, stage by stage through
les_step (the per-stage path: node records, network inference overwriting the eddy
viscosity, face kernel), in both precisions.

1. A network with constant output c = C_s^2 (zero output weights, b3 = softplus^-1(C_s^2)):
   the learned closure is then the paper's Smagorinsky model (Subgrid Scale Modeling) up to
   the FP32 rounding of c, so four closure steps must match the oracle's own Smagorinsky
   steps. Bar: FP64 relative L2 <= 1e-12 + 1e-6 E, mixed <= 2e-5, where E is the relative
   size of the whole subgrid effect on the state (oracle with C_s against oracle with
   C_s = 0) and 1e-6 covers the FP32 rounding of c (6e-8 relative) with margin.
2. A random network at initialisation scale, input range wide open (no fallback except
   |S| = 0, where mu_t = 0 anyway): three closure steps against the oracle's closure step
   (oracle/mlp.py closure_step, the FP64 network at every stage). The GPU evaluates the
   network with split-BF16 products, relative error of c below 1e-3 on such networks; that
   error reaches the state only through the subgrid flux. Bar: relative L2 per component
   <= 2e-3 E + 1e-12 (FP64), and that plus 2e-5 (mixed), with E as above for this network.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from gpu_cases import case, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _announce(what):
    print(f"[gpu] {what}", flush=True)


def _random_net(seed):
    rng = np.random.default_rng(seed)
    th = np.empty(omlp.NPARAMS)
    th[omlp.OFF_W1:omlp.OFF_B1] = rng.normal(scale=1 / math.sqrt(6), size=omlp.OFF_B1)
    th[omlp.OFF_B1:omlp.OFF_W2] = rng.normal(scale=0.1, size=64)
    th[omlp.OFF_W2:omlp.OFF_B2] = rng.normal(scale=1 / 8, size=64 * 64)
    th[omlp.OFF_B2:omlp.OFF_W3] = rng.normal(scale=0.1, size=64)
    th[omlp.OFF_W3:omlp.OFF_B3] = rng.normal(scale=1 / 8, size=64)
    th[omlp.OFF_B3] = -3.0
    return th.astype(np.float32).astype(np.float64)


def _gpu_closure_run(torch, p, xyz, q, theta, norm_arrays, precision, nsteps):
    from paper_2212_12365_amd.lesmi import Context, les_mlp_norm
    ctx = Context(p.replace(precision=precision, closure=1), xyz)
    nm = les_mlp_norm.from_arrays(*norm_arrays)
    ctx.mlp_set_network(torch.from_numpy(theta.astype(np.float32)).cuda(), nm)
    g = torch.from_numpy(q).cuda()
    dt = ctx.step(g, nsteps, cfl=0.5)
    out = g.cpu().numpy()
    ctx.close()
    return out, dt


OPEN = (np.zeros(6), np.ones(6), np.full(6, -1e30), np.full(6, 1e30))


@pytest.mark.parametrize("precision", [0, 1])
def test_constant_network_closure_steps_match_smagorinsky(torch, precision):
    _announce(f"closure steps, constant network, precision={precision}")
    p, xyz, q = case("jet_small")
    o = oracle.Oracle(p, xyz)
    q = o.apply_bc(q)
    cs2 = p.cs ** 2
    th = np.zeros(omlp.NPARAMS)
    th[omlp.OFF_B3] = math.log(math.expm1(cs2))
    th = th.astype(np.float32).astype(np.float64)
    got, dt = _gpu_closure_run(torch, p, xyz, q, th, OPEN, precision, 4)
    ref, dtref = o.step(q, 4, cfl=0.5)
    nosgs, _ = oracle.Oracle(p.replace(cs=0.0), xyz).step(q, 4, cfl=0.5)
    E = rel_l2(ref, nosgs)
    err = rel_l2(got, ref)
    print("constant-network closure vs Smagorinsky oracle", err, "subgrid effect", E)
    assert np.all(E > 1e-9)   # the subgrid model acts on this field
    bar = 1e-12 + 1e-6 * E if precision == 0 else 2e-5 + 1e-6 * E
    assert np.all(err <= bar), (err, bar)
    # The last step's dt is reduced from a state that already differs by the FP32 rounding
    # of c (about 1e-8 here): relative 1e-6.
    assert abs(dt - dtref) <= 1e-6 * dtref


@pytest.mark.parametrize("precision", [0, 1])
def test_network_closure_steps_match_oracle_closure_steps(torch, precision):
    _announce(f"closure steps, random network, precision={precision}")
    p, xyz, q = case("jet_small")
    o = oracle.Oracle(p, xyz)
    q = o.apply_bc(q)
    cs2 = p.cs ** 2
    th = _random_net(5)
    got, dt = _gpu_closure_run(torch, p, xyz, q, th, OPEN, precision, 3)
    ref, dtref = omlp.closure_step(o, th, OPEN, cs2, q, 3, cfl=0.5)
    nosgs, _ = oracle.Oracle(p.replace(cs=0.0), xyz).step(q, 3, cfl=0.5)
    E = rel_l2(ref, nosgs)
    err = rel_l2(got, ref)
    print("network closure vs oracle closure step", err, "subgrid effect", E)
    assert np.all(E > 1e-9)
    bar = 2e-3 * E + (1e-12 if precision == 0 else 2e-5)
    assert np.all(err <= bar), (err, bar)
    assert abs(dt - dtref) <= 1e-6 * dtref
