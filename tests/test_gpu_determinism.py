"""Repeatability of the HIP path: two runs from the same state are bitwise equal, and a run
stopped, copied to the host (a checkpoint) and resumed in a fresh context equals the
straight run bitwise. Both hold because every reduction has a fixed order or is a minimum."""
import numpy as np
import pytest

import oracle
from gpu_cases import case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _start(name):
    p, xyz, q = case(name)
    if p.bc[0] != 0:
        q = oracle.Oracle(p, xyz).apply_bc(q)
    return p, xyz, q


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["jet_ragged", "skew_odd"])
def test_two_runs_bitwise_equal(torch, name, precision):
    print(f"[gpu] repeat {name} precision={precision}", flush=True)
    from paper_2212_12365_amd.lesmi import Context
    p, xyz, q = _start(name)
    outs = []
    for _ in range(2):
        ctx = Context(p.replace(precision=precision), xyz)
        g = torch.from_numpy(q).cuda()
        dt = ctx.step(g, 4, cfl=0.5)
        r = ctx.residual(g)
        outs.append((g.cpu().numpy(), r.cpu().numpy(), dt))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("precision", [0, 1])
def test_checkpoint_resume_bitwise_equal(torch, precision):
    print(f"[gpu] checkpoint/resume precision={precision}", flush=True)
    from paper_2212_12365_amd.lesmi import Context
    p, xyz, q = _start("jet_small")
    pp = p.replace(precision=precision)
    ctx = Context(pp, xyz)
    g = torch.from_numpy(q).cuda()
    dt_straight = ctx.step(g, 6, cfl=0.5)
    straight = g.cpu().numpy()
    ctx.close()
    ctx = Context(pp, xyz)
    g = torch.from_numpy(q).cuda()
    ctx.step(g, 3, cfl=0.5)
    saved = g.cpu().numpy().copy()  # the checkpoint: the conserved state on the host
    ctx.close()
    ctx = Context(pp, xyz)
    g = torch.from_numpy(saved).cuda()
    dt_resumed = ctx.step(g, 3, cfl=0.5)
    assert np.array_equal(g.cpu().numpy(), straight)
    assert dt_resumed == dt_straight
    ctx.close()
