"""les_step replays a captured HIP graph of one Runge-Kutta step (the default) or launches the
kernels one by one (les_set_graph(ctx, 0)); both run the same kernels in the same order, so
the states must agree bit for bit. The sequence exercises the recapture triggers (a new state
pointer, a fixed dt that changes, CFL and fixed-dt modes, a new tuning, a new network) and
replays with eager work on the same stream in between, several replays per call."""
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


def _sequence(torch, ctx, q, closure_nets=None):
    g = torch.from_numpy(q).cuda()
    g2 = torch.from_numpy(q).cuda()
    out = []
    out.append(ctx.step(g, 3, cfl=0.5))
    out.append(ctx.residual(g).cpu().numpy())        # eager work between replays
    out.append(ctx.step(g, 2, cfl=0.5))
    out.append(ctx.step(g, 2, cfl=0.0, dt_fixed=1e-4))
    out.append(ctx.step(g, 1, cfl=0.0, dt_fixed=2e-4))
    out.append(ctx.step(g2, 2, cfl=0.5))               # another state array
    ctx.set_tuning(0, 4)
    out.append(ctx.step(g, 2, cfl=0.5))
    if closure_nets:
        ctx.mlp_set_network(*closure_nets[1])
        out.append(ctx.step(g, 2, cfl=0.5))
    out.append(g.cpu().numpy())
    out.append(g2.cpu().numpy())
    return out


@pytest.mark.parametrize("precision,closure", [(0, 0), (1, 0), (0, 1)])
def test_graph_replay_equals_direct_launches(torch, precision, closure):
    print(f"[gpu] graph replay precision={precision} closure={closure}", flush=True)
    from paper_2212_12365_amd.lesmi import Context, les_mlp_norm
    p, xyz, q = case("jet_ragged")
    q = oracle.Oracle(p, xyz).apply_bc(q)
    pp = p.replace(precision=precision, closure=closure)
    nets = None
    if closure:
        from test_gpu_closure_steps import _random_net
        th = [torch.from_numpy(_random_net(seed).astype(np.float32)).cuda() for seed in (2, 3)]
        nm = [les_mlp_norm.from_arrays([0] * 6, [1] * 6, [-1e30] * 6, [1e30] * 6),
              les_mlp_norm.from_arrays([0.1] * 6, [0.9] * 6, [-1e30] * 6, [1e30] * 6)]
        nets = [(th[0], nm[0]), (th[1], nm[1])]
    results = []
    for graph in (True, False):
        ctx = Context(pp, xyz)
        ctx.set_graph(graph)
        if nets:
            ctx.mlp_set_network(*nets[0])
        results.append(_sequence(torch, ctx, q, nets))
        ctx.close()
    a, b = results
    assert len(a) == len(b)
    for x, y in zip(a, b):
        if isinstance(x, float):
            assert x == y
        else:
            assert np.array_equal(x, y)
