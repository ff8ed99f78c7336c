"""Long-run checks of the full workloads (minutes; not collected by pytest). Run on a machine
with an MI355X, from the repository root:

    python tests/long_runs.py [--steps 500]

1. Jet 256 x 128 x 128, FP64: the GPU run against the oracle run step for step. Every 10
   steps both accumulate (rho, u, v, w, p); after the run the centreline mean axial velocity
   and the kinetic-energy history are compared (bar: 1 %).
2. Jet 384 x 192 x 192: the mixed form against the FP64 form on the GPU from the same
   state; relative L2 and Linf of rho, u and E every 50 steps.
Each result is one JSON line on stdout.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def jet_vs_oracle(torch, steps, every=10):
    import oracle
    import synthetic as sy
    from paper_2212_12365_amd.lesmi import Context
    p, xyz, q = sy.make_case("jet", (256, 128, 128), seed=0)
    o = oracle.Oracle(p, xyz)
    q = o.apply_bc(q)
    ctx = Context(p, xyz)
    g = torch.from_numpy(q).cuda()
    ctx.stats_reset()
    x = q.copy()
    s1 = np.zeros((5,) + p.shape)
    ke_gpu, ke_ref = [], []
    t0 = time.perf_counter()
    for n in range(every, steps + 1, every):
        x, _ = o.step(x, every, cfl=0.5)
        s1 += oracle.primitives(x, p.gamma)
        ctx.step(g, every, cfl=0.5)
        ctx.stats_accumulate(g)
        if n % 50 == 0:
            ke_ref.append(o.diagnostics(x)[0])
            ke_gpu.append(ctx.diagnostics(g)[0])
            print(json.dumps({"progress": n, "elapsed_s": round(time.perf_counter() - t0, 1)}),
                  flush=True)
    mean, _, count = ctx.stats_read()
    mean = mean.cpu().numpy()
    mref = s1 / count
    cl = mean[1, :, 0, :].mean(0)
    cl_ref = mref[1, :, 0, :].mean(0)
    ke_gpu, ke_ref = np.array(ke_gpu), np.array(ke_ref)
    state = g.cpu().numpy()
    out = {"check": "jet 256x128x128 FP64 GPU vs oracle", "steps": steps,
           "samples": count,
           "centreline_mean_u_max_rel_err": float(np.max(np.abs(cl - cl_ref)) / np.max(np.abs(cl_ref))),
           "kinetic_energy_max_rel_err": float(np.max(np.abs(ke_gpu - ke_ref) / np.abs(ke_ref))),
           "state_rel_l2": [float(v) for v in
                            np.sqrt(((state - x) ** 2).reshape(5, -1).sum(1)) /
                            np.sqrt((x ** 2).reshape(5, -1).sum(1))]}
    ctx.close()
    return out


def mixed_vs_fp64(torch, steps, every=50):
    import synthetic as sy
    from paper_2212_12365_amd.lesmi import Context
    p, xyz, q = sy.make_case("jet", (384, 192, 192), seed=0)
    c64 = Context(p, xyz)
    c32 = Context(p.replace(precision=1), xyz)
    g64 = torch.from_numpy(q).cuda()
    c64.apply_bc(g64)
    g32 = g64.clone()
    rows = []

    def rel(a, b):
        return [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)),
                float((a - b).abs().max() / b.abs().max())]

    for n in range(every, steps + 1, every):
        c64.step(g64, every, cfl=0.5)
        c32.step(g32, every, cfl=0.5)
        rows.append({"step": n, "rho": rel(g32[0], g64[0]),
                     "u": rel(g32[1] / g32[0], g64[1] / g64[0]), "E": rel(g32[4], g64[4])})
    c64.close()
    c32.close()
    return {"check": "jet 384x192x192 mixed vs FP64 (GPU), [rel L2, rel Linf]",
            "every": every, "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--skip-oracle", action="store_true")
    a = ap.parse_args()
    import torch
    print(json.dumps(mixed_vs_fp64(torch, a.steps)), flush=True)
    if not a.skip_oracle:
        res = jet_vs_oracle(torch, a.steps)
        print(json.dumps(res), flush=True)
        ok = res["centreline_mean_u_max_rel_err"] <= 1e-2 and \
            res["kinetic_energy_max_rel_err"] <= 1e-2
        sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
