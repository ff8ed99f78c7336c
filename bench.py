#!/usr/bin/env python3
"""Throughput benchmark of the LES hot path on one MI355X.

One benchmark step is one full Runge-Kutta step (time-step reduction, five stages of two
kernels each, boundary conditions) of the synthetic M = 1.4 jet on the 256 x 128 x 128
curvilinear grid in FP64, with the state resident in HBM. The JSON line reports
Mcell-RKstage/s (updated nodes x 5 stages x steps / wall time), the roofline position of the
dominant kernel (the face kernel, timed live with HIP events on the stream it runs on), the
same workload in the mixed-precision form, the 16-member batched ensemble against the same
members run one after another, the 384 x 192 x 192 jet in FP64, mixed precision (with its
error against the FP64 run) and mixed precision with the learned closure, and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per updated node and Runge-Kutta stage (metrics stored, halos served on
# chip): read the stage input Q^(l-1) (40 B) and Q^(0) (40 B), write Q^(l) (40 B), read the
# metrics S and J^-1; stage 1 reads Q^(0) once. FP64: S 72 B + J^-1 8 B, stage 1 160 B,
# stages 2-5 200 B. Mixed: S stored in FP32 (36 B), stage 1 124 B, stages 2-5 164 B.
BYTES_PER_CELL_STAGE = {"fp64": (160.0 + 4 * 200.0) / 5.0, "mixed": (124.0 + 4 * 164.0) / 5.0}
STAGE_SOURCES = ["paper_2212_12365_amd/csrc/les_stage.hip", "paper_2212_12365_amd/csrc/les_device.h"]
JET_GRID = (256, 128, 128)
# The meshes of the paper's mesh table (Computational Performance Assessment), as (n_xi,
# n_eta, n_zeta) = axial, radial and azimuthal points, in the table's order (meshes 1-10).
PAPER_MESHES = [(200, 150, 40), (400, 150, 40), (800, 150, 40), (400, 75, 40), (400, 300, 40),
                (400, 150, 10), (400, 150, 60), (800, 300, 120), (200, 75, 40), (200, 75, 20)]


def stage_kernel_hash():
    h = hashlib.sha256()
    for rel in STAGE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    with the current stage-kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "stage_fp64_jet256_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_hash:
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, xyz, q, steps):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = oracle.Oracle(params, xyz)
    q = o.apply_bc(q)
    t0 = time.perf_counter()
    o.step(q, steps, cfl=0.5)
    t = time.perf_counter() - t0
    # One step again on a single thread.
    oracle.set_threads(1)
    t1 = time.perf_counter()
    o.step(q, 1, cfl=0.5)
    t1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    box = params.bc[0] == 0  # a periodic box updates every node; the jet its interior
    upd = params.ni * params.nj * params.nk if box else (params.ni - 2) * (params.nj - 2) * params.nk
    kind = "box" if box else "jet"
    return {"value": round(upd * 5 * steps / t / 1e6, 3), "unit": "Mcell-RKstage/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} RK steps (= {5 * steps} stages, with time-step reduction and "
                      f"boundary conditions) of the same {kind} {params.ni}x{params.nj}x{params.nk} "
                      f"FP64 workload, {t:.1f} s on {threads} OpenMP threads; then 1 step on "
                      f"1 thread, {t1:.1f} s",
            "single_thread_value": round(upd * 5 / t1 / 1e6, 3),
            "host_cpu": host_cpu()}


REPEATS = 5


def timed_repeats(torch, run, reset, repeats=REPEATS):
    """Wall times of `repeats` runs of run(), each from the state reset() restores, with a
    device synchronisation on both sides of every timed run."""
    walls = []
    for _ in range(repeats):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    return walls


def median(xs):
    xs = sorted(xs)
    m = len(xs) // 2
    return xs[m] if len(xs) % 2 else 0.5 * (xs[m - 1] + xs[m])


def run_form(torch, params, xyz, q, steps, warmup, repeats=REPEATS):
    """Times `steps` RK steps of one context `repeats` times from the same warmed-up state
    (the median is reported), then once more with the stage kernels bracketed by HIP events
    (kernel times only; that run is not part of the throughput figure)."""
    from paper_2212_12365_amd.lesmi import Context
    ctx = Context(params, xyz)
    g = torch.from_numpy(q).to("cuda")
    ctx.apply_bc(g)
    upd = ctx.updated_nodes()
    if warmup:
        ctx.step(g, warmup, cfl=0.5)
    start = g.clone()
    walls = timed_repeats(torch, lambda: ctx.step(g, steps, cfl=0.5), lambda: g.copy_(start),
                          repeats)
    wall = median(walls)
    g.copy_(start)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.step(g, steps, cfl=0.5)
    torch.cuda.synchronize()
    nodes_ms, faces_ms, stages = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    return {"updated_nodes": upd, "wall_s": wall, "walls_s": walls, "nodes_ms": nodes_ms,
            "faces_ms": faces_ms, "stages": stages, "rate": upd * 5 * steps / wall / 1e6}


def mesh_sweep(torch, steps, warmup, grids=None):
    """FP64 and mixed-form throughput of the synthetic jet on each of the paper's meshes
    (or on the given grids)."""
    import synthetic as sy
    rows = []
    for m, n in enumerate(grids or PAPER_MESHES, 1):
        p, xyz, q = sy.make_case("jet", n, seed=0)
        f64 = run_form(torch, p, xyz, q, steps, warmup)
        mx = run_form(torch, p.replace(precision=1), xyz, q, steps, warmup)
        row = {"mesh": m, "grid": list(n), "nodes": n[0] * n[1] * n[2],
               "fp64": round(f64["rate"], 1), "mixed": round(mx["rate"], 1),
               "fp64_face_kernel_us": round(f64["faces_ms"] * 1e3 / max(f64["stages"], 1), 2),
               "fp64_node_kernel_us": round(f64["nodes_ms"] * 1e3 / max(f64["stages"], 1), 2)}
        print(json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
    return rows


def run_batched(torch, steps, warmup):
    """The 16-member mixed-precision ensemble: one after another through les_step, then as
    one batch (persistent launches, graph-replayed steps, autotuned launch shape)."""
    import synthetic as sy
    from paper_2212_12365_amd.lesmi import Batch, Context
    members = sy.make_ensemble(precision=1)
    ctxs, states = [], []
    for p, xyz, q in members:
        c = Context(p, xyz)
        g = torch.from_numpy(q).to("cuda")
        c.apply_bc(g)
        ctxs.append(c)
        states.append(g)
    upd = sum(c.updated_nodes() for c in ctxs)
    for c, g in zip(ctxs, states):
        c.step(g, warmup, cfl=0.5)
    start = [s.clone() for s in states]

    def reset():
        for g, g0 in zip(states, start):
            g.copy_(g0)

    def sequential():
        for c, g in zip(ctxs, states):
            c.step(g, steps, cfl=0.5)

    t_seq = median(timed_repeats(torch, sequential, reset))
    reset()
    b = Batch(ctxs)
    tile, kmin = b.autotune(states)
    b.step(states, 1, cfl=0.5)   # captures the step graph
    t_b = median(timed_repeats(torch, lambda: b.step(states, steps, cfl=0.5), reset))
    b.close()
    for c in ctxs:
        c.close()
    bm = BYTES_PER_CELL_STAGE["mixed"]
    rate = upd * 5 * steps / t_b / 1e6
    return {"value": round(rate, 3), "steps": steps,
            "members": "4x64x64x64, 4x96x64x64, 4x128x96x96, 4x160x96x96 jets, mixed, seeds 0-15",
            "updated_nodes": upd, "ms_per_step": round(t_b * 1e3 / steps, 4),
            "hbm_roofline_pct": round(100 * rate * 1e6 * bm / (HBM_PEAK_GBS * 1e9), 2),
            "tuning": {"tile": tile, "kmin": kmin},
            "sequential_value": round(upd * 5 * steps / t_seq / 1e6, 3),
            "speedup_vs_sequential": round(t_seq / t_b, 3)}


def run_c3(torch, steps, warmup):
    """The 384 x 192 x 192 jet: the mixed form stepped beside the FP64 form from the same
    state (relative errors of rho, u and E after `steps` steps), and the mixed form with the
    learned closure against the mixed form with Smagorinsky (throughput, with a network
    trained briefly on a filtered 256 x 128 x 128 run and its training data's input range,
    so the fallback acts where the flow leaves that range)."""
    import synthetic as sy
    from paper_2212_12365_amd import closure
    from paper_2212_12365_amd.lesmi import Context
    n = (384, 192, 192)
    params, xyz, q = sy.make_case("jet", n, seed=0)
    out = {"grid": list(n)}

    def timed(ctx, g):
        ctx.step(g, warmup, cfl=0.5)
        g0 = g.clone()
        walls = timed_repeats(torch, lambda: ctx.step(g, steps, cfl=0.5), lambda: g.copy_(g0))
        return median(walls)

    c64 = Context(params, xyz)
    g64 = torch.from_numpy(q).to("cuda")
    c64.apply_bc(g64)
    upd = c64.updated_nodes()
    start = g64.clone()
    t64 = timed(c64, g64)
    c32 = Context(params.replace(precision=1), xyz)
    g32 = start.clone()
    t32 = timed(c32, g32)
    # error of the mixed run against the FP64 run after the same warmup + steps
    rho64, rho32 = g64[0], g32[0]
    u64, u32 = g64[1] / g64[0], g32[1] / g32[0]

    def rel(a, b):
        return {"rel_l2": float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)),
                "rel_linf": float((a - b).abs().max() / b.abs().max())}

    out["fp64_value"] = round(upd * 5 * steps / t64 / 1e6, 3)
    out["mixed_value"] = round(upd * 5 * steps / t32 / 1e6, 3)
    out["mixed_speedup_vs_fp64"] = round(t64 / t32, 3)
    out["mixed_vs_fp64_after_steps"] = {"steps": warmup + steps, "rho": rel(rho32, rho64),
                                        "u": rel(u32, u64), "E": rel(g32[4], g64[4])}
    del g64, c64
    # A network trained by the library's own kernels on a short FP64 run of the
    # 256 x 128 x 128 jet filtered onto 128 x 64 x 64 (the invariants are scale-free), with
    # the input range of its training data: the fallback to C_s^2 acts where the
    # 384 x 192 x 192 run leaves that range.
    trained = closure.run((256, 128, 128), spinup=300, every=100, count=3, steps=300,
                          batch=4096, post_steps=0, log=lambda m: None, return_network=True)
    cm = Context(params.replace(precision=1, closure=1), xyz)
    cm.mlp_set_network(trained["theta"], trained["norm"])
    gm = start.clone()
    tm = timed(cm, gm)
    evaluations = params.ni * params.nj * params.nk * 5 * (warmup + REPEATS * steps)
    out["learned_closure_value"] = round(upd * 5 * steps / tm / 1e6, 3)
    out["learned_closure_cost_vs_smagorinsky"] = round(tm / t32, 3)
    out["learned_closure_fallback_fraction"] = round(cm.mlp_fallback_count() / evaluations, 5)
    out["learned_closure_training"] = {
        "fine_grid": trained["fine_grid"], "coarse_grid": trained["coarse_grid"],
        "adam_steps": trained["adam_steps"], "heldout_gain_vs_cs2": round(trained["gain"], 4),
        "heldout_gain_vs_best_constant": round(trained["gain_vs_best_constant"], 4)}
    out["steps"] = steps
    return out


def copy_calibration(gib=1.0, reps=5):
    """A plain device copy of known size, for scaling HBM counter readings."""
    import torch
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8,
                      "reps": reps}), flush=True)


# Algorithmic bytes per node: one running-statistics sample reads q (40 B) and reads and
# writes the sums and the sums of squares (5 + 5 FP64 each: 160 B).
STATS_BYTES_PER_NODE = 200
# A dual-time pseudo-stage: the residual launch reads Q^(l-1) (40 B), the metrics and J^-1
# (80 B) and writes the residual (40 B); the update reads Q^(0), the residual, Q^n (and
# Q^(n-1) for the second-order step), the local pseudo-time step and J, and writes Q^(l)
# (176 B for the backward-Euler first step); once per iteration the local pseudo-time step
# reads q, the metrics and J^-1 and writes it (128 B).
DUAL_BYTES_PER_NODE_STAGE = 160 + 176
DUAL_BYTES_PER_NODE_ITER = 128
# Far-field noise: floating-point operations of one (observer, time, surface node) term of
# the surface integral, counting each division and square root as one: the distance and
# its unit vector (12), the retarded time and the interpolation weight (5), the seven
# interpolated sources (21), the two projections (10), the three terms and the sums (12).
FWH_FLOP_PER_TERM = 60
FP64_VECTOR_PEAK_TFLOPS = 78.6


def event_time(torch, fn, reps):
    """Average GPU time of fn() over reps calls, from HIP events on torch's current stream
    (the stream the library launches on when no stream is given)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def run_rows(torch, cpu=True):
    """The rows beyond the explicit step on the 256 x 128 x 128 jet, each timed on the GPU and
    set against its roofline, with the oracle timed beside it on a bounded sample:
    * grid metrics: les_init_grid (once per run);
    * diagnostics: les_diagnostics (HBM-bound: 48 B per node), with its return to the host;
    * running statistics: one les_stats_accumulate sample (HBM-bound: 200 B per node), and
      the azimuthal reduction;
    * far-field noise: les_fwh_pressure on a control surface around the jet (x from 2 to 6,
      r = 1.5, both caps) with 256 samples of an acoustic monopole field, 64 observers on an
      arc at 30 jet diameters and 256 observer times (FP64 arithmetic-bound);
    * dual time: one backward-Euler physical step of four times the explicit CFL-0.5 step,
      four pseudo-time iterations at cfl_tau 1."""
    import math
    import numpy as np
    import synthetic as sy
    from paper_2212_12365_amd.lesmi import FWH, Context
    if cpu:  # the oracle serves only the CPU legs timed beside the rows
        import oracle
        from oracle import dualtime, fwh
        from oracle.stats import RunningStats
    p, xyz, q = sy.make_case("jet", JET_GRID, seed=0)
    N = p.ni * p.nj * p.nk
    Context(p, xyz).close()  # warm-up (module load)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = Context(p, xyz)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    g = torch.from_numpy(q).cuda()
    ctx.apply_bc(g)
    upd = ctx.updated_nodes()
    rows = {}

    # Grid metrics (once per run): les_init_grid, including the upload of the coordinates.
    mt = {"workload": "jet 256x128x128 grid: metrics, J^-1, J and boundary normals",
          "ms_per_init": round(t_init * 1e3, 2)}
    if cpu:
        t0 = time.perf_counter()
        oracle.Oracle(p, xyz)
        t_o = time.perf_counter() - t0
        mt["oracle"] = {"ms_per_init": round(t_o * 1e3, 1), "kind": "oracle",
                        "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                        "sample": "the oracle's metrics and J^-1 of the same grid"}
    rows["a1_metrics"] = mt

    # Diagnostics (volume-weighted kinetic energy and conserved totals, fixed-order sums):
    # q and J^-1 read once, 48 B per node; the call returns to the host.
    walls = []
    for _ in range(10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.diagnostics(g)
        walls.append(time.perf_counter() - t0)
    t_dg = median(walls)
    dg = {"workload": "jet 256x128x128 FP64 state", "us_per_call": round(t_dg * 1e6, 1),
          "value": round(N / t_dg / 1e6, 1), "unit": "Mnode/s",
          "roofline": {"bound": "hbm", "achieved": round(48 * N / t_dg / 1e9, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(48 * N / t_dg / 1e9 / HBM_PEAK_GBS, 4),
                       "bytes_per_node": 48, "note": "wall time of the call, with its return"}}
    if cpu:
        o = oracle.Oracle(p, xyz)
        t0 = time.perf_counter()
        for _ in range(3):
            o.diagnostics(q)
        t_o = (time.perf_counter() - t0) / 3
        del o
        dg["oracle"] = {"value": round(N / t_o / 1e6, 1), "unit": "Mnode/s", "kind": "oracle",
                        "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                        "sample": f"3 calls on the same state, {t_o * 1e3:.1f} ms each"}
    rows["a12_diagnostics"] = dg

    # Running statistics.
    ctx.stats_reset()
    ctx.stats_accumulate(g)
    t_acc = event_time(torch, lambda: ctx.stats_accumulate(g), 50)
    t_az = event_time(torch, lambda: ctx.stats_azimuthal(), 5)
    gbs = STATS_BYTES_PER_NODE * N / t_acc / 1e9
    st = {"workload": "jet 256x128x128 FP64 state, one sample per call",
          "accumulate_us": round(t_acc * 1e6, 2),
          "value": round(N / t_acc / 1e6, 1), "unit": "Mnode-samples/s",
          "azimuthal_reduction_us": round(t_az * 1e6, 2),
          "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "kernel": "k_stats_acc", "bytes_per_node": STATS_BYTES_PER_NODE}}
    if cpu:
        ctx_state = g.cpu().numpy()
        rs = RunningStats(p.shape, p.gamma)
        t0 = time.perf_counter()
        for _ in range(3):
            rs.add(ctx_state)
        t_o = (time.perf_counter() - t0) / 3
        st["oracle"] = {"value": round(N / t_o / 1e6, 2), "unit": "Mnode-samples/s",
                        "kind": "oracle", "cores": 1,
                        "sample": f"3 samples of the same state (numpy), {t_o:.2f} s each"}
    rows["f1_statistics"] = st

    # Dual time.
    g2 = g.clone()
    dt_expl = ctx.step(g2, 1, cfl=0.5)
    dt = 4.0 * dt_expl
    sub = 4
    g2.copy_(g)
    ctx.dual_step(g2, 1, dt, 1, 1.0)  # allocates the buffers; warm-up
    walls = []
    for _ in range(REPEATS):
        g2.copy_(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.dual_step(g2, 1, dt, sub, 1.0)
        walls.append(time.perf_counter() - t0)
    t_d = median(walls)
    rate = upd * 5 * sub / t_d / 1e6
    bpn = DUAL_BYTES_PER_NODE_STAGE + DUAL_BYTES_PER_NODE_ITER / 5.0
    gbs = rate * 1e6 * bpn / 1e9
    du = {"workload": "jet 256x128x128 FP64, one backward-Euler step of 4x the explicit "
                      "CFL-0.5 step, 4 pseudo-time iterations at cfl_tau 1",
          "ms_per_physical_step": round(t_d * 1e3, 3),
          "value": round(rate, 1), "unit": "Mcell-pseudo-stage/s",
          "residual_history": [float(x) for x in res[0]],
          "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "bytes_per_node_stage": bpn}}
    if cpu:
        o = oracle.Oracle(p, xyz)
        qo = o.apply_bc(q)
        t0 = time.perf_counter()
        dualtime.dual_step(o, qo, None, 1, dt, 1, 1.0)
        t_o = time.perf_counter() - t0
        du["oracle"] = {"value": round(upd * 5 / t_o / 1e6, 2), "unit": "Mcell-pseudo-stage/s",
                        "kind": "oracle", "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                                      os.cpu_count() or 1)),
                        "sample": f"one pseudo-time iteration (5 stages) of the same step, "
                                  f"{t_o:.1f} s"}
        del o
    rows["f4_dual_time"] = du

    # Far-field noise.
    r_of_j = np.hypot(xyz[1, 0, :, 0], xyz[2, 0, :, 0])
    x_of_i = xyz[0, 0, 0, :]
    js = int(np.argmin(np.abs(r_of_j - 1.5)))
    i1, i2 = int(np.argmin(np.abs(x_of_i - 2.0))), int(np.argmin(np.abs(x_of_i - 6.0)))
    src = np.array([0.5 * (x_of_i[i1] + x_of_i[i2]), 0.0, 0.0])
    M, T, A = 256, 4.0, 1e-4
    omega, dtau = 2 * math.pi / T, T / 32
    rho0, c0, p0, gam = p.rho_inf, 1.0, p.p_inf, p.gamma
    f = FWH(ctx, xyz, i1, i2, js, caps=3, capacity=M, dtau=dtau)
    X = torch.from_numpy(xyz).cuda()
    d = X - torch.tensor(src, dtype=torch.float64, device="cuda").view(3, 1, 1, 1)
    R = torch.sqrt((d * d).sum(0))
    gq = torch.empty_like(g)
    for m in range(M):
        tr = m * dtau - R / c0
        fv = A * torch.sin(omega * tr)
        fd = A * omega * torch.cos(omega * tr)
        ur = fv / (4 * math.pi * R * R) + fd / (4 * math.pi * R * c0)
        pp = rho0 * fd / (4 * math.pi * R)
        rho = rho0 + pp / c0 ** 2
        u = ur * d / R
        gq[0] = rho
        gq[1:4] = rho * u
        gq[4] = (p0 + pp) / (gam - 1.0) + 0.5 * rho * (u * u).sum(0)
        f.sample(gq)
    del X, d, R
    D = 30.0
    ang = np.linspace(0.0, math.pi, 64)
    obs = src[None, :] + D * np.stack([np.cos(ang), np.sin(ang), 0 * ang], axis=1)
    times = np.linspace(38.0, 54.0, 256)
    pr, _, skipped = f.pressure(obs, times, c0, p0)   # also forms the sources once
    walls = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr, _, skipped = f.pressure(obs, times, c0, p0)
        walls.append(time.perf_counter() - t0)
    t_f = median(walls)
    terms = len(obs) * len(times) * f.ns
    tf = FWH_FLOP_PER_TERM * terms / t_f / 1e12
    fw = {"workload": f"jet 256x128x128 control surface ({f.ns} nodes), {M} samples, "
                      f"{len(obs)} observers x {len(times)} times",
          "ms_per_call": round(t_f * 1e3, 3), "skipped_terms": int(skipped),
          "value": round(terms / t_f / 1e9, 3), "unit": "Gterm/s",
          "roofline": {"bound": "alu", "achieved": round(tf, 3),
                       "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
                       "kernel": "k_fwh_integrate", "flop_per_term": FWH_FLOP_PER_TERM}}
    if cpu:
        o = oracle.Oracle(p, xyz)
        ids, y, nrm, dS = fwh.jet_surface(o.S, xyz, i1, i2, js)
        del o
        idt = torch.from_numpy(np.asarray(ids, dtype=np.int64)).cuda()
        rho_s = np.empty((M, len(ids)))
        u_s = np.empty((M, len(ids), 3))
        p_s = np.empty((M, len(ids)))
        Xs = torch.from_numpy(xyz.reshape(3, -1)).cuda()[:, idt]
        ds = Xs - torch.tensor(src, dtype=torch.float64, device="cuda").view(3, 1)
        Rs = torch.sqrt((ds * ds).sum(0))
        for m in range(M):  # the same monopole samples at the surface nodes
            tr = m * dtau - Rs / c0
            fd = A * omega * torch.cos(omega * tr)
            fv = A * torch.sin(omega * tr)
            ur = fv / (4 * math.pi * Rs * Rs) + fd / (4 * math.pi * Rs * c0)
            pp = rho0 * fd / (4 * math.pi * Rs)
            rho_s[m] = (rho0 + pp / c0 ** 2).cpu().numpy()
            u_s[m] = (ur * ds / Rs).T.cpu().numpy()
            p_s[m] = (p0 + pp).cpu().numpy()
        no, nt = 4, 16
        t0 = time.perf_counter()
        fwh.fwh_pressure(y, nrm, dS, rho_s, u_s, p_s, 0.0, dtau, rho0, c0, p0, obs[:no],
                         times[:nt])
        t_o = time.perf_counter() - t0
        fw["oracle"] = {"value": round(no * nt * len(ids) / t_o / 1e9, 5), "unit": "Gterm/s",
                        "kind": "oracle", "cores": 1,
                        "sample": f"{no} observers x {nt} times (numpy), {t_o:.2f} s"}
    f.close()
    rows["f3_fwh"] = fw
    ctx.close()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-forms", dest="forms", action="store_false",
                    help="time the FP64 form only (skip the mixed-precision and batched runs)")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="RK steps timed for the batched ensemble and its sequential baseline")
    ap.add_argument("--cpu-steps", type=int, default=15,
                    help="RK steps of the oracle timed for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="only time the CPU oracle on the Taylor-Green box (20 steps) and the "
                         "384x192x192 jet (2 steps) and print one JSON line, then exit")
    ap.add_argument("--mesh-sweep", action="store_true",
                    help="only time the FP64 and mixed forms of the jet on the paper's ten "
                         "meshes (its mesh table) and print one JSON line, then exit")
    ap.add_argument("--sweep-grids", default="",
                    help="with --mesh-sweep: grids to time instead of the paper's meshes, "
                         "e.g. 768x384x384,384x192x192")
    ap.add_argument("--closure-only", action="store_true",
                    help="only train the closure network briefly (256x128x128 FP64 run filtered "
                         "onto 128x64x64) and time learned-closure steps of the 384x192x192 "
                         "mixed jet (for counter runs of the closure kernels), then exit")
    ap.add_argument("--rows-only", action="store_true",
                    help="only measure the statistics, far-field noise and dual-time rows on "
                         "the 256x128x128 jet (with the oracle beside them unless "
                         "--cpu-steps 0) and print one JSON line, then exit")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only time the mixed-precision form of the jet workload and print its "
                         "figures (for counter runs of its kernels), then exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this library runs the whole grid on one GPU; multi-GPU runs "
                                   "(--gpus > 1) are not supported"}), flush=True)
        sys.exit(2)

    if args.oracle_configs:
        import synthetic as sy
        rows = []
        for name, grid, steps in (("tgv", 32, 20), ("jet", (384, 192, 192), 2)):
            p, xyz, q = sy.make_case(name, grid, seed=0)
            r = cpu_baseline(p, xyz, q, steps)
            r["workload"] = f"{name} {grid}"
            print(json.dumps(r), file=sys.stderr, flush=True)
            rows.append(r)
        print(json.dumps({"oracle_configs": rows}), flush=True)
        return

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    import synthetic as sy

    if args.mesh_sweep:
        grids = [tuple(int(x) for x in g.split("x")) for g in args.sweep_grids.split(",") if g]
        rows = mesh_sweep(torch, args.steps, args.warmup, grids or None)
        print(json.dumps({"mesh_sweep": rows, "unit": "Mcell-RKstage/s", "steps": args.steps,
                          "warmup": args.warmup, "workload": "synthetic jet, CFL 0.5, Smagorinsky"}),
              flush=True)
        return
    if args.rows_only:
        print(json.dumps({"rows": run_rows(torch, cpu=args.cpu_steps > 0)}), flush=True)
        return
    if args.closure_only:
        from paper_2212_12365_amd import closure
        from paper_2212_12365_amd.lesmi import Context
        t0 = time.perf_counter()
        trained = closure.run((256, 128, 128), spinup=100, every=50, count=3, steps=100,
                              batch=4096, post_steps=0, log=lambda m: None, return_network=True)
        t_train = time.perf_counter() - t0
        p3, xyz3, q3 = sy.make_case("jet", (384, 192, 192), seed=0)
        cm = Context(p3.replace(precision=1, closure=1), xyz3)
        cm.mlp_set_network(trained["theta"], trained["norm"])
        g = torch.from_numpy(q3).to("cuda")
        cm.apply_bc(g)
        cm.step(g, args.warmup, cfl=0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cm.step(g, args.steps, cfl=0.5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(json.dumps({"form": "mixed + learned closure", "workload": "jet 384x192x192",
                          "ms_per_step": round(wall * 1e3 / max(args.steps, 1), 3),
                          "training_s": round(t_train, 2),
                          "heldout_gain_vs_cs2": round(trained["gain"], 4)}), flush=True)
        return
    params, xyz, q = sy.make_case("jet", JET_GRID, seed=0)
    if args.mixed_only:
        mx = run_form(torch, params.replace(precision=1), xyz, q, args.steps, args.warmup)
        print(json.dumps({"form": "mixed", "workload": "jet 256x128x128 mixed, CFL 0.5",
                          "value": round(mx["rate"], 3), "unit": "Mcell-RKstage/s",
                          "face_kernel_us": round(mx["faces_ms"] * 1e3 / max(mx["stages"], 1), 2),
                          "node_kernel_us": round(mx["nodes_ms"] * 1e3 / max(mx["stages"], 1), 2)}),
              flush=True)
        return
    f64 = run_form(torch, params, xyz, q, args.steps, args.warmup)
    upd = f64["updated_nodes"]
    value = f64["rate"]
    # Dominant kernel: the face kernel (fluxes, flux differences, stage update), timed by
    # HIP events recorded on the stream it is launched on.
    bpc = BYTES_PER_CELL_STAGE["fp64"]
    face_s = f64["faces_ms"] / 1e3 / max(f64["stages"], 1)
    node_s = f64["nodes_ms"] / 1e3 / max(f64["stages"], 1)
    per_launch = bpc * upd
    achieved = per_launch / face_s / 1e9
    khash = stage_kernel_hash()
    forms = {"fp64": {"value": round(value, 3),
                      "hbm_roofline_pct": round(100 * value * 1e6 * bpc / (HBM_PEAK_GBS * 1e9), 2),
                      "face_kernel_us": round(face_s * 1e6, 2),
                      "node_kernel_us": round(node_s * 1e6, 2)}}
    if args.forms:
        mp = params.replace(precision=1)
        mx = run_form(torch, mp, xyz, q, args.steps, args.warmup)
        bm = BYTES_PER_CELL_STAGE["mixed"]
        forms["mixed"] = {
            "value": round(mx["rate"], 3),
            "hbm_roofline_pct": round(100 * mx["rate"] * 1e6 * bm / (HBM_PEAK_GBS * 1e9), 2),
            "face_kernel_us": round(mx["faces_ms"] * 1e3 / max(mx["stages"], 1), 2),
            "node_kernel_us": round(mx["nodes_ms"] * 1e3 / max(mx["stages"], 1), 2),
            "speedup_vs_fp64": round(mx["rate"] / value, 3)}
    if args.forms:
        forms["batched"] = run_batched(torch, args.batch_steps, 2)
        forms["jet384"] = run_c3(torch, args.batch_steps, 2)
    out = {
        "metric": "Mcell-RKstage updates/s and % HBM roofline, FP64 vs mixed vs batched",
        "value": round(value, 3),
        "unit": "Mcell-RKstage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jet 256x128x128 FP64, CFL 0.5, Smagorinsky",
                   "grid": list(JET_GRID), "updated_nodes": upd, "forms": forms},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(khash),
                     "kernel": "k_stage_planes (face fluxes, flux differences, stage update)",
                     "avg_launch_us": round(face_s * 1e6, 2), "launches": f64["stages"],
                     "algorithmic_bytes_per_launch": per_launch,
                     "kernel_source_hash": khash},
    }
    if args.forms:
        out["rows"] = run_rows(torch, cpu=args.cpu_steps > 0)
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(params, xyz, q, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
