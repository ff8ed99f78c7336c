#!/usr/bin/env python3
"""Throughput benchmark of the LES hot path on one MI355X.

One benchmark step is one full Runge-Kutta step (time-step reduction, five stage kernels,
boundary conditions) of the synthetic M = 1.4 jet on the 256 x 128 x 128 curvilinear grid in
FP64, with the state resident in HBM. The JSON line reports Mcell-RKstage/s (updated nodes x
5 stages x steps / wall time), the roofline position of the stage kernel (timed live with
HIP events on the stream it runs on), and the CPU oracle timed on a bounded sample of the
same workload.
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
# Algorithmic bytes per updated node and stage of the fused FP64 stage kernel: read the
# stage input Q^(l-1) (40 B) and Q^(0) (40 B), write Q^(l) (40 B), read the metrics
# S (72 B) and J^-1 (8 B); stage 1 reads Q^(0) once (160 B), stages 2-5 move 200 B.
BYTES_PER_CELL_STAGE = {"fp64": (160.0 + 4 * 200.0) / 5.0}
STAGE_SOURCES = ["paper_2212_12365_amd/csrc/les_stage.hip", "paper_2212_12365_amd/csrc/les_device.h"]


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


def cpu_baseline(params, xyz, q, steps):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = oracle.Oracle(params, xyz)
    q = o.apply_bc(q)
    t0 = time.perf_counter()
    o.step(q, steps, cfl=0.5)
    t = time.perf_counter() - t0
    upd = (params.ni - 2) * (params.nj - 2) * params.nk
    return {"value": upd * 5 * steps / t / 1e6, "unit": "Mcell-RKstage/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} RK step(s) (= {5 * steps} stages) of the same jet "
                      f"{params.ni}x{params.nj}x{params.nk} FP64 workload, {t:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="RK steps of the oracle timed for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs the whole grid on one GPU; multi-GPU runs "
                                   "(--gpus > 1) are not supported"}), flush=True)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    import synthetic as sy
    from paper_2212_12365_amd.lesmi import Context

    n = (256, 128, 128)
    params, xyz, q = sy.make_case("jet", n, seed=0)
    ctx = Context(params, xyz)
    g = torch.from_numpy(q).to("cuda")
    ctx.apply_bc(g)
    upd = ctx.updated_nodes()
    if args.warmup:
        ctx.step(g, args.warmup, cfl=0.5)
    torch.cuda.synchronize()

    ctx.profile(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(g, args.steps, cfl=0.5)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, launches = ctx.profile_read()
    ctx.profile(False)
    ev_ms = e0.elapsed_time(e1)

    value = upd * 5 * args.steps / wall / 1e6
    bpc = BYTES_PER_CELL_STAGE["fp64"]
    avg_s = stage_ms / 1e3 / max(launches, 1)
    per_launch = bpc * upd
    achieved = per_launch / avg_s / 1e9
    khash = stage_kernel_hash()
    traffic = measured_traffic(khash)
    out = {
        "metric": "Mcell-RKstage updates/s and % HBM roofline, FP64 vs mixed vs batched",
        "value": round(value, 3),
        "unit": "Mcell-RKstage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jet 256x128x128 FP64, CFL 0.5",
                   "grid": list(n), "updated_nodes": upd, "precision": "fp64",
                   "closure": "smagorinsky",
                   "hbm_roofline_pct_whole_step": round(100 * value * 1e6 * bpc / (HBM_PEAK_GBS * 1e9), 2),
                   "event_ms_per_step": round(ev_ms / args.steps, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "RK stage kernel(s)",
                     "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
                     "algorithmic_bytes_per_launch": per_launch,
                     "kernel_source_hash": khash},
    }
    ctx.close()
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(params, xyz, q, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
