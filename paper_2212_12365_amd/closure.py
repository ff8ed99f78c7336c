"""Training and evaluation driver of the learned subgrid closure.

Orchestration only: the training data (box filter and least-squares target), the network's
forward and backward passes, the Adam updates and the inference all run in the library's
kernels through the C ABI (les_filter_target, les_mlp_loss_grad, les_mlp_adam,
les_mlp_coefficient). The driver draws the random numbers of training (the initial weights
and the minibatch node numbers) from a seeded numpy generator and passes them in.
"""
from __future__ import annotations

import math

import numpy as np

from . import lesmi

NIN, NH = 6, 64


def init_params(cs2, seed=0):
    """Initial network: weights N(0, 1/fan_in), zero hidden biases, and the output bias set
    so that an untrained network predicts c = C_s^2 (softplus(b3) = cs2)."""
    import torch
    rng = np.random.default_rng(seed)
    th = np.zeros(lesmi.MLP_NPARAMS, dtype=np.float64)
    o = 0
    th[o:o + NH * NIN] = rng.normal(0.0, 1.0 / math.sqrt(NIN), NH * NIN)
    o += NH * NIN + NH
    th[o:o + NH * NH] = rng.normal(0.0, 1.0 / math.sqrt(NH), NH * NH)
    o += NH * NH + NH
    th[o:o + NH] = rng.normal(0.0, 0.1 / math.sqrt(NH), NH)
    th[-1] = math.log(math.expm1(cs2))
    return torch.from_numpy(th.astype(np.float32)).cuda()


def training_pool(weight):
    """Node numbers with weight > 0 (int64 numpy)."""
    w = weight.reshape(-1).cpu().numpy()
    return np.nonzero(w > 0)[0]


def train(feat, target, weight, cs2, steps=400, batch=4096, lr=2e-3, seed=0, widen=0.1,
          log_every=0):
    """Fits the network to the targets of the nodes with weight > 0.

    feat [6][n], target [n], weight [n]: float32 GPU tensors (one or several snapshots laid
    end to end). Returns (theta, norm, losses)."""
    import torch
    n = target.numel()
    feat = feat.reshape(6, n).contiguous()
    target = target.reshape(n).contiguous()
    weight = weight.reshape(n).contiguous()
    norm = lesmi.mlp_fit_norm(feat, weight, widen)
    theta = init_params(cs2, seed)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    pool = training_pool(weight)
    if pool.size == 0:
        raise ValueError("no training node has weight > 0")
    rng = np.random.default_rng(seed + 1)
    work = torch.empty(lesmi.mlp_work_size(batch), dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, steps + 1):
        sel = rng.choice(pool, size=batch, replace=pool.size < batch)
        idx = torch.from_numpy(sel.astype(np.int32)).cuda()
        grad, loss = lesmi.mlp_loss_grad(theta, norm, feat, target, weight, idx, 1.0 / batch,
                                         work=work)
        lesmi.mlp_adam(theta, grad, m, v, step, lr)
        if log_every and (step % log_every == 0 or step == 1):
            losses.append((step, float(loss.item())))
    return theta, norm, losses


def evaluate(theta, norm, cs2, feat, smag, target, weight):
    """Weighted mean-square error of the network's coefficient and of the constant C_s^2
    against the targets (nodes with weight > 0), and the fallback fraction there."""
    n = target.numel()
    c, _ = lesmi.mlp_coefficient(theta, norm, cs2, feat.reshape(6, n).contiguous(),
                                 smag.reshape(n).contiguous())
    c = c.cpu().numpy().astype(np.float64)
    y = target.reshape(n).cpu().numpy().astype(np.float64)
    w = weight.reshape(n).cpu().numpy().astype(np.float64)
    f = feat.reshape(6, n).cpu().numpy()
    s = smag.reshape(n).cpu().numpy()
    lo, hi = np.array(list(norm.lo)), np.array(list(norm.hi))
    ok = np.all(np.isfinite(f), axis=0) & (s > 0) & np.all((f >= lo[:, None]) &
                                                          (f <= hi[:, None]), axis=0)
    sel = w > 0
    wsum = w[sel].sum()
    mse_mlp = float(np.sum(w[sel] * (c[sel] - y[sel]) ** 2) / wsum)
    mse_smag = float(np.sum(w[sel] * (cs2 - y[sel]) ** 2) / wsum)
    ybar = float(np.sum(w[sel] * y[sel]) / wsum)
    mse_const = float(np.sum(w[sel] * (ybar - y[sel]) ** 2) / wsum)
    return {"mse_mlp": mse_mlp, "mse_smagorinsky": mse_smag, "mse_best_constant": mse_const,
            "gain": 1.0 - mse_mlp / mse_smag if mse_smag > 0 else 0.0,
            "gain_vs_best_constant": 1.0 - mse_mlp / mse_const if mse_const > 0 else 0.0,
            "mean_target": ybar, "fallback_fraction": float(np.mean(~ok[sel])),
            "nodes": int(sel.sum())}


def snapshots(fine, coarse, q_fine, every, count, smin, cfl=0.5):
    """Advances the fine run and, every `every` steps, collects the filtered training data
    on the coarse grid. Returns a list of dicts (see lesmi.filter_target)."""
    out = []
    for _ in range(count):
        fine.step(q_fine, every, cfl=cfl)
        out.append(lesmi.filter_target(fine, coarse, q_fine, smin))
    return out


def stack(snaps, key):
    """Concatenates one field of several snapshots (inputs as [6][n])."""
    import torch
    if key == "feat":
        return torch.cat([d["feat"].reshape(6, -1) for d in snaps], dim=1).contiguous()
    return torch.cat([d[key].reshape(-1) for d in snaps]).contiguous()


def aposteriori(fine, coarse, xyzc, q_fine, q_start, theta, norm, fine_steps, smin,
                checkpoints=1, log=print):
    """A-posteriori comparison: from the filtered state q_start, coarse runs (mixed form)
    with the Smagorinsky closure and with the learned closure advance over the time the fine
    run advances in `fine_steps` steps (coarse dt = 2 x the fine run's dt, fixed), and their
    velocity fields are compared with the filtered fine solution at `checkpoints` equally
    spaced times (the last one at the end). Returns the relative L2 errors of u at each
    checkpoint, per closure."""
    import torch
    from .lesmi import Context
    checkpoints = max(1, int(checkpoints))
    seg = fine_steps // checkpoints
    seg -= seg % 2
    if seg < 2:
        raise ValueError("fine_steps too small for the checkpoints")
    dt_f = fine.step(q_fine, 1, cfl=0.5)
    refs = []
    for m in range(checkpoints):
        fine.step(q_fine, seg - 1 if m == 0 else seg, cfl=0.0, dt_fixed=dt_f)
        ref = lesmi.filter_target(fine, coarse, q_fine, smin)["q"]
        refs.append(ref[1:4] / ref[0])
        log(f"a-posteriori: fine reference {m + 1}/{checkpoints}")
    coarse_params = coarse.params
    out = {"fine_dt": dt_f, "coarse_steps": [(m + 1) * (seg // 2) for m in range(checkpoints)]}
    inner = (slice(None), slice(None), slice(1, -1), slice(1, -1))
    for name, closure_id in (("smagorinsky", 0), ("learned", 1)):
        c = Context(coarse_params.replace(precision=1, closure=closure_id), xyzc)
        if closure_id == 1:
            c.mlp_set_network(theta, norm)
        g = q_start.clone()
        c.apply_bc(g)
        errs = []
        for m in range(checkpoints):
            c.step(g, seg // 2, cfl=0.0, dt_fixed=2.0 * dt_f)
            u = g[1:4] / g[0]
            u_ref = refs[m]
            err = (torch.linalg.vector_norm((u - u_ref)[inner]) /
                   torch.linalg.vector_norm(u_ref[inner]))
            errs.append(float(err))
        out[f"u_rel_l2_{name}"] = errs
        if closure_id == 1:
            out["fallback_evaluations"] = c.mlp_fallback_count()
        c.close()
        log(f"a-posteriori {name}: u rel-L2 vs filtered fine at coarse steps "
            f"{out['coarse_steps']}: " + ", ".join(f"{e:.4e}" for e in errs))
    return out


def run(fine_shape=(768, 384, 384), spinup=1200, every=200, count=3, steps=600, batch=8192,
        lr=2e-3, seed=0, smin=1.0, post_steps=1000, checkpoints=5, log=print,
        return_network=False):
    """End-to-end training of the closure on the jet: an FP64 run on the fine grid (seeded
    jet field), `count` snapshots box-filtered onto the grid of half the nodes per direction,
    training on all but the last snapshot and evaluation on the last; then, if post_steps > 0,
    the a-posteriori comparison over post_steps fine steps at `checkpoints` equally spaced
    times. Returns a dict (with the trained
    network under "theta" and "norm" if return_network)."""
    import time as _time
    import torch
    import synthetic as sy
    from .lesmi import Context
    t0 = _time.perf_counter()
    fine_shape = tuple(fine_shape)
    coarse_shape = tuple(n // 2 for n in fine_shape)
    pf, xyzf, qf = sy.make_case("jet", fine_shape, seed=seed)
    xyzc = np.ascontiguousarray(xyzf.reshape(3, coarse_shape[2], 2, coarse_shape[1], 2,
                                             coarse_shape[0], 2).mean(axis=(2, 4, 6)))
    fine = Context(pf, xyzf)
    coarse = Context(sy.jet_params(coarse_shape), xyzc)
    del xyzf
    g = torch.from_numpy(qf).cuda()
    del qf
    fine.apply_bc(g)
    log(f"fine {fine_shape} ready in {_time.perf_counter() - t0:.1f} s")
    t1 = _time.perf_counter()
    done = 0
    while done < spinup:
        n = min(100, spinup - done)
        fine.step(g, n, cfl=0.5)
        done += n
        log(f"fine run: {done}/{spinup} steps")
    snaps = []
    for c in range(count):
        fine.step(g, every, cfl=0.5)
        snaps.append(lesmi.filter_target(fine, coarse, g, smin))
        log(f"snapshot {c + 1}/{count} after {spinup + (c + 1) * every} steps")
    t_run = _time.perf_counter() - t1
    cs2 = coarse.params.cs ** 2
    train_snaps, test = snaps[:-1], snaps[-1]
    t2 = _time.perf_counter()
    theta, norm, losses = train(stack(train_snaps, "feat"), stack(train_snaps, "target"),
                                stack(train_snaps, "weight"), cs2, steps=steps, batch=batch,
                                lr=lr, seed=seed, log_every=max(steps // 6, 1))
    torch.cuda.synchronize()
    t_train = _time.perf_counter() - t2
    res = evaluate(theta, norm, cs2, test["feat"], test["smag"], test["target"], test["weight"])
    res.update({"fine_grid": list(fine_shape), "coarse_grid": list(coarse_shape),
                "fine_steps": spinup + count * every, "snapshot_every": every,
                "train_snapshots": count - 1, "adam_steps": steps, "batch": batch,
                "losses": losses, "fine_run_s": round(t_run, 1), "train_s": round(t_train, 2)})
    if post_steps > 0:
        res["aposteriori"] = aposteriori(fine, coarse, xyzc, g, test["q"], theta, norm,
                                         post_steps, smin, checkpoints, log)
    fine.close()
    coarse.close()
    if return_network:
        res["theta"], res["norm"] = theta, norm
    return res


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="train the learned closure on a filtered fine run")
    ap.add_argument("--fine", default="768,384,384")
    ap.add_argument("--spinup", type=int, default=1200)
    ap.add_argument("--every", type=int, default=200)
    ap.add_argument("--count", type=int, default=3)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--post-steps", type=int, default=1000)
    ap.add_argument("--checkpoints", type=int, default=5)
    a = ap.parse_args()
    out = run(tuple(int(x) for x in a.fine.split(",")), a.spinup, a.every, a.count, a.steps,
              a.batch, post_steps=a.post_steps, checkpoints=a.checkpoints,
              log=lambda m: print(m, flush=True))
    print(json.dumps(out), flush=True)
