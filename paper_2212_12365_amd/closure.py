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
