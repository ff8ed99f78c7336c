"""The allocation-free training entry point (les_mlp_loss_grad_noalloc) against
les_mlp_loss_grad, through the C ABI.

The two share the gradient kernels and the grid for a given sample count, and the
allocation-free form only keeps the per-wave partial gradients in the library's static device
array instead of the caller's workspace, so loss and gradient must agree bit for bit. Two
calls in a row, the second with fewer samples (fewer waves, so partials left over from the
first call stay in the array and must not be read), then the size limit.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = np.empty(4673)
    th[:384] = rng.normal(scale=1 / math.sqrt(6), size=384)
    th[384:448] = rng.normal(scale=0.1, size=64)
    th[448:4544] = rng.normal(scale=1 / 8, size=4096)
    th[4544:4608] = rng.normal(scale=0.1, size=64)
    th[4608:4672] = rng.normal(scale=1 / 8, size=64)
    th[4672] = -3.0
    return th.astype(np.float32)


def test_noalloc_loss_grad_equals_workspace_form(torch):
    print("[gpu] allocation-free loss/gradient entry point", flush=True)
    from paper_2212_12365_amd import lesmi
    rng = np.random.default_rng(11)
    nfeat = 20000
    feat = torch.from_numpy(rng.normal(size=(6, nfeat)).astype(np.float32)).cuda()
    target = torch.from_numpy((0.03 * rng.random(nfeat)).astype(np.float32)).cuda()
    weight = torch.from_numpy((rng.random(nfeat) > 0.2).astype(np.float32)).cuda()
    theta = torch.from_numpy(_theta(3)).cuda()
    norm = lesmi.les_mlp_norm.from_arrays(0.1 * rng.normal(size=6), 1.0 + 0.1 * rng.random(6),
                                          [-1e30] * 6, [1e30] * 6)
    grad = torch.empty(lesmi.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for n in (lesmi.MLP_NOALLOC_MAX_SAMPLES, 3000):
        idx = torch.from_numpy(rng.integers(0, nfeat, n).astype(np.int32)).cuda()
        inv = 1.0 / n
        ref_g, ref_l = lesmi.mlp_loss_grad(theta, norm, feat, target, weight, idx, inv)
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        lesmi.mlp_loss_grad_noalloc(theta, norm, feat, target, weight, idx, inv, grad, loss)
        torch.cuda.synchronize()
        g, r = grad.cpu().numpy(), ref_g.cpu().numpy()
        print(f"n={n}: loss {loss.item():.6e} vs {ref_l.item():.6e}, "
              f"max |dgrad| {np.abs(g - r).max():.3e}", flush=True)
        assert np.all(np.isfinite(g)) and np.abs(r).max() > 0
        assert np.array_equal(g, r), n
        assert loss.item() == ref_l.item(), n
    # beyond the static array: refused before any launch
    n = lesmi.MLP_NOALLOC_MAX_SAMPLES + 1
    idx = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(lesmi.LesError) as e:
        lesmi.mlp_loss_grad_noalloc(theta, norm, feat, target, weight, idx, 1.0, grad, loss)
    assert e.value.code == lesmi.LES_EINVAL
