"""GPU parity of the L1 + SSIM loss (igs_l1_ssim_loss_grad) through the C ABI against the FP64
oracle (oracle/ssimref.py).

Tolerances: the kernel accumulates the local moments in fp64, so the loss terms agree with the
oracle to 1e-9 relative.  The gradient stores the three partial-derivative maps in fp32 and blurs
them in fp32, and its three terms cancel where the image is flat, so each entry is held to
1e-4 of its value plus 1e-5 of the sum of the magnitudes of its terms (the oracle's
``ssim_grad_cond``, scaled like the gradient) and of the L1 term.
"""
import numpy as np
import pytest
import torch

from oracle import ssimref as sr
from paper_2407_01866_amd import synth
import paper_2407_01866_amd._native as nat

pytestmark = pytest.mark.gpu

WEIGHT = 0.1


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_loss_grad(x, y, weight=WEIGHT):
    d = dev()
    n, H, W = x.shape
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(d)
    yt = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(d)
    g = torch.empty_like(xt)
    loss = torch.zeros(4, dtype=torch.float64, device=d)
    ws = torch.empty(nat.igs_l1_ssim_workspace_size(n, H, W), dtype=torch.uint8, device=d)
    nat.igs_l1_ssim_loss_grad(xt, yt, n, H, W, weight, g, loss, ws, ws.numel())
    torch.cuda.synchronize()
    return loss.cpu().numpy(), g.cpu().numpy().astype(np.float64)


def check_grad(g, x, y, weight=WEIGHT, ref=None, cond=None):
    count = x.size
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    if ref is None:
        ref = sr.l1_ssim_loss_grad(x64, y64, weight)[1]
    if cond is None:
        cond = sr.ssim_grad_cond(x64, y64)
    tol = 1e-4 * np.abs(ref) + 1e-5 * (1.0 + weight * cond) / count
    err = np.abs(g - ref)
    bad = err > tol
    assert not bad.any(), (f"{int(bad.sum())} of {g.size} entries off; worst excess "
                           f"{float((err / tol).max()):.3g}x tolerance")


def check_loss(loss, x, y, weight=WEIGHT):
    (L, l1, mse, s), _ = sr.l1_ssim_loss_grad(x.astype(np.float64), y.astype(np.float64), weight)
    for got, want in zip(loss, (L, l1, mse, s)):
        assert abs(got - want) <= 1e-9 * max(abs(want), 1e-3), (got, want)


def pair(seed, n, H, W):
    """A target from the synthetic image generator and a rendering-like approximation of it:
    the target plus smooth and pixel noise, so there are flat, textured and edge regions."""
    rng = np.random.default_rng(seed)
    if n % 3 == 0:
        y = np.concatenate([synth.gen_image(seed + k, H, W, 3, 20) for k in range(n // 3)])
    else:
        y = rng.random((n, H, W))
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    smooth = 0.05 * np.sin(2 * np.pi * (hh / max(H, 2) * 1.3 + ww / max(W, 2) * 0.7))
    x = y + smooth[None] + rng.normal(0.0, 0.03, size=(n, H, W))
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("n,H,W", [(3, 64, 96), (1, 17, 33), (9, 50, 70), (2, 1, 77), (1, 90, 1),
                                   (2, 5, 7), (3, 32, 16), (4, 48, 130), (3, 256, 256)])
def test_l1_ssim_matches_oracle(n, H, W):
    print(f"[ssim] n={n} H={H} W={W}", flush=True)
    x, y = pair(100 + H + W, n, H, W)
    loss, g = gpu_loss_grad(x, y)
    check_loss(loss, x, y)
    check_grad(g, x, y)


@pytest.mark.parametrize("weight", [0.0, 1.0, 0.37])
def test_weights(weight):
    print(f"[ssim] weight={weight}", flush=True)
    x, y = pair(7, 3, 40, 45)
    loss, g = gpu_loss_grad(x, y, weight)
    check_loss(loss, x, y, weight)
    check_grad(g, x, y, weight)


def test_identical_images_give_zero_loss_and_gradient():
    print("[ssim] identical", flush=True)
    _, y = pair(8, 3, 70, 90)
    loss, g = gpu_loss_grad(y, y)
    assert abs(loss[3] - 1.0) <= 1e-12 and abs(loss[0]) <= 1e-12 and loss[1] == 0 and loss[2] == 0
    cond = sr.ssim_grad_cond(y.astype(np.float64), y.astype(np.float64))
    assert np.all(np.abs(g) <= 1e-5 * WEIGHT * cond / y.size)


def test_constant_images():
    print("[ssim] constant", flush=True)
    x = np.full((2, 40, 50), 0.25, np.float32)
    y = np.full((2, 40, 50), 0.75, np.float32)
    loss, g = gpu_loss_grad(x, y)
    check_loss(loss, x, y)
    check_grad(g, x, y)


def test_exact_equality_gives_zero_l1_sign():
    """Where image == target the L1 term contributes nothing (sign 0) on both sides."""
    print("[ssim] equal pixels", flush=True)
    x, y = pair(9, 3, 33, 47)
    x[:, ::3, ::2] = y[:, ::3, ::2]
    loss, g = gpu_loss_grad(x, y)
    check_loss(loss, x, y)
    check_grad(g, x, y)


def test_texture_2048_n9_sampled():
    """Full size of the texture-stack workload (2048^2, n = 9): the gradient at sampled pixels
    (corners, edges and interior) against the oracle evaluated on the 21 x 21 neighbourhood that
    determines it, the L1 and MSE terms in full, and the SSIM term through a full-size property
    (an image against itself)."""
    d = dev()
    n, H, W = 9, 2048, 2048
    print(f"[ssim] texture n={n} H={H} W={W}", flush=True)
    x, y = pair(2000, n, H, W)
    loss, g = gpu_loss_grad(x, y)
    dd = x.astype(np.float64) - y.astype(np.float64)
    assert abs(loss[1] - np.abs(dd).mean()) <= 1e-9 * np.abs(dd).mean()
    assert abs(loss[2] - (dd * dd).mean()) <= 1e-9 * (dd * dd).mean()
    assert 0.0 < loss[3] < 1.0
    assert abs(loss[0] - (loss[1] + WEIGHT * (1.0 - loss[3]))) <= 1e-12
    rng = np.random.default_rng(5)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (3, 1000), (1000, 2044), (7, 9)]
    pts += [tuple(p) for p in rng.integers(0, [H, W], size=(60, 2))]
    count = x.size
    for (h, w) in pts:
        h0, h1 = max(0, h - 10), min(H, h + 11)
        w0, w1 = max(0, w - 10), min(W, w + 11)
        xc = x[:, h0:h1, w0:w1].astype(np.float64)
        yc = y[:, h0:h1, w0:w1].astype(np.float64)
        # dL/dx at (h, w) depends only on pixels within 10 of it; a crop boundary that is not
        # the image's lies exactly 10 away, so the crop's own zero extension does not reach it
        ref = (np.sign(xc - yc) - WEIGHT * sr.ssim_grad(xc, yc)) / count
        cond = sr.ssim_grad_cond(xc, yc)
        i, j = h - h0, w - w0
        tol = 1e-4 * np.abs(ref[:, i, j]) + 1e-5 * (1.0 + WEIGHT * cond[:, i, j]) / count
        err = np.abs(g[:, h, w] - ref[:, i, j])
        assert np.all(err <= tol), (h, w, err, tol)
    same, gs = gpu_loss_grad(y, y)
    assert abs(same[3] - 1.0) <= 1e-12 and abs(same[0]) <= 1e-12
    assert np.abs(gs).max() <= 1e-3 / count
    del d
