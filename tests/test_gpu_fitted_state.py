"""GPU parity of the whole frame at a fitted-like state of the texture workload (2048 x 2048,
n = 9, N = 100,000, K = 10), through the C ABI, against the FP64 oracle (Sec. 3.2 Eq. 5 and
the adjoint of Sec. 3.3).

The parameters come from ``synth.gen_fitted_like``: the spread a texture fit reaches after a few
dozen Adam iterations (strongly anisotropic and image-sized Gaussians, one covering every tile,
colours outside [0, 1], means past the border, angles on the clamp values), plus a dense cluster
whose tiles hold up to ~450 candidates, more than one LDS batch of the forward (192) and of the
adjoint (256).  The oracle never sees anything the GPU computed.

Checked, on every pixel and every Gaussian:
* tile hit lists bit-exact;
* top-K sets bit-exact wherever an fp32 ranking decides them for certain, and at every near-tie
  pixel a valid selection whose pixel equals the oracle's blend over the GPU's own set;
* pixels within 1e-5 relative (+1e-7);
* the two-pass adjoint with a seeded upstream gradient (zeroed at near-tie pixels, so both sides
  differentiate the same selection) at the 1e-4 row bar;
* the single-pass L1 kernel (render, loss and adjoint per tile) against a target 0.02-0.1 away
  from the oracle's image: the loss to 1e-6 relative, and the gradient at the 1e-4 row bar for
  every Gaussian that no near-tie pixel retains (at such a pixel the kernel's own, equally valid,
  selection decides its L1 gradient's terms there).
"""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_2407_01866_amd import synth
from test_gpu_render import check_forward, check_grad, check_tile_lists, gpu_ids, near_tie_mask

pytestmark = pytest.mark.gpu

SEED = 2600
H = W = 2048
N, n, K = 100000, 9, 10
TIE_FRAC_FITTED = 1e-3   # measured 822 of 4,194,304 (2.0e-4) for this seed; a sanity bound


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_texture_2048_fitted_like_state_full_frame():
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    print(f"[fitted] gen_fitted_like({SEED}) {H}x{W} n={n} N={N} K={K}", flush=True)
    p = synth.gen_fitted_like(SEED, H, W, N, n)
    p64 = p.astype(np.float64)
    r = Renderer(N, n, H, W, K, device=d)
    pt = torch.from_numpy(p).to(d)
    img, saved = r.render(pt)
    torch.cuda.synchronize()
    ids, ranges, vals = gpu_ids(r, saved, H, W, K)
    check_tile_lists(p64, H, W, ranges, vals)
    cnt = ranges[:, 1] - ranges[:, 0]
    print(f"[fitted] pairs {int(cnt.sum())}, largest hit set {int(cnt.max())}, tiles above 192 "
          f"{int((cnt > 192).sum())}, above 256 {int((cnt > 256).sum())}", flush=True)
    assert (cnt > 256).sum() > 0
    ref = cref.render(p64, H, W, K)
    tie = near_tie_mask(ref)
    img_np = img.cpu().numpy()
    nt = check_forward(img_np.astype(np.float64), ids, ref, K, tie, p64, (H, W))
    assert nt < TIE_FRAC_FITTED * H * W

    # two-pass adjoint, seeded upstream gradient zeroed at near-tie pixels
    g = synth.gen_grad_image(SEED + 1, n, H, W)
    g[:, tie] = 0.0
    o = cref.render_tiles(p64, H, W, K, grad_img=g.astype(np.float64), want=())
    gp = r.backward(pt, img, torch.from_numpy(g).to(d), saved)
    torch.cuda.synchronize()
    check_grad(gp.cpu().numpy().astype(np.float64), o["grad"], o["grad_abs"])
    del o, gp

    # single-pass L1 kernel against a target 0.02-0.1 away from the oracle's image
    rng = np.random.default_rng(SEED + 2)
    off = rng.uniform(0.02, 0.1, size=(n, H, W)) * rng.choice([-1.0, 1.0], size=(n, H, W))
    t1 = (ref["img"] - off).astype(np.float32)
    d64 = ref["img"] - t1.astype(np.float64)
    o1 = cref.render_tiles(p64, H, W, K, grad_img=np.sign(d64) / (n * H * W), want=())
    loss = torch.zeros(2, dtype=torch.float64, device=d)
    gp1 = torch.empty((5 + n, N), device=d)
    r.l1_grad_into(pt, torch.from_numpy(t1).to(d), loss, gp1, r.new_saved())
    torch.cuda.synchronize()
    l1 = np.abs(d64).mean()
    assert abs(float(loss[0]) - l1) <= 1e-6 * l1, (float(loss[0]), l1)
    # Gaussians retained at a near-tie pixel by either side are left out of the exact comparison
    ys, xs = np.nonzero(tie)
    held = np.unique(np.concatenate([ref["topk"][ys, xs].ravel(), ids[ys, xs].ravel()]))
    keep = np.setdiff1d(np.arange(N), held[held >= 0])
    print(f"[fitted] single-pass gradient: {len(keep)} Gaussians compared, "
          f"{N - len(keep)} retained at near-tie pixels", flush=True)
    check_grad(gp1.cpu().numpy().astype(np.float64)[:, keep], o1["grad"][:, keep],
               o1["grad_abs"][:, keep])
