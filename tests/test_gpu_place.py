"""GPU parity of the Gaussian placement entry points (igs_init_gaussians for Eq. 6,
igs_add_gaussians for Eq. 7) through the C ABI against the FP64 oracle (oracle/initref.py).

Both sides invert the same cumulative distribution at the same caller-supplied uniforms, so the
sampled pixels are compared exactly; only a uniform that falls within 1e-9 (relative) of a
boundary between two pixels' cumulative probabilities may resolve to either neighbour, and the
test then checks the pixel is valid under the oracle's distribution within that margin."""
import numpy as np
import pytest
import torch

from oracle import initref as ir
from paper_2407_01866_amd import synth
import paper_2407_01866_amd._native as nat

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run_place(target, uniforms, lam=0.3, image=None, scale=5.0, N_total=None, first=0,
              with_fit=True):
    d = dev()
    n, H, W = target.shape
    count = uniforms.size
    N_total = count + first if N_total is None else N_total
    tt = torch.from_numpy(np.ascontiguousarray(target, np.float32)).to(d)
    ut = torch.from_numpy(np.ascontiguousarray(uniforms, np.float32)).to(d)
    rp = torch.full((5 + n, N_total), -7.0, device=d)
    fp = torch.full((5 + n, N_total), -7.0, device=d) if with_fit else None
    ws = torch.empty(nat.igs_place_workspace_size(H, W), dtype=torch.uint8, device=d)
    if image is None:
        nat.igs_init_gaussians(tt, n, H, W, lam, ut, count, scale, rp, fp, N_total, first, ws,
                               ws.numel())
    else:
        it = torch.from_numpy(np.ascontiguousarray(image, np.float32)).to(d)
        nat.igs_add_gaussians(it, tt, n, H, W, ut, count, scale, rp, fp, N_total, first, ws,
                              ws.numel())
    torch.cuda.synchronize()
    return rp.cpu().numpy(), (fp.cpu().numpy() if with_fit else None)


def pixels_of(rp, W, first, count):
    mx, my = rp[0, first:first + count], rp[1, first:first + count]
    return ((my - 0.5).astype(np.int64) * W + (mx - 0.5).astype(np.int64))


def check_pixels(got, prob, uniforms, tol=1e-9):
    ref = ir.sample_pixels(prob, uniforms)
    cdf = np.cumsum(prob.ravel())
    t = uniforms.astype(np.float64) * cdf[-1]
    bad = np.nonzero(got != ref)[0]
    for i in bad:
        k = got[i]
        lo = cdf[k - 1] if k > 0 else 0.0
        assert prob.ravel()[k] > 0 or lo == cdf[k], (i, k)
        assert lo <= t[i] + tol and cdf[k] >= t[i] - tol, (i, k, ref[i], t[i], lo, cdf[k])
    assert bad.size <= max(2, uniforms.size // 10000), f"{bad.size} samples differ"


def check_params(rp, fp, target, pix, first, count, scale=5.0, N_total=None):
    n, H, W = target.shape
    h, w = pix // W, pix % W
    cols = slice(first, first + count)
    assert np.array_equal(rp[0, cols], (w + 0.5).astype(np.float32))
    assert np.array_equal(rp[1, cols], (h + 0.5).astype(np.float32))
    assert np.all(rp[2, cols] == 0) and np.all(rp[3:5, cols] == np.float32(scale))
    assert np.array_equal(rp[5:, cols], target[:, h, w].astype(np.float32))
    if fp is not None:
        assert np.allclose(fp[0, cols], (w + 0.5) / W, rtol=1e-7)
        assert np.allclose(fp[1, cols], (h + 0.5) / H, rtol=1e-7)
        assert np.all(fp[2, cols] == 0) and np.allclose(fp[3:5, cols], 1.0 / scale, rtol=1e-7)
        assert np.array_equal(fp[5:, cols], rp[5:, cols])
    others = np.ones(rp.shape[1], bool)
    others[cols] = False
    assert np.all(rp[:, others] == -7.0)
    if fp is not None:
        assert np.all(fp[:, others] == -7.0)


@pytest.mark.parametrize("n,H,W,lam", [(3, 64, 96, 0.3), (9, 50, 70, 0.3), (1, 1, 77, 0.3),
                                       (1, 90, 1, 0.0), (2, 5, 7, 1.0), (3, 256, 256, 0.0),
                                       (3, 33, 47, 0.7)])
def test_init_matches_oracle(n, H, W, lam):
    print(f"[place] init n={n} H={H} W={W} lam={lam}", flush=True)
    rng = np.random.default_rng(H * 131 + W)
    if n % 3 == 0:
        tgt = np.concatenate([synth.gen_image(H + k, H, W, 3, 10) for k in range(n // 3)])
    else:
        tgt = rng.random((n, H, W)).astype(np.float32)
    u = rng.random(777).astype(np.float32)
    rp, fp = run_place(tgt, u, lam)
    pix = pixels_of(rp, W, 0, u.size)
    check_pixels(pix, ir.init_probabilities(tgt.astype(np.float64), lam), u)
    check_params(rp, fp, tgt, pix, 0, u.size)


def test_init_constant_target_is_uniform_and_offsets_respected():
    print("[place] constant target", flush=True)
    tgt = np.full((3, 40, 30), 0.25, np.float32)
    u = np.random.default_rng(3).random(300).astype(np.float32)
    rp, fp = run_place(tgt, u, 0.3, N_total=1000, first=123, scale=2.5)
    pix = pixels_of(rp, 30, 123, 300)
    check_pixels(pix, ir.init_probabilities(tgt.astype(np.float64), 0.3), u)
    check_params(rp, fp, tgt, pix, 123, 300, scale=2.5)


def test_add_samples_only_pixels_with_error():
    print("[place] add, sparse error", flush=True)
    rng = np.random.default_rng(4)
    tgt = rng.random((3, 48, 64)).astype(np.float32)
    img = tgt.copy()
    spots = [(5, 7), (20, 40), (47, 63)]
    for (h, w), e in zip(spots, (0.1, 0.3, 0.6)):
        img[1, h, w] += e
    u = rng.random(2000).astype(np.float32)
    rp, fp = run_place(tgt, u, image=img, N_total=2500, first=500, with_fit=False)
    pix = pixels_of(rp, 64, 500, 2000)
    assert set(np.unique(pix)) <= {h * 64 + w for h, w in spots}
    check_pixels(pix, ir.error_probabilities(img.astype(np.float64), tgt.astype(np.float64)), u)
    check_params(rp, None, tgt, pix, 500, 2000)


def test_add_matches_oracle_on_a_render_like_image():
    print("[place] add", flush=True)
    rng = np.random.default_rng(5)
    tgt = synth.gen_image(77, 96, 80, 3, 20)
    img = (tgt + rng.normal(0, 0.05, tgt.shape)).astype(np.float32)
    u = rng.random(1500).astype(np.float32)
    rp, fp = run_place(tgt, u, image=img)
    pix = pixels_of(rp, 80, 0, 1500)
    check_pixels(pix, ir.error_probabilities(img.astype(np.float64), tgt.astype(np.float64)), u)
    check_params(rp, fp, tgt, pix, 0, 1500)


def test_zero_count_writes_nothing():
    tgt = np.random.default_rng(6).random((3, 20, 20)).astype(np.float32)
    rp, fp = run_place(tgt, np.zeros(0, np.float32), N_total=10, first=10)
    assert np.all(rp == -7.0) and np.all(fp == -7.0)


def test_init_texture_2048_n9_N50000():
    """Half of the texture workload's budget placed by Eq. 6 at full size (2048^2, n = 9)."""
    print("[place] texture 2048^2 n=9", flush=True)
    w = synth.workload(2)
    tgt = w.target()
    u = np.random.default_rng(7).random(w.N // 2).astype(np.float32)
    rp, fp = run_place(tgt, u, 0.3, N_total=w.N, first=0)
    pix = pixels_of(rp, w.W, 0, u.size)
    check_pixels(pix, ir.init_probabilities(tgt.astype(np.float64), 0.3), u)
    check_params(rp, fp, tgt, pix, 0, u.size, N_total=w.N)
