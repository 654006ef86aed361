"""GPU parity of the single-pass L1 evaluation (igs_render_l1_grad and its batched form): render,
L1 comparison and adjoint of each tile in one kernel.

It evaluates the float expressions of the fused render + L1 pair (igs_render_l1, then
igs_render_backward_l1) in the same order: the same top-K ranking and double-precision weights,
the same per-pixel sign decisions and g . c_r, the same per-pair records and the same
fixed-order reductions.  Loss and gradient must therefore be identical to that pair's, which is
itself pinned to the FP64 oracle (test_gpu_fused).  Independently of the pair, the single-pass
gradient is checked against the oracle on targets built so that every sign is decided far from
0 and no pixel lies in a top-K near tie.
"""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_2407_01866_amd import synth
import paper_2407_01866_amd._native as nat

from test_gpu_render import check_grad, near_tie_mask

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _pair_and_single(p, tgt, H, W, K, capacity=None):
    """(loss, grad) of the fused pair and of the single-pass call, on one renderer."""
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    n, N = p.shape[0] - 5, p.shape[1]
    r = Renderer(N, n, H, W, K, device=d)
    pt = torch.from_numpy(np.ascontiguousarray(p)).to(d)
    tt = torch.from_numpy(np.ascontiguousarray(tgt)).to(d)
    if capacity is None:
        r.render(pt)                                       # sizes the pair buffer
    else:
        r.set_capacity(capacity)
    img = torch.empty((n, H, W), device=d)
    sa, sb = r.new_saved(), r.new_saved()
    la = torch.zeros(2, dtype=torch.float64, device=d)
    lb = torch.full((2,), -1.0, dtype=torch.float64, device=d)
    ga = torch.empty((5 + n, N), device=d)
    gb = torch.full((5 + n, N), float("nan"), device=d)
    r.render_l1_into(pt, tt, img, la, sa)
    r.backward_l1_into(pt, sa, ga)
    r.l1_grad_into(pt, tt, lb, gb, sb)
    torch.cuda.synchronize()
    # the binning state both calls leave behind is the same
    assert torch.equal(r.status_of(sa), r.status_of(sb))
    return r, sb, (la, ga), (lb, gb)


def assert_identical(a, b):
    (la, ga), (lb, gb) = a, b
    assert torch.equal(la, lb), (la.tolist(), lb.tolist())
    assert ga.shape == gb.shape
    assert torch.equal(ga, gb), f"{int((ga != gb).sum())} gradient entries differ"


def _target(H, W, n):
    if n % 3 == 0:
        return synth.gen_image(5 + H, H, W, n, 20)
    return np.random.default_rng(H).random((n, H, W), dtype=np.float64).astype(np.float32)


@pytest.mark.parametrize("H,W,n,N,K", [(256, 256, 3, 2000, 10), (200, 136, 9, 700, 10),
                                       (17, 33, 1, 40, 1), (90, 77, 16, 300, 32),
                                       (64, 48, 4, 150, 5), (72, 40, 16, 250, 8),
                                       (33, 160, 3, 0, 10)])
def test_single_pass_equals_fused_pair(H, W, n, N, K):
    """Ragged tails, every channel-count variant (1, 3, 4, 9, 16) and list lengths 1 to 32, and
    the empty set (the loss of an all-zero image)."""
    print(f"[single-pass] H={H} W={W} n={n} N={N} K={K}", flush=True)
    p = synth.gen_gaussians(11 + N, H, W, N, n)
    _, saved, a, b = _pair_and_single(p, _target(H, W, n), H, W, K)
    assert_identical(a, b)
    if N == 0:
        t = _target(H, W, n).astype(np.float64)
        np.testing.assert_allclose(b[0].cpu().numpy(), [np.abs(t).mean(), (t * t).mean()],
                                   rtol=1e-12)


def test_single_pass_large_hit_sets():
    """Hit sets of 500 members (more than one forward LDS batch of 192 and one adjoint batch of
    256): the blend reads colours from memory and the adjoint runs two batches per tile."""
    H, W, n, N, K = 48, 64, 3, 500, 10
    print(f"[single-pass] large hit sets H={H} W={W} N={N}", flush=True)
    p = synth.gen_gaussians(7, H, W, N, n)
    p[3:5] = np.float32(40.0)                               # every circle covers every tile
    r, saved, a, b = _pair_and_single(p, _target(H, W, n), H, W, K)
    assert int(r.status_of(saved)[nat.STAT_MAX_LIST]) == N
    assert_identical(a, b)


def test_single_pass_big_footprints():
    """Gaussians covering 244 to 400 tiles (both gradient reduction paths)."""
    from test_gpu_render import big_footprint_params
    p, H, W = big_footprint_params()
    print(f"[single-pass] big footprints H={H} W={W}", flush=True)
    _, _, a, b = _pair_and_single(p, _target(H, W, 3), H, W, 10)
    assert_identical(a, b)


def test_single_pass_on_overflow_matches_pair():
    """A pair buffer too small for the hit lists: both paths report the overflow, give the loss of
    an all-zero image and a zero gradient."""
    H, W, n, N, K = 64, 64, 3, 300, 10
    p = synth.gen_gaussians(3, H, W, N, n)
    r, saved, a, b = _pair_and_single(p, _target(H, W, n), H, W, K, capacity=64)
    assert int(r.status_of(saved)[nat.STAT_OVERFLOW]) != 0
    assert_identical(a, b)
    assert not bool(b[1].any())


@pytest.mark.parametrize("H,W,n,N,K,seed", [(96, 80, 3, 300, 10, 7), (50, 70, 9, 120, 4, 2),
                                            (40, 40, 1, 60, 1, 3)])
def test_single_pass_gradient_matches_oracle(H, W, n, N, K, seed):
    """Targets = oracle image -/+ an offset of 0.02..0.1, so every sign is decided far from 0."""
    print(f"[single-pass-oracle] H={H} W={W} n={n} N={N} K={K} seed={seed}", flush=True)
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    p = synth.gen_gaussians(seed, H, W, N, n)
    p64 = p.astype(np.float64)
    ref = cref.render(p64, H, W, K)
    tie = near_tie_mask(ref)
    assert tie.sum() == 0, "seed chosen to have no near-tie pixel"
    rng = np.random.default_rng(seed + 99)
    off = rng.uniform(0.02, 0.1, size=(n, H, W)) * rng.choice([-1.0, 1.0], size=(n, H, W))
    tgt = (ref["img"] - off).astype(np.float32)
    g = np.sign(ref["img"] - tgt.astype(np.float64)) / (n * H * W)
    o = cref.render(p64, H, W, K, grad_img=g)
    r = Renderer(N, n, H, W, K, device=d)
    pt = torch.from_numpy(p).to(d)
    r.render(pt)                                          # sizes the pair buffer
    saved = r.new_saved()
    loss = torch.zeros(2, dtype=torch.float64, device=d)
    gp = torch.empty((5 + n, N), device=d)
    r.l1_grad_into(pt, torch.from_numpy(tgt).to(d), loss, gp, saved)
    torch.cuda.synchronize()
    check_grad(gp.cpu().numpy().astype(np.float64), o["grad"], o["grad_abs"])
    d64 = ref["img"] - tgt.astype(np.float64)
    l1_ref, mse_ref = np.abs(d64).mean(), (d64 * d64).mean()
    assert abs(float(loss[0]) - l1_ref) <= 1e-6 * l1_ref
    assert abs(float(loss[1]) - mse_ref) <= 1e-5 * mse_ref


def test_single_pass_texture_2048_n9_N100000_equals_pair():
    """The benchmark's workload (2048^2, n = 9, N = 100k) in the launch configuration it times."""
    w = synth.workload(2)
    print(f"[single-pass] {w.name}", flush=True)
    _, _, a, b = _pair_and_single(w.gaussians(), w.target(), w.H, w.W, w.K)
    assert_identical(a, b)


def test_single_pass_batched_equals_plain():
    from paper_2407_01866_amd.render import BatchRenderer, Renderer
    d = dev()
    sizes = [(64, 96, 300), (130, 47, 150), (16, 16, 20), (200, 180, 900)]
    n, K = 3, 10
    print(f"[single-pass] batch {sizes}", flush=True)
    ps = [synth.gen_gaussians(40 + b, H, W, N, n) for b, (H, W, N) in enumerate(sizes)]
    ps[3][3:5, :5] = 150.0          # boxes of every tile of image 3: the cooperative binning path
    ts = [synth.gen_image(60 + b, H, W, n, 10) for b, (H, W, N) in enumerate(sizes)]
    br = BatchRenderer(sizes, n, K, device=d)
    bp = br.pack_params(ps)
    br.render(bp)                                          # sizes the pair buffer
    saved = br.new_saved()
    loss = torch.zeros((len(sizes), 2), dtype=torch.float64, device=d)
    gp = torch.empty((5 + n, br.N), device=d)
    br.l1_grad_into(bp, br.pack_images([torch.from_numpy(t) for t in ts]), loss, gp, saved)
    torch.cuda.synchronize()
    for b, (H, W, N) in enumerate(sizes):
        r = Renderer(N, n, H, W, K, device=d)
        pt = torch.from_numpy(ps[b]).to(d)
        r.render(pt)
        sv = r.new_saved()
        lo = torch.zeros(2, dtype=torch.float64, device=d)
        g1 = torch.empty((5 + n, N), device=d)
        r.l1_grad_into(pt, torch.from_numpy(ts[b]).to(d), lo, g1, sv)
        torch.cuda.synchronize()
        go = br.gauss_off[b]
        assert torch.equal(gp[:, go:go + N], g1), b
        assert torch.equal(loss[b], lo), b


def test_single_pass_fitters_track_fused_fitters():
    """20 graph-replayed iterations: the single-pass fitter's parameters and PSNR equal those of
    the fitter that runs the fused pair, plain and batched."""
    from paper_2407_01866_amd.fit import BatchFitter, PlainFitter
    d = dev()
    n, K = 3, 10
    w = synth.workload(0)
    tg = torch.from_numpy(w.target()).to(d)
    p0 = torch.from_numpy(w.gaussians()).to(d)
    a = PlainFitter(tg, p0, K, fused=True)
    b = PlainFitter(tg, p0, K, single_pass=True)
    a.run(20, report_every=20)
    b.run(20, report_every=20)
    assert a.psnr() == b.psnr()
    assert torch.equal(a.fit, b.fit) and torch.equal(a.rend, b.rend)
    sizes = [(64, 96, 400), (32, 48, 100)]
    tgs = [torch.from_numpy(synth.gen_image(40 + i, H, W, n, 10)).to(d)
           for i, (H, W, _) in enumerate(sizes)]
    pss = [torch.from_numpy(synth.gen_gaussians(50 + i, H, W, N, n)).to(d)
           for i, (H, W, N) in enumerate(sizes)]
    ba = BatchFitter(tgs, pss, K, fused=True)
    bb = BatchFitter(tgs, pss, K, single_pass=True)
    ba.run(20, report_every=20)
    bb.run(20, report_every=20)
    assert ba.psnrs() == bb.psnrs()
    assert torch.equal(ba.fit, bb.fit)


def test_single_pass_rejects_more_than_16_channels():
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    H = W = 32
    n, N, K = 17, 10, 4
    r = Renderer(N, n, H, W, K, device=d)
    p = torch.from_numpy(synth.gen_gaussians(1, H, W, N, n)).to(d)
    with pytest.raises(nat.IGSError) as e:
        r.l1_grad_into(p, torch.zeros((n, H, W), device=d),
                       torch.zeros(2, dtype=torch.float64, device=d),
                       torch.empty((5 + n, N), device=d), r.new_saved())
    assert e.value.status == nat.IGS_ERR_UNSUPPORTED


def test_single_pass_hit_set_beyond_16_bit_slots():
    """One 16 x 16 tile hit by 70,000 Gaussians (|S_j| > 65535, Sec. 3.2 ranks all of them): the
    single-pass kernel keeps its retained slots on chip at full width, so its loss and gradient
    match the oracle; the two-pass adjoint's 16-bit slots cannot address such a set, so the render
    marks its gradient as unusable and a two-pass fitter skips the step and raises, while a
    single-pass fitter steps."""
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    H = W = 16
    n, N, K = 3, 70000, 10
    print(f"[single-pass] |S_j| = {N} on one tile", flush=True)
    p = synth.gen_gaussians(70, H, W, N, n)
    p64 = p.astype(np.float64)
    ref = cref.render(p64, H, W, K)
    assert not near_tie_mask(ref).any(), "seed chosen to have no near-tie pixel"
    rng = np.random.default_rng(170)
    off = rng.uniform(0.02, 0.1, size=(n, H, W)) * rng.choice([-1.0, 1.0], size=(n, H, W))
    tgt = (ref["img"] - off).astype(np.float32)
    d64 = ref["img"] - tgt.astype(np.float64)
    o = cref.render(p64, H, W, K, grad_img=np.sign(d64) / (n * H * W))
    r = Renderer(N, n, H, W, K, device=d)
    pt = torch.from_numpy(p).to(d)
    tt = torch.from_numpy(tgt).to(d)
    saved = r.bin(pt)
    st = r.status_of(saved).cpu()
    assert int(st[nat.STAT_MAX_LIST]) == N and int(st[nat.STAT_SLOT_OVERFLOW]) == 1
    saved = r.new_saved()
    loss = torch.zeros(2, dtype=torch.float64, device=d)
    gp = torch.empty((5 + n, N), device=d)
    r.l1_grad_into(pt, tt, loss, gp, saved)
    torch.cuda.synchronize()
    st = r.status_of(saved).cpu()
    assert int(st[nat.STAT_SKIP]) == 0 and int(st[nat.STAT_OVERFLOW]) == 0
    check_grad(gp.cpu().numpy().astype(np.float64), o["grad"], o["grad_abs"])
    assert abs(float(loss[0]) - np.abs(d64).mean()) <= 1e-6 * np.abs(d64).mean()
    # the fused two-pass render reports the unusable slots in the skip word
    img = torch.empty((n, H, W), device=d)
    sv2 = r.new_saved()
    r.render_l1_into(pt, tt, img, torch.zeros(2, dtype=torch.float64, device=d), sv2)
    torch.cuda.synchronize()
    assert int(r.status_of(sv2)[nat.STAT_SKIP].item()) == 1
    two = PlainFitter(tt, pt, K)
    with pytest.raises(RuntimeError, match="65535"):
        two.advance_to(1, use_graph=False)
    assert two.steps_done() == 0
    one = PlainFitter(tt, pt, K, single_pass=True)
    one.advance_to(2, use_graph=False)
    assert one.steps_done() == 2
