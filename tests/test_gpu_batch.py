"""GPU tests of the batched path: many images of uneven size and Gaussian count rendered,
differentiated and fitted with one launch per phase must give every image exactly what the plain
single-image path gives it (images are independent), and hence what the oracle gives."""
import numpy as np
import pytest
import torch

from oracle import cref, fitref
from paper_2407_01866_amd import synth

pytestmark = pytest.mark.gpu

SIZES = [(64, 96, 300), (17, 33, 40), (128, 128, 800), (1, 50, 5), (200, 136, 800), (32, 32, 0),
         (48, 80, 150)]


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def make_batch(sizes, n=3, seed=0):
    params = [synth.gen_gaussians(seed + 31 * b, H, W, N, n) for b, (H, W, N) in enumerate(sizes)]
    return params


def test_batched_render_equals_plain_renders():
    from paper_2407_01866_amd.render import BatchRenderer, Renderer
    d = dev()
    n, K = 3, 10
    params = make_batch(SIZES, n)
    print(f"[batch] {SIZES}", flush=True)
    br = BatchRenderer(SIZES, n, K, device=d)
    imgs, saved = br.render(br.pack_params([torch.from_numpy(p) for p in params]))
    torch.cuda.synchronize()
    views = br.image_views(imgs)
    slots = br.slots(saved)
    ranges, vals = br.tile_lists(saved)
    ranges, vals = ranges.cpu().numpy(), vals.cpu().numpy()
    for b, ((H, W, N), p) in enumerate(zip(SIZES, params)):
        r = Renderer(N, n, H, W, K, device=d)
        img, sv = r.render(torch.from_numpy(p).to(d))
        torch.cuda.synchronize()
        assert torch.equal(views[b], img), f"image {b} differs"
        assert torch.equal(slots[b], r.slots(sv)), f"slots of image {b} differ"
        pr, pv = r.tile_lists(sv)
        pr, pv = pr.cpu().numpy(), pv.cpu().numpy()
        t0 = br.descs[b].tile_off
        go = br.descs[b].gauss_off
        for t in range(pr.shape[0]):
            a = vals[ranges[t0 + t, 0]:ranges[t0 + t, 1]] - go
            assert np.array_equal(a, pv[pr[t, 0]:pr[t, 1]])


def test_batched_render_matches_oracle_per_image():
    from paper_2407_01866_amd.render import BatchRenderer
    d = dev()
    n, K = 3, 10
    params = make_batch(SIZES, n, seed=5)
    br = BatchRenderer(SIZES, n, K, device=d)
    imgs, _ = br.render(br.pack_params([torch.from_numpy(p) for p in params]))
    torch.cuda.synchronize()
    for b, ((H, W, N), p) in enumerate(zip(SIZES, params)):
        ref = cref.render(p.astype(np.float64), H, W, K)
        ok = ref["margin"] > 0                        # near ties: see test_gpu_render
        got = br.image_views(imgs)[b].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref["img"])[:, ok]
        assert np.all(err <= 1e-5 * np.abs(ref["img"][:, ok]) + 1e-7), (b, err.max())


def test_batched_backward_equals_plain_backward():
    from paper_2407_01866_amd.render import BatchRenderer, Renderer
    d = dev()
    n, K = 3, 10
    params = make_batch(SIZES, n, seed=9)
    br = BatchRenderer(SIZES, n, K, device=d)
    pt = br.pack_params([torch.from_numpy(p) for p in params])
    imgs, saved = br.render(pt)
    g = torch.from_numpy(synth.gen_grad_image(3, 1, 1, n * br.P).reshape(-1)).to(d)
    gp = torch.empty_like(pt)
    br.backward_into(pt, imgs, g, saved, gp)
    torch.cuda.synchronize()
    gviews = br.image_views(g)
    for b, ((H, W, N), p) in enumerate(zip(SIZES, params)):
        if N == 0:
            continue
        r = Renderer(N, n, H, W, K, device=d)
        pb = torch.from_numpy(p).to(d)
        img, sv = r.render(pb)
        ref = r.backward(pb, img, gviews[b].contiguous(), sv)
        go = br.descs[b].gauss_off
        got = gp[:, go:go + N]
        # the same per-tile records summed in the same emit order: identical bits
        assert torch.equal(got, ref), b


def test_tile_queue_is_stable_largest_first():
    from paper_2407_01866_amd.render import BatchRenderer
    d = dev()
    params = make_batch(SIZES, 3, seed=2)
    br = BatchRenderer(SIZES, 3, 10, device=d)
    _, saved = br.render(br.pack_params([torch.from_numpy(p) for p in params]))
    q = br.tile_queue(saved).cpu().numpy()
    ranges, _ = br.tile_lists(saved)
    cnt = (ranges[:, 1] - ranges[:, 0]).cpu().numpy()
    assert np.array_equal(np.sort(q), np.arange(br.T))
    expect = np.array(sorted(range(br.T), key=lambda t: (-cnt[t], t)))
    assert np.array_equal(q, expect)


def test_batched_l1_and_adam_match_reference():
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd.render import BatchRenderer
    d = dev()
    n = 3
    sizes = [(40, 70, 50), (16, 16, 0), (90, 33, 120)]
    br = BatchRenderer(sizes, n, 10, device=d)
    imgs = [torch.from_numpy(synth.gen_image(b, H, W, n, 4)) for b, (H, W, _) in enumerate(sizes)]
    tgts = [torch.from_numpy(synth.gen_image(10 + b, H, W, n, 4)) for b, (H, W, _) in enumerate(sizes)]
    I, T = br.pack_images(imgs), br.pack_images(tgts)
    G = torch.empty_like(I)
    loss = torch.zeros((3, 2), dtype=torch.float64, device=d)
    ws = torch.empty(nat.igs_l1_batched_workspace_size(br.descs, n), dtype=torch.uint8, device=d)
    nat.igs_l1_loss_grad_batched(I, T, br.descs, br.d_descs, n, G, loss, ws, ws.numel())
    torch.cuda.synchronize()
    for b in range(3):
        l_ref, g_ref = fitref.l1_loss_grad(imgs[b].numpy(), tgts[b].numpy())
        assert loss[b, 0].item() == pytest.approx(l_ref, rel=1e-13)
        np.testing.assert_allclose(br.image_views(G)[b].cpu().numpy(), g_ref, rtol=1e-6)
    # Adam: per-image normalization of the mean and per-image inverse-scale floor
    params = [synth.gen_gaussians(70 + b, H, W, N, n) for b, (H, W, N) in enumerate(sizes)]
    fits = [fitref.to_fit_space(p.astype(np.float64), H, W) for p, (H, W, _) in zip(params, sizes)]
    fit = torch.from_numpy(np.concatenate(fits, axis=1).astype(np.float32)).to(d)
    rend = torch.empty_like(fit)
    m, v = torch.zeros_like(fit), torch.zeros_like(fit)
    step = torch.zeros(1, dtype=torch.int32, device=d)
    grads = [np.random.default_rng(b).standard_normal((5 + n, N)) * 1e-3 for b, (_, _, N) in enumerate(sizes)]
    gt = torch.from_numpy(np.concatenate(grads, axis=1).astype(np.float32)).to(d)
    nat.igs_adam_step_batched(fit, rend, gt, m, v, step, br.descs, br.d_descs, n, fitref.LR_MU,
                              fitref.LR_TH, fitref.LR_S, fitref.LR_C)
    torch.cuda.synchronize()
    for b, (H, W, N) in enumerate(sizes):
        go = br.descs[b].gauss_off
        gf = fitref.grad_to_fit_space(grads[b].astype(np.float32).astype(np.float64), fits[b], H, W)
        ref, _, _ = fitref.adam_step(fits[b].astype(np.float32).astype(np.float64), gf,
                                     np.zeros_like(gf), np.zeros_like(gf), 1, fitref.row_lrs(n),
                                     H=H, W=W)
        np.testing.assert_allclose(fit[:, go:go + N].cpu().numpy(), ref, rtol=2e-5, atol=2e-6)
        np.testing.assert_allclose(rend[:, go:go + N].cpu().numpy(),
                                   fitref.to_render_space(ref, H, W), rtol=2e-5, atol=2e-5)


def test_batch_fitter_tracks_plain_fitters():
    from paper_2407_01866_amd.fit import BatchFitter, PlainFitter
    d = dev()
    n, K = 3, 10
    sizes = [(64, 96, 400), (128, 64, 600), (32, 48, 100)]
    tg = [torch.from_numpy(synth.gen_image(40 + b, H, W, n, 10)).to(d) for b, (H, W, _) in enumerate(sizes)]
    ps = [torch.from_numpy(synth.gen_gaussians(50 + b, H, W, N, n)).to(d) for b, (H, W, N) in enumerate(sizes)]
    bf = BatchFitter(tg, ps, K)
    bf.run(40, report_every=40)
    bp = bf.psnrs()
    for b in range(len(sizes)):
        pf = PlainFitter(tg[b], ps[b], K)
        pf.run(40, report_every=40)
        # every kernel of the batched iteration evaluates each image exactly as the plain one
        assert pf.psnr() == bp[b], b
        assert torch.equal(bf.image_params(b), pf.rend), b


def test_batched_ssim_loss_equals_plain_calls():
    """igs_l1_ssim_loss_grad_batched gives every image the gradient igs_l1_ssim_loss_grad gives it
    alone (bit for bit: the same per-pixel operations) and its loss terms (sums in another
    order)."""
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd.render import BatchRenderer
    d = dev()
    n = 3
    sizes = [(64, 96, 10), (130, 47, 10), (5, 7, 10), (300, 200, 10), (1, 77, 10), (128, 32, 10)]
    print(f"[batch-ssim] {len(sizes)} images", flush=True)
    br = BatchRenderer(sizes, n, 10, device=d)
    rng = np.random.default_rng(12)
    imgs = [torch.from_numpy(synth.gen_image(80 + b, H, W, n, 6)) for b, (H, W, _) in enumerate(sizes)]
    tgts = [torch.from_numpy((synth.gen_image(80 + b, H, W, n, 6) +
                              rng.normal(0, 0.05, (n, H, W))).astype(np.float32))
            for b, (H, W, _) in enumerate(sizes)]
    I, T = br.pack_images(imgs), br.pack_images(tgts)
    G = torch.empty_like(I)
    loss = torch.zeros((len(sizes), 4), dtype=torch.float64, device=d)
    ws = torch.empty(nat.igs_l1_ssim_batched_workspace_size(br.descs, n), dtype=torch.uint8,
                     device=d)
    nat.igs_l1_ssim_loss_grad_batched(I, T, br.descs, br.d_descs, n, 0.1, G, loss, ws, ws.numel())
    torch.cuda.synchronize()
    gv = br.image_views(G)
    for b, (H, W, _) in enumerate(sizes):
        x, y = imgs[b].to(d), tgts[b].to(d)
        g = torch.empty_like(x)
        lo = torch.zeros(4, dtype=torch.float64, device=d)
        w1 = torch.empty(nat.igs_l1_ssim_workspace_size(n, H, W), dtype=torch.uint8, device=d)
        nat.igs_l1_ssim_loss_grad(x, y, n, H, W, 0.1, g, lo, w1, w1.numel())
        torch.cuda.synchronize()
        assert torch.equal(gv[b], g), b
        assert np.allclose(loss[b].cpu().numpy(), lo.cpu().numpy(), rtol=1e-12, atol=1e-15), b


def test_batch_fitter_with_ssim_tracks_plain_fitters():
    from paper_2407_01866_amd.fit import BatchFitter, PlainFitter
    d = dev()
    n, K = 3, 10
    sizes = [(64, 96, 400), (200, 136, 900), (32, 48, 100)]
    tg = [torch.from_numpy(synth.gen_image(40 + b, H, W, n, 10)).to(d) for b, (H, W, _) in enumerate(sizes)]
    ps = [torch.from_numpy(synth.gen_gaussians(50 + b, H, W, N, n)).to(d) for b, (H, W, N) in enumerate(sizes)]
    bf = BatchFitter(tg, ps, K, ssim_weight=0.1)
    bf.run(30, report_every=30)
    bp = bf.psnrs()
    for b in range(len(sizes)):
        pf = PlainFitter(tg[b], ps[b], K, ssim_weight=0.1)
        pf.run(30, report_every=30)
        assert torch.equal(bf.image_params(b), pf.rend), b
        assert abs(pf.psnr() - bp[b]) < 1e-9, b
