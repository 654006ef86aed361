"""GPU tests of the fitting loop (render + L1 gradient + adjoint + Adam in HIP) and of the
measurement hooks used by the benchmark."""
import math

import numpy as np
import pytest
import torch

from paper_2407_01866_amd import synth

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def make_fitter(cfg=0, **kw):
    from paper_2407_01866_amd.fit import PlainFitter
    w = synth.workload(cfg)
    d = dev()
    print(f"[fit] {w.name}", flush=True)
    return PlainFitter(torch.from_numpy(w.target()).to(d), torch.from_numpy(w.gaussians()).to(d),
                       w.K, **kw), w


def test_fit_256_psnr_rises():
    f, w = make_fitter(0)
    rep = f.run(300, report_every=50)
    ps = [p for _, p in rep]
    print(ps)
    assert all(b > a for a, b in zip(ps, ps[1:])), ps
    assert ps[-1] > ps[0] + 2.0


def test_fit_1024_N20000_1000_iters_psnr_each_100():
    f, w = make_fitter(1)
    rep = f.run(1000, report_every=100)
    ps = [p for _, p in rep]
    print("PSNR per 100 iterations:", [round(p, 3) for p in ps], flush=True)
    assert len(ps) == 10
    assert all(b > a for a, b in zip(ps, ps[1:])), ps


@pytest.mark.parametrize("ssim_weight", [0.0, 0.1])
def test_graph_replay_matches_eager_steps(ssim_weight):
    fa, _ = make_fitter(0, ssim_weight=ssim_weight)
    fb, _ = make_fitter(0, ssim_weight=ssim_weight)
    fb.capture()
    for _ in range(4):
        fa.step_async()
        fb.step()
    torch.cuda.synchronize()
    assert int(fa.step_count.item()) == int(fb.step_count.item()) == 4
    # the iteration is deterministic (no float atomics anywhere): identical states
    assert torch.equal(fb.fit, fa.fit) and torch.equal(fb.m, fa.m) and torch.equal(fb.v, fa.v)
    assert fa.psnr() == fb.psnr()


@pytest.mark.parametrize("mode", ["separate", "fused", "ssim"])
def test_first_step_equals_its_pieces(mode):
    """One fitter iteration equals the library's pieces chained by hand through the C ABI from
    the same seeded state: render, the loss gradient (L1, or L1 + 0.1 SSIM), the adjoint and the
    Adam step in the fitter's units.  Each piece is checked against the oracle on seeded inputs
    in its own test (render and adjoint, L1, SSIM, Adam), so this covers the fitter's plumbing;
    every step is deterministic, so the comparison is exact."""
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd.fit import AdamConfig
    from paper_2407_01866_amd.render import Renderer
    kw = {"ssim_weight": 0.1} if mode == "ssim" else {"fused": mode == "fused"}
    f, w = make_fitter(0, **kw)
    d = f.dev
    fit, rend = f.fit.clone(), f.rend.clone()
    f.step_async()
    r = Renderer(w.N, w.n, w.H, w.W, w.K, device=d)
    tgt = f.target
    gp = torch.empty_like(rend)
    if mode == "fused":
        img = torch.empty_like(tgt)
        loss = torch.zeros(2, dtype=torch.float64, device=d)
        r.render(rend)                                    # sizes the pair buffer
        saved = r.new_saved()
        r.render_l1_into(rend, tgt, img, loss, saved)
        r.backward_l1_into(rend, saved, gp)
    else:
        img, saved = r.render(rend)
        g = torch.empty_like(img)
        if mode == "ssim":
            loss = torch.zeros(4, dtype=torch.float64, device=d)
            ws = torch.empty(nat.igs_l1_ssim_workspace_size(w.n, w.H, w.W), dtype=torch.uint8,
                             device=d)
            nat.igs_l1_ssim_loss_grad(img, tgt, w.n, w.H, w.W, 0.1, g, loss, ws, ws.numel())
        else:
            loss = torch.zeros(2, dtype=torch.float64, device=d)
            ws = torch.empty(nat.igs_l1_workspace_size(img.numel()), dtype=torch.uint8, device=d)
            nat.igs_l1_loss_grad(img, tgt, w.n, w.H, w.W, g, loss, ws, ws.numel())
        r.backward_into(rend, img, g, saved, gp)
    a = AdamConfig()
    m, v = torch.zeros_like(fit), torch.zeros_like(fit)
    step = torch.zeros(1, dtype=torch.int32, device=d)
    nat.igs_adam_step(fit, rend, gp, m, v, step, w.N, w.n, w.H, w.W, a.lr_mu, a.lr_theta,
                      a.lr_inv_scale, a.lr_color, a.beta1, a.beta2, a.eps, 1.0 / max(w.H, w.W),
                      a.inv_scale_hi)
    torch.cuda.synchronize()
    assert torch.equal(f.image, img)
    if mode != "fused":
        assert torch.equal(f.grad_image, g)
    assert torch.equal(f.loss, loss)
    assert torch.equal(f.grad_params, gp)
    assert torch.equal(f.fit, fit) and torch.equal(f.rend, rend)
    assert torch.equal(f.m, m) and torch.equal(f.v, v) and int(f.step_count.item()) == 1


def test_fit_256_with_ssim_term_improves_psnr_and_ssim():
    f, w = make_fitter(0, ssim_weight=0.1)
    f.run(1, report_every=1)
    ssim0 = f.ssim()
    rep = f.run(300, report_every=100)
    ps = [p for _, p in rep]
    print("PSNR", ps, "SSIM", ssim0, "->", f.ssim(), flush=True)
    assert all(b > a for a, b in zip(ps, ps[1:])), ps
    assert f.ssim() > ssim0 + 0.05
    loss = f.loss.cpu().numpy()
    assert abs(loss[0] - (loss[1] + 0.1 * (1.0 - loss[3]))) <= 1e-12


def test_checkpoint_resume_reproduces_next_report():
    """Resuming from a checkpoint continues exactly the same trajectory (every step is
    deterministic); a fitter that did not load the state is far off."""
    f, w = make_fitter(0)
    f.run(60, report_every=60, use_graph=False)
    sd = f.state_dict()
    a = f.run(40, report_every=40, use_graph=False)[-1][1]
    g, _ = make_fitter(0)
    g.load_state_dict(sd)
    assert g.steps_done() == 60
    b = g.run(40, report_every=40, use_graph=False)[-1][1]
    assert a == b
    assert torch.equal(f.fit, g.fit)
    h, _ = make_fitter(0)
    c = h.run(40, report_every=40, use_graph=False)[-1][1]
    assert abs(c - a) > 0.5


def test_phase_timers_record_every_phase():
    from paper_2407_01866_amd import _native as nat
    f, _ = make_fitter(0)
    nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(True)
    for _ in range(3):
        f.step_async()
    torch.cuda.synchronize()
    t = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    # every phase of the two-pass iteration; the single-pass kernel is not part of it
    for phase, (ms, calls) in t.items():
        if phase == "raster_fit":
            assert calls == 0, (phase, ms, calls)
        else:
            assert calls == 3 and ms > 0, (phase, ms, calls)
    t = nat.igs_timing_read(reset=True)
    assert all(c == 0 for _, c in t.values())
    # the single-pass iteration: binning, the one raster kernel, the gradient reduction (which
    # also finishes the loss) and Adam
    f, _ = make_fitter(0, single_pass=True)
    nat.igs_timing_enable(True)
    for _ in range(2):
        f.step_async()
    torch.cuda.synchronize()
    t = nat.igs_timing_read(reset=True)
    nat.igs_timing_enable(False)
    for phase, (ms, calls) in t.items():
        if phase in ("raster_fwd", "raster_bwd", "loss"):
            assert calls == 0, (phase, ms, calls)
        else:
            assert calls == 2 and ms > 0, (phase, ms, calls)


def test_overflowed_iteration_is_a_no_op_and_is_repeated():
    """A render that overflows the pair buffer (forced by a tiny capacity) must leave the fitter's
    state untouched; advancing then grows the buffer and applies the iteration."""
    f, w = make_fitter(0, pair_capacity=500)
    fit0, m0 = f.fit.clone(), f.m.clone()
    f.step_async()
    torch.cuda.synchronize()
    assert int(f.status()[1]) == 1
    assert f.steps_done() == 0
    assert torch.equal(f.fit, fit0) and torch.equal(f.m, m0)
    f.advance_to(3, use_graph=False)
    assert f.steps_done() == 3 and f.r.cap > 500
    assert not torch.equal(f.fit, fit0)


# --------------------------------------------------------------- placement and densification


def _target256():
    w = synth.workload(0)
    return torch.from_numpy(w.target()).to(dev()), w


def test_from_target_places_gaussians_as_the_oracle():
    """The fitter's initial Gaussians are Eq. 6 samples at the generator's uniforms (pixel
    centres, rotation 0, 5 px, target colours), up to the fitter's own unit conversion."""
    from oracle import initref as ir
    from paper_2407_01866_amd.fit import PlainFitter
    t, w = _target256()
    f = PlainFitter.from_target(t, 4000, w.K, seed=3)
    assert f.N == 2000 and [s for s, _ in f.growth] == [500, 1000, 1500, 2000]
    gen = torch.Generator(device=t.device)
    gen.manual_seed(3)
    u = torch.rand(2000, generator=gen, device=t.device).cpu().numpy()
    ref = ir.init_gaussians(w.target().astype(np.float64), u)
    got = f.rend.cpu().numpy().astype(np.float64)
    # the sampled pixel of every Gaussian (a uniform within 1e-9 of a boundary may pick either
    # neighbour; none does at this seed)
    assert np.array_equal(np.floor(got[0]), np.floor(ref[0]))
    assert np.array_equal(np.floor(got[1]), np.floor(ref[1]))
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)


def test_densify_equals_direct_placement_call():
    """The fitter's error-guided addition is igs_add_gaussians on a render of its current
    parameters with the next uniforms of its generator; new columns start with zero Adam
    moments."""
    from paper_2407_01866_amd import _native as nat
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.render import Renderer
    t, w = _target256()
    f = PlainFitter.from_target(t, 2400, w.K, seed=5)
    f.run(40, report_every=40)
    img, _ = Renderer(f.N, w.n, w.H, w.W, w.K, device=t.device).render(f.rend.clone(),
                                                                       keep_state=False)
    fit0, m0 = f.fit.clone(), f.m.clone()
    state = f.gen.get_state()
    f.densify(300)
    gen = torch.Generator(device=t.device)
    gen.set_state(state)
    u = torch.rand(300, generator=gen, device=t.device)
    rp = torch.zeros((5 + w.n, 1500), device=t.device)
    fp = torch.zeros_like(rp)
    ws = torch.empty(nat.igs_place_workspace_size(w.H, w.W), dtype=torch.uint8, device=t.device)
    nat.igs_add_gaussians(img, f.target, w.n, w.H, w.W, u, 300, 5.0, rp, fp, 1500, 1200, ws,
                          ws.numel())
    torch.cuda.synchronize()
    assert f.N == 1500
    assert torch.equal(f.rend[:, 1200:], rp[:, 1200:])
    assert torch.equal(f.fit[:, 1200:], fp[:, 1200:])
    assert torch.equal(f.fit[:, :1200], fit0) and torch.equal(f.m[:, :1200], m0)
    assert torch.count_nonzero(f.m[:, 1200:]) == 0 and torch.count_nonzero(f.v[:, 1200:]) == 0


def test_progressive_fit_grows_on_schedule_and_beats_random_init():
    """The progressive schedule (Sec. 4.1: half the budget placed by Eq. 6, an eighth more by Eq. 7
    every 500 iterations) against the same fit held at its initial half.  Both start from the same
    Eq. 6 draws, so their reports agree exactly until the first addition; the progressive fit then
    grows on schedule and its PSNR keeps rising.  The paper gives no figure for what the additions
    gain (its ablation table has no such row), and on this small target the half budget already
    fits about as well within these iterations, so the two final PSNRs are printed, not ranked."""
    from paper_2407_01866_amd.fit import PlainFitter
    t, w = _target256()
    f = PlainFitter.from_target(t, 3000, w.K, seed=1)
    rep = f.run(1100, report_every=100)
    ps = [p for _, p in rep]
    print("progressive PSNR", [round(p, 2) for p in ps], "N", f.N, flush=True)
    assert f.N == 1500 + 2 * 375 and f.steps_done() == 1100
    fixed = PlainFitter.from_target(t, 1500, w.K, progressive=False, seed=1)
    pf = [p for _, p in fixed.run(1100, report_every=100)]
    print("fixed 1500 PSNR", [round(p, 2) for p in pf], flush=True)
    assert ps[:4] == pf[:4]                    # iterations 100..400: no addition yet
    assert ps[-1] > ps[0] and max(ps[5:]) > ps[4]   # rises, and recovers from the first addition
    g = PlainFitter(t, torch.from_numpy(synth.gen_gaussians(9, w.H, w.W, 3000, w.n)).to(t.device),
                    w.K)
    h = PlainFitter.from_target(t, 3000, w.K, progressive=False, seed=1)
    pg = g.run(300, report_every=300)[-1][1]
    ph = h.run(300, report_every=300)[-1][1]
    print("300 iterations: random init", pg, "content-adaptive", ph, flush=True)
    assert ph > pg + 1.0


def test_checkpoint_resume_across_a_densification():
    from paper_2407_01866_amd.fit import PlainFitter
    t, w = _target256()
    f = PlainFitter.from_target(t, 2000, w.K, seed=2)
    f.run(520, report_every=520)
    assert f.N == 1250
    sd = f.state_dict()
    a = f.run(500, report_every=500)[-1][1]
    g = PlainFitter.from_target(t, 2000, w.K, seed=2)
    g.load_state_dict(sd)
    assert g.N == 1250 and g.steps_done() == 520 and g.growth == sd["growth"]
    b = g.run(500, report_every=500)[-1][1]
    assert g.N == f.N == 1500
    assert a == b and torch.equal(f.fit, g.fit)
