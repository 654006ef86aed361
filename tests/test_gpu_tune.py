"""Launch settings (one workgroup per tile or persistent tile queues, forward culling on or off,
the forward's LDS batch size, the length of its register-resident list) must not change a single
output bit, and the autotuner must leave the fitter's state as it was."""
import numpy as np
import pytest
import torch

from paper_2407_01866_amd import synth
import paper_2407_01866_amd._native as nat

pytestmark = pytest.mark.gpu

CONFIGS = [(0, 0, 1, 0, 0), (0, 0, 0, 0, 0), (1, 0, 1, 0, 0), (1, 4, 0, 0, 0), (1, 1, 1, 0, 0),
           (1, 8, 1, 0, 0), (0, 0, 1, 64, 0), (0, 0, 1, 128, 16), (1, 0, 1, 256, 32),
           (0, 0, 0, 96, 32)]


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def default_config():
    yield
    nat.igs_set_launch_config(0, 0, 1)


def _plain_outputs(p, tgt, H, W, K):
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    n, N = p.shape[0] - 5, p.shape[1]
    r = Renderer(N, n, H, W, K, pair_capacity=40 * N + 4096, device=d)
    pt = torch.from_numpy(p).to(d)
    img = torch.empty((n, H, W), device=d)
    sv = r.new_saved()
    r.render_into(pt, img, sv)
    g = torch.from_numpy(synth.gen_grad_image(3, n, H, W)).to(d)
    gp = torch.empty((5 + n, N), device=d)
    r.backward_into(pt, img, g, sv, gp)
    img2 = torch.empty_like(img)
    sv2 = r.new_saved()
    loss = torch.zeros(2, dtype=torch.float64, device=d)
    gp2 = torch.empty_like(gp)
    r.render_l1_into(pt, torch.from_numpy(tgt).to(d), img2, loss, sv2)
    r.backward_l1_into(pt, sv2, gp2)
    loss3 = torch.zeros(2, dtype=torch.float64, device=d)
    gp3 = torch.empty_like(gp)
    r.l1_grad_into(pt, torch.from_numpy(tgt).to(d), loss3, gp3, r.new_saved())
    torch.cuda.synchronize()
    assert int(r.status_of(sv)[nat.STAT_OVERFLOW]) == 0
    return img, r.slots(sv), gp, img2, loss, gp2, loss3, gp3


@pytest.mark.parametrize("H,W,n,N,K", [(512, 384, 3, 3000, 10), (200, 136, 9, 900, 16),
                                       (70, 90, 1, 300, 1)])
def test_launch_configs_give_identical_results(H, W, n, N, K):
    print(f"[tune] H={H} W={W} n={n} N={N} K={K}", flush=True)
    p = synth.gen_gaussians(31 + N, H, W, N, n)
    p[3:5, :3] = 200.0                       # a few Gaussians over every tile
    tgt = synth.gen_image(7, H, W, n, 20) if n % 3 == 0 else \
        np.random.default_rng(2).random((n, H, W)).astype(np.float32)
    nat.igs_set_launch_config(0, 0, 1)
    ref = _plain_outputs(p, tgt, H, W, K)
    for cfg in CONFIGS[1:]:
        nat.igs_set_launch_config(*cfg)
        got = _plain_outputs(p, tgt, H, W, K)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), cfg


def test_launch_configs_batched_identical():
    from paper_2407_01866_amd.render import BatchRenderer
    d = dev()
    sizes = [(64, 96, 300), (130, 47, 150), (16, 16, 20), (256, 180, 1200)]
    n, K = 3, 10
    ps = [synth.gen_gaussians(60 + b, H, W, N, n) for b, (H, W, N) in enumerate(sizes)]
    outs = []
    for cfg in CONFIGS:
        nat.igs_set_launch_config(*cfg)
        br = BatchRenderer(sizes, n, K, pair_capacity=200000, device=d)
        bp = br.pack_params([torch.from_numpy(q) for q in ps])
        imgs = br.new_images()
        sv = br.new_saved()
        br.render_into(bp, imgs, sv)
        g = torch.from_numpy(synth.gen_grad_image(5, 1, 1, n * br.P).reshape(-1)).to(d)
        gp = torch.empty_like(bp)
        br.backward_into(bp, imgs, g, sv, gp)
        tg = br.pack_images([torch.from_numpy(synth.gen_image(70 + b, H, W, n, 10))
                             for b, (H, W, _) in enumerate(sizes)])
        loss = torch.zeros((len(sizes), 2), dtype=torch.float64, device=d)
        gp1 = torch.empty_like(bp)
        br.l1_grad_into(bp, tg, loss, gp1, br.new_saved())
        torch.cuda.synchronize()
        outs.append((imgs, gp, loss, gp1))
    for cfg, got in zip(CONFIGS[1:], outs[1:]):
        for a, b in zip(got, outs[0]):
            assert torch.equal(a, b), cfg


def test_autotune_restores_fitter_state():
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.tune import autotune
    d = dev()
    w = synth.workload(0)
    f = PlainFitter(torch.from_numpy(w.target()).to(d), torch.from_numpy(w.gaussians()).to(d),
                    w.K, headroom=3.0)
    f.advance_to(3, use_graph=False)
    fit0, step0 = f.fit.clone(), f.steps_done()
    best, times = autotune(f, candidates=[(0, 0, 1, 0, 0), (1, 0, 1, 128, 16)], iters=2,
                           warmup=1)
    assert best in times and len(times) == 2 and all(t > 0 for t in times.values())
    assert f.steps_done() == step0 and torch.equal(f.fit, fit0)
    assert nat.igs_get_launch_config().as_tuple() == best




def test_autotune_coordinate_descent_of_a_single_pass_fitter():
    """Scheduling and culling first, then the LDS batch, then the list length; every trial
    restores the fitter, and the fitter keeps the winner."""
    from paper_2407_01866_amd.fit import PlainFitter
    from paper_2407_01866_amd.tune import FWD_BATCHES, SINGLE_PASS_SCHEDULES, autotune
    d = dev()
    w = synth.workload(0)
    f = PlainFitter(torch.from_numpy(w.target()).to(d), torch.from_numpy(w.gaussians()).to(d),
                    w.K, headroom=3.0, single_pass=True)
    f.advance_to(3, use_graph=False)
    fit0, step0 = f.fit.clone(), f.steps_done()
    best, times = autotune(f, iters=2, warmup=1)
    assert {c[:3] for c in times} == set(SINGLE_PASS_SCHEDULES)
    assert {c[3] for c in times} == set(FWD_BATCHES) and {c[4] for c in times} == {0, 16}
    assert len(times) == len(SINGLE_PASS_SCHEDULES) + len(FWD_BATCHES) - 1 + 1
    assert best in times and f.launch_config == best
    assert f.steps_done() == step0 and torch.equal(f.fit, fit0)
    nat.igs_set_launch_config(0, 0, 1)


def test_fitters_apply_their_own_launch_settings():
    """Two fitters tuned differently, stepped alternately on one thread: each step runs under its
    own fitter's settings (and, every setting being result-invariant, both match an untuned
    fitter bit for bit)."""
    from paper_2407_01866_amd.fit import PlainFitter
    w = synth.workload(0)
    d = dev()
    t = torch.from_numpy(w.target()).to(d)
    p = torch.from_numpy(w.gaussians()).to(d)
    fa = PlainFitter(t, p, w.K)
    fb = PlainFitter(t, p, w.K)
    fc = PlainFitter(t, p, w.K)
    fa.launch_config = (1, 4, 0, 128, 16)
    fb.launch_config = (0, 0, 1, 0, 0)
    nat.igs_set_launch_config(1, 6, 1)
    for _ in range(3):
        fa.step_async()
        assert nat.igs_get_launch_config().as_tuple() == (1, 4, 0, 128, 16)
        fb.step_async()
        assert nat.igs_get_launch_config().as_tuple() == (0, 0, 1, 0, 0)
        fc.step_async()                      # no own settings: the thread's current ones
        assert nat.igs_get_launch_config().as_tuple() == (0, 0, 1, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(fa.fit, fc.fit) and torch.equal(fb.fit, fc.fit)
