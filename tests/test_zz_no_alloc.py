"""The no-allocation single-pass call (igs_render_l1_grad_noalloc) against igs_render_l1_grad,
through the C ABI: the same loss, gradient and saved state bit for bit, on two calls in a row
(the second on a smaller problem, so it runs on what the first left in the static workspace)."""
import numpy as np
import pytest
import torch

from paper_2407_01866_amd import _native as nat
from paper_2407_01866_amd import synth

pytestmark = pytest.mark.gpu

CASES = [(256, 256, 3, 2000, 10, 11), (96, 80, 3, 300, 10, 12)]   # second smaller


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _problem(H, W, n, N, K, seed, d):
    from paper_2407_01866_amd.render import Renderer
    p = torch.from_numpy(synth.gen_gaussians(seed, H, W, N, n)).to(d)
    t = torch.from_numpy(synth.gen_image(seed, H, W, n, 10)).to(d)
    r = Renderer(N, n, H, W, K, device=d)
    r.render(p, keep_state=False)                 # sizes the pair buffer
    return r, p, t


def test_noalloc_matches_workspace_call_on_two_calls_in_a_row():
    d = dev()
    probs = [_problem(*c, d) for c in CASES]
    ref = []
    for r, p, t in probs:
        loss = torch.zeros(2, dtype=torch.float64, device=d)
        gp = torch.empty((5 + r.n, r.N), device=d)
        saved = r.new_saved()
        r.l1_grad_into(p, t, loss, gp, saved)
        ref.append((loss, gp, saved))
    torch.cuda.synchronize()
    got = []
    for (r, p, t), c in zip(probs, CASES):
        print(f"[noalloc] H={c[0]} W={c[1]} n={c[2]} N={c[3]} K={c[4]} cap={r.cap}", flush=True)
        ws, _ = nat.igs_render_buffer_sizes(r.N, r.n, r.H, r.W, r.K, 16, 16, r.cap)
        assert ws <= nat.IGS_NOALLOC_SCRATCH_BYTES
        loss = torch.full((2,), -1.0, dtype=torch.float64, device=d)
        gp = torch.full((5 + r.n, r.N), float("nan"), device=d)
        saved = r.new_saved()
        nat.igs_render_l1_grad_noalloc(p, r.N, r.n, r.H, r.W, r.K, 16, 16, r.cap, t, loss, gp,
                                       saved, saved.numel())
        got.append((loss, gp, saved))
    torch.cuda.synchronize()
    for (r, _, _), (l0, g0, s0), (l1, g1, s1) in zip(probs, ref, got):
        assert int(r.status_of(s1)[nat.STAT_OVERFLOW]) == 0
        assert torch.equal(l0, l1), (l0, l1)
        assert torch.equal(g0, g1)
        assert torch.equal(r.status_of(s0), r.status_of(s1))
        ra, va = r.tile_lists(s0)
        rb, vb = r.tile_lists(s1)
        assert torch.equal(ra, rb) and torch.equal(va, vb)
        assert float(l1[0]) > 0 and np.isfinite(g1.cpu().numpy()).all()


def test_noalloc_rejects_a_workspace_beyond_its_array():
    d = dev()
    H = W = 64
    n, N, K = 3, 10, 10
    cap = 1 << 24
    ws, sv = nat.igs_render_buffer_sizes(N, n, H, W, K, 16, 16, cap)
    assert ws > nat.IGS_NOALLOC_SCRATCH_BYTES
    p = torch.from_numpy(synth.gen_gaussians(1, H, W, N, n)).to(d)
    saved = torch.empty(sv, dtype=torch.uint8, device=d)
    with pytest.raises(nat.IGSError) as e:
        nat.igs_render_l1_grad_noalloc(p, N, n, H, W, K, 16, 16, cap,
                                       torch.zeros((n, H, W), device=d),
                                       torch.zeros(2, dtype=torch.float64, device=d),
                                       torch.empty((5 + n, N), device=d), saved, sv)
    assert e.value.status == nat.IGS_ERR_WORKSPACE
