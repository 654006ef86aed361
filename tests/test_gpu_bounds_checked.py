"""The bounds-checked build (libimagegs_debug.so: the same sources compiled with IGS_BOUNDS_CHECK,
so the kernels validate every index into their LDS batches and into the pair arrays against the
buffer sizes) runs the parity workloads with no index out of range, and its results are bit for
bit those of the normal build.

Workloads: the fitted-like state of the texture workload at full size (hit sets longer than one
LDS batch, Gaussians on thousands of tiles; Sec. 3.2 binning and ranking, Eq. 5 blend, Sec. 3.3
adjoint) through the single-pass and the two-pass iteration; a batch of uneven images with a
cooperative-binning Gaussian; 70,000 Gaussians on one tile (|S_j| > 65535); point queries.
"""
import numpy as np
import pytest
import torch

from paper_2407_01866_amd import _native as nat
from paper_2407_01866_amd import synth

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def debug_lib():
    dev()
    # built by __graft_entry__.build() beside the normal library; a missing build is a failure
    return nat.load(nat.LIB_DEBUG_PATH)


def both(debug_lib, fn):
    """fn() under the normal build and under the bounds-checked one; returns both results and the
    violation mask the checked build reported for its run."""
    torch.cuda.synchronize()
    assert nat.igs_bounds_violations() is None  # the normal build has no checks
    a = fn()
    torch.cuda.synchronize()
    with nat.using(debug_lib):
        assert nat.igs_bounds_violations() == 0  # clears anything left from earlier runs
        b = fn()
        torch.cuda.synchronize()
        v = nat.igs_bounds_violations()
    return a, b, v


def test_bounds_checked_fitted_state_single_and_two_pass(debug_lib):
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    H = W = 2048
    n, N, K = 9, 100000, 10
    print("[bounds] fitted-like 2048^2, single-pass and two-pass", flush=True)
    p = torch.from_numpy(synth.gen_fitted_like(2600, H, W, N, n)).to(d)
    t = torch.from_numpy(synth.gen_image(2601, H, W, n, 10)).to(d)
    r = Renderer(N, n, H, W, K, device=d)
    r.render(p, keep_state=False)  # sizes the pair buffer

    def single():
        loss = torch.zeros(2, dtype=torch.float64, device=d)
        g = torch.empty((5 + n, N), device=d)
        saved = r.new_saved()
        r.l1_grad_into(p, t, loss, g, saved)
        return loss, g, r.status_of(saved)[:6].clone()

    def two_pass():
        loss = torch.zeros(2, dtype=torch.float64, device=d)
        img = torch.empty((n, H, W), device=d)
        g = torch.empty((5 + n, N), device=d)
        saved = r.new_saved()
        r.render_l1_into(p, t, img, loss, saved)
        r.backward_l1_into(p, saved, g)
        return loss, img, g

    a, b, v = both(debug_lib, single)
    assert v == 0, f"bounds violations at sites {v:#x}"
    assert int(a[2][nat.STAT_MAX_LIST]) > 256  # hit sets longer than one LDS batch occur
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    a, b, v = both(debug_lib, two_pass)
    assert v == 0, f"bounds violations at sites {v:#x}"
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_bounds_checked_batch_and_long_hit_set(debug_lib):
    from paper_2407_01866_amd.render import BatchRenderer, Renderer
    d = dev()
    sizes = [(64, 96, 300), (130, 47, 150), (16, 16, 20), (200, 180, 900)]
    n, K = 3, 10
    print(f"[bounds] batch {sizes}", flush=True)
    ps = [synth.gen_gaussians(40 + b, H, W, N, n) for b, (H, W, N) in enumerate(sizes)]
    ps[3][3:5, :5] = 150.0  # boxes of every tile of image 3: the cooperative binning path
    ts = [synth.gen_image(60 + b, H, W, n, 10) for b, (H, W, N) in enumerate(sizes)]
    br = BatchRenderer(sizes, n, K, device=d)
    bp = br.pack_params(ps)
    br.render(bp)
    tt = br.pack_images([torch.from_numpy(x) for x in ts])

    def batch():
        loss = torch.zeros((len(sizes), 2), dtype=torch.float64, device=d)
        g = torch.empty((5 + n, br.N), device=d)
        br.l1_grad_into(bp, tt, loss, g, br.new_saved())
        return loss, g

    a, b, v = both(debug_lib, batch)
    assert v == 0, f"bounds violations at sites {v:#x}"
    for x, y in zip(a, b):
        assert torch.equal(x, y)

    print("[bounds] |S_j| = 70000 on one tile", flush=True)
    H = W = 16
    N = 70000
    p = torch.from_numpy(synth.gen_gaussians(70, H, W, N, n)).to(d)
    t = torch.from_numpy(synth.gen_image(71, H, W, n, 10)).to(d)
    r = Renderer(N, n, H, W, K, device=d)
    r.bin(p)

    def long_set():
        loss = torch.zeros(2, dtype=torch.float64, device=d)
        g = torch.empty((5 + n, N), device=d)
        r.l1_grad_into(p, t, loss, g, r.new_saved())
        return loss, g

    a, b, v = both(debug_lib, long_set)
    assert v == 0, f"bounds violations at sites {v:#x}"
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_bounds_checked_point_queries(debug_lib):
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    H, W, n, N, K = 512, 384, 3, 20000, 10
    print("[bounds] point queries", flush=True)
    p = torch.from_numpy(synth.gen_gaussians(90, H, W, N, n)).to(d)
    pts = torch.from_numpy(
        np.random.default_rng(91).uniform(0, 1, size=(50000, 2)).astype(np.float32)
        * np.array([W, H], np.float32)).to(d)
    r = Renderer(N, n, H, W, K, device=d)

    def query():
        saved = r.bin(p)
        return (r.query(p, saved, pts),)

    a, b, v = both(debug_lib, query)
    assert v == 0, f"bounds violations at sites {v:#x}"
    assert torch.equal(a[0], b[0])
