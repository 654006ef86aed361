"""Binning (Sec. 3.2: the hit sets S_j of every tile, in ascending Gaussian index) under each plan
of the pair sort, against the oracle's brute-force tile lists, together with the tile statistics
of the status block (pair count, largest |S_j|, E_fwd = sum_j |S_j| npx_j and
E_bwd = sum_j min(K, |S_j|) npx_j, npx_j = the tile's pixels inside the image).

Plans by the number of tile-key bits b = ceil(log2 T): up to 16 bits a stable partition by the
top min(8, b) bits followed by one workgroup per group (with the Gaussian index packed into the
key when both fit 32 bits, else looked up per pair), above 16 bits LSD passes.  The cases cover
b = 1 (one tile), 8 (one tile per group), 12 and 14 with packed keys, 16 with looked-up indices
and 17 (LSD passes).
"""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_2407_01866_amd import _native as nat
from paper_2407_01866_amd import synth

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def expected(p64, H, W, K):
    counts, lists = cref.tile_lists(p64, H, W)
    tx_n = (W + 15) // 16
    t = np.arange(counts.size)
    tx, ty = t % tx_n, t // tx_n
    npx = (np.minimum(W - tx * 16, 16) * np.minimum(H - ty * 16, 16)).astype(np.int64)
    stats = {nat.STAT_PAIRS: int(counts.sum()), nat.STAT_MAX_LIST: int(counts.max()),
             nat.STAT_EVALS_FWD: int((counts * npx).sum()),
             nat.STAT_EVALS_BWD: int((np.minimum(counts, K) * npx).sum())}
    return counts, lists, stats


CASES = [
    # H, W, N, smin, smax: tile-key bits
    (16, 16, 3000, 1.0, 12.0),       # 1
    (256, 256, 2000, 1.0, 12.0),     # 8
    (600, 1000, 20000, 1.0, 30.0),   # 12, ragged edge tiles
    (2048, 2048, 30000, 1.0, 40.0),  # 14
    (2912, 2896, 65537, 1.0, 12.0),  # 16, Gaussian index looked up (17 + 16 bits)
    (4128, 4112, 3000, 4.0, 60.0),   # 17: LSD passes
]


@pytest.mark.parametrize("H,W,N,smin,smax", CASES)
def test_tile_lists_and_statistics(H, W, N, smin, smax):
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    n, K = 3, 10
    print(f"[binning] H={H} W={W} N={N} sigma {smin}-{smax}", flush=True)
    p = synth.gen_gaussians(7 + H + W, H, W, N, n, smin=smin, smax=smax)
    r = Renderer(N, n, H, W, K, device=d)
    saved = r.bin(torch.from_numpy(p).to(d))
    torch.cuda.synchronize()
    st = r.status_of(saved).cpu().numpy()
    ranges, vals = (x.cpu().numpy() for x in r.tile_lists(saved))
    counts, lists, stats = expected(p.astype(np.float64), H, W, K)
    assert st[nat.STAT_OVERFLOW] == 0 and st[nat.STAT_SKIP] == 0
    for k, v in stats.items():
        assert int(st[k]) == v, (k, int(st[k]), v)
    assert st[nat.STAT_SLOT_OVERFLOW] == (1 if stats[nat.STAT_MAX_LIST] > 0xFFFF else 0)
    assert np.array_equal(ranges[:, 1] - ranges[:, 0], counts)
    # tiles in order, each list at its own place, empty tiles [0, 0)
    nz = counts > 0
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    assert np.array_equal(ranges[nz, 0], start[nz])
    assert not ranges[~nz].any()
    assert np.array_equal(vals[: counts.sum()], lists)


def test_single_pass_reports_the_same_statistics():
    """The single-pass L1 iteration sums the binning's per-group statistics in its gradient
    reduction instead of a kernel of its own; its status block must equal binning alone's."""
    from paper_2407_01866_amd.render import Renderer
    d = dev()
    H, W, N, n, K = 600, 1000, 20000, 3, 10
    print(f"[binning] single-pass statistics H={H} W={W} N={N}", flush=True)
    p = torch.from_numpy(synth.gen_gaussians(11, H, W, N, n, smin=1.0, smax=30.0)).to(d)
    t = torch.from_numpy(synth.gen_image(12, H, W, n, 10)).to(d)
    r = Renderer(N, n, H, W, K, device=d)
    ref = r.status_of(r.bin(p)).cpu().clone()
    saved = r.new_saved()
    loss = torch.zeros(2, dtype=torch.float64, device=d)
    g = torch.empty((5 + n, N), device=d)
    r.l1_grad_into(p, t, loss, g, saved)
    torch.cuda.synchronize()
    st = r.status_of(saved).cpu()
    assert torch.equal(st[:7], ref[:7]), (st[:7].tolist(), ref[:7].tolist())
    assert int(st[nat.STAT_EVALS_FWD]) > 0
