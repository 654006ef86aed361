"""Pins for the FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: closed forms of Eq. 1, 2 and 5
for one and two Gaussians, the K >= |S_j| reduction to the normalized Eq. 4 blend, the K = 1
nearest-Gaussian partition, partition of unity, the symmetries of Eq. 2, an independent NumPy
implementation (explicit covariance inverse, matrix-form adjoint) and central finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import cref, dense, fitref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def make_params(rng, N, n, H, W, smin=1.0, smax=12.0):
    p = np.empty((5 + n, N))
    p[0] = rng.uniform(0, W, N)
    p[1] = rng.uniform(0, H, N)
    p[2] = rng.uniform(0, math.pi, N)
    p[3] = np.exp(rng.uniform(math.log(smin), math.log(smax), N))
    p[4] = np.exp(rng.uniform(math.log(smin), math.log(smax), N))
    p[5:] = rng.uniform(0, 1, (n, N))
    return p.astype(np.float32).astype(np.float64)


def tiles_hit_by_segments(mx, my, r, H, W, tile):
    """Independent tile test: the circle meets the closed rectangle iff the centre lies inside it
    or one of its four edges (segments) comes within r of the centre."""
    def seg_dist2(px, py, ax, ay, bx, by):
        vx, vy = bx - ax, by - ay
        L2 = vx * vx + vy * vy
        t = 0.0 if L2 == 0 else max(0.0, min(1.0, ((px - ax) * vx + (py - ay) * vy) / L2))
        cx, cy = ax + t * vx, ay + t * vy
        return (px - cx) ** 2 + (py - cy) ** 2

    hits = []
    tx_n, ty_n = (W + tile - 1) // tile, (H + tile - 1) // tile
    for ty in range(ty_n):
        for tx in range(tx_n):
            x0, y0 = tx * tile, ty * tile
            x1, y1 = min(x0 + tile, W), min(y0 + tile, H)
            inside = x0 <= mx <= x1 and y0 <= my <= y1
            d2 = min(seg_dist2(mx, my, x0, y0, x1, y0), seg_dist2(mx, my, x1, y0, x1, y1),
                     seg_dist2(mx, my, x1, y1, x0, y1), seg_dist2(mx, my, x0, y1, x0, y0))
            if inside or d2 <= r * r:
                hits.append(ty * tx_n + tx)
    return hits


def pixel_tile(H, W, tile):
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return (hh // tile) * ((W + tile - 1) // tile) + ww // tile


# --------------------------------------------------------------------------- single Gaussian


@pytest.mark.parametrize("seed", range(6))
def test_single_gaussian_support_and_colour(seed):
    rng = np.random.default_rng(seed)
    H, W, n, tile = 70, 90, 3, 16
    p = make_params(rng, 1, n, H, W, 1.0, 9.0)
    r = 3.0 * max(p[3, 0], p[4, 0])
    hits = set(tiles_hit_by_segments(p[0, 0], p[1, 0], r, H, W, tile))
    counts, _ = cref.tile_lists(p, H, W, tile)
    assert set(np.nonzero(counts)[0].tolist()) == hits
    g = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, K=10, tile=tile, grad_img=g)
    covered = np.isin(pixel_tile(H, W, tile), list(hits))
    for ch in range(n):
        # one candidate: weight 1, the pixel takes the Gaussian's colour exactly
        assert np.array_equal(o["img"][ch][covered], np.full(covered.sum(), p[5 + ch, 0]))
        assert np.all(o["img"][ch][~covered] == 0)
        assert o["grad"][5 + ch, 0] == pytest.approx(g[ch][covered].sum(), rel=1e-12, abs=1e-12)
    # with a single candidate the blend weight is 1 regardless of geometry: no geometry gradient
    assert np.all(o["grad"][:5] == 0)
    assert np.all(o["topk"][covered][:, 0] == 0) and np.all(o["topk"][~covered] == -1)


@pytest.mark.parametrize("theta,axis_swap", [(0.0, False), (math.pi / 2, True)])
def test_single_gaussian_quadratic_form_closed_form(theta, axis_swap):
    H = W = 48
    p = np.array([[20.25], [27.5], [theta], [3.5], [1.75], [0.3]])
    o = cref.render(p, H, W, K=4)
    q = o["qsel"][..., 0]
    hh, ww = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    sx, sy = (p[4, 0], p[3, 0]) if axis_swap else (p[3, 0], p[4, 0])
    closed = ((ww - p[0, 0]) / sx) ** 2 + ((hh - p[1, 0]) / sy) ** 2
    m = np.isfinite(q)
    assert m.sum() > 100
    np.testing.assert_allclose(q[m], closed[m], rtol=1e-13, atol=1e-12)


def test_isotropic_gaussian_independent_of_theta():
    H = W = 32
    base = np.array([[14.0], [17.0], [0.0], [2.5], [2.5], [1.0]])
    ref = cref.render(base, H, W, K=2)["qsel"][..., 0]
    for th in (0.3, 1.1, 2.9):
        p = base.copy()
        p[2, 0] = th
        q = cref.render(p, H, W, K=2)["qsel"][..., 0]
        m = np.isfinite(ref)
        np.testing.assert_allclose(q[m], ref[m], rtol=1e-13)


def test_tile_test_tangency_and_clipping():
    # edge tangency: circle r = 6 about (22, 8) touches x = 16, the right edge of tile 0
    p = np.array([[22.0], [8.0], [0.0], [2.0], [1.0], [1.0]])
    counts, _ = cref.tile_lists(p, 32, 64, 16)
    assert counts[0] == 1 and counts[1] == 1 and counts[2] == 0
    p[0, 0] = 22.0 + 2.0 ** -20
    counts, _ = cref.tile_lists(p, 32, 64, 16)
    assert counts[0] == 0
    # corner tangency (9, 12, 15 triangle): r = 15 about (25, 28) touches the corner (16, 16)
    p = np.array([[25.0], [28.0], [0.0], [5.0], [1.0], [1.0]])
    counts, _ = cref.tile_lists(p, 64, 64, 16)
    assert counts[0] == 1
    p[1, 0] = 28.0 + 2.0 ** -20
    counts, _ = cref.tile_lists(p, 64, 64, 16)
    assert counts[0] == 0
    # the last tile of a 40-wide image is clipped to [32, 40]: centre at x = 47 needs r >= 7
    p = np.array([[47.0], [8.0], [0.0], [2.0], [1.0], [1.0]])       # r = 6
    counts, _ = cref.tile_lists(p, 16, 40, 16)
    assert counts.sum() == 0
    p[3, 0] = 2.5                                                     # r = 7.5
    counts, _ = cref.tile_lists(p, 16, 40, 16)
    assert counts.tolist() == [0, 0, 1]


@pytest.mark.parametrize("seed", range(3))
def test_tile_lists_match_segment_test(seed):
    rng = np.random.default_rng(100 + seed)
    H, W, tile = 80, 112, 16
    p = make_params(rng, 40, 1, H, W, 0.5, 10.0)
    p[0] = rng.uniform(-30, W + 30, 40)     # include centres outside the image
    p[1] = rng.uniform(-30, H + 30, 40)
    counts, lists = cref.tile_lists(p, H, W, tile)
    T = cref.num_tiles(H, W, tile)
    members = [set() for _ in range(T)]
    off = np.concatenate([[0], np.cumsum(counts)])
    for t in range(T):
        seg = lists[off[t]:off[t + 1]]
        assert np.all(np.diff(seg) > 0)          # ascending Gaussian index
        members[t] = set(seg.tolist())
    for i in range(40):
        r = 3.0 * max(p[3, i], p[4, i])
        for t in tiles_hit_by_segments(p[0, i], p[1, i], r, H, W, tile):
            assert i in members[t]
    assert sum(len(m) for m in members) == sum(
        len(tiles_hit_by_segments(p[0, i], p[1, i], 3.0 * max(p[3, i], p[4, i]), H, W, tile)) for i in range(40))


# --------------------------------------------------------------------------- two Gaussians


def test_two_gaussians_logistic_blend_and_gradients():
    H = W = 16
    p = np.array([[5.3, 10.9], [6.1, 9.7], [0.0, 0.0], [3.0, 2.2], [2.0, 4.1],
                  [0.9, 0.1], [0.2, 0.7]])
    g = np.random.default_rng(7).standard_normal((2, H, W))
    o = cref.render(p, H, W, K=10, grad_img=g)
    hh, ww = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    q1 = ((ww - p[0, 0]) / p[3, 0]) ** 2 + ((hh - p[1, 0]) / p[4, 0]) ** 2
    q2 = ((ww - p[0, 1]) / p[3, 1]) ** 2 + ((hh - p[1, 1]) / p[4, 1]) ** 2
    sig = 1.0 / (1.0 + np.exp(-(q2 - q1) / 2))            # weight of Gaussian 1
    for ch in range(2):
        c1, c2 = p[5 + ch, 0], p[5 + ch, 1]
        np.testing.assert_allclose(o["img"][ch], c2 + (c1 - c2) * sig, rtol=1e-13, atol=1e-15)
    gr = o["grad"]
    np.testing.assert_allclose(gr[5:, 0], (g * sig).sum(axis=(1, 2)), rtol=1e-12)
    np.testing.assert_allclose(gr[5:, 1], (g * (1 - sig)).sum(axis=(1, 2)), rtol=1e-12)
    # dc_r/dq1 = -1/2 (c1 - c2) sig (1 - sig); dq1/dmu_x1 = -2 (x - mu_x1) / s1^2
    dc = np.stack([p[5 + ch, 0] - p[5 + ch, 1] for ch in range(2)])[:, None, None]
    dcr_dq1 = -0.5 * dc * sig * (1 - sig)
    dmx1 = (g * dcr_dq1 * (-2.0 * (ww - p[0, 0]) / p[3, 0] ** 2)).sum()
    ds1 = (g * dcr_dq1 * (-2.0 * (ww - p[0, 0]) ** 2 / p[3, 0] ** 3)).sum()
    dmy2 = (g * (-dcr_dq1) * (-2.0 * (hh - p[1, 1]) / p[4, 1] ** 2)).sum()
    assert gr[0, 0] == pytest.approx(dmx1, rel=1e-11)
    assert gr[3, 0] == pytest.approx(ds1, rel=1e-11)
    assert gr[1, 1] == pytest.approx(dmy2, rel=1e-11)


# --------------------------------------------------------------------------- special cases of K


def test_K_at_least_members_is_normalized_eq4():
    """One 16x16 tile, every Gaussian hits it, K >= N: Eq. 5 is Eq. 4 normalized by sum G."""
    rng = np.random.default_rng(3)
    H = W = 16
    N, n = 12, 4
    p = make_params(rng, N, n, H, W, 2.0, 8.0)
    o = cref.render(p, H, W, K=16)
    hh, ww = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    X = np.stack([ww.ravel(), hh.ravel()], 1)
    G = np.empty((H * W, N))
    for i in range(N):
        c, s = math.cos(p[2, i]), math.sin(p[2, i])
        R = np.array([[c, -s], [s, c]])
        Sig = R @ np.diag([p[3, i] ** 2, p[4, i] ** 2]) @ R.T
        d = X - p[0:2, i]
        G[:, i] = np.exp(-0.5 * np.einsum("pi,ij,pj->p", d, np.linalg.inv(Sig), d))
    ref = (G @ p[5:].T) / G.sum(1, keepdims=True)
    np.testing.assert_allclose(o["img"].reshape(n, -1).T, ref, rtol=1e-11)


def test_K1_is_nearest_gaussian_partition():
    rng = np.random.default_rng(4)
    H, W, n = 48, 64, 2
    p = make_params(rng, 30, n, H, W, 2.0, 10.0)
    g = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, K=1, grad_img=g)
    d = dense.render(p, H, W, K=1)
    q = np.where(dense.membership(p, H, W), d["q"], np.inf)
    arg = np.argmin(q, axis=1).reshape(H, W)
    has = np.isfinite(q.min(axis=1)).reshape(H, W)
    assert np.array_equal(o["topk"][..., 0][has], arg[has])
    for ch in range(n):
        np.testing.assert_array_equal(o["img"][ch][has], p[5 + ch][arg[has]])
        cell = np.array([g[ch][has & (arg == i)].sum() for i in range(30)])
        np.testing.assert_allclose(o["grad"][5 + ch], cell, rtol=1e-12, atol=1e-12)
    assert np.all(o["grad"][:5] == 0)


def test_partition_of_unity():
    rng = np.random.default_rng(5)
    H, W, n = 64, 48, 3
    p = make_params(rng, 50, n, H, W)
    p[5:] = np.array([0.25, 0.5, 0.75])[:, None]
    g = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, K=10, grad_img=g)
    has = o["topk"][..., 0] >= 0
    for ch in range(n):
        np.testing.assert_allclose(o["img"][ch][has], p[5 + ch, 0], rtol=1e-14)
    scale = np.abs(g).sum()
    assert np.abs(o["grad"][:5]).max() < 1e-12 * scale


def test_empty_tiles_are_zero():
    p = np.array([[4.0], [4.0], [0.3], [1.0], [1.0], [0.7]])
    o = cref.render(p, 64, 64, K=3)
    assert np.all(o["img"][0, 16:, :] == 0) and np.all(o["img"][0, :, 16:] == 0)
    assert np.all(o["topk"][16:, :] == -1)


# --------------------------------------------------------------------------- invariants


def gap_mask(qsel, K, rel=1e-9):
    qk, qk1 = qsel[..., K - 1], qsel[..., K]
    return ~(np.isfinite(qk1) & (qk1 - qk <= rel * (1 + qk1)))


@pytest.mark.parametrize("kind", ["theta_plus_pi", "swap_axes", "permute"])
def test_invariants(kind):
    rng = np.random.default_rng(11)
    H, W, n, K = 48, 48, 3, 5
    N = 60
    p = make_params(rng, N, n, H, W)
    ref = cref.render(p, H, W, K)
    q = p.copy()
    perm = None
    if kind == "theta_plus_pi":
        q[2] += math.pi
    elif kind == "swap_axes":
        q[3], q[4] = p[4].copy(), p[3].copy()
        q[2] += math.pi / 2
    else:
        perm = rng.permutation(N)
        q = p[:, perm]
    o = cref.render(q, H, W, K)
    np.testing.assert_allclose(o["img"], ref["img"], rtol=1e-11, atol=1e-13)
    ok = gap_mask(ref["qsel"], K)
    tk = o["topk"] if perm is None else np.where(o["topk"] >= 0, perm[np.maximum(o["topk"], 0)], -1)
    assert np.array_equal(tk[ok], ref["topk"][ok])


# --------------------------------------------------------------------------- independent NumPy


@pytest.mark.parametrize("K", [1, 2, 3, 10, 64])
@pytest.mark.parametrize("shape", [(48, 48), (40, 56), (33, 17)])
def test_c_oracle_matches_numpy_dense(K, shape):
    H, W = shape
    rng = np.random.default_rng(K * 1000 + H)
    n = 3
    p = make_params(rng, 60, n, H, W, 1.5, 9.0)
    g = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, K, grad_img=g)
    d = dense.render(p, H, W, K, grad_img=g)
    ok = gap_mask(o["qsel"], K)
    assert ok.mean() > 0.99
    assert np.array_equal(o["topk"][ok], d["topk"][ok])
    np.testing.assert_allclose(o["img"][:, ok], d["img"][:, ok], rtol=1e-10, atol=1e-12)
    if ok.all():
        scale = np.abs(d["grad"]).max(axis=1, keepdims=True)
        np.testing.assert_allclose(o["grad"], d["grad"], rtol=1e-8, atol=1e-10 * scale.max())


def test_dense_mode_equals_tile_mode():
    rng = np.random.default_rng(21)
    H, W = 40, 72
    p = make_params(rng, 80, 2, H, W)
    np.testing.assert_array_equal(cref.render_dense(p, H, W, 10), cref.render(p, H, W, 10)["img"])


# --------------------------------------------------------------------------- finite differences


@pytest.mark.parametrize("seed", range(3))
def test_gradients_match_central_differences(seed):
    rng = np.random.default_rng(200 + seed)
    H, W, n, K, N = 32, 32, 2, 4, 14
    p = make_params(rng, N, n, H, W, 2.0, 9.0)
    r = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, K, grad_img=r)
    checked = 0
    for row in range(5 + n):
        for i in range(N):
            h = 1e-6 * max(1.0, abs(p[row, i]))
            pp, pm = p.copy(), p.copy()
            pp[row, i] += h
            pm[row, i] -= h
            op, om = cref.render(pp, H, W, K), cref.render(pm, H, W, K)
            # the selection is held fixed by the adjoint: skip steps that change S_j or S_j^K
            if not (np.array_equal(op["topk"], o["topk"]) and np.array_equal(om["topk"], o["topk"])):
                continue
            fd = ((r * op["img"]).sum() - (r * om["img"]).sum()) / (2 * h)
            assert o["grad"][row, i] == pytest.approx(fd, rel=2e-6, abs=1e-7), (row, i)
            checked += 1
    assert checked > 0.8 * (5 + n) * N


def test_grad_for_gaussians_matches_full_gradient():
    rng = np.random.default_rng(31)
    H, W, n, K = 64, 80, 3, 6
    p = make_params(rng, 120, n, H, W)
    g = rng.standard_normal((n, H, W))
    full = cref.render(p, H, W, K, grad_img=g)["grad"]
    ids = [0, 7, 55, 119]
    np.testing.assert_allclose(cref.grad_for_gaussians(p, H, W, K, g, ids), full[:, ids], rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------- fitting reference


def test_adam_first_step_moves_by_learning_rate():
    rng = np.random.default_rng(1)
    n = 3
    H, W = 64, 32
    fp = np.abs(rng.standard_normal((5 + n, 10))) * 0.1 + 0.5
    fp[2] = 1.0
    g = rng.standard_normal((5 + n, 10))
    lrs = fitref.row_lrs(n)
    newp, m, v = fitref.adam_step(fp, g, np.zeros_like(g), np.zeros_like(g), 1, lrs, H=H, W=W)
    # bias-corrected first step: m_hat / sqrt(v_hat) = sign(g)
    np.testing.assert_allclose(newp, fp - lrs[:, None] * np.sign(g), rtol=1e-6)


def _adam_vs_torch(step_fn, steps=6, seed=3):
    """Largest difference between ``step_fn`` (the oracle's Adam signature) and torch.optim.Adam
    followed by the fitter's clamps (theta to [0, pi], Sec. 3.1; 1/s to [1/max(H, W), 4]) over
    ``steps`` steps with per-row learning rates (Sec. 4.1) and gradients that change sign and
    size every step.  Parameters start next to every bound with gradients that push across it."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(seed)
    n, N, H, W = 3, 12, 40, 64
    p = rng.uniform(0.2, 0.8, (5 + n, N))
    p[2] = rng.uniform(0.5, 2.5, N)
    p[3:5] = rng.uniform(0.1, 3.0, (2, N))
    # theta at 0 and pi, 1/s at 4 and at 1/max(H, W), each pushed outward by the first gradients
    p[2, 0], p[2, 1] = 1e-4, math.pi - 1e-4
    p[3, 2], p[4, 3] = 4.0 - 1e-4, 1.0 / W + 1e-5
    lrs = fitref.row_lrs(n)
    grads = rng.standard_normal((steps, 5 + n, N)) * rng.uniform(0.1, 10.0, (steps, 5 + n, 1))
    grads[:, 2, 0], grads[:, 2, 1] = 1.0, -1.0
    grads[:, 3, 2], grads[:, 4, 3] = -1.0, 1.0
    rows = [torch.tensor(p[r], dtype=torch.float64, requires_grad=True) for r in range(5 + n)]
    opt = torch.optim.Adam([{"params": [rows[r]], "lr": float(lrs[r])} for r in range(5 + n)])
    q, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    worst = 0.0
    for t in range(steps):
        for r in range(5 + n):
            rows[r].grad = torch.tensor(grads[t, r], dtype=torch.float64)
        opt.step()
        with torch.no_grad():
            rows[2].clamp_(0.0, math.pi)
            rows[3].clamp_(1.0 / max(H, W), 4.0)
            rows[4].clamp_(1.0 / max(H, W), 4.0)
        q, m, v = step_fn(q, grads[t], m, v, t + 1, lrs, H=H, W=W)
        ref = np.stack([x.detach().numpy() for x in rows])
        worst = max(worst, float(np.abs(q - ref).max()))
    return worst, q


def test_adam_matches_torch_adam_with_clamps_over_several_steps():
    """The Adam reference (Sec. 4.1; beta1, beta2, eps as PyTorch's defaults) against PyTorch's own
    optimizer over six steps, with the clamps of Sec. 3.1 reached in both directions."""
    worst, q = _adam_vs_torch(fitref.adam_step)
    assert worst < 1e-13, worst
    assert q[2, 0] == 0.0 and q[2, 1] == math.pi
    assert q[3, 2] == 4.0 and q[4, 3] == 1.0 / 64


def test_adam_pin_catches_planted_mistakes():
    """The torch comparison above fails for swapped betas, a missing clamp, a missing bias
    correction and a wrong eps, each planted in the oracle's Adam."""
    import functools
    from unittest import mock

    swapped = functools.partial(fitref.adam_step, b1=0.999, b2=0.9)
    assert _adam_vs_torch(swapped)[0] > 1e-6
    with mock.patch.object(fitref.np, "clip", lambda x, lo, hi: x):
        assert _adam_vs_torch(fitref.adam_step)[0] > 1e-6

    def no_bias_correction(p, g, m, v, step, lrs, **kw):
        return fitref.adam_step(p, g, m, v, 10 ** 6, lrs, **kw)
    assert _adam_vs_torch(no_bias_correction)[0] > 1e-6

    assert _adam_vs_torch(functools.partial(fitref.adam_step, eps=1e-4))[0] > 1e-6


def test_paper_constants_fix_parameter_count():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    H, W, n = c["restoration_budget"]["image"]
    bits = c["param_bits"]["value"]
    # 10K Gaussians of 5+n float16 parameters: 160 KB, 78.64x, 0.305 bpp (Sec. 4.2, Sec. 5.2)
    N = 10000
    nbytes = N * (5 + n) * bits // 8
    assert nbytes == c["restoration_budget"]["model_bytes"]
    assert round(H * W * 3 / nbytes, 2) == c["restoration_budget"]["compression_ratio"]
    assert round(nbytes * 8 / (H * W), 3) == c["lod_bpp"]["bpp_max"]
    lr = c["learning_rates"]
    assert list(fitref.row_lrs(1)) == [lr["mu"], lr["mu"], lr["theta"], lr["s"], lr["s"], lr["c"]]
    assert c["top_k"]["value"] == 10 and c["tile_size"]["value"] == 16


def test_reparam_chain_rule_matches_finite_differences():
    rng = np.random.default_rng(9)
    H, W, n = 40, 56, 2
    rp = make_params(rng, 10, n, H, W, 2.0, 7.0)
    fp = fitref.to_fit_space(rp, H, W)
    r = rng.standard_normal((n, H, W))
    g_render = cref.render(rp, H, W, 4, grad_img=r)["grad"]
    g_fit = fitref.grad_to_fit_space(g_render, fp, H, W)
    base = cref.render(rp, H, W, 4)["topk"]
    for row in (0, 1, 3, 4):
        for i in range(0, 10, 3):
            h = 1e-7 * max(1.0, abs(fp[row, i]))
            a, b = fp.copy(), fp.copy()
            a[row, i] += h
            b[row, i] -= h
            oa = cref.render(fitref.to_render_space(a, H, W), H, W, 4)
            ob = cref.render(fitref.to_render_space(b, H, W), H, W, 4)
            if not (np.array_equal(oa["topk"], base) and np.array_equal(ob["topk"], base)):
                continue
            fd = ((r * oa["img"]).sum() - (r * ob["img"]).sum()) / (2 * h)
            assert g_fit[row, i] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_l1_gradient_and_psnr():
    img = np.array([[[0.5, 0.2], [0.1, 0.9]]])
    tgt = np.array([[[0.4, 0.2], [0.3, 0.9]]])
    loss, g = fitref.l1_loss_grad(img, tgt)
    assert loss == pytest.approx((0.1 + 0.2) / 4)
    np.testing.assert_array_equal(g, np.array([[[0.25, 0.0], [-0.25, 0.0]]]))
    assert fitref.psnr(img, tgt) == pytest.approx(10 * math.log10(1 / ((0.01 + 0.04) / 4)))


def test_exact_ties_keep_lower_index():
    """Duplicated geometry gives exactly equal q; the lower Gaussian index ranks first."""
    H = W = 16
    geo = [7.3, 8.6, 0.4, 3.0, 2.0]
    cols = [0.1, 0.4, 0.9]
    p = np.array([[geo[r] for _ in cols] for r in range(5)] + [cols])
    p = p[:, [2, 0, 1]]            # indices 0, 1, 2 carry colours 0.9, 0.1, 0.4
    o = cref.render(p, H, W, K=1)
    assert np.all(o["topk"][..., 0] == 0)
    assert np.all(o["img"][0] == 0.9)
    o = cref.render(p, H, W, K=2)
    assert np.all(o["topk"] == np.array([0, 1]))
    np.testing.assert_allclose(o["img"][0], 0.5, rtol=1e-15)


def test_gradient_conditioning_bounds_the_gradient():
    """grad_abs sums the terms' magnitudes: it bounds |grad| and equals it for colour rows when
    the upstream gradient is non-negative."""
    rng = np.random.default_rng(41)
    H, W, n = 48, 40, 2
    p = make_params(rng, 50, n, H, W)
    g = rng.standard_normal((n, H, W))
    o = cref.render(p, H, W, 6, grad_img=g)
    assert np.all(o["grad_abs"] >= np.abs(o["grad"]) * (1 - 1e-12))
    o = cref.render(p, H, W, 6, grad_img=np.abs(g))
    np.testing.assert_allclose(o["grad_abs"][5:], o["grad"][5:], rtol=1e-12)


# --------------------------------------------------------------------------- near-tie margin


def test_margin_without_rounding_is_the_selection_gap():
    """gamma = 0: the margin is q_(K+1) - q_(K), the gap the ranking has to decide (Sec. 3.2)."""
    rng = np.random.default_rng(41)
    H, W, n, K = 48, 40, 3, 6
    p = make_params(rng, 150, n, H, W)
    o = cref.render(p, H, W, K, gamma=0.0)
    gap = o["qsel"][..., K] - o["qsel"][..., K - 1]
    full = np.isfinite(o["qsel"][..., K])
    np.testing.assert_array_equal(o["margin"][full], gap[full])
    assert np.all(np.isinf(o["margin"][~full]))


def test_rank_scale_is_q_for_axis_aligned_gaussians():
    """For theta = 0 nothing cancels in e = R^T d / s, so the rounding scale M equals q; at
    theta = pi/4 on the diagonal through the mean, e1 = sqrt(2)|d| and e2 = 0 while
    M = 2 dx^2 (1/s1^2 + 1/s2^2)."""
    H, W = 32, 32
    p = np.array([[15.3], [16.8], [0.0], [3.0], [5.0], [0.2], [0.4], [0.6]])
    idx, q, mb = cref.rank_pixel(p, H, W, 20, 9)
    assert idx.tolist() == [0]
    assert mb[0] == pytest.approx(q[0], rel=1e-15)
    p2 = np.array([[16.5], [16.5], [math.pi / 4], [3.0], [5.0], [0.2], [0.4], [0.6]])
    idx, q, mb = cref.rank_pixel(p2, H, W, 20, 20)
    dx = 20.5 - 16.5
    assert q[0] == pytest.approx(2 * dx * dx / 9.0, rel=1e-14)
    assert mb[0] == pytest.approx(2 * dx * dx * (1 / 9.0 + 1 / 25.0), rel=1e-14)


def test_rank_pixel_and_blend_set_reproduce_the_render():
    """The pixel ranking lists S_j in the render's order (its first K are the render's top-K with
    the same q) and the blend over that set is the rendered colour; one Gaussian blends to its
    colour, two to the logistic form of Eq. 5."""
    rng = np.random.default_rng(42)
    H, W, n, K = 40, 56, 3, 5
    p = make_params(rng, 120, n, H, W)
    o = cref.render(p, H, W, K)
    counts, lists = cref.tile_lists(p, H, W)
    for h, w in [(0, 0), (17, 33), (39, 55), (25, 4)]:
        idx, q, mb = cref.rank_pixel(p, H, W, h, w)
        t = (h // 16) * ((W + 15) // 16) + w // 16
        assert sorted(idx.tolist()) == lists[counts[:t].sum():counts[:t + 1].sum()].tolist()
        k = min(K, len(idx))
        assert idx[:k].tolist() == o["topk"][h, w, :k].tolist()
        np.testing.assert_allclose(q[: k + 1], o["qsel"][h, w, : k + 1][np.isfinite(o["qsel"][h, w, : k + 1])], rtol=1e-15)
        assert np.all(mb >= q * (1 - 1e-15))
        np.testing.assert_allclose(cref.blend_set(p, h, w, idx[:k]), o["img"][:, h, w], rtol=1e-13)
        assert np.array_equal(cref.blend_set(p, h, w, idx[:1]), p[5:, idx[0]])
        a, b = idx[0], idx[1]
        sig = 1.0 / (1.0 + math.exp(-(q[1] - q[0]) / 2))
        np.testing.assert_allclose(cref.blend_set(p, h, w, [a, b]),
                                   p[5:, b] + (p[5:, a] - p[5:, b]) * sig, rtol=1e-13)


def test_positive_margin_means_perturbations_keep_the_set():
    """Brute force: moving every candidate's q by up to gamma M (random signs and sizes, and the
    worst case) never changes the retained set where the margin is positive, and the worst case
    does change it where the margin is negative."""
    rng = np.random.default_rng(43)
    H, W, n, K = 32, 32, 3, 4
    p = make_params(rng, 90, n, H, W)
    gam = 1e-2                                  # large, so that both cases occur
    o = cref.render(p, H, W, K, gamma=gam)
    seen_pos = seen_neg = 0
    for h in range(0, H, 3):
        for w in range(0, W, 3):
            idx, q, mb = cref.rank_pixel(p, H, W, h, w)
            if len(idx) <= K:
                assert np.isinf(o["margin"][h, w])
                continue
            base = set(idx[:K].tolist())
            worst = q.copy()
            worst[:K] += gam * mb[:K]
            worst[K:] -= gam * mb[K:]
            worst_set = set(idx[np.lexsort((idx, worst))[:K]].tolist())
            if o["margin"][h, w] > 0:
                seen_pos += 1
                for _ in range(5):
                    pert = q + gam * mb * rng.uniform(-1, 1, len(q))
                    assert set(idx[np.lexsort((idx, pert))[:K]].tolist()) == base
                assert worst_set == base
            elif o["margin"][h, w] < 0:
                seen_neg += 1
                assert worst_set != base
    assert seen_pos > 10 and seen_neg > 3, (seen_pos, seen_neg)
