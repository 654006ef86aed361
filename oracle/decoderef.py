"""NumPy FP64 reference for the decoding side of the representation.  Test infrastructure only:
the tests, the smoke check and the benchmark's CPU baseline may use it, nothing on the product
path.

* Random access (Sec. 1, Sec. 3.2): the colour at an arbitrary point (x, y) of the image plane
  [0, W) x [0, H) is Eq. 5 evaluated at that point: the point belongs to tile
  (floor(x / 16), floor(y / 16)); S_j is every Gaussian whose 3-sigma enclosing circle meets that
  tile's closed rectangle (clipped to the image); its members are ranked by q at the point (then
  by index) and the top K blended.  Points outside the image have colour 0.  At a pixel centre
  this is the rendered pixel.
* Storage (Sec. 4.1): the trained attributes, i.e. the fitter's parameters (mean normalized to
  [0,1]^2, rotation, inverse scales, colour), rounded to IEEE float16 (nearest, ties to even),
  and decoded back into the renderer's units (mean times (W, H), scale = 1 / inverse scale) in
  float32 arithmetic.  A prefix of the stored set (its first N' Gaussians) is a level of detail.
"""
from __future__ import annotations

import numpy as np


def _tile_members(p, H, W, tx, ty, tile=16):
    """Members of S_j for tile (tx, ty): the circle of radius 3 max(s1, s2) about the mean meets
    the closed rectangle [x0, x1] x [y0, y1] clipped to the image (tangency counts)."""
    x0, y0 = float(tx * tile), float(ty * tile)
    x1, y1 = float(min(x0 + tile, W)), float(min(y0 + tile, H))
    mx, my = p[0], p[1]
    dx = mx - np.clip(mx, x0, x1)
    dy = my - np.clip(my, y0, y1)
    r = 3.0 * np.maximum(p[3], p[4])
    return np.nonzero(dx * dx + dy * dy <= r * r)[0]


def evaluate_points(params, H, W, K, points, tile=16):
    """Colours [n][M] of the representation at points [2][M] (x row, y row), in FP64."""
    p = np.asarray(params, np.float64)
    n = p.shape[0] - 5
    pts = np.asarray(points, np.float64)
    M = pts.shape[1]
    out = np.zeros((n, M))
    tiles_x, tiles_y = (W + tile - 1) // tile, (H + tile - 1) // tile
    cache = {}
    for i in range(M):
        x, y = pts[0, i], pts[1, i]
        if not (0.0 <= x < W and 0.0 <= y < H):
            continue
        tx = min(int(np.floor(x / tile)), tiles_x - 1)
        ty = min(int(np.floor(y / tile)), tiles_y - 1)
        if (tx, ty) not in cache:
            cache[(tx, ty)] = _tile_members(p, H, W, tx, ty, tile)
        mem = cache[(tx, ty)]
        if mem.size == 0:
            continue
        dx, dy = x - p[0, mem], y - p[1, mem]
        c, s = np.cos(p[2, mem]), np.sin(p[2, mem])
        e1 = c * dx + s * dy
        e2 = -s * dx + c * dy
        q = e1 * e1 / (p[3, mem] ** 2) + e2 * e2 / (p[4, mem] ** 2)     # Eq. 1 exponent x -2
        order = np.lexsort((mem, q))[:K]                               # by q, then by index
        w = np.exp(-0.5 * (q[order] - q[order[0]]))                     # Eq. 5, shifted
        out[:, i] = (p[5:, mem[order]] * w).sum(axis=1) / w.sum()
    return out


def near_tie_points(params, H, W, K, points, tile=16, rel=1e-5):
    """Points whose K-th and (K+1)-th ranked q are closer than rel * (1 + q_(K+1)): there an
    float32 ranking may keep either candidate."""
    p = np.asarray(params, np.float64)
    pts = np.asarray(points, np.float64)
    tiles_x, tiles_y = (W + tile - 1) // tile, (H + tile - 1) // tile
    out = np.zeros(pts.shape[1], bool)
    for i in range(pts.shape[1]):
        x, y = pts[0, i], pts[1, i]
        if not (0.0 <= x < W and 0.0 <= y < H):
            continue
        tx = min(int(np.floor(x / tile)), tiles_x - 1)
        ty = min(int(np.floor(y / tile)), tiles_y - 1)
        mem = _tile_members(p, H, W, tx, ty, tile)
        if mem.size <= K:
            continue
        dx, dy = x - p[0, mem], y - p[1, mem]
        c, s = np.cos(p[2, mem]), np.sin(p[2, mem])
        q = np.sort((c * dx + s * dy) ** 2 / p[3, mem] ** 2 +
                    (-s * dx + c * dy) ** 2 / p[4, mem] ** 2)
        out[i] = q[K] - q[K - 1] <= rel * (1.0 + q[K])
    return out


def to_fp16(fit_params):
    """IEEE float16 bit patterns (uint16) of the fitter's parameters, nearest, ties to even."""
    return np.asarray(fit_params, np.float32).astype(np.float16).view(np.uint16)


def decode_fp16(stored, H, W, n_prefix=None):
    """float32 renderer parameters [5+n][n_prefix] of the first n_prefix stored Gaussians."""
    f = np.asarray(stored, np.uint16).view(np.float16).astype(np.float32)
    if n_prefix is not None:
        f = f[:, :n_prefix]
    out = f.copy()
    out[0] = f[0] * np.float32(W)
    out[1] = f[1] * np.float32(H)
    out[3] = np.float32(1.0) / f[3]
    out[4] = np.float32(1.0) / f[4]
    return out
