"""ctypes wrapper of the C oracle (oracle.c).  Test infrastructure only.

All entry points take the parameter set as float64 [5+n][N] (float32 inputs are promoted
exactly) and return NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from . import build as _build

_lib = None
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp = ctypes.c_void_p
        ci = ctypes.c_int
        L.orc_num_tiles.argtypes = [ci, ci, ci, ci]
        L.orc_num_tiles.restype = ci
        L.orc_tile_lists.argtypes = [_f64p, ci, ci, ci, ci, ci, ci, _i32p, ci, _i64p, vp, ctypes.c_int64]
        L.orc_tile_lists.restype = ci
        L.orc_render_tiles.argtypes = [_f64p, ci, ci, ci, ci, ci, ci, ci, _i32p, ci, vp, vp, vp, vp,
                                       vp, vp, ci, ctypes.c_double, vp]
        L.orc_render_tiles.restype = ci
        L.orc_rank_pixel.argtypes = [_f64p, ci, ci, ci, ci, ci, ci, ci, ci, vp, vp, vp, ci]
        L.orc_rank_pixel.restype = ci
        L.orc_blend_set.argtypes = [_f64p, ci, ci, ci, ci, _i32p, ci, _f64p]
        L.orc_blend_set.restype = ci
        L.orc_render_dense.argtypes = [_f64p, ci, ci, ci, ci, ci, ci, ci, vp, ci]
        L.orc_render_dense.restype = ci
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ci
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(params: np.ndarray) -> Tuple[np.ndarray, int, int]:
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.ndim != 2 or p.shape[0] < 6:
        raise ValueError("params must be [5+n][N]")
    return p, p.shape[1], p.shape[0] - 5


def num_tiles(H: int, W: int, tile: int = 16) -> int:
    return (H + tile - 1) // tile * ((W + tile - 1) // tile)


def max_threads() -> int:
    return lib().orc_max_threads()


def tile_lists(params, H, W, tile=16, tiles: Optional[Sequence[int]] = None):
    """S_j for the listed tiles (all tiles by default): returns (counts[int64], members[int32])."""
    p, N, n = _prep(params)
    T = num_tiles(H, W, tile)
    t = np.arange(T, dtype=np.int32) if tiles is None else np.ascontiguousarray(tiles, dtype=np.int32)
    counts = np.zeros(len(t), dtype=np.int64)
    rc = lib().orc_tile_lists(p, N, n, H, W, tile, tile, t, len(t), counts, None, 0)
    if rc != 0:
        raise RuntimeError(f"orc_tile_lists failed: {rc}")
    lists = np.zeros(max(1, int(counts.sum())), dtype=np.int32)
    rc = lib().orc_tile_lists(p, N, n, H, W, tile, tile, t, len(t), counts, _ptr(lists), lists.size)
    if rc != 0:
        raise RuntimeError(f"orc_tile_lists failed: {rc}")
    return counts, lists[: int(counts.sum())]


# Unit roundoff of float32, and the multiple of it times M (orc's rank_scale) that bounds the error
# of q = |e|^2 evaluated in float32 from float32 rotation-scale rows and offsets: each component
# e_a carries at most ~4 roundings of its two products' magnitudes (the two inputs, the product,
# the sum), squaring doubles that to ~8 of M, and the final square and sum add 2 more; 16 leaves
# room for second-order terms.
U32 = 2.0 ** -24
TIE_GAMMA = 16.0 * U32


def render_tiles(params, H, W, K, tile=16, tiles=None, grad_img=None, want=("img", "topk", "qsel"),
                 nthreads=0, gamma=TIE_GAMMA):
    """Render the listed tiles; returns dict with compact per-tile arrays and, when ``grad_img``
    ([n][H][W]) is given, ``grad`` [5+n][N] holding the listed tiles' contributions and
    ``grad_abs`` [5+n][N], the sums of the terms' magnitudes before cancellation.  With "margin"
    in ``want``: per pixel, how far the retained set is from changing when every q is perturbed
    by up to gamma M (non-positive: a near tie, where several selections are correct)."""
    p, N, n = _prep(params)
    T = num_tiles(H, W, tile)
    t = np.arange(T, dtype=np.int32) if tiles is None else np.ascontiguousarray(tiles, dtype=np.int32)
    tp = tile * tile
    out = {}
    img = np.zeros((len(t), n, tp)) if "img" in want else None
    topk = np.zeros((len(t), tp, K), dtype=np.int32) if "topk" in want else None
    qsel = np.zeros((len(t), tp, K + 1)) if "qsel" in want else None
    margin = np.zeros((len(t), tp)) if "margin" in want else None
    g = None
    grad = gabs = None
    if grad_img is not None:
        g = np.ascontiguousarray(grad_img, dtype=np.float64)
        if g.shape != (n, H, W):
            raise ValueError("grad_img must be [n][H][W]")
        grad = np.zeros((5 + n, N))
        gabs = np.zeros((5 + n, N))
    rc = lib().orc_render_tiles(p, N, n, H, W, K, tile, tile, t, len(t), _ptr(img), _ptr(topk),
                                _ptr(qsel), _ptr(g), _ptr(grad), _ptr(gabs), nthreads, gamma,
                                _ptr(margin))
    if rc != 0:
        raise RuntimeError(f"orc_render_tiles failed: {rc}")
    out["tiles"] = t
    if img is not None:
        out["img"] = img
    if topk is not None:
        out["topk"] = topk
    if qsel is not None:
        out["qsel"] = qsel
    if margin is not None:
        out["margin"] = margin
    if grad is not None:
        out["grad"] = grad
        out["grad_abs"] = gabs
    return out


def _tiles_to_planar(arr: np.ndarray, tiles: np.ndarray, H: int, W: int, tile: int, fill=0.0):
    """[ntiles][C][tile*tile] -> [C][H][W] (tiles not listed keep ``fill``)."""
    C = arr.shape[1]
    tx_n = (W + tile - 1) // tile
    out = np.full((C, H, W), fill, dtype=arr.dtype)
    for a, t in enumerate(tiles):
        tx, ty = t % tx_n, t // tx_n
        x0, y0 = tx * tile, ty * tile
        x1, y1 = min(x0 + tile, W), min(y0 + tile, H)
        blk = arr[a].reshape(C, tile, tile)
        out[:, y0:y1, x0:x1] = blk[:, : y1 - y0, : x1 - x0]
    return out


def render(params, H, W, K, tile=16, grad_img=None, nthreads=0, gamma=TIE_GAMMA):
    """Full-image oracle: image [n][H][W], topk [H][W][K] (Gaussian ids, -1 unused),
    qsel [H][W][K+1], margin [H][W] (see render_tiles) and, with ``grad_img``, the full gradient
    [5+n][N]."""
    r = render_tiles(params, H, W, K, tile, None, grad_img, want=("img", "topk", "qsel", "margin"),
                     nthreads=nthreads, gamma=gamma)
    t = r["tiles"]
    out = {
        "img": _tiles_to_planar(r["img"], t, H, W, tile),
        "topk": np.moveaxis(_tiles_to_planar(np.moveaxis(r["topk"], 2, 1), t, H, W, tile, -1), 0, 2),
        "qsel": np.moveaxis(_tiles_to_planar(np.moveaxis(r["qsel"], 2, 1), t, H, W, tile, np.inf), 0, 2),
        "margin": _tiles_to_planar(r["margin"][:, None, :], t, H, W, tile, np.inf)[0],
    }
    if "grad" in r:
        out["grad"] = r["grad"]
        out["grad_abs"] = r["grad_abs"]
    return out


def rank_pixel(params, H, W, h, w, tile=16):
    """Every member of the hit set of pixel (h, w)'s tile ranked there by (q, index):
    (idx int32, q, M) in rank order (M: the rounding scale of q, see render_tiles)."""
    p, N, n = _prep(params)
    m = lib().orc_rank_pixel(p, N, n, H, W, tile, tile, h, w, None, None, None, 0)
    if m < 0:
        raise RuntimeError(f"orc_rank_pixel failed: {m}")
    idx = np.zeros(max(m, 1), dtype=np.int32)
    q = np.zeros(max(m, 1))
    mb = np.zeros(max(m, 1))
    lib().orc_rank_pixel(p, N, n, H, W, tile, tile, h, w, _ptr(idx), _ptr(q), _ptr(mb), m)
    return idx[:m], q[:m], mb[:m]


def blend_set(params, h, w, ids) -> np.ndarray:
    """Eq. 5 over the given Gaussians at the centre of pixel (h, w): colour [n]."""
    p, N, n = _prep(params)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    out = np.zeros(n)
    rc = lib().orc_blend_set(p, N, n, h, w, ids, len(ids), out)
    if rc != 0:
        raise RuntimeError(f"orc_blend_set failed: {rc}")
    return out


def render_dense(params, H, W, K, tile=16, nthreads=0) -> np.ndarray:
    p, N, n = _prep(params)
    img = np.zeros((n, H, W))
    rc = lib().orc_render_dense(p, N, n, H, W, K, tile, tile, _ptr(img), nthreads)
    if rc != 0:
        raise RuntimeError(f"orc_render_dense failed: {rc}")
    return img


def grad_for_gaussians(params, H, W, K, grad_img, gids: Sequence[int], tile=16, nthreads=0,
                       with_abs=False):
    """Exact gradient rows for the Gaussians ``gids`` ([5+n][len(gids)]): renders every tile whose
    S_j contains one of them, which holds every pixel that can select them.  With ``with_abs``
    also returns the matching ``grad_abs`` rows."""
    p, N, n = _prep(params)
    gids = np.asarray(gids, dtype=np.int64)
    sub = p[:, gids]
    counts, _ = tile_lists(sub, H, W, tile)
    tiles = np.nonzero(counts > 0)[0].astype(np.int32)
    r = render_tiles(p, H, W, K, tile, tiles, grad_img, want=(), nthreads=nthreads)
    if with_abs:
        return r["grad"][:, gids], r["grad_abs"][:, gids]
    return r["grad"][:, gids]
