"""Seeded synthetic inputs for the Image-GS renderer (images and Gaussian parameter sets).

This module only draws random inputs; it contains none of the renderer's arithmetic, so both the
HIP path and the FP64 oracle can be fed from it without sharing any of the method's code.

The paper evaluates on 2K x 2K RGB images and 9-channel texture stacks (Sec. 4.1, "Dataset") that
are not available here.  These generators stand in for them with images of the same sizes and
channel counts: smooth sinusoidal gradients (low-frequency content), axis-aligned rectangles
(sharp edges, the non-uniform feature distribution the method targets) and mild Gaussian noise.
Gaussian parameters follow the layout of Eq. 3 (mean, angle, two scales, n-channel colour).

Every generator is driven by ``numpy.random.default_rng(seed)`` (PCG64), computed in float64 and
returned as float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

N_SINUSOIDS = 8


def gen_image(seed: int, H: int, W: int, C: int = 3, n_rect: int = 20) -> np.ndarray:
    """Planar float32 image [C][H][W] with values in [0, 1].

    Base value 0.5, plus 8 plane-wave sinusoids a*sin(2*pi*f*(u*cos(phi) + v*sin(phi)) + psi) with
    u = (w + 1/2)/W, v = (h + 1/2)/H, f ~ U[0.5, 3] cycles per image, phi ~ U[0, 2 pi) and, per
    channel, a ~ U[0, 1/16], psi ~ U[0, 2 pi); plus ``n_rect`` axis-aligned rectangles (uniform
    corner, side lengths log-uniform in [0.02, 0.3] of the image side, additive per-channel offset
    ~ U[-0.3, 0.3]); plus N(0, 0.02^2) noise; clamped to [0, 1].
    """
    rng = np.random.default_rng(seed)
    img = np.full((C, H, W), 0.5, dtype=np.float64)
    u = (np.arange(W, dtype=np.float64) + 0.5) / W
    v = (np.arange(H, dtype=np.float64) + 0.5) / H
    for _ in range(N_SINUSOIDS):
        f = rng.uniform(0.5, 3.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        amp = rng.uniform(0.0, 1.0 / 16.0, size=C)
        psi = rng.uniform(0.0, 2.0 * math.pi, size=C)
        au = 2.0 * math.pi * f * math.cos(phi) * u          # [W]
        bv = 2.0 * math.pi * f * math.sin(phi) * v          # [H]
        for ch in range(C):
            # sin(a + b + psi) = sin(a + psi) cos(b) + cos(a + psi) sin(b): two outer products
            sa, ca = np.sin(au + psi[ch]), np.cos(au + psi[ch])
            img[ch] += amp[ch] * (np.outer(np.cos(bv), sa) + np.outer(np.sin(bv), ca))
    lo, hi = math.log(0.02), math.log(0.3)
    for _ in range(n_rect):
        x0 = rng.uniform(0.0, W)
        y0 = rng.uniform(0.0, H)
        rw = math.exp(rng.uniform(lo, hi)) * W
        rh = math.exp(rng.uniform(lo, hi)) * H
        off = rng.uniform(-0.3, 0.3, size=C)
        xa, xb = int(math.floor(x0)), min(W, int(math.ceil(x0 + rw)))
        ya, yb = int(math.floor(y0)), min(H, int(math.ceil(y0 + rh)))
        img[:, ya:yb, xa:xb] += off[:, None, None]
    img += rng.normal(0.0, 0.02, size=img.shape)
    np.clip(img, 0.0, 1.0, out=img)
    return img.astype(np.float32)


def gen_texture_stack(seed: int, H: int, W: int, n_maps: int = 3, n_rect: int = 200) -> np.ndarray:
    """n_maps independent 3-channel maps (seeds seed, seed+1, ...) concatenated: [3*n_maps][H][W]."""
    return np.concatenate([gen_image(seed + k, H, W, 3, n_rect) for k in range(n_maps)], axis=0)


def gen_gaussians(seed: int, H: int, W: int, N: int, n: int,
                  smin: float = 1.0, smax: float = 12.0) -> np.ndarray:
    """Gaussian parameters, float32 structure-of-arrays [5+n][N] in pixel units.

    Rows: mu_x ~ U[0, W), mu_y ~ U[0, H), theta ~ U[0, pi), s_1, s_2 independently log-uniform in
    [smin, smax] pixels, then n colour rows ~ U[0, 1].
    """
    rng = np.random.default_rng(seed)
    p = np.empty((5 + n, N), dtype=np.float64)
    p[0] = rng.uniform(0.0, W, size=N)
    p[1] = rng.uniform(0.0, H, size=N)
    p[2] = rng.uniform(0.0, math.pi, size=N)
    p[3] = np.exp(rng.uniform(math.log(smin), math.log(smax), size=N))
    p[4] = np.exp(rng.uniform(math.log(smin), math.log(smax), size=N))
    p[5:] = rng.uniform(0.0, 1.0, size=(n, N))
    out = p.astype(np.float32)
    # float32 rounding may push a draw onto the open upper bound; keep the half-open ranges
    out[0] = np.minimum(out[0], np.nextafter(np.float32(W), np.float32(0)))
    out[1] = np.minimum(out[1], np.nextafter(np.float32(H), np.float32(0)))
    out[2] = np.minimum(out[2], np.nextafter(np.float32(math.pi), np.float32(0)))
    return out


def gen_fitted_like(seed: int, H: int, W: int, N: int, n: int) -> np.ndarray:
    """A parameter set with the spread of a texture fit a few dozen Adam iterations in, float32
    [5+n][N] in pixel units.  Fitting stretches some Gaussians across large parts of the image,
    makes many strongly anisotropic, pushes colours outside [0, 1], means a little past the border
    and angles onto the clamp values 0 and pi; this draws such a set directly:

    * the base set as ``gen_gaussians`` (scales 1-12 px);
    * 2.5% elongated: the long scale log-uniform in [20, 80] px, the short one in [1, 20] px;
    * 30 large: the long scale log-uniform in [100, 600] px, the short one in [10, 80] px,
      and one of them isotropic at max(H, W) px with its mean inside the image (it covers every
      tile);
    * a cluster of 600 Gaussians of 1-6 px with means in a 48 x 48 px square, so that a few tiles
      hold several hundred candidates;
    * 5% of the colours redrawn from U[-0.35, 1.35]; 5% of the angles set to exactly 0 or pi;
      1% of the means redrawn from U[-25, W + 25] x U[-25, H + 25].
    """
    rng = np.random.default_rng(seed)
    p = gen_gaussians(seed + 1, H, W, N, n).astype(np.float64)
    big = float(max(H, W))
    idx = rng.permutation(N)
    n_el = int(round(0.025 * N))
    n_lg = min(30, max(0, N - n_el))
    n_cl = min(600, max(0, N - n_el - n_lg))
    el, lg, cl = idx[:n_el], idx[n_el:n_el + n_lg], idx[n_el + n_lg:n_el + n_lg + n_cl]

    def logu(a, b, size):
        return np.exp(rng.uniform(math.log(a), math.log(b), size=size))

    for sel, (la, lb), (sa, sb) in ((el, (20.0, 80.0), (1.0, 20.0)),
                                    (lg, (100.0, 600.0), (10.0, 80.0))):
        long_ = logu(la, max(lb, la), len(sel))
        short = logu(sa, sb, len(sel))
        first = rng.random(len(sel)) < 0.5
        p[3, sel] = np.where(first, long_, short)
        p[4, sel] = np.where(first, short, long_)
    if n_lg >= 1:
        p[3, lg[0]] = big
        p[4, lg[0]] = big
        p[0, lg[0]] = rng.uniform(0.25 * W, 0.75 * W)
        p[1, lg[0]] = rng.uniform(0.25 * H, 0.75 * H)
    if n_cl:
        cx = rng.uniform(0.0, max(W - 48.0, 0.0))
        cy = rng.uniform(0.0, max(H - 48.0, 0.0))
        p[0, cl] = cx + rng.uniform(0.0, min(48.0, W), size=n_cl)
        p[1, cl] = cy + rng.uniform(0.0, min(48.0, H), size=n_cl)
        p[3, cl] = logu(1.0, 6.0, n_cl)
        p[4, cl] = logu(1.0, 6.0, n_cl)
    col = rng.random((n, N)) < 0.05
    p[5:][col] = rng.uniform(-0.35, 1.35, size=int(col.sum()))
    ang = rng.random(N) < 0.05
    p[2, ang] = np.where(rng.random(int(ang.sum())) < 0.5, 0.0, math.pi)
    mu = rng.random(N) < 0.01
    p[0, mu] = rng.uniform(-25.0, W + 25.0, size=int(mu.sum()))
    p[1, mu] = rng.uniform(-25.0, H + 25.0, size=int(mu.sum()))
    return p.astype(np.float32)


def gen_grad_image(seed: int, n: int, H: int, W: int) -> np.ndarray:
    """A seeded upstream gradient / linear functional r ~ N(0,1), float32 [n][H][W]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, H, W)).astype(np.float32)


# ----------------------------------------------------------------------------------------------
# Workloads.  Image seed = 1000*config + item, Gaussian seed = image seed + 500.
# ----------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    H: int
    W: int
    n: int
    N: int
    n_rect: int
    smin: float
    smax: float
    K: int = 10
    tile: int = 16
    texture: bool = False
    image_seed: int = 0

    @property
    def gauss_seed(self) -> int:
        return self.image_seed + 500

    def target(self) -> np.ndarray:
        if self.texture:
            return gen_texture_stack(self.image_seed, self.H, self.W, self.n // 3, self.n_rect)
        return gen_image(self.image_seed, self.H, self.W, self.n, self.n_rect)

    def gaussians(self) -> np.ndarray:
        return gen_gaussians(self.gauss_seed, self.H, self.W, self.N, self.n, self.smin, self.smax)


def workload(config: int, item: int = 0) -> Workload:
    """The plain single-image workloads: 0 (256^2, 2k), 1 (1024^2, 20k), 2 (2048^2 x 9ch, 100k),
    4 (4096^2, 500k, sigma 0.5-8 px)."""
    seed = 1000 * config + item
    if config == 0:
        return Workload("plain-256x256-n3-N2000", 256, 256, 3, 2000, 20, 1.0, 12.0, image_seed=seed)
    if config == 1:
        return Workload("fit-1024x1024-n3-N20000", 1024, 1024, 3, 20000, 200, 1.0, 12.0, image_seed=seed)
    if config == 2:
        return Workload("texture-2048x2048-n9-N100000", 2048, 2048, 9, 100000, 200, 1.0, 12.0,
                        texture=True, image_seed=seed)
    if config == 4:
        return Workload("large-4096x4096-n3-N500000", 4096, 4096, 3, 500000, 2000, 0.5, 8.0, image_seed=seed)
    raise ValueError(f"no plain workload for config {config}")


def batch_workloads(count: int = 64, seed: int = 3000) -> List[Workload]:
    """Uneven batch: H, W uniform over {256, 512, 1024, 2048}; N proportional to pixel count with
    +-30% jitter, clipped to [5000, 80000]; 3-channel images with 200 rectangles."""
    rng = np.random.default_rng(seed)
    sides = np.array([256, 512, 1024, 2048])
    out = []
    for b in range(count):
        H = int(rng.choice(sides))
        W = int(rng.choice(sides))
        jit = rng.uniform(-0.3, 0.3)
        N = int(np.clip(round(80000 * H * W / 2048 ** 2 * (1 + jit)), 5000, 80000))
        out.append(Workload(f"batch{b}-{H}x{W}-N{N}", H, W, 3, N, 200, 1.0, 12.0, image_seed=seed + b))
    return out


def small_batch_workloads(count: int = 16, seed: int = 4100) -> List[Workload]:
    """16 images of 1024^2 with 30k Gaussians each, sigma 0.5-8 px, 2000 rectangles."""
    return [Workload(f"b16-{b}", 1024, 1024, 3, 30000, 2000, 0.5, 8.0, image_seed=seed + b)
            for b in range(count)]
