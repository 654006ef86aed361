"""NumPy FP64 reference for the paper's Gaussian placement around the renderer: content-adaptive
initialization (Sec. 3.3, Eq. 6) and error-guided addition of Gaussians (Sec. 3.3, Eq. 7).
Test infrastructure only: the tests, the smoke check and the benchmark's CPU baseline may use
it, nothing on the product path.

Readings (both sides):
* the image gradient is taken per channel with central differences inside the image and
  one-sided differences at its border (zero along an axis of length 1); ||grad I(x)||_2 is the
  Euclidean norm over both directions and all channels;
* Eq. 6: P_init(x) = (1 - lambda) ||grad I(x)|| / sum ||grad I|| + lambda / (H W); when the image
  has no gradient anywhere the first term is taken as zero and P_init as uniform;
* Eq. 7: P_add(x) = e(x) / sum e with e(x) = sum over channels of |rendered - target| (the L1
  error of the pixel); uniform when the render equals the target everywhere;
* each Gaussian's pixel is drawn independently (with replacement) by inverting the cumulative
  distribution over pixels in row-major order at a caller-supplied uniform u in [0, 1): the
  first pixel whose cumulative probability exceeds u;
* a Gaussian placed at pixel (h, w) has mean (w + 1/2, h + 1/2) in pixels, rotation 0, both
  scales 5 px (Sec. 4.1) and the target's colour at that pixel.
"""
from __future__ import annotations

import numpy as np

LAMBDA_INIT = 0.3
SCALE_INIT = 5.0


def _axis_gradient(a, axis):
    """Central differences inside, one-sided differences at both ends, zero for length 1."""
    a = np.asarray(a, np.float64)
    n = a.shape[axis]
    g = np.zeros_like(a)
    if n < 2:
        return g
    sl = lambda s: tuple(s if k == axis else slice(None) for k in range(a.ndim))  # noqa: E731
    g[sl(slice(1, n - 1))] = (a[sl(slice(2, n))] - a[sl(slice(0, n - 2))]) / 2.0
    g[sl(slice(0, 1))] = a[sl(slice(1, 2))] - a[sl(slice(0, 1))]
    g[sl(slice(n - 1, n))] = a[sl(slice(n - 1, n))] - a[sl(slice(n - 2, n - 1))]
    return g


def gradient_magnitude(img):
    """||grad I(x)||_2 over both directions and all channels of an [n][H][W] image -> [H][W]."""
    img = np.asarray(img, np.float64)
    gy = _axis_gradient(img, 1)
    gx = _axis_gradient(img, 2)
    return np.sqrt((gx * gx + gy * gy).sum(axis=0))


def init_probabilities(target, lam=LAMBDA_INIT):
    """Eq. 6 over the pixels of the target, [H][W], summing to 1."""
    g = gradient_magnitude(target)
    H, W = g.shape
    total = g.sum()
    if total <= 0:
        return np.full((H, W), 1.0 / (H * W))
    return (1.0 - lam) * g / total + lam / (H * W)


def error_probabilities(image, target):
    """Eq. 7 over the pixels, [H][W], summing to 1."""
    e = np.abs(np.asarray(image, np.float64) - np.asarray(target, np.float64)).sum(axis=0)
    total = e.sum()
    if total <= 0:
        return np.full(e.shape, 1.0 / e.size)
    return e / total


def sample_pixels(prob, uniforms):
    """Row-major pixel index of each uniform by inverting the cumulative distribution."""
    cdf = np.cumsum(np.asarray(prob, np.float64).ravel())
    t = np.asarray(uniforms, np.float64) * cdf[-1]
    return np.minimum(np.searchsorted(cdf, t, side="right"), cdf.size - 1)


def gaussians_at(pixels, target, scale=SCALE_INIT):
    """[5+n][count] render-space parameters of Gaussians placed at the given row-major pixels."""
    target = np.asarray(target, np.float64)
    n, H, W = target.shape
    pixels = np.asarray(pixels)
    h, w = pixels // W, pixels % W
    out = np.zeros((5 + n, pixels.size))
    out[0] = w + 0.5
    out[1] = h + 0.5
    out[2] = 0.0
    out[3] = scale
    out[4] = scale
    out[5:] = target[:, h, w]
    return out


def init_gaussians(target, uniforms, lam=LAMBDA_INIT, scale=SCALE_INIT):
    """Content-adaptive initialization: Eq. 6 sampling, target colours, 5 px, rotation 0."""
    return gaussians_at(sample_pixels(init_probabilities(target, lam), uniforms), target, scale)


def add_gaussians(image, target, uniforms, scale=SCALE_INIT):
    """Error-guided addition: Eq. 7 sampling, initialized like the content-adaptive ones."""
    return gaussians_at(sample_pixels(error_probabilities(image, target), uniforms), target,
                        scale)


def progressive_schedule(budget, every=500):
    """Active Gaussian count per step: budget/2 at the start, budget/8 more every 500 steps until
    the budget is reached (Sec. 4.1).  Returns the list of (step, count added)."""
    first = budget // 2
    steps = [(0, first)]
    active, k = first, 1
    while active < budget:
        add = min(budget // 8, budget - active)
        if add <= 0:
            add = budget - active
        steps.append((k * every, add))
        active += add
        k += 1
    return steps
