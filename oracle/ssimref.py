"""NumPy FP64 reference for the SSIM term of the fitting loss.  Test infrastructure only: the
tests, the smoke check and the benchmark's CPU baseline may use it, nothing on the product path.

The paper fits against L1 + 0.1 * L_SSIM (Sec. 3.3, Sec. 4.1) without spelling out the SSIM
variant.  Reading used here (both sides):

* L_SSIM = 1 - SSIM, SSIM = the mean of the structural-similarity map of Wang et al. (2004) over
  all n*H*W positions (every channel on its own);
* local statistics are weighted means under an 11 x 11 Gaussian window with sigma = 1.5, its
  weights normalized to sum 1, centred on every pixel; the image is extended by zeros outside
  [0, H) x [0, W), so the map has the image's size and every pixel receives a gradient;
* C1 = (0.01)^2, C2 = (0.03)^2 (dynamic range 1);
* the map at a pixel is (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)) with
  mx, my the local means, sxx, syy the local variances and sxy the local covariance, each taken as
  a weighted second moment minus the product of the means.

The total loss of a fitting step is L = L1 + 0.1 * (1 - SSIM); its gradient with respect to the
rendered image x (target y fixed) follows by the chain rule through the five local moments
(mx, my, E[x^2], E[y^2], E[xy]): for a weighted mean M(a)(p) = sum_q w(q - p) a(q), the
derivative of sum_p F(M(x)(p), ...) with respect to x(q) is sum_p w(q - p) dF/dM(p) = M(dF/dM)(q)
because the window is symmetric and zero outside the image.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
SSIM_WEIGHT = 0.1


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """1D weights exp(-t^2 / (2 sigma^2)), t = -r..r, normalized to sum 1 (the 2D window is the
    outer product, which then also sums to 1)."""
    r = size // 2
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(t * t) / (2.0 * sigma * sigma))
    return w / w.sum()


def window_mean(a: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """Weighted local mean of every plane of a [..., H, W] array: out[h, x] = sum over (u, v) of
    w[u] w[v] a[h + u - r, x + v - r], with a = 0 outside the image.  Written as the plain sum over
    the window's 121 offsets."""
    w = gaussian_window() if w is None else w
    a = np.asarray(a, np.float64)
    r = len(w) // 2
    H, W = a.shape[-2:]
    pad = [(0, 0)] * (a.ndim - 2) + [(r, r), (r, r)]
    ap = np.pad(a, pad)
    out = np.zeros_like(a)
    for u in range(len(w)):
        for v in range(len(w)):
            out += w[u] * w[v] * ap[..., u:u + H, v:v + W]
    return out


def moments(x, y, w=None):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = window_mean(x, w), window_mean(y, w)
    exx, eyy, exy = window_mean(x * x, w), window_mean(y * y, w), window_mean(x * y, w)
    return mx, my, exx, eyy, exy


def ssim_map(x, y, w=None, c1=C1, c2=C2):
    """The per-pixel SSIM map of two [n, H, W] stacks (channels independent)."""
    mx, my, exx, eyy, exy = moments(x, y, w)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    num = (2.0 * mx * my + c1) * (2.0 * sxy + c2)
    den = (mx * mx + my * my + c1) * (sxx + syy + c2)
    return num / den


def ssim(x, y, **kw) -> float:
    return float(ssim_map(x, y, **kw).mean())


def map_partials(x, y, w=None, c1=C1, c2=C2):
    """The SSIM map S and its partial derivatives with respect to the moments mx, E[x^2] and E[xy]
    (the target's moments are constants), by the quotient rule on S = A1 A2 / (B1 B2) with
    A1 = 2 mx my + C1, A2 = 2 (E[xy] - mx my) + C2, B1 = mx^2 + my^2 + C1,
    B2 = (E[x^2] - mx^2) + (E[y^2] - my^2) + C2:
      dA1/dmx = 2 my, dA2/dmx = -2 my, dB1/dmx = 2 mx, dB2/dmx = -2 mx,
      dB2/dE[x^2] = 1, dA2/dE[xy] = 2."""
    mx, my, exx, eyy, exy = moments(x, y, w)
    a1 = 2.0 * mx * my + c1
    a2 = 2.0 * (exy - mx * my) + c2
    b1 = mx * mx + my * my + c1
    b2 = (exx - mx * mx) + (eyy - my * my) + c2
    num, den = a1 * a2, b1 * b2
    s = num / den
    dnum_dmx = 2.0 * my * a2 + a1 * (-2.0 * my)
    dden_dmx = 2.0 * mx * b2 + b1 * (-2.0 * mx)
    d_mx = (dnum_dmx * den - num * dden_dmx) / (den * den)
    d_exx = -num * b1 / (den * den)
    d_exy = 2.0 * a1 / den
    return s, d_mx, d_exx, d_exy


def ssim_grad(x, y, w=None, **kw):
    """d(sum of the SSIM map)/dx, [n, H, W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    _, d_mx, d_exx, d_exy = map_partials(x, y, w, **kw)
    return window_mean(d_mx, w) + 2.0 * x * window_mean(d_exx, w) + y * window_mean(d_exy, w)


def ssim_grad_cond(x, y, w=None, **kw):
    """Sum of the magnitudes of the three terms of ssim_grad before they cancel: the scale of the
    rounding error of any evaluation that stores the partials and blurs them in fp32."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    _, d_mx, d_exx, d_exy = map_partials(x, y, w, **kw)
    return (window_mean(np.abs(d_mx), w) + 2.0 * np.abs(x) * window_mean(np.abs(d_exx), w)
            + np.abs(y) * window_mean(np.abs(d_exy), w))


def l1_ssim_loss_grad(x, y, weight=SSIM_WEIGHT):
    """L = mean|x - y| + weight * (1 - SSIM) and dL/dx; also the L1 mean, the MSE and SSIM.
    Returns (L, L1, MSE, SSIM), grad."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    count = x.size
    d = x - y
    l1 = np.abs(d).mean()
    mse = (d * d).mean()
    s = ssim(x, y)
    g = np.sign(d) / count - weight * ssim_grad(x, y) / count
    return (l1 + weight * (1.0 - s), l1, mse, s), g
