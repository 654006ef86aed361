"""NumPy FP64 reference for the fitting loop around the renderer.  Test infrastructure only.

* L1 loss (Sec. 3.3 and Sec. 4.1 name L1 + 0.1 SSIM; the workloads here use the L1 term alone),
  taken as the mean over n*H*W with sign(0) = 0;
* PSNR = 10 log10(1/MSE) over all channels (Sec. 4.1 metrics);
* Adam (Sec. 4.1, constant per-group learning rates for mu, c, s, theta = 5e-4, 5e-3, 2e-3, 2e-3)
  with PyTorch's default beta1, beta2, eps and bias correction, applied in the fitter's
  parameterization: mean normalized to [0,1]^2 (Sec. 4.1), inverse scales 1/s (Sec. 3.3 footnote,
  Sec. 4.1), theta in radians clipped to [0, pi] (Sec. 3.1) and raw colours.
"""
from __future__ import annotations

import math

import numpy as np

LR_MU, LR_C, LR_S, LR_TH = 5e-4, 5e-3, 2e-3, 2e-3


def l1_loss_grad(img, target):
    d = np.asarray(img, np.float64) - np.asarray(target, np.float64)
    return np.abs(d).mean(), np.sign(d) / d.size


def psnr(img, target):
    mse = np.mean((np.asarray(img, np.float64) - np.asarray(target, np.float64)) ** 2)
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else math.inf


def row_lrs(n):
    return np.array([LR_MU, LR_MU, LR_TH, LR_S, LR_S] + [LR_C] * n)


def to_fit_space(render_params, H, W):
    """Render parameters (pixels, s) -> fitter parameters (normalized mean, 1/s)."""
    p = np.array(render_params, dtype=np.float64)
    p[0] /= W
    p[1] /= H
    p[3] = 1.0 / p[3]
    p[4] = 1.0 / p[4]
    return p


def to_render_space(fit_params, H, W):
    p = np.array(fit_params, dtype=np.float64)
    p[0] *= W
    p[1] *= H
    p[3] = 1.0 / p[3]
    p[4] = 1.0 / p[4]
    return p


def grad_to_fit_space(grad_render, fit_params, H, W):
    """Chain rule: dL/dmu_norm = (W, H) dL/dmu_px ; dL/du = -s^2 dL/ds = -dL/ds / u^2."""
    g = np.array(grad_render, dtype=np.float64)
    u = np.asarray(fit_params, np.float64)[3:5]
    g[0] *= W
    g[1] *= H
    g[3:5] = -g[3:5] / (u * u)
    return g


def adam_step(fit_params, grad_fit, m, v, step, lrs, b1=0.9, b2=0.999, eps=1e-8,
              u_lo=None, u_hi=4.0, H=None, W=None):
    """One Adam step (step counts from 1); returns new (params, m, v).  theta is clipped to
    [0, pi]; the inverse scales to [1/max(H, W), u_hi] when H and W are given."""
    p = np.array(fit_params, np.float64)
    g = np.asarray(grad_fit, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p - np.asarray(lrs)[:, None] * mh / (np.sqrt(vh) + eps)
    p[2] = np.clip(p[2], 0.0, math.pi)
    if u_lo is None and H is not None:
        u_lo = 1.0 / max(H, W)
    if u_lo is not None:
        p[3:5] = np.clip(p[3:5], u_lo, u_hi)
    return p, m, v
