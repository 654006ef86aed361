"""Pins of the FP64 SSIM reference (oracle/ssimref.py) against what fixes it independently:

* the window's weighted mean equals SciPy's Gaussian filter with zero extension (a library
  routine: pins the window size, sigma, normalization and the border reading);
* SSIM of an image with itself is 1 at every pixel and its gradient there is 0 (the maximum);
* for constant images the map has a closed form in the window mass inside the image (pins C1,
  C2, the factors of 2 and the border reading once more);
* a brute-force per-pixel evaluation in the three-factor form of Wang et al. (luminance, contrast,
  structure with C3 = C2/2) using centred sums agrees with the moment form;
* central finite differences of the whole loss L1 + 0.1 (1 - SSIM) agree with the analytic
  gradient at every pixel of a small stack;
* symmetry in its two arguments and equivariance under transposition.
"""
import numpy as np
import pytest
import scipy.ndimage

from oracle import ssimref as sr


def _rand_pair(seed, shape, gap=0.0):
    rng = np.random.default_rng(seed)
    y = rng.random(shape)
    sign = rng.choice([-1.0, 1.0], size=shape)
    x = y + sign * (gap + rng.random(shape) * 0.3)
    return x, y


def test_window_is_normalized_gaussian_11_sigma_1_5():
    w = sr.gaussian_window()
    assert w.shape == (11,)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w[::-1], rtol=0, atol=0)
    assert np.isclose(w[6] / w[5], np.exp(-1.0 / (2 * 1.5 ** 2)), rtol=1e-14)


@pytest.mark.parametrize("shape", [(1, 7, 9), (3, 20, 33), (2, 12, 5)])
def test_window_mean_equals_scipy_gaussian_filter_with_zero_extension(shape):
    a = np.random.default_rng(1).standard_normal(shape)
    ours = sr.window_mean(a)
    for c in range(shape[0]):
        # radius = int(truncate * sigma + 0.5) = 5 taps each side; weights normalized to 1
        ref = scipy.ndimage.gaussian_filter(a[c], sigma=1.5, mode="constant", cval=0.0,
                                            truncate=5.0 / 1.5)
        assert np.allclose(ours[c], ref, rtol=1e-13, atol=1e-15)


def test_identical_images_give_one_and_zero_gradient():
    x = np.random.default_rng(2).random((2, 15, 18))
    s = sr.ssim_map(x, x)
    assert np.allclose(s, 1.0, rtol=0, atol=1e-13)
    g = sr.ssim_grad(x, x)
    scale = np.abs(sr.ssim_grad_cond(x, x)).max()
    assert np.abs(g).max() <= 1e-13 * scale


def _mass(n, size=11, sigma=1.5):
    w = sr.gaussian_window(size, sigma)
    r = size // 2
    m = np.zeros(n)
    for i in range(n):
        for u in range(size):
            if 0 <= i + u - r < n:
                m[i] += w[u]
    return m


@pytest.mark.parametrize("a,b", [(0.3, 0.7), (0.5, 0.5), (0.0, 0.9), (1.0, 0.2)])
def test_constant_images_closed_form(a, b):
    H, W = 19, 23
    x = np.full((1, H, W), a)
    y = np.full((1, H, W), b)
    M = _mass(H)[:, None] * _mass(W)[None, :]
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    # mx = a M, my = b M, E[x^2] = a^2 M, E[xy] = a b M, so the variances are a^2 M (1 - M), ...
    num = (2 * a * b * M * M + c1) * (2 * a * b * M * (1 - M) + c2)
    den = ((a * a + b * b) * M * M + c1) * ((a * a + b * b) * M * (1 - M) + c2)
    # rtol: fp64 rounding of E[y^2] - my^2 (about 1e-16) against C2 = 9e-4
    assert np.allclose(sr.ssim_map(x, y)[0], num / den, rtol=1e-10, atol=0)
    # far from the border the whole window is inside: the luminance term alone remains
    interior = sr.ssim_map(x, y)[0, 5:-5, 5:-5]
    assert np.allclose(interior, (2 * a * b + c1) / (a * a + b * b + c1), rtol=1e-12)


def _brute_force_map(x, y):
    """Per pixel, the centred weighted statistics over the zero-extended window and the product
    of luminance, contrast and structure (C3 = C2 / 2)."""
    w = sr.gaussian_window()
    r = 5
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    c3 = c2 / 2
    n, H, W = x.shape
    out = np.zeros_like(x)
    for c in range(n):
        for h in range(H):
            for v in range(W):
                vals = []
                for du in range(-r, r + 1):
                    for dv in range(-r, r + 1):
                        hh, vv = h + du, v + dv
                        inside = 0 <= hh < H and 0 <= vv < W
                        vals.append((w[du + r] * w[dv + r],
                                     x[c, hh, vv] if inside else 0.0,
                                     y[c, hh, vv] if inside else 0.0))
                mux = sum(k * p for k, p, _ in vals)
                muy = sum(k * q for k, _, q in vals)
                vx = sum(k * (p - mux) ** 2 for k, p, _ in vals)
                vy = sum(k * (q - muy) ** 2 for k, _, q in vals)
                cxy = sum(k * (p - mux) * (q - muy) for k, p, q in vals)
                sx, sy = np.sqrt(vx), np.sqrt(vy)
                lum = (2 * mux * muy + c1) / (mux * mux + muy * muy + c1)
                con = (2 * sx * sy + c2) / (vx + vy + c2)
                stru = (cxy + c3) / (sx * sy + c3)
                out[c, h, v] = lum * con * stru
    return out


def test_brute_force_three_factor_form():
    x, y = _rand_pair(3, (2, 7, 9))
    assert np.allclose(sr.ssim_map(x, y), _brute_force_map(x, y), rtol=1e-11, atol=1e-13)


def test_loss_gradient_matches_central_differences():
    x, y = _rand_pair(4, (2, 12, 14), gap=0.05)   # |x - y| >= 0.05: L1 is smooth there
    (L, l1, mse, s), g = sr.l1_ssim_loss_grad(x, y)
    d = x - y
    assert np.isclose(l1, np.abs(d).mean()) and np.isclose(mse, (d * d).mean())
    assert np.isclose(L, l1 + 0.1 * (1 - s), rtol=1e-15)
    h = 1e-6
    fd = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp = x.copy()
        xp[idx] += h
        xm = x.copy()
        xm[idx] -= h
        fd[idx] = (sr.l1_ssim_loss_grad(xp, y)[0][0] - sr.l1_ssim_loss_grad(xm, y)[0][0]) / (2 * h)
    err = np.abs(fd - g)
    assert err.max() <= 1e-7 * np.abs(g).max(), err.max() / np.abs(g).max()
    # the SSIM part alone, which is what the stencil kernels compute
    gs = sr.ssim_grad(x, y)
    fds = np.zeros_like(x)
    for idx in list(np.ndindex(x.shape))[::7]:
        xp = x.copy()
        xp[idx] += h
        xm = x.copy()
        xm[idx] -= h
        fds[idx] = (sr.ssim_map(xp, y).sum() - sr.ssim_map(xm, y).sum()) / (2 * h)
        assert abs(fds[idx] - gs[idx]) <= 1e-6 * np.abs(gs).max()


def test_symmetry_and_transposition():
    x, y = _rand_pair(5, (2, 10, 13))
    assert np.allclose(sr.ssim_map(x, y), sr.ssim_map(y, x), rtol=1e-14, atol=0)
    xt, yt = x.transpose(0, 2, 1), y.transpose(0, 2, 1)
    assert np.allclose(sr.ssim_map(xt, yt), sr.ssim_map(x, y).transpose(0, 2, 1), rtol=1e-13)
    assert np.allclose(sr.ssim_grad(xt, yt), sr.ssim_grad(x, y).transpose(0, 2, 1), rtol=1e-12,
                       atol=1e-12 * np.abs(sr.ssim_grad_cond(x, y)).max())


def test_planted_mistakes_fail_the_pins():
    """Wrong constants or a wrong window are caught by the closed form and the library check."""
    a, b = 0.3, 0.7
    x = np.full((1, 19, 23), a)
    y = np.full((1, 19, 23), b)
    good = sr.ssim_map(x, y)
    for kw in ({"c1": 0.03 ** 2, "c2": 0.01 ** 2}, {"c1": 0.01, "c2": 0.03}):
        assert not np.allclose(sr.ssim_map(x, y, **kw), good, rtol=1e-6)
    z = np.random.default_rng(6).standard_normal((1, 12, 12))
    ref = scipy.ndimage.gaussian_filter(z[0], sigma=1.5, mode="constant", truncate=5.0 / 1.5)
    for w in (sr.gaussian_window(11, 1.0), sr.gaussian_window(9, 1.5)):
        assert not np.allclose(sr.window_mean(z, w)[0], ref, rtol=1e-6)
