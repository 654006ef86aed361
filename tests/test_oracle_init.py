"""Pins of the FP64 placement reference (oracle/initref.py): content-adaptive initialization
(Eq. 6) and error-guided addition (Eq. 7), against NumPy's gradient routine, closed forms of the
two distributions, a brute-force sampler and sampling frequencies."""
import numpy as np
import pytest

from oracle import initref as ir


@pytest.mark.parametrize("shape", [(3, 9, 13), (1, 2, 7), (9, 5, 2), (2, 16, 16)])
def test_gradient_magnitude_equals_numpy_gradient(shape):
    img = np.random.default_rng(1).random(shape)
    gy = np.gradient(img, axis=1)
    gx = np.gradient(img, axis=2)
    ref = np.sqrt((gx * gx + gy * gy).sum(axis=0))
    assert np.allclose(ir.gradient_magnitude(img), ref, rtol=1e-14, atol=0)


def test_gradient_along_a_length_one_axis_is_zero():
    img = np.random.default_rng(2).random((2, 1, 6))
    gx = np.gradient(img, axis=2)
    assert np.allclose(ir.gradient_magnitude(img), np.sqrt((gx * gx).sum(axis=0)), rtol=1e-14)
    assert np.all(ir.gradient_magnitude(np.ones((1, 1, 1))) == 0)


def test_eq6_is_a_distribution_and_lambda_one_is_uniform():
    t = np.random.default_rng(3).random((3, 12, 10))
    for lam in (0.0, 0.3, 1.0):
        p = ir.init_probabilities(t, lam)
        assert p.shape == (12, 10) and np.all(p >= 0) and abs(p.sum() - 1.0) < 1e-12
    assert np.allclose(ir.init_probabilities(t, 1.0), 1.0 / 120, rtol=1e-14)


def test_eq6_linear_ramp_is_uniform():
    """Central and one-sided differences of a linear function are exact and equal: the gradient
    magnitude is the same at every pixel, so every lambda gives the uniform distribution."""
    H, W = 8, 11
    h, w = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    t = np.stack([0.02 * w + 0.01 * h, 0.5 - 0.03 * h, 0.004 * w])
    for lam in (0.0, 0.3):
        assert np.allclose(ir.init_probabilities(t, lam), 1.0 / (H * W), rtol=1e-12)


def test_eq6_step_edge_closed_form():
    """A vertical step of height d between columns k-1 and k: the central differences at those
    two columns are d/2, zero elsewhere."""
    H, W, k, d, lam = 6, 10, 4, 0.8, 0.3
    t = np.zeros((1, H, W))
    t[0, :, k:] = d
    p = ir.init_probabilities(t, lam)
    ref = np.full((H, W), lam / (H * W))
    ref[:, k - 1:k + 1] += (1 - lam) / (2 * H)
    assert np.allclose(p, ref, rtol=1e-13)


def test_eq6_constant_image_is_uniform():
    assert np.allclose(ir.init_probabilities(np.full((3, 5, 7), 0.4), 0.3), 1 / 35)


def test_eq7_closed_forms():
    t = np.random.default_rng(4).random((3, 5, 6))
    img = t.copy()
    assert np.allclose(ir.error_probabilities(img, t), 1 / 30)
    img[1, 2, 3] += 0.25
    img[0, 4, 0] -= 0.75
    p = ir.error_probabilities(img, t)
    ref = np.zeros((5, 6))
    ref[2, 3], ref[4, 0] = 0.25, 0.75
    assert np.allclose(p, ref, rtol=1e-12, atol=1e-15)


def test_sampling_boundaries_and_zero_probability_pixels():
    p = np.array([0.25, 0.0, 0.5, 0.25])
    u = np.array([0.0, 0.2499, 0.25, 0.7499, 0.75, 0.999999])
    assert list(ir.sample_pixels(p, u)) == [0, 0, 2, 2, 3, 3]
    p2 = np.array([0.0, 0.0, 1.0, 0.0])
    assert list(ir.sample_pixels(p2, [0.0, 0.5, 0.9999999])) == [2, 2, 2]


def _brute_sample(prob, u):
    flat = np.asarray(prob, np.float64).ravel()
    out = []
    for x in u:
        acc, t = 0.0, x * flat.sum()
        for k, v in enumerate(flat):
            acc += v
            if acc > t:
                break
        out.append(k)
    return np.array(out)


def test_sampling_equals_brute_force():
    rng = np.random.default_rng(5)
    p = rng.random((7, 9)) * (rng.random((7, 9)) > 0.3)
    p /= p.sum()
    u = rng.random(500)
    assert np.array_equal(ir.sample_pixels(p, u), _brute_sample(p, u))


def test_sampling_frequencies():
    rng = np.random.default_rng(6)
    p = np.array([0.1, 0.4, 0.05, 0.3, 0.15])
    n = 200_000
    counts = np.bincount(ir.sample_pixels(p, rng.random(n)), minlength=5)
    sd = np.sqrt(n * p * (1 - p))
    assert np.all(np.abs(counts - n * p) < 5 * sd)


def test_gaussians_at_pixels():
    t = np.random.default_rng(7).random((2, 4, 5))
    g = ir.gaussians_at(np.array([0, 7, 19]), t)
    assert np.allclose(g[0], [0.5, 2.5, 4.5]) and np.allclose(g[1], [0.5, 1.5, 3.5])
    assert np.all(g[2] == 0) and np.all(g[3:5] == 5.0)
    assert np.allclose(g[5:, 1], t[:, 1, 2]) and np.allclose(g[5:, 2], t[:, 3, 4])


def test_progressive_schedule():
    assert ir.progressive_schedule(1000) == [(0, 500), (500, 125), (1000, 125), (1500, 125),
                                             (2000, 125)]
    s = ir.progressive_schedule(100)
    assert s[0] == (0, 50) and sum(a for _, a in s) == 100
