"""Pins of the decoding reference (oracle/decoderef.py): point evaluation against the C oracle's
render at pixel centres and against closed forms at arbitrary points; float16 storage against
known IEEE bit patterns (nearest, ties to even) and exact round trips."""
import math

import numpy as np
import pytest

from oracle import cref, decoderef as dr
from paper_2407_01866_amd import synth


@pytest.mark.parametrize("H,W,N,n,K", [(40, 56, 120, 3, 10), (33, 17, 60, 2, 1), (20, 20, 30, 1, 32)])
def test_points_at_pixel_centres_equal_the_render(H, W, N, n, K):
    p = synth.gen_gaussians(H + W, H, W, N, n).astype(np.float64)
    img = cref.render(p, H, W, K)["img"]
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pts = np.stack([ww.ravel() + 0.5, hh.ravel() + 0.5])
    got = dr.evaluate_points(p, H, W, K, pts)
    assert np.allclose(got, img.reshape(n, -1), rtol=1e-12, atol=1e-14)


def test_points_outside_are_zero():
    p = synth.gen_gaussians(1, 30, 30, 40, 3).astype(np.float64)
    pts = np.array([[-0.1, 30.0, 5.0, 5.0, np.nan], [5.0, 5.0, -1e-9, 30.0, 3.0]])
    assert np.all(dr.evaluate_points(p, 30, 30, 10, pts) == 0)


def test_single_gaussian_closed_form():
    """One Gaussian: its colour wherever its circle meets the point's tile, 0 elsewhere."""
    p = np.array([[20.3], [18.7], [0.4], [2.0], [1.0], [0.25], [0.75]])
    pts = np.array([[17.9, 31.99, 0.2, 47.5, 20.3], [16.01, 17.5, 0.3, 47.5, 40.0]])
    got = dr.evaluate_points(p, 48, 48, 10, pts)
    # circle of radius 6 about (20.3, 18.7): tile (1, 1) holds the mean; tile (0, 0)'s nearest
    # corner (16, 16) is sqrt(4.3^2 + 2.7^2) = 5.08 away (member); tile (2, 2) starts 11.7 away in
    # x and tile (1, 2) 13.3 away in y (not members)
    expect = np.array([[0.25, 0.25, 0.25, 0.0, 0.0], [0.75, 0.75, 0.75, 0.0, 0.0]])
    assert np.allclose(got, expect, rtol=0, atol=0)


def test_two_gaussians_blend_at_fractional_points():
    p = np.array([[10.0, 14.0], [8.0, 9.5], [0.0, 1.1], [3.0, 2.0], [1.5, 2.5],
                  [1.0, 0.0], [0.0, 1.0]])
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 16, size=(2, 50))
    got = dr.evaluate_points(p, 16, 16, 2, pts)

    def q(i, x, y):
        c, s = math.cos(p[2, i]), math.sin(p[2, i])
        dx, dy = x - p[0, i], y - p[1, i]
        return (c * dx + s * dy) ** 2 / p[3, i] ** 2 + (-s * dx + c * dy) ** 2 / p[4, i] ** 2

    for j in range(50):
        g = [math.exp(-0.5 * q(i, pts[0, j], pts[1, j])) for i in range(2)]
        assert abs(got[0, j] - g[0] / sum(g)) < 1e-12 and abs(got[1, j] - g[1] / sum(g)) < 1e-12


def test_fp16_bit_patterns():
    vals = np.array([0.1, 1.0 / 3.0, 1.0, 65504.0, 2049.0, 2051.0, 6e-8, -2.5, 0.0])
    bits = dr.to_fp16(vals.reshape(1, -1))[0]
    assert [int(b) for b in bits] == [0x2E66, 0x3555, 0x3C00, 0x7BFF, 0x6800, 0x6802, 0x0001,
                                      0xC100, 0x0000]


def test_fp16_decode_round_trip_and_prefix():
    H, W, n, N = 64, 96, 3, 20
    rng = np.random.default_rng(4)
    fit = np.empty((5 + n, N), np.float32)
    # values exactly representable in float16 decode exactly
    fit[0] = rng.integers(0, 1024, N) / 1024.0
    fit[1] = rng.integers(0, 1024, N) / 1024.0
    fit[2] = rng.integers(0, 256, N) / 128.0
    fit[3] = 0.25
    fit[4] = 0.5
    fit[5:] = rng.integers(0, 256, (n, N)) / 256.0
    dec = dr.decode_fp16(dr.to_fp16(fit), H, W, 12)
    assert dec.shape == (5 + n, 12)
    assert np.array_equal(dec[0], fit[0, :12] * W) and np.array_equal(dec[1], fit[1, :12] * H)
    assert np.all(dec[3] == 4.0) and np.all(dec[4] == 2.0)
    assert np.array_equal(dec[2], fit[2, :12]) and np.array_equal(dec[5:], fit[5:, :12])
