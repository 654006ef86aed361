"""Independent NumPy FP64 evaluation of the Image-GS renderer for tiny inputs.  Test
infrastructure only.

Unlike ``oracle.c`` it builds each covariance explicitly as R S S^T R^T (Eq. 2), inverts it with
``numpy.linalg.inv`` and evaluates the Mahalanobis form of Eq. 1 as d^T Sigma^{-1} d; the tile
test uses the distance from the mean to the rectangle written as max(x0 - mu, 0, mu - x1); the
ranking uses ``numpy.lexsort``; the adjoint is derived in matrix form
(dq/dmu = -2 Sigma^{-1} d, dq/dSigma^{-1} = d d^T, Sigma^{-1} = R S^{-2} R^T).
Memory is O(H*W*N): keep H*W*N below a few million.
"""
from __future__ import annotations

import numpy as np


def _rot(th):
    c, s = np.cos(th), np.sin(th)
    R = np.empty(th.shape + (2, 2))
    R[..., 0, 0], R[..., 0, 1], R[..., 1, 0], R[..., 1, 1] = c, -s, s, c
    return R


def _geometry(p):
    mu = p[0:2].T                       # [N,2]
    th = p[2]
    s = p[3:5].T                        # [N,2]
    R = _rot(th)
    S = np.zeros(th.shape + (2, 2))
    S[:, 0, 0], S[:, 1, 1] = s[:, 0], s[:, 1]
    Sigma = R @ S @ np.swapaxes(S, 1, 2) @ np.swapaxes(R, 1, 2)   # Eq. 2
    return mu, th, s, R, np.linalg.inv(Sigma)


def _pixels(H, W):
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return np.stack([ww.ravel() + 0.5, hh.ravel() + 0.5], axis=1), hh.ravel(), ww.ravel()


def membership(params, H, W, tile=16):
    """[H*W, N] bool: is Gaussian i in S_j of the pixel's tile (3-sigma enclosing circle vs tile)."""
    p = np.asarray(params, dtype=np.float64)
    _, hh, ww = _pixels(H, W)
    x0 = (ww // tile) * tile
    y0 = (hh // tile) * tile
    x1 = np.minimum(x0 + tile, W)
    y1 = np.minimum(y0 + tile, H)
    mx, my = p[0][None, :], p[1][None, :]
    ddx = np.maximum(np.maximum(x0[:, None] - mx, mx - x1[:, None]), 0.0)
    ddy = np.maximum(np.maximum(y0[:, None] - my, my - y1[:, None]), 0.0)
    r = 3.0 * np.maximum(p[3], p[4])[None, :]
    return ddx * ddx + ddy * ddy <= r * r


def render(params, H, W, K, tile=16, grad_img=None):
    """Returns dict(img [n][H][W], topk [H][W][K] (-1 unused), q [H*W][N]) and, with ``grad_img``,
    grad [5+n][N] of sum(grad_img * img) with the selection held fixed."""
    p = np.asarray(params, dtype=np.float64)
    N, n = p.shape[1], p.shape[0] - 5
    col = p[5:].T                                          # [N,n]
    mu, th, s, R, Sinv = _geometry(p)
    X, hh, ww = _pixels(H, W)
    d = X[:, None, :] - mu[None, :, :]                     # [P,N,2]
    q = np.einsum("pni,nij,pnj->pn", d, Sinv, d)   # Eq. 1 exponent (times -2)
    mem = membership(p, H, W, tile)
    qm = np.where(mem, q, np.inf)
    idx = np.broadcast_to(np.arange(N), qm.shape)
    order = np.lexsort((idx, qm), axis=-1)[:, :K]          # by q, then by index
    if order.shape[1] < K:                                 # K > N: pad with empty slots
        qm = np.concatenate([qm, np.full((qm.shape[0], 1), np.inf)], axis=1)
        order = np.concatenate([order, np.full((order.shape[0], K - order.shape[1]), N)], axis=1)
    qk = np.take_along_axis(qm, order, axis=1)
    valid = np.isfinite(qk)
    P = H * W
    img = np.zeros((P, n))
    topk = np.where(valid, order, -1)
    anyv = valid[:, 0]
    # Eq. 5, multiplied through by exp(q_min/2) (unchanged ratio, avoids underflow)
    G = np.where(valid, np.exp(-0.5 * (qk - qk[:, :1])), 0.0)
    Z = G.sum(axis=1)
    Zs = np.where(anyv, Z, 1.0)
    img = np.einsum("pk,pkc->pc", G, col[np.where(valid, order, 0)]) / Zs[:, None]
    img[~anyv] = 0.0
    out = {"img": img.T.reshape(n, H, W), "topk": topk.reshape(H, W, K), "q": q[:, :N]}
    if grad_img is None:
        return out
    g = np.asarray(grad_img, dtype=np.float64).reshape(n, P).T        # [P,n]
    alpha = G / Zs[:, None]                                             # [P,K]
    sel = np.where(valid, order, 0)
    grad = np.zeros((5 + n, N))
    # colour: dL/dc_i = sum_x alpha_i(x) g(x)
    for k in range(K):
        np.add.at(grad[5:].T, sel[:, k], (alpha[:, k:k + 1] * g) * valid[:, k:k + 1])
    # dL/dq_i = -1/2 alpha_i g.(c_i - c_r)
    dLdq = -0.5 * alpha * np.einsum("pc,pkc->pk", g, col[sel] - img[:, None, :])
    dLdq = np.where(valid, dLdq, 0.0)
    dk = np.take_along_axis(d, sel[:, :, None], axis=1)                # [P,K,2]
    Sk = Sinv[sel]                                                       # [P,K,2,2]
    # dq/dmu = -2 Sigma^{-1} d
    dq_dmu = -2.0 * np.einsum("pkij,pkj->pki", Sk, dk)
    for a in range(2):
        np.add.at(grad[a], sel.ravel(), (dLdq * dq_dmu[..., a]).ravel())
    # dq/dtheta = d^T (dSigma^{-1}/dtheta) d, dq/ds_a = d^T (dSigma^{-1}/ds_a) d
    c, sn = np.cos(th), np.sin(th)
    dR = np.empty(th.shape + (2, 2))
    dR[:, 0, 0], dR[:, 0, 1], dR[:, 1, 0], dR[:, 1, 1] = -sn, -c, c, -sn
    Sm2 = np.zeros(th.shape + (2, 2))
    Sm2[:, 0, 0], Sm2[:, 1, 1] = s[:, 0] ** -2, s[:, 1] ** -2
    RT = np.swapaxes(R, 1, 2)
    dSinv_dth = dR @ Sm2 @ RT + R @ Sm2 @ np.swapaxes(dR, 1, 2)
    dSinv_ds = []
    for a in range(2):
        D = np.zeros(th.shape + (2, 2))
        D[:, a, a] = -2.0 * s[:, a] ** -3
        dSinv_ds.append(R @ D @ RT)
    for row, M in ((2, dSinv_dth), (3, dSinv_ds[0]), (4, dSinv_ds[1])):
        val = np.einsum("pki,pkij,pkj->pk", dk, M[sel], dk)
        np.add.at(grad[row], sel.ravel(), (dLdq * val).ravel())
    out["grad"] = grad
    return out
