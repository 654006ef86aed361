"""Python front end of libimagegs: device buffers for the C ABI, a render/adjoint pair, and the
``torch.autograd.Function`` used for fitting.  Every step of the renderer runs in the HIP library;
this module only allocates torch tensors and calls the ABI (see ``_native``).
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _native as nat

TILE = nat.IGS_TILE


def _aligned_bytes(nbytes: int, device) -> torch.Tensor:
    """A uint8 device buffer of ``nbytes`` whose data pointer is 256-byte aligned."""
    raw = torch.empty(max(1, nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + max(1, nbytes)]


def initial_pair_capacity(N: int, H: int, W: int) -> int:
    """A first guess for the number of (tile, Gaussian) pairs: 16 per Gaussian, at least 64k."""
    return max(1 << 16, 16 * N)


class Renderer:
    """Scratch workspace for one problem shape (N, n, H, W, K) and a pair capacity that grows
    when the device reports an overflow.  Saved forward state is allocated per render call so that
    several renders may be pending an adjoint at once."""

    def __init__(self, N: int, n: int, H: int, W: int, K: int = 10,
                 pair_capacity: Optional[int] = None, device="cuda"):
        self.N, self.n, self.H, self.W, self.K = N, n, H, W, K
        self.device = torch.device(device)
        self.cap = int(pair_capacity or initial_pair_capacity(N, H, W))
        self._alloc()

    def _alloc(self):
        self.ws_bytes, self.saved_bytes = nat.igs_render_buffer_sizes(
            self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap)
        self.offsets = nat.igs_saved_offsets(self.N, self.n, self.H, self.W, self.K, TILE, TILE,
                                             self.cap)
        self.ws = _aligned_bytes(self.ws_bytes, self.device)

    def set_capacity(self, cap: int) -> None:
        if cap != self.cap:
            self.cap = int(cap)
            self._alloc()

    def new_saved(self) -> torch.Tensor:
        return _aligned_bytes(self.saved_bytes, self.device)

    # -------------------------------------------------------------------------- raw entry points

    def render_into(self, params: torch.Tensor, image: torch.Tensor,
                    saved: Optional[torch.Tensor]) -> None:
        """Enqueue one forward render (no synchronization, no overflow handling)."""
        if saved is None:
            need = self.ws_bytes + self.saved_bytes
            if self.ws.numel() < need:
                self.ws = _aligned_bytes(need, self.device)
            nat.igs_render(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap,
                           image, None, 0, self.ws, self.ws.numel())
        else:
            nat.igs_render(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap,
                           image, saved, saved.numel(), self.ws, self.ws.numel())

    def backward_into(self, params, image, grad_image, saved, grad_params) -> None:
        nat.igs_render_backward(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE,
                                self.cap, image, grad_image, saved, saved.numel(), grad_params,
                                self.ws, self.ws.numel())

    def render_l1_into(self, params, target, image, loss_out, saved) -> None:
        """Forward render fused with the mean-absolute-error loss against ``target``
        (loss_out: float64[2] = mean |d|, mean d^2); ``saved`` is required."""
        nat.igs_render_l1(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap,
                          target, image, loss_out, saved, saved.numel(), self.ws, self.ws.numel())

    def backward_l1_into(self, params, saved, grad_params) -> None:
        """Gradient of the fused forward's mean absolute error (no gradient image needed)."""
        nat.igs_render_backward_l1(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE,
                                   self.cap, saved, saved.numel(), grad_params, self.ws,
                                   self.ws.numel())

    def l1_grad_into(self, params, target, loss_out, grad_params, saved) -> None:
        """Mean absolute error against ``target`` and its gradient in one rasterization pass (the
        same numbers as render_l1_into + backward_l1_into, without an image)."""
        nat.igs_render_l1_grad(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE,
                               self.cap, target, loss_out, grad_params, saved, saved.numel(),
                               self.ws, self.ws.numel())

    def status_of(self, saved: Optional[torch.Tensor]) -> torch.Tensor:
        """The int64[8] device status block of a saved state (or of the workspace copy)."""
        buf = saved if saved is not None else self.ws[self.ws_bytes:]
        return buf[:64].view(torch.int64)

    # --------------------------------------------------------------------------- checked calls

    def render(self, params: torch.Tensor, keep_state: bool = True
               ) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        """Render and, if the pair capacity was too small, grow it to the reported size and render
        again (one 64-byte device-to-host read per call).  Returns (image, saved or None)."""
        image = torch.empty((self.n, self.H, self.W), dtype=torch.float32, device=self.device)
        for _ in range(2):
            saved = self.new_saved() if keep_state else None
            self.render_into(params, image, saved)
            st = self.status_of(saved).cpu()
            if int(st[nat.STAT_OVERFLOW]) == 0:
                if keep_state and int(st[nat.STAT_SLOT_OVERFLOW]) != 0:
                    raise RuntimeError("a tile hit set exceeds 65535 Gaussians: the saved top-K "
                                       "slots cannot be used for the adjoint")
                return image, saved
            self.set_capacity(int(int(st[nat.STAT_PAIRS]) * 1.25) + 1024)
        raise RuntimeError("pair capacity overflow persisted after resizing")

    def bin(self, params: torch.Tensor) -> torch.Tensor:
        """Binning alone (the tile lists point queries read), growing the pair capacity on
        overflow like ``render``.  Returns the saved state."""
        for _ in range(2):
            saved = self.new_saved()
            nat.igs_bin(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap,
                        saved, saved.numel(), self.ws, self.ws.numel())
            st = self.status_of(saved).cpu()
            if int(st[nat.STAT_OVERFLOW]) == 0:
                return saved
            self.set_capacity(int(int(st[nat.STAT_PAIRS]) * 1.25) + 1024)
        raise RuntimeError("pair capacity overflow persisted after resizing")

    def query_into(self, params, saved, points, out, sort: bool = True) -> None:
        """Colours [M][n] at points [M][2] ((x, y) in pixels) from the tile lists in ``saved``
        (written by ``bin`` or a render of the same parameters).  ``sort``: group the points by
        tile first (for scattered points; results are the same either way)."""
        M = int(points.shape[0])
        ws, nbytes = None, 0
        if sort and M > 0:
            nbytes = nat.igs_query_workspace_size(M, self.N, self.n, self.H, self.W)
            if getattr(self, "_qws", None) is None or self._qws.numel() < nbytes:
                self._qws = _aligned_bytes(nbytes, self.device)
            ws = self._qws
        nat.igs_query(params, self.N, self.n, self.H, self.W, self.K, TILE, TILE, self.cap, saved,
                      saved.numel(), points, M, out, ws, nbytes)

    def query(self, params, saved, points, sort: bool = True) -> torch.Tensor:
        out = torch.empty((int(points.shape[0]), self.n), dtype=torch.float32,
                          device=self.device)
        self.query_into(params, saved, points.contiguous(), out, sort)
        return out

    def backward(self, params, image, grad_image, saved) -> torch.Tensor:
        gp = torch.empty((5 + self.n, self.N), dtype=torch.float32, device=self.device)
        self.backward_into(params, image, grad_image.contiguous(), saved, gp)
        return gp

    # ------------------------------------------------------------------------------ inspection

    def tile_lists(self, saved: torch.Tensor):
        """(ranges int32[T][2], sorted Gaussian indices int32[P]) of a saved state."""
        T = ((self.H + TILE - 1) // TILE) * ((self.W + TILE - 1) // TILE)
        o = self.offsets
        st = self.status_of(saved).cpu()
        P = int(st[nat.STAT_PAIRS])
        ranges = saved[o["ranges"]:o["ranges"] + 8 * T].view(torch.int32).view(T, 2)
        vals = saved[o["vals"]:o["vals"] + 4 * min(P, self.cap)].view(torch.int32)
        return ranges, vals

    def slots(self, saved: torch.Tensor) -> torch.Tensor:
        """Saved top-K slots as int32 [K][H][W] (-1 = unused)."""
        o = self.offsets
        n = self.K * self.H * self.W
        s = saved[o["slots"]:o["slots"] + 2 * n].view(torch.int16).to(torch.int32) & 0xFFFF
        s = s.view(self.K, self.H, self.W)
        return torch.where(s == 0xFFFF, torch.full_like(s, -1), s)


def pack_params(means: torch.Tensor, theta: torch.Tensor, scales: torch.Tensor,
                colors: torch.Tensor) -> torch.Tensor:
    """[N,2], [N], [N,2], [N,n] -> float32 SoA [5+n][N] in the renderer's row order."""
    return torch.cat([means.T, theta[None], scales.T, colors.T], dim=0).float().contiguous()


_cache = {}


def renderer_for(N, n, H, W, K, device) -> Renderer:
    key = (N, n, H, W, K, str(device))
    r = _cache.get(key)
    if r is None:
        r = Renderer(N, n, H, W, K, device=device)
        _cache[key] = r
    return r


def render(params: torch.Tensor, H: int, W: int, K: int = 10) -> torch.Tensor:
    """Render a [5+n][N] float32 parameter set (pixel units) into an [n][H][W] image."""
    n, N = params.shape[0] - 5, params.shape[1]
    r = renderer_for(N, n, H, W, K, params.device)
    img, _ = r.render(params.contiguous(), keep_state=False)
    return img


class RenderFn(torch.autograd.Function):
    """Differentiable Image-GS render in the fitter's parameterization.

    Inputs: means [N,2] normalized to [0,1]^2 (x by W, y by H), theta [N], inverse scales [N,2]
    (1/s in 1/pixels), colors [N,n]; H, W, K.  Output: [n,H,W].  The parameters are gathered into
    the [5+n][N] fitter layout of igs_adam_step (a copy), converted to render units by
    igs_fit_to_render, rendered, and the backward runs the HIP adjoint through the K retained
    Gaussians and igs_grad_to_fit for the chain rule back to the fitter's units."""

    @staticmethod
    def forward(ctx, means, theta, inv_scales, colors, H: int, W: int, K: int = 10):
        N, n = means.shape[0], colors.shape[1]
        fit = torch.cat([means.T, theta.reshape(1, N), inv_scales.T, colors.T], dim=0)
        fit = fit.float().contiguous()
        params = torch.empty_like(fit)
        if N > 0:
            nat.igs_fit_to_render(fit, params, N, n, H, W)
        r = renderer_for(N, n, H, W, K, means.device)
        image, saved = r.render(params, keep_state=True)
        ctx.r, ctx.saved_state = r, saved
        ctx.H, ctx.W, ctx.N, ctx.n = H, W, N, n
        ctx.save_for_backward(fit, params, image)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        fit, params, image = ctx.saved_tensors
        gp = ctx.r.backward(params, image, grad_image.float().contiguous(), ctx.saved_state)
        g = torch.empty_like(gp)
        if ctx.N > 0:
            nat.igs_grad_to_fit(fit, gp, g, ctx.N, ctx.n, ctx.H, ctx.W)
        return (g[0:2].T.contiguous(), g[2].clone(), g[3:5].T.contiguous(), g[5:].T.contiguous(),
                None, None, None)


class BatchRenderer:
    """Device buffers for rendering a batch of images of uneven size and Gaussian count with one
    launch per phase.  ``sizes`` is a list of (H, W, N); parameters are the concatenation of the
    images' [5+n][N_b] sets along the Gaussian axis; images are concatenated planar blocks (see
    ``image_views``)."""

    def __init__(self, sizes, n: int, K: int = 10, pair_capacity: Optional[int] = None,
                 device="cuda"):
        self.sizes = [tuple(int(v) for v in s) for s in sizes]
        self.n, self.K, self.B = n, K, len(self.sizes)
        self.device = torch.device(device)
        H = [s[0] for s in self.sizes]
        W = [s[1] for s in self.sizes]
        N = [s[2] for s in self.sizes]
        self.descs, (self.N, self.T, self.P, self.loss_blocks) = nat.igs_batch_describe(H, W, N, n)
        self.d_descs = nat.descs_to_device(self.descs, self.device)
        self.gauss_off = [d.gauss_off for d in self.descs]
        self.pix_off = [d.pix_off for d in self.descs]
        self.cap = int(pair_capacity or initial_pair_capacity(self.N, 0, 0))
        self._alloc()

    def _alloc(self):
        self.ws_bytes, self.saved_bytes = nat.igs_batch_buffer_sizes(self.descs, self.n, self.K,
                                                                     self.cap)
        self.offsets = nat.igs_batch_saved_offsets(self.descs, self.n, self.K, self.cap)
        self.ws = _aligned_bytes(self.ws_bytes, self.device)

    def set_capacity(self, cap: int) -> None:
        if cap != self.cap:
            self.cap = int(cap)
            self._alloc()

    def new_saved(self) -> torch.Tensor:
        return _aligned_bytes(self.saved_bytes, self.device)

    def new_images(self) -> torch.Tensor:
        return torch.empty(self.n * self.P, dtype=torch.float32, device=self.device)

    def image_views(self, flat: torch.Tensor):
        """[n][H][W] views of each image inside a concatenated buffer."""
        out = []
        for (H, W, _), po in zip(self.sizes, self.pix_off):
            out.append(flat[self.n * po:self.n * (po + H * W)].view(self.n, H, W))
        return out

    def pack_images(self, images) -> torch.Tensor:
        return torch.cat([im.reshape(-1) for im in images]).to(self.device, torch.float32).contiguous()

    def pack_params(self, params_list) -> torch.Tensor:
        return torch.cat([torch.as_tensor(p) for p in params_list], dim=1).to(
            self.device, torch.float32).contiguous()

    def render_into(self, params, images, saved) -> None:
        nat.igs_render_batched(params, self.descs, self.d_descs, self.n, self.K, self.cap, images,
                               saved, saved.numel(), self.ws, self.ws.numel())

    def backward_into(self, params, images, grad_images, saved, grad_params) -> None:
        nat.igs_render_backward_batched(params, self.descs, self.d_descs, self.n, self.K, self.cap,
                                        images, grad_images, saved, saved.numel(), grad_params,
                                        self.ws, self.ws.numel())

    def render_l1_into(self, params, targets, images, loss_out, saved) -> None:
        nat.igs_render_l1_batched(params, self.descs, self.d_descs, self.n, self.K, self.cap,
                                  targets, images, loss_out, saved, saved.numel(), self.ws,
                                  self.ws.numel())

    def backward_l1_into(self, params, saved, grad_params) -> None:
        nat.igs_render_backward_l1_batched(params, self.descs, self.d_descs, self.n, self.K,
                                           self.cap, saved, saved.numel(), grad_params, self.ws,
                                           self.ws.numel())

    def l1_grad_into(self, params, targets, loss_out, grad_params, saved) -> None:
        nat.igs_render_l1_grad_batched(params, self.descs, self.d_descs, self.n, self.K, self.cap,
                                       targets, loss_out, grad_params, saved, saved.numel(),
                                       self.ws, self.ws.numel())

    def status_of(self, saved: torch.Tensor) -> torch.Tensor:
        return saved[:64].view(torch.int64)

    def render(self, params, keep_state=True):
        images = self.new_images()
        for _ in range(2):
            saved = self.new_saved()
            self.render_into(params, images, saved)
            st = self.status_of(saved).cpu()
            if int(st[nat.STAT_OVERFLOW]) == 0:
                return images, saved
            self.set_capacity(int(int(st[nat.STAT_PAIRS]) * 1.25) + 1024)
        raise RuntimeError("pair capacity overflow persisted after resizing")

    def tile_lists(self, saved):
        o = self.offsets
        P = int(self.status_of(saved)[nat.STAT_PAIRS])
        ranges = saved[o["ranges"]:o["ranges"] + 8 * self.T].view(torch.int32).view(self.T, 2)
        vals = saved[o["vals"]:o["vals"] + 4 * min(P, self.cap)].view(torch.int32)
        return ranges, vals

    def tile_queue(self, saved) -> torch.Tensor:
        o = self.offsets
        return saved[o["order"]:o["order"] + 4 * self.T].view(torch.int32)

    def slots(self, saved):
        """Per image: slots int32 [K][H][W] (-1 unused)."""
        o = self.offsets
        raw = saved[o["slots"]:o["slots"] + 2 * self.K * self.P].view(torch.int16).to(torch.int32) & 0xFFFF
        raw = torch.where(raw == 0xFFFF, torch.full_like(raw, -1), raw)
        return [raw[self.K * po:self.K * (po + H * W)].view(self.K, H, W)
                for (H, W, _), po in zip(self.sizes, self.pix_off)]


class Decoder:
    """A stored representation (float16 fitter parameters, Sec. 4.1) decoded for use: the first
    ``n_prefix`` Gaussians (a level of detail of a progressive fit; all by default) in the
    renderer's units, binned once, then rendered or sampled at arbitrary points."""

    def __init__(self, stored: torch.Tensor, n: int, H: int, W: int, K: int = 10,
                 n_prefix: Optional[int] = None):
        self.device = stored.device
        N_stored = int(stored.shape[1])
        N = N_stored if n_prefix is None else int(n_prefix)
        self.n, self.H, self.W, self.K, self.N = n, H, W, K, N
        self.params = torch.empty((5 + n, N), dtype=torch.float32, device=self.device)
        nat.igs_decode_fp16(stored.contiguous(), N_stored, n, N, H, W, self.params)
        self.r = Renderer(N, n, H, W, K, device=self.device)
        self.saved = self.r.bin(self.params)

    def query(self, points: torch.Tensor) -> torch.Tensor:
        """Colours [M][n] at points [M][2] ((x, y) in pixels)."""
        return self.r.query(self.params, self.saved, points)

    def render(self) -> torch.Tensor:
        img, _ = self.r.render(self.params, keep_state=False)
        return img


def store_fp16(fit_params: torch.Tensor) -> torch.Tensor:
    """The float16 storage of a [5+n][N] float32 set of fitter parameters (int16 bit patterns)."""
    n, N = fit_params.shape[0] - 5, fit_params.shape[1]
    out = torch.empty((5 + n, N), dtype=torch.int16, device=fit_params.device)
    nat.igs_params_to_fp16(fit_params.contiguous(), N, n, out)
    return out
