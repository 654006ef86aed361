"""Fitting loop around the renderer (Image-GS Sec. 3.3 and Sec. 4.1): every iteration renders the
Gaussians, takes the loss gradient against the target (L1, fused into the render pass for up to
16 channels, or the paper's L1 + 0.1 SSIM as a separate stencil step), runs the adjoint and
applies one Adam step with the paper's constant per-group
learning rates, in the fitter's parameterization (mean normalized to [0,1]^2, inverse scales
1/s).  Every step is a libimagegs kernel; an
iteration enqueues with no host synchronization and can be captured as one HIP graph.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import torch

from . import _native as nat
from .render import Renderer, _aligned_bytes

# Sec. 4.1: learning rates of (mu, c, s, theta), constant throughout training
LR_MU, LR_COLOR, LR_SCALE, LR_THETA = 5e-4, 5e-3, 2e-3, 2e-3
# the fused render+L1 entry points record 2-bit loss signs per channel
MAX_FUSED_CHANNELS = 16
# Sec. 4.1: initial scale of every placed Gaussian (pixels), weight of the uniform term of Eq. 6,
# and the period of the error-guided additions
INIT_SCALE = 5.0
LAMBDA_INIT = 0.3
GROW_EVERY = 500


def _check_single_pass(single_pass: bool, ssim_weight: float, fused: bool, n: int) -> bool:
    if not single_pass:
        return False
    if ssim_weight > 0:
        raise ValueError("the single-pass kernel evaluates the L1 loss only")
    if not fused or n > MAX_FUSED_CHANNELS:
        raise ValueError(f"the single-pass kernel needs the fused L1 path (n <= {MAX_FUSED_CHANNELS})")
    return True


def progressive_growth(budget: int, every: int = GROW_EVERY) -> List[Tuple[int, int]]:
    """(step, count) of the error-guided additions after the initial budget // 2 Gaussians
    (Sec. 4.1): budget // 8 more every 500 steps until the budget is reached (the last addition
    tops up what integer division leaves)."""
    out, active, k = [], budget // 2, 1
    while active < budget:
        add = min(max(budget // 8, 1), budget - active)
        out.append((k * every, add))
        active += add
        k += 1
    return out


@dataclass
class AdamConfig:
    lr_mu: float = LR_MU
    lr_theta: float = LR_THETA
    lr_inv_scale: float = LR_SCALE
    lr_color: float = LR_COLOR
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    inv_scale_hi: float = 4.0       # 1/s <= 4, i.e. s >= 0.25 px; 1/s >= 1/max(H, W)


class _FitLoop:
    """Iteration bookkeeping shared by the plain and batched fitters: graph capture, the device
    step counter, repetition of iterations whose render overflowed the pair buffer, and the
    fitter's own raster launch settings (``launch_config``: a (persistent, wgs_per_cu, fwd_cull,
    fwd_batch, k_unroll) tuple applied on the enqueueing thread before every eager step and
    capture; None keeps the thread's current settings)."""

    graph = None
    launch_config = None

    def _apply_launch_config(self) -> None:
        if self.launch_config is not None:
            nat.igs_set_launch_config(*self.launch_config)

    def capture(self) -> None:
        """Capture one iteration as a HIP graph (the library allocates nothing, so buffers and
        kernel arguments stay valid across replays)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step_async()
        self.graph = g

    def step(self) -> None:
        if self.graph is not None:
            self.graph.replay()
        else:
            self.step_async()

    def status(self) -> torch.Tensor:
        """Status block of the last render (synchronizes)."""
        self.status_host.copy_(self.r.status_of(self.saved))
        return self.status_host

    def steps_done(self) -> int:
        return int(self.step_count.item())

    def grow(self, factor: float = 1.5) -> None:
        """Enlarge the pair buffer to ``factor`` times the larger of the current capacity and the
        last render's requirement; drops the captured graph (it is re-captured on demand).  Raises
        if the last iteration was skipped for a hit set too long for the two-pass adjoint's 16-bit
        slots (the single-pass path has no such limit)."""
        st = self.status()
        if int(st[nat.STAT_SKIP]) != 0 and int(st[nat.STAT_OVERFLOW]) == 0:
            raise RuntimeError("a tile hit set exceeds 65535 Gaussians, more than the two-pass "
                               "adjoint's 16-bit slots address; fit with single_pass=True")
        need = max(self.r.cap, int(st[nat.STAT_PAIRS]))
        self.r.set_capacity(int(need * factor) + 1024)
        self.saved = self.r.new_saved()
        self.graph = None

    def advance_to(self, target: int, use_graph: bool = True, max_rounds: int = 8) -> None:
        """Run iterations until exactly ``target`` have been applied (skipped ones repeat)."""
        for _ in range(max_rounds):
            missing = target - self.steps_done()
            if missing <= 0:
                return
            if use_graph and self.graph is None:
                self.capture()
            for _ in range(missing):
                self.step() if use_graph else self.step_async()
            if self.steps_done() < target:
                self.grow()
        raise RuntimeError("pair buffer kept overflowing")

    def run(self, iters: int, report_every: int = 100, use_graph: bool = True):
        """Fit for ``iters`` iterations; returns (iteration, PSNR of that iteration's render)
        every ``report_every`` iterations (and at the last)."""
        start = self.steps_done()
        out = []
        it = 0
        while it < iters:
            it = min(iters, (it // report_every + 1) * report_every)
            self.advance_to(start + it, use_graph)
            out.append((it, self.psnr()))
        return out

    def _skip_word(self) -> torch.Tensor:
        """The status word that makes Adam skip an iteration whose gradient is unusable."""
        return self.r.status_of(self.saved)[nat.STAT_SKIP:nat.STAT_SKIP + 1]

    def snapshot(self) -> dict:
        return self.state_dict()

    def restore(self, sd: dict) -> None:
        self.load_state_dict(sd)


class PlainFitter(_FitLoop):
    """Fits one image.  ``render_params`` is the initial [5+n][N] float32 set in pixel units."""

    def __init__(self, target: torch.Tensor, render_params: torch.Tensor, K: int = 10,
                 adam: Optional[AdamConfig] = None, headroom: float = 1.25,
                 pair_capacity: Optional[int] = None, fused: Optional[bool] = None,
                 ssim_weight: float = 0.0, single_pass: bool = False):
        if target.dim() != 3:
            raise ValueError("target must be [n][H][W]")
        # ssim_weight > 0: the loss is L1 + ssim_weight * (1 - SSIM) (the paper uses 0.1); the
        # SSIM term needs neighbouring pixels of the rendered image, so that path renders, takes
        # the loss gradient image and runs the adjoint as separate steps
        self.ssim_weight = float(ssim_weight)
        if self.ssim_weight < 0:
            raise ValueError("ssim_weight must be >= 0")
        if self.ssim_weight > 0 and fused:
            raise ValueError("the SSIM term is not fused into the render pass")
        self.dev = target.device
        self.target = target.contiguous().float()
        self.n, self.H, self.W = self.target.shape
        self.N = render_params.shape[1]
        self.K = K
        self.adam = adam or AdamConfig()
        # fused: the forward computes the L1 loss and its gradient record in the same pass and the
        # adjoint reads that record (no gradient image); otherwise render, L1, adjoint separately
        if self.ssim_weight > 0:
            self.fused = False
        else:
            self.fused = (self.n <= MAX_FUSED_CHANNELS) if fused is None else bool(fused)
        # single_pass: render, L1 and adjoint of every tile in one kernel (same loss and gradient
        # as the fused pair, no image); self.image is then rendered only when densifying
        self.single_pass = _check_single_pass(single_pass, self.ssim_weight, self.fused, self.n)
        self.rend = render_params.to(self.dev).float().contiguous().clone()
        self.fit = torch.empty_like(self.rend)
        self.fit.copy_(self.rend)
        self.fit[0] /= self.W
        self.fit[1] /= self.H
        self.fit[3:5] = 1.0 / self.fit[3:5]
        # render parameters are always derived from the fitter's by the library's conversion
        nat.igs_fit_to_render(self.fit, self.rend, self.N, self.n, self.H, self.W)
        self.m = torch.zeros_like(self.rend)
        self.v = torch.zeros_like(self.rend)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.r = Renderer(self.N, self.n, self.H, self.W, K, pair_capacity=pair_capacity,
                          device=self.dev)
        self.image = torch.empty_like(self.target)
        self.grad_image = torch.empty_like(self.target)
        self.grad_params = torch.empty_like(self.rend)
        # L1 alone: [mean |x - y|, MSE]; with SSIM: [L, mean |x - y|, MSE, SSIM]
        self.loss = torch.zeros(4 if self.ssim_weight > 0 else 2, dtype=torch.float64,
                                device=self.dev)
        if self.ssim_weight > 0:
            self.l1_ws = _aligned_bytes(
                nat.igs_l1_ssim_workspace_size(self.n, self.H, self.W), self.dev)
        else:
            self.l1_ws = _aligned_bytes(nat.igs_l1_workspace_size(self.target.numel()), self.dev)
        if pair_capacity is None:
            # size the pair buffer from a binning of the initial state, with headroom for growth
            P = int(self.r.status_of(self.r.bin(self.rend))[nat.STAT_PAIRS])
            self.r.set_capacity(max(1024, int(P * headroom)))
        self.saved = self.r.new_saved()
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.status_host = torch.zeros(8, dtype=torch.int64).pin_memory()
        self.headroom = headroom
        self.growth: List[Tuple[int, int]] = []     # pending (step, count) additions
        self.gen: Optional[torch.Generator] = None
        self.scale_init = INIT_SCALE
        self.place_ws: Optional[torch.Tensor] = None

    @classmethod
    def from_target(cls, target: torch.Tensor, budget: int, K: int = 10, progressive: bool = True,
                    lambda_init: float = LAMBDA_INIT, scale: float = INIT_SCALE, seed: int = 0,
                    **kw) -> "PlainFitter":
        """The paper's fit from scratch (Sec. 3.3, Sec. 4.1): budget // 2 Gaussians (all of them
        when not progressive) placed by content-adaptive sampling (Eq. 6), then budget // 8 more
        every 500 iterations placed where the render's error is largest (Eq. 7).  Random numbers
        come from a device generator seeded with ``seed``."""
        target = target.contiguous().float()
        n, H, W = target.shape
        dev = target.device
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        N0 = budget // 2 if progressive else budget
        rp = torch.empty((5 + n, N0), dtype=torch.float32, device=dev)
        ws = _aligned_bytes(nat.igs_place_workspace_size(H, W), dev)
        u = torch.rand(N0, generator=gen, device=dev)
        nat.igs_init_gaussians(target, n, H, W, lambda_init, u, N0, scale, rp, None, N0, 0, ws,
                               ws.numel())
        f = cls(target, rp, K, **kw)
        f.gen, f.place_ws, f.scale_init = gen, ws, float(scale)
        f.growth = progressive_growth(budget) if progressive else []
        return f

    # ----------------------------------------------------------------------- densification

    def _resize(self, N_new: int) -> None:
        """Grow (or shrink, when loading a checkpoint) every per-Gaussian buffer to N_new
        columns, keeping the common columns; new Adam moments are zero."""
        def cols(t):
            out = torch.zeros((5 + self.n, N_new), dtype=t.dtype, device=self.dev)
            k = min(self.N, N_new)
            out[:, :k] = t[:, :k]
            return out
        self.fit, self.rend, self.m, self.v = (cols(t) for t in (self.fit, self.rend, self.m,
                                                                 self.v))
        self.grad_params = torch.empty_like(self.rend)
        self.N = N_new
        self.r = Renderer(self.N, self.n, self.H, self.W, self.K, device=self.dev)
        self.graph = None

    def _size_pairs(self) -> None:
        P = int(self.r.status_of(self.r.bin(self.rend))[nat.STAT_PAIRS])
        self.r.set_capacity(max(1024, int(P * self.headroom)))
        self.saved = self.r.new_saved()

    def densify(self, count: int) -> None:
        """Error-guided addition of ``count`` Gaussians (Eq. 7) from a render of the current
        parameters (every loss path renders them the same way, growing the pair buffer if needed),
        initialized like the content-adaptive ones (Sec. 4.1); drops the captured graph."""
        if count <= 0:
            return
        if self.gen is None:
            self.gen = torch.Generator(device=self.dev)
            self.gen.manual_seed(0)
        if self.place_ws is None:
            self.place_ws = _aligned_bytes(nat.igs_place_workspace_size(self.H, self.W),
                                           self.dev)
        img, _ = self.r.render(self.rend, keep_state=False)
        self.image.copy_(img)
        N_old = self.N
        self._resize(N_old + count)
        u = torch.rand(count, generator=self.gen, device=self.dev)
        nat.igs_add_gaussians(self.image, self.target, self.n, self.H, self.W, u, count,
                              self.scale_init, self.rend, self.fit, self.N, N_old, self.place_ws,
                              self.place_ws.numel())
        self._size_pairs()

    def advance_to(self, target: int, use_graph: bool = True, max_rounds: int = 8) -> None:
        """As the base loop, with the pending error-guided additions applied when the fit reaches
        their step."""
        while self.growth and self.growth[0][0] <= target:
            step, count = self.growth[0]
            super().advance_to(step, use_graph, max_rounds)
            self.growth.pop(0)
            self.densify(count)
        super().advance_to(target, use_graph, max_rounds)

    # ------------------------------------------------------------------------------- one step

    def step_async(self) -> None:
        """Enqueue one iteration on the current stream (no synchronization)."""
        self._apply_launch_config()
        a = self.adam
        if self.single_pass:
            self.r.l1_grad_into(self.rend, self.target, self.loss, self.grad_params, self.saved)
        elif self.fused:
            self.r.render_l1_into(self.rend, self.target, self.image, self.loss, self.saved)
            self.r.backward_l1_into(self.rend, self.saved, self.grad_params)
        else:
            self.r.render_into(self.rend, self.image, self.saved)
            if self.ssim_weight > 0:
                nat.igs_l1_ssim_loss_grad(self.image, self.target, self.n, self.H, self.W,
                                          self.ssim_weight, self.grad_image, self.loss,
                                          self.l1_ws, self.l1_ws.numel())
            else:
                nat.igs_l1_loss_grad(self.image, self.target, self.n, self.H, self.W,
                                     self.grad_image, self.loss, self.l1_ws, self.l1_ws.numel())
            self.r.backward_into(self.rend, self.image, self.grad_image, self.saved,
                                 self.grad_params)
        # an iteration whose render overflowed the pair buffer (or, two-pass, whose hit sets are
        # too long for 16-bit slots) changes nothing and does not count; the host notices from the
        # step counter, grows the buffer and repeats it (or raises)
        nat.igs_adam_step(self.fit, self.rend, self.grad_params, self.m, self.v, self.step_count,
                          self.N, self.n, self.H, self.W, a.lr_mu, a.lr_theta, a.lr_inv_scale,
                          a.lr_color, a.beta1, a.beta2, a.eps, 1.0 / max(self.H, self.W),
                          a.inv_scale_hi, skip_flag=self._skip_word())

    # --------------------------------------------------------------------------- bookkeeping

    def psnr(self) -> float:
        mse = float(self.loss[2 if self.ssim_weight > 0 else 1].item())
        return 10.0 * math.log10(1.0 / mse) if mse > 0 else math.inf

    def ssim(self) -> float:
        """SSIM of the last iteration's render (only with the SSIM term in the loss)."""
        if self.ssim_weight <= 0:
            raise RuntimeError("the loss has no SSIM term")
        return float(self.loss[3].item())

    def state_dict(self) -> dict:
        return {"fit": self.fit.clone(), "m": self.m.clone(), "v": self.v.clone(),
                "step": self.step_count.clone(), "H": self.H, "W": self.W, "K": self.K,
                "growth": list(self.growth),
                "gen": None if self.gen is None else self.gen.get_state()}

    def load_state_dict(self, sd: dict) -> None:
        N = int(sd["fit"].shape[1])
        if N != self.N:
            self._resize(N)
            self.fit.copy_(sd["fit"])
            nat.igs_fit_to_render(self.fit, self.rend, self.N, self.n, self.H, self.W)
            self._size_pairs()
        self.fit.copy_(sd["fit"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step_count.copy_(sd["step"])
        nat.igs_fit_to_render(self.fit, self.rend, self.N, self.n, self.H, self.W)
        self.growth = list(sd.get("growth", []))
        if sd.get("gen") is not None:
            if self.gen is None:
                self.gen = torch.Generator(device=self.dev)
            self.gen.set_state(sd["gen"])


class BatchFitter(_FitLoop):
    """Fits many images of uneven size and Gaussian count at once: every iteration is one batched
    render, one batched L1 gradient, one batched adjoint and one batched Adam step (one launch per
    phase over all images), captured as one HIP graph.  Each image is fitted exactly as a
    ``PlainFitter`` would fit it alone."""

    def __init__(self, targets: List[torch.Tensor], render_params: List[torch.Tensor], K: int = 10,
                 adam: Optional[AdamConfig] = None, headroom: float = 1.25,
                 pair_capacity: Optional[int] = None, device=None, fused: Optional[bool] = None,
                 ssim_weight: float = 0.0, single_pass: bool = False):
        from .render import BatchRenderer
        self.dev = torch.device(device) if device is not None else targets[0].device
        self.n = int(targets[0].shape[0])
        self.K = K
        self.adam = adam or AdamConfig()
        self.ssim_weight = float(ssim_weight)
        if self.ssim_weight < 0:
            raise ValueError("ssim_weight must be >= 0")
        if self.ssim_weight > 0 and fused:
            raise ValueError("the SSIM term is not fused into the render pass")
        if self.ssim_weight > 0:
            self.fused = False
        else:
            self.fused = (self.n <= MAX_FUSED_CHANNELS) if fused is None else bool(fused)
        self.single_pass = _check_single_pass(single_pass, self.ssim_weight, self.fused, self.n)
        sizes = [(int(t.shape[1]), int(t.shape[2]), int(p.shape[1]))
                 for t, p in zip(targets, render_params)]
        self.r = BatchRenderer(sizes, self.n, K, pair_capacity=pair_capacity, device=self.dev)
        self.B, self.N = self.r.B, self.r.N
        self.target = self.r.pack_images(targets)
        rend = self.r.pack_params(render_params)
        # fitter parameterization: mean / (W, H) of its own image, inverse scales
        self.fit = rend.clone()
        for (H, W, N), go in zip(sizes, self.r.gauss_off):
            self.fit[0, go:go + N] /= W
            self.fit[1, go:go + N] /= H
        self.fit[3:5] = 1.0 / self.fit[3:5]
        self.rend = torch.empty_like(self.fit)
        nat.igs_fit_to_render_batched(self.fit, self.rend, self.r.descs, self.r.d_descs, self.n)
        self.m = torch.zeros_like(self.fit)
        self.v = torch.zeros_like(self.fit)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.image = self.r.new_images()
        self.grad_image = torch.empty_like(self.image)
        self.grad_params = torch.empty_like(self.fit)
        # L1 alone: per image [mean |x - y|, MSE]; with SSIM: [L, mean |x - y|, MSE, SSIM]
        self.loss = torch.zeros((self.B, 4 if self.ssim_weight > 0 else 2), dtype=torch.float64,
                                device=self.dev)
        if self.ssim_weight > 0:
            self.l1_ws = _aligned_bytes(
                nat.igs_l1_ssim_batched_workspace_size(self.r.descs, self.n), self.dev)
        else:
            self.l1_ws = _aligned_bytes(nat.igs_l1_batched_workspace_size(self.r.descs, self.n),
                                        self.dev)
        if pair_capacity is None:
            _, saved = self.r.render(self.rend)
            P = int(self.r.status_of(saved)[nat.STAT_PAIRS])
            self.r.set_capacity(max(1024, int(P * headroom)))
        self.saved = self.r.new_saved()
        self.graph = None
        self.status_host = torch.zeros(8, dtype=torch.int64).pin_memory()

    def step_async(self) -> None:
        self._apply_launch_config()
        a = self.adam
        r = self.r
        if self.single_pass:
            r.l1_grad_into(self.rend, self.target, self.loss, self.grad_params, self.saved)
        elif self.fused:
            r.render_l1_into(self.rend, self.target, self.image, self.loss, self.saved)
            r.backward_l1_into(self.rend, self.saved, self.grad_params)
        else:
            r.render_into(self.rend, self.image, self.saved)
            if self.ssim_weight > 0:
                nat.igs_l1_ssim_loss_grad_batched(self.image, self.target, r.descs, r.d_descs,
                                                  self.n, self.ssim_weight, self.grad_image,
                                                  self.loss, self.l1_ws, self.l1_ws.numel())
            else:
                nat.igs_l1_loss_grad_batched(self.image, self.target, r.descs, r.d_descs, self.n,
                                             self.grad_image, self.loss, self.l1_ws,
                                             self.l1_ws.numel())
            r.backward_into(self.rend, self.image, self.grad_image, self.saved, self.grad_params)
        nat.igs_adam_step_batched(self.fit, self.rend, self.grad_params, self.m, self.v,
                                  self.step_count, r.descs, r.d_descs, self.n, a.lr_mu, a.lr_theta,
                                  a.lr_inv_scale, a.lr_color, a.beta1, a.beta2, a.eps,
                                  a.inv_scale_hi, skip_flag=self._skip_word())

    def psnrs(self) -> List[float]:
        mse = self.loss[:, 2 if self.ssim_weight > 0 else 1].cpu().tolist()
        return [10.0 * math.log10(1.0 / m) if m > 0 else math.inf for m in mse]

    def psnr(self) -> float:
        """Mean PSNR over the batch (per-image values: ``psnrs``)."""
        return sum(self.psnrs()) / self.B

    def image_params(self, b: int) -> torch.Tensor:
        go, N = self.r.gauss_off[b], self.r.sizes[b][2]
        return self.rend[:, go:go + N]

    def state_dict(self) -> dict:
        return {"fit": self.fit.clone(), "m": self.m.clone(), "v": self.v.clone(),
                "step": self.step_count.clone(), "sizes": list(self.r.sizes), "K": self.K}

    def load_state_dict(self, sd: dict) -> None:
        self.fit.copy_(sd["fit"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step_count.copy_(sd["step"])
        nat.igs_fit_to_render_batched(self.fit, self.rend, self.r.descs, self.r.d_descs, self.n)
