"""ctypes binding of libimagegs.so (include/imagegs.h).  Argument marshalling only: every step of
the renderer runs in the library's HIP kernels; torch tensors are used for device memory and the
current HIP stream.  Importing works without a GPU; calling the compute entry points needs one.
There is no fallback: a missing library raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libimagegs.so")
# the bounds-checked build of the same sources (build.py --debug); see igs_bounds_violations
LIB_DEBUG_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libimagegs_debug.so")

IGS_OK = 0
IGS_ERR_INVALID_ARG = -1
IGS_ERR_WORKSPACE = -2
IGS_ERR_HIP = -3
IGS_ERR_UNSUPPORTED = -4
IGS_MAX_K = 32
IGS_MAX_CHANNELS = 32
IGS_TILE = 16
IGS_STATUS_WORDS = 8
IGS_NOALLOC_SCRATCH_BYTES = 64 << 20

# status block words (int64 at byte 0 of the saved state)
(STAT_PAIRS, STAT_OVERFLOW, STAT_MAX_LIST, STAT_SLOT_OVERFLOW, STAT_EVALS_FWD, STAT_EVALS_BWD,
 STAT_SKIP) = range(7)

EXPORTED = ("igs_abi_version", "igs_status_string", "igs_render_buffer_sizes", "igs_saved_offsets",
            "igs_render",
            "igs_render_backward", "igs_l1_workspace_size", "igs_l1_loss_grad", "igs_adam_step",
            "igs_fit_to_render", "igs_grad_to_fit", "igs_bounds_violations",
            "igs_timing_enable", "igs_timing_read", "igs_batch_describe",
            "igs_batch_buffer_sizes", "igs_batch_saved_offsets", "igs_render_batched",
            "igs_render_backward_batched", "igs_l1_batched_workspace_size",
            "igs_l1_loss_grad_batched", "igs_adam_step_batched", "igs_fit_to_render_batched",
            "igs_render_l1", "igs_render_backward_l1", "igs_render_l1_batched",
            "igs_render_backward_l1_batched", "igs_set_launch_config", "igs_get_launch_config",
            "igs_l1_ssim_workspace_size", "igs_l1_ssim_loss_grad", "igs_place_workspace_size",
            "igs_init_gaussians", "igs_add_gaussians", "igs_bin", "igs_query",
            "igs_query_workspace_size", "igs_l1_ssim_batched_workspace_size",
            "igs_l1_ssim_loss_grad_batched",
            "igs_params_to_fp16", "igs_decode_fp16", "igs_render_l1_grad",
            "igs_render_l1_grad_noalloc",
            "igs_render_l1_grad_batched")

PHASES = ("binning", "raster_fwd", "raster_bwd", "loss", "adam", "grad_reduce", "raster_fit")


class ImageDesc(ctypes.Structure):
    """Mirror of igs_image_desc (include/imagegs.h)."""
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("N", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("tile_off", ctypes.c_int32), ("gauss_off", ctypes.c_int32),
                ("l1_block_off", ctypes.c_int32), ("pix_off", ctypes.c_int64),
                ("ssim_block_off", ctypes.c_int64)]


class LaunchConfig(ctypes.Structure):
    """Mirror of igs_launch_config (include/imagegs.h)."""
    _fields_ = [("persistent", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("fwd_cull", ctypes.c_int32), ("fwd_batch", ctypes.c_int32),
                ("k_unroll", ctypes.c_int32)]

    def as_tuple(self):
        return (self.persistent, self.wgs_per_cu, self.fwd_cull, self.fwd_batch, self.k_unroll)

    def __repr__(self):
        return (f"LaunchConfig(persistent={self.persistent}, wgs_per_cu={self.wgs_per_cu}, "
                f"fwd_cull={self.fwd_cull}, fwd_batch={self.fwd_batch}, "
                f"k_unroll={self.k_unroll})")


class IGSError(RuntimeError):
    def __init__(self, func: str, status: int):
        super().__init__(f"{func} failed: {status} ({_status_name(status)})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The library every wrapper below calls (libimagegs.so unless `using` selected another)."""
    global _lib
    if _lib is not None:
        return _lib
    _lib = load(LIB_PATH)
    return _lib


class using:
    """Context manager: the wrappers call the given loaded library (e.g. load(LIB_DEBUG_PATH))
    inside the block, and the previous one afterwards."""

    def __init__(self, L: ctypes.CDLL):
        self.L, self.prev = L, None

    def __enter__(self):
        global _lib
        self.prev, _lib = _lib, self.L
        return self.L

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev
        return False


def load(path: str) -> ctypes.CDLL:
    """Loads a build of libimagegs and declares its entry points (argument marshalling only)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python paper_2407_01866_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(path)
    i32, i64, sz, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    f32 = ctypes.c_float
    L.igs_abi_version.argtypes = []
    L.igs_abi_version.restype = i32
    L.igs_status_string.argtypes = [i32]
    L.igs_status_string.restype = ctypes.c_char_p
    L.igs_render_buffer_sizes.argtypes = [i32, i32, i32, i32, i32, i32, i32, i64,
                                          ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.igs_render_buffer_sizes.restype = i32
    L.igs_saved_offsets.argtypes = [i32, i32, i32, i32, i32, i32, i32, i64, ctypes.POINTER(i64)]
    L.igs_saved_offsets.restype = i32
    L.igs_render.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, vp, sz, vp, sz, vp]
    L.igs_render.restype = i32
    L.igs_render_backward.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, vp, vp, sz,
                                      vp, vp, sz, vp]
    L.igs_render_backward.restype = i32
    L.igs_l1_workspace_size.argtypes = [i64, ctypes.POINTER(sz)]
    L.igs_l1_workspace_size.restype = i32
    L.igs_l1_loss_grad.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]
    L.igs_l1_loss_grad.restype = i32
    L.igs_l1_ssim_workspace_size.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
    L.igs_l1_ssim_workspace_size.restype = i32
    L.igs_l1_ssim_loss_grad.argtypes = [vp, vp, i32, i32, i32, ctypes.c_double, vp, vp, vp, sz,
                                        vp]
    L.igs_l1_ssim_loss_grad.restype = i32
    L.igs_bin.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, sz, vp, sz, vp]
    L.igs_bin.restype = i32
    L.igs_query.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, sz, vp, i32, vp, vp,
                            sz, vp]
    L.igs_query_workspace_size.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.igs_query_workspace_size.restype = i32
    L.igs_query.restype = i32
    L.igs_params_to_fp16.argtypes = [vp, i32, i32, vp, vp]
    L.igs_params_to_fp16.restype = i32
    L.igs_decode_fp16.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    L.igs_decode_fp16.restype = i32
    L.igs_place_workspace_size.argtypes = [i32, i32, ctypes.POINTER(sz)]
    L.igs_place_workspace_size.restype = i32
    L.igs_init_gaussians.argtypes = [vp, i32, i32, i32, ctypes.c_double, vp, i32, f32, vp, vp, i32,
                                     i32, vp, sz, vp]
    L.igs_init_gaussians.restype = i32
    L.igs_add_gaussians.argtypes = [vp, vp, i32, i32, i32, vp, i32, f32, vp, vp, i32, i32, vp, sz,
                                    vp]
    L.igs_add_gaussians.restype = i32
    L.igs_adam_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, f32, f32, f32, f32,
                                f32, f32, f32, f32, f32, vp]
    L.igs_adam_step.restype = i32
    L.igs_fit_to_render.argtypes = [vp, vp, i32, i32, i32, i32, vp]
    L.igs_fit_to_render.restype = i32
    L.igs_grad_to_fit.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
    L.igs_grad_to_fit.restype = i32
    dp = ctypes.POINTER(ImageDesc)
    i32p = ctypes.POINTER(i32)
    L.igs_l1_ssim_batched_workspace_size.argtypes = [dp, i32, i32, ctypes.POINTER(sz)]
    L.igs_l1_ssim_batched_workspace_size.restype = i32
    L.igs_l1_ssim_loss_grad_batched.argtypes = [vp, vp, dp, vp, i32, i32, ctypes.c_double, vp, vp,
                                                vp, sz, vp]
    L.igs_l1_ssim_loss_grad_batched.restype = i32
    L.igs_batch_describe.argtypes = [i32, i32, i32p, i32p, i32p, dp, ctypes.POINTER(i64)]
    L.igs_batch_describe.restype = i32
    L.igs_batch_buffer_sizes.argtypes = [dp, i32, i32, i32, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.igs_batch_buffer_sizes.restype = i32
    L.igs_batch_saved_offsets.argtypes = [dp, i32, i32, i32, i64, ctypes.POINTER(i64)]
    L.igs_batch_saved_offsets.restype = i32
    L.igs_render_batched.argtypes = [vp, dp, vp, i32, i32, i32, i64, vp, vp, sz, vp, sz, vp]
    L.igs_render_batched.restype = i32
    L.igs_render_backward_batched.argtypes = [vp, dp, vp, i32, i32, i32, i64, vp, vp, vp, sz, vp,
                                              vp, sz, vp]
    L.igs_render_backward_batched.restype = i32
    L.igs_l1_batched_workspace_size.argtypes = [dp, i32, i32, ctypes.POINTER(sz)]
    L.igs_l1_batched_workspace_size.restype = i32
    L.igs_l1_loss_grad_batched.argtypes = [vp, vp, dp, vp, i32, i32, vp, vp, vp, sz, vp]
    L.igs_l1_loss_grad_batched.restype = i32
    L.igs_adam_step_batched.argtypes = [vp, vp, vp, vp, vp, vp, vp, dp, vp, i32, i32, f32, f32, f32,
                                        f32, f32, f32, f32, f32, vp]
    L.igs_adam_step_batched.restype = i32
    L.igs_fit_to_render_batched.argtypes = [vp, vp, dp, vp, i32, i32, vp]
    L.igs_fit_to_render_batched.restype = i32
    L.igs_render_l1.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, vp, vp, vp, sz, vp,
                                sz, vp]
    L.igs_render_l1.restype = i32
    L.igs_render_backward_l1.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, sz, vp, vp,
                                         sz, vp]
    L.igs_render_backward_l1.restype = i32
    L.igs_render_l1_batched.argtypes = [vp, dp, vp, i32, i32, i32, i64, vp, vp, vp, vp, sz, vp, sz,
                                        vp]
    L.igs_render_l1_batched.restype = i32
    L.igs_render_backward_l1_batched.argtypes = [vp, dp, vp, i32, i32, i32, i64, vp, sz, vp, vp,
                                                 sz, vp]
    L.igs_render_backward_l1_batched.restype = i32
    L.igs_render_l1_grad.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, vp, vp, vp,
                                     sz, vp, sz, vp]
    L.igs_render_l1_grad.restype = i32
    L.igs_render_l1_grad_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i64, vp, vp,
                                             vp, vp, sz, vp]
    L.igs_render_l1_grad_noalloc.restype = i32
    L.igs_render_l1_grad_batched.argtypes = [vp, dp, vp, i32, i32, i32, i64, vp, vp, vp, vp, sz,
                                             vp, sz, vp]
    L.igs_render_l1_grad_batched.restype = i32
    L.igs_set_launch_config.argtypes = [ctypes.POINTER(LaunchConfig)]
    L.igs_set_launch_config.restype = i32
    L.igs_get_launch_config.argtypes = [ctypes.POINTER(LaunchConfig)]
    L.igs_get_launch_config.restype = i32
    L.igs_timing_enable.argtypes = [i32]
    L.igs_timing_enable.restype = i32
    L.igs_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
    L.igs_timing_read.restype = i32
    L.igs_bounds_violations.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    L.igs_bounds_violations.restype = i32
    return L


def _status_name(s: int) -> str:
    try:
        return lib().igs_status_string(s).decode()
    except Exception:  # pragma: no cover - only while reporting another failure
        return "?"


def _check(func: str, s: int) -> None:
    if s != IGS_OK:
        raise IGSError(func, s)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _f32(t: torch.Tensor, name: str) -> int:
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return _ptr(t)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


# ------------------------------------------------------------------------------- entry points


def igs_abi_version() -> int:
    return lib().igs_abi_version()


def igs_status_string(s: int) -> str:
    return lib().igs_status_string(s).decode()


def igs_render_buffer_sizes(N: int, n: int, H: int, W: int, K: int, tile_h: int = IGS_TILE,
                            tile_w: int = IGS_TILE, pair_capacity: int = 1) -> Tuple[int, int]:
    ws, sv = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check("igs_render_buffer_sizes",
           lib().igs_render_buffer_sizes(N, n, H, W, K, tile_h, tile_w, pair_capacity,
                                         ctypes.byref(ws), ctypes.byref(sv)))
    return ws.value, sv.value


def igs_saved_offsets(N: int, n: int, H: int, W: int, K: int, tile_h: int = IGS_TILE,
                      tile_w: int = IGS_TILE, pair_capacity: int = 1) -> dict:
    out = (ctypes.c_int64 * 6)()
    _check("igs_saved_offsets",
           lib().igs_saved_offsets(N, n, H, W, K, tile_h, tile_w, pair_capacity, out))
    return dict(zip(("status", "ranges", "vals", "slots", "aux", "total"), list(out)))


def igs_render(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, image, saved, saved_bytes,
               workspace, ws_bytes, stream=None) -> None:
    _check("igs_render", lib().igs_render(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _f32(image, "image"), _ptr(saved), saved_bytes, _ptr(workspace), ws_bytes,
        _stream(stream)))


def igs_render_backward(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, image, grad_image,
                        saved, saved_bytes, grad_params, workspace, ws_bytes, stream=None) -> None:
    _check("igs_render_backward", lib().igs_render_backward(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _f32(image, "image"), _f32(grad_image, "grad_image"), _ptr(saved), saved_bytes,
        _f32(grad_params, "grad_params") if N > 0 else None, _ptr(workspace), ws_bytes,
        _stream(stream)))


def igs_render_l1(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, target, image, loss_out,
                  saved, saved_bytes, workspace, ws_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[2]")
    _check("igs_render_l1", lib().igs_render_l1(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _f32(target, "target"), _f32(image, "image"), _ptr(loss_out), _ptr(saved), saved_bytes,
        _ptr(workspace), ws_bytes, _stream(stream)))


def igs_render_backward_l1(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, saved,
                           saved_bytes, grad_params, workspace, ws_bytes, stream=None) -> None:
    _check("igs_render_backward_l1", lib().igs_render_backward_l1(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _ptr(saved), saved_bytes, _f32(grad_params, "grad_params") if N > 0 else None,
        _ptr(workspace), ws_bytes, _stream(stream)))


def igs_render_l1_grad(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, target, loss_out,
                       grad_params, saved, saved_bytes, workspace, ws_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[2]")
    _check("igs_render_l1_grad", lib().igs_render_l1_grad(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _f32(target, "target"), _ptr(loss_out), _f32(grad_params, "grad_params") if N > 0 else None,
        _ptr(saved), saved_bytes, _ptr(workspace), ws_bytes, _stream(stream)))


def igs_render_l1_grad_noalloc(params, N, n, H, W, K, tile_h, tile_w, pair_capacity, target,
                               loss_out, grad_params, saved, saved_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[2]")
    _check("igs_render_l1_grad_noalloc", lib().igs_render_l1_grad_noalloc(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, pair_capacity,
        _f32(target, "target"), _ptr(loss_out), _f32(grad_params, "grad_params") if N > 0 else None,
        _ptr(saved), saved_bytes, _stream(stream)))


def igs_l1_workspace_size(count: int) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_l1_workspace_size", lib().igs_l1_workspace_size(count, ctypes.byref(ws)))
    return ws.value


def igs_l1_loss_grad(image, target, n, H, W, grad_image, loss_out, workspace, ws_bytes,
                     stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[2]")
    _check("igs_l1_loss_grad", lib().igs_l1_loss_grad(
        _f32(image, "image"), _f32(target, "target"), n, H, W, _f32(grad_image, "grad_image"),
        _ptr(loss_out), _ptr(workspace), ws_bytes, _stream(stream)))


def igs_l1_ssim_workspace_size(n: int, H: int, W: int) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_l1_ssim_workspace_size",
           lib().igs_l1_ssim_workspace_size(n, H, W, ctypes.byref(ws)))
    return ws.value


def igs_l1_ssim_loss_grad(image, target, n, H, W, ssim_weight, grad_image, loss_out, workspace,
                          ws_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64 or loss_out.numel() < 4:
        raise TypeError("loss_out must be float64[4]")
    _check("igs_l1_ssim_loss_grad", lib().igs_l1_ssim_loss_grad(
        _f32(image, "image"), _f32(target, "target"), n, H, W, float(ssim_weight),
        _f32(grad_image, "grad_image"), _ptr(loss_out), _ptr(workspace), ws_bytes,
        _stream(stream)))


def igs_bin(params, N, n, H, W, K, tile_h, tile_w, cap, saved, saved_bytes, workspace, ws_bytes,
            stream=None) -> None:
    _check("igs_bin", lib().igs_bin(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, cap,
        _ptr(saved), saved_bytes, _ptr(workspace), ws_bytes, _stream(stream)))


def igs_query_workspace_size(M: int, N: int, n: int, H: int, W: int) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_query_workspace_size",
           lib().igs_query_workspace_size(M, N, n, H, W, ctypes.byref(ws)))
    return ws.value


def igs_query(params, N, n, H, W, K, tile_h, tile_w, cap, saved, saved_bytes, points, M, out,
              workspace=None, ws_bytes=0, stream=None) -> None:
    _check("igs_query", lib().igs_query(
        _f32(params, "params") if N > 0 else None, N, n, H, W, K, tile_h, tile_w, cap,
        _ptr(saved), saved_bytes, _f32(points, "points") if M > 0 else None, M,
        _f32(out, "out") if M > 0 else None, _ptr(workspace), ws_bytes, _stream(stream)))


def igs_params_to_fp16(params, N, n, out, stream=None) -> None:
    if out.dtype not in (torch.int16, torch.float16):
        raise TypeError("out must be a 16-bit tensor")
    _check("igs_params_to_fp16", lib().igs_params_to_fp16(
        _f32(params, "params") if N > 0 else None, N, n, _ptr(out) if N > 0 else None,
        _stream(stream)))


def igs_decode_fp16(stored, N_stored, n, N_prefix, H, W, render_params, stream=None) -> None:
    if stored.dtype not in (torch.int16, torch.float16):
        raise TypeError("stored must be a 16-bit tensor")
    _check("igs_decode_fp16", lib().igs_decode_fp16(
        _ptr(stored), N_stored, n, N_prefix, H, W,
        _f32(render_params, "render_params") if N_prefix > 0 else None, _stream(stream)))


def igs_place_workspace_size(H: int, W: int) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_place_workspace_size", lib().igs_place_workspace_size(H, W, ctypes.byref(ws)))
    return ws.value


def igs_init_gaussians(target, n, H, W, lambda_init, uniforms, count, scale, render_params,
                       fit_params, N_total, first, workspace, ws_bytes, stream=None) -> None:
    _check("igs_init_gaussians", lib().igs_init_gaussians(
        _f32(target, "target"), n, H, W, float(lambda_init), _f32(uniforms, "uniforms"), count,
        float(scale), _f32(render_params, "render_params"),
        None if fit_params is None else _f32(fit_params, "fit_params"), N_total, first,
        _ptr(workspace), ws_bytes, _stream(stream)))


def igs_add_gaussians(image, target, n, H, W, uniforms, count, scale, render_params, fit_params,
                      N_total, first, workspace, ws_bytes, stream=None) -> None:
    _check("igs_add_gaussians", lib().igs_add_gaussians(
        _f32(image, "image"), _f32(target, "target"), n, H, W, _f32(uniforms, "uniforms"), count,
        float(scale), _f32(render_params, "render_params"),
        None if fit_params is None else _f32(fit_params, "fit_params"), N_total, first,
        _ptr(workspace), ws_bytes, _stream(stream)))


def igs_adam_step(fit_params, render_params, grad_render, m, v, step, N, n, H, W, lr_mu, lr_theta,
                  lr_inv_scale, lr_color, beta1=0.9, beta2=0.999, eps=1e-8, inv_scale_lo=None,
                  inv_scale_hi=4.0, skip_flag=None, stream=None) -> None:
    """skip_flag: optional device int64 tensor (e.g. the render status's overflow word); when
    non-zero at execution time the step changes nothing."""
    if step.dtype != torch.int32:
        raise TypeError("step must be int32[1]")
    if inv_scale_lo is None:
        inv_scale_lo = 1.0 / max(H, W)
    _check("igs_adam_step", lib().igs_adam_step(
        _f32(fit_params, "fit_params"), _f32(render_params, "render_params"),
        _f32(grad_render, "grad_render"), _f32(m, "m"), _f32(v, "v"), _ptr(step),
        _ptr(skip_flag), N, n, H, W,
        lr_mu, lr_theta, lr_inv_scale, lr_color, beta1, beta2, eps, inv_scale_lo, inv_scale_hi,
        _stream(stream)))


def igs_fit_to_render(fit_params, render_params, N, n, H, W, stream=None) -> None:
    _check("igs_fit_to_render", lib().igs_fit_to_render(
        _f32(fit_params, "fit_params"), _f32(render_params, "render_params"), N, n, H, W,
        _stream(stream)))


def igs_grad_to_fit(fit_params, grad_render, grad_fit, N, n, H, W, stream=None) -> None:
    _check("igs_grad_to_fit", lib().igs_grad_to_fit(
        _f32(fit_params, "fit_params"), _f32(grad_render, "grad_render"),
        _f32(grad_fit, "grad_fit"), N, n, H, W, _stream(stream)))


def igs_set_launch_config(persistent: int = 0, wgs_per_cu: int = 0, fwd_cull: int = 1,
                          fwd_batch: int = 0, k_unroll: int = 0) -> None:
    cfg = LaunchConfig(persistent, wgs_per_cu, fwd_cull, fwd_batch, k_unroll)
    _check("igs_set_launch_config", lib().igs_set_launch_config(ctypes.byref(cfg)))


def igs_get_launch_config() -> LaunchConfig:
    cfg = LaunchConfig()
    _check("igs_get_launch_config", lib().igs_get_launch_config(ctypes.byref(cfg)))
    return cfg


def igs_bounds_violations() -> Optional[int]:
    """The sites (bit mask) where the bounds-checked build met an out-of-range index since the
    last call, or None for a normal build (which has no checks).  Synchronizes the device."""
    out = ctypes.c_uint32(0)
    st = lib().igs_bounds_violations(ctypes.byref(out))
    if st == IGS_ERR_UNSUPPORTED:
        return None
    _check("igs_bounds_violations", st)
    return int(out.value)


def igs_timing_enable(on: bool) -> None:
    _check("igs_timing_enable", lib().igs_timing_enable(1 if on else 0))


def igs_timing_read(reset: bool = True) -> dict:
    """{phase: (total_ms, calls)} accumulated since the last reset (waits for the events)."""
    ms = (ctypes.c_double * len(PHASES))()
    calls = (ctypes.c_int64 * len(PHASES))()
    _check("igs_timing_read", lib().igs_timing_read(ms, calls, 1 if reset else 0))
    return {p: (ms[i], calls[i]) for i, p in enumerate(PHASES)}


# ------------------------------------------------------------------------------------ batches


def igs_batch_describe(H, W, N, n: int):
    """Host descriptors (ctypes array of ImageDesc) and totals (Ntot, T, pixels, loss blocks)."""
    B = len(H)
    arr = (ImageDesc * B)()
    tot = (ctypes.c_int64 * 4)()
    h = (ctypes.c_int32 * B)(*H)
    w = (ctypes.c_int32 * B)(*W)
    g = (ctypes.c_int32 * B)(*N)
    _check("igs_batch_describe", lib().igs_batch_describe(B, n, h, w, g, arr, tot))
    return arr, tuple(tot)


def descs_to_device(descs, device) -> torch.Tensor:
    """Copy host descriptors into a device byte tensor (the kernels' copy)."""
    raw = bytes(descs)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


def igs_batch_buffer_sizes(descs, n, K, pair_capacity) -> Tuple[int, int]:
    ws, sv = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check("igs_batch_buffer_sizes", lib().igs_batch_buffer_sizes(
        descs, len(descs), n, K, pair_capacity, ctypes.byref(ws), ctypes.byref(sv)))
    return ws.value, sv.value


def igs_batch_saved_offsets(descs, n, K, pair_capacity) -> dict:
    out = (ctypes.c_int64 * 7)()
    _check("igs_batch_saved_offsets",
           lib().igs_batch_saved_offsets(descs, len(descs), n, K, pair_capacity, out))
    return dict(zip(("status", "ranges", "vals", "slots", "aux", "total", "order"), list(out)))


def igs_render_batched(params, descs, d_descs, n, K, pair_capacity, images, saved, saved_bytes,
                       workspace, ws_bytes, stream=None) -> None:
    _check("igs_render_batched", lib().igs_render_batched(
        _f32(params, "params") if params.numel() else None, descs, _ptr(d_descs), len(descs), n,
        K, pair_capacity, _f32(images, "images"), _ptr(saved), saved_bytes, _ptr(workspace),
        ws_bytes, _stream(stream)))


def igs_render_backward_batched(params, descs, d_descs, n, K, pair_capacity, images, grad_images,
                                saved, saved_bytes, grad_params, workspace, ws_bytes,
                                stream=None) -> None:
    _check("igs_render_backward_batched", lib().igs_render_backward_batched(
        _f32(params, "params") if params.numel() else None, descs, _ptr(d_descs), len(descs), n,
        K, pair_capacity, _f32(images, "images"), _f32(grad_images, "grad_images"), _ptr(saved),
        saved_bytes, _f32(grad_params, "grad_params") if grad_params.numel() else None,
        _ptr(workspace), ws_bytes, _stream(stream)))


def igs_render_l1_batched(params, descs, d_descs, n, K, pair_capacity, targets, images, loss_out,
                          saved, saved_bytes, workspace, ws_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[B][2]")
    _check("igs_render_l1_batched", lib().igs_render_l1_batched(
        _f32(params, "params") if params.numel() else None, descs, _ptr(d_descs), len(descs), n,
        K, pair_capacity, _f32(targets, "targets"), _f32(images, "images"), _ptr(loss_out),
        _ptr(saved), saved_bytes, _ptr(workspace), ws_bytes, _stream(stream)))


def igs_render_backward_l1_batched(params, descs, d_descs, n, K, pair_capacity, saved, saved_bytes,
                                   grad_params, workspace, ws_bytes, stream=None) -> None:
    _check("igs_render_backward_l1_batched", lib().igs_render_backward_l1_batched(
        _f32(params, "params") if params.numel() else None, descs, _ptr(d_descs), len(descs), n,
        K, pair_capacity, _ptr(saved), saved_bytes,
        _f32(grad_params, "grad_params") if grad_params.numel() else None, _ptr(workspace),
        ws_bytes, _stream(stream)))


def igs_render_l1_grad_batched(params, descs, d_descs, n, K, pair_capacity, targets, loss_out,
                               grad_params, saved, saved_bytes, workspace, ws_bytes,
                               stream=None) -> None:
    if loss_out.dtype != torch.float64:
        raise TypeError("loss_out must be float64[B][2]")
    _check("igs_render_l1_grad_batched", lib().igs_render_l1_grad_batched(
        _f32(params, "params") if params.numel() else None, descs, _ptr(d_descs), len(descs), n,
        K, pair_capacity, _f32(targets, "targets"), _ptr(loss_out),
        _f32(grad_params, "grad_params") if grad_params.numel() else None, _ptr(saved),
        saved_bytes, _ptr(workspace), ws_bytes, _stream(stream)))


def igs_l1_batched_workspace_size(descs, n) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_l1_batched_workspace_size",
           lib().igs_l1_batched_workspace_size(descs, len(descs), n, ctypes.byref(ws)))
    return ws.value


def igs_l1_loss_grad_batched(images, targets, descs, d_descs, n, grad_images, loss_out, workspace,
                             ws_bytes, stream=None) -> None:
    _check("igs_l1_loss_grad_batched", lib().igs_l1_loss_grad_batched(
        _f32(images, "images"), _f32(targets, "targets"), descs, _ptr(d_descs), len(descs), n,
        _f32(grad_images, "grad_images"), _ptr(loss_out), _ptr(workspace), ws_bytes,
        _stream(stream)))


def igs_l1_ssim_batched_workspace_size(descs, n) -> int:
    ws = ctypes.c_size_t(0)
    _check("igs_l1_ssim_batched_workspace_size",
           lib().igs_l1_ssim_batched_workspace_size(descs, len(descs), n, ctypes.byref(ws)))
    return ws.value


def igs_l1_ssim_loss_grad_batched(images, targets, descs, d_descs, n, ssim_weight, grad_images,
                                  loss_out, workspace, ws_bytes, stream=None) -> None:
    if loss_out.dtype != torch.float64 or loss_out.numel() < 4 * len(descs):
        raise TypeError("loss_out must be float64[B][4]")
    _check("igs_l1_ssim_loss_grad_batched", lib().igs_l1_ssim_loss_grad_batched(
        _f32(images, "images"), _f32(targets, "targets"), descs, _ptr(d_descs), len(descs), n,
        float(ssim_weight), _f32(grad_images, "grad_images"), _ptr(loss_out), _ptr(workspace),
        ws_bytes, _stream(stream)))


def igs_adam_step_batched(fit_params, render_params, grad_render, m, v, step, descs, d_descs, n,
                          lr_mu, lr_theta, lr_inv_scale, lr_color, beta1=0.9, beta2=0.999,
                          eps=1e-8, inv_scale_hi=4.0, skip_flag=None, stream=None) -> None:
    _check("igs_adam_step_batched", lib().igs_adam_step_batched(
        _f32(fit_params, "fit_params"), _f32(render_params, "render_params"),
        _f32(grad_render, "grad_render"), _f32(m, "m"), _f32(v, "v"), _ptr(step),
        _ptr(skip_flag), descs, _ptr(d_descs), len(descs), n, lr_mu, lr_theta, lr_inv_scale,
        lr_color, beta1, beta2, eps, inv_scale_hi, _stream(stream)))


def igs_fit_to_render_batched(fit_params, render_params, descs, d_descs, n, stream=None) -> None:
    _check("igs_fit_to_render_batched", lib().igs_fit_to_render_batched(
        _f32(fit_params, "fit_params"), _f32(render_params, "render_params"), descs,
        _ptr(d_descs), len(descs), n, _stream(stream)))
