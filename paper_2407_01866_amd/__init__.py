"""Image-GS renderer for MI355X (gfx950): hand-written HIP kernels behind a small C ABI
(``include/imagegs.h``, ``libimagegs.so``), with a thin ctypes binding (``_native``), a
``torch.autograd.Function`` (``render.RenderFn``) and a fitter (``fit``).

Submodules are imported on use; importing the package itself touches neither the GPU nor the
native library.
"""

__all__ = ["_native", "render", "fit", "synth", "build"]
