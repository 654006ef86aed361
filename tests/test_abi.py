"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function the
header declares, and validates arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imagegs.h")


@pytest.fixture(scope="module")
def nat():
    from paper_2407_01866_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2407_01866_amd import build
        build.build()
    _native.lib()
    return _native


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(igs_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(nat):
    names = declared_functions()
    assert len(names) >= 9
    L = ctypes.CDLL(nat.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(nat.EXPORTED)


def test_bounds_checked_build_exports_the_same_symbols(nat):
    """The bounds-checked build (libimagegs_debug.so) has the same C ABI; the normal build
    reports that it has no checks."""
    if not os.path.exists(nat.LIB_DEBUG_PATH):
        from paper_2407_01866_amd import build
        build.build(debug=True)
    D = nat.load(nat.LIB_DEBUG_PATH)
    for name in declared_functions():
        assert hasattr(D, name), name
    out = ctypes.c_uint32(7)
    assert nat.lib().igs_bounds_violations(ctypes.byref(out)) == nat.IGS_ERR_UNSUPPORTED
    assert out.value == 0
    assert nat.lib().igs_bounds_violations(None) == nat.IGS_ERR_INVALID_ARG
    assert D.igs_abi_version() == nat.igs_abi_version()


def test_abi_version_and_status_strings(nat):
    assert nat.igs_abi_version() == 3
    assert nat.igs_status_string(0) == "ok"
    for s in (-1, -2, -3, -4):
        assert nat.igs_status_string(s) not in ("ok", "unknown status")


def test_buffer_sizes_scale_with_problem(nat):
    ws1, sv1 = nat.igs_render_buffer_sizes(1000, 3, 256, 256, 10, 16, 16, 20000)
    ws2, sv2 = nat.igs_render_buffer_sizes(1000, 3, 256, 256, 10, 16, 16, 40000)
    assert ws2 > ws1 and sv2 > sv1
    ws3, sv3 = nat.igs_render_buffer_sizes(1000, 3, 512, 256, 10, 16, 16, 20000)
    assert sv3 > sv1
    off = nat.igs_saved_offsets(1000, 3, 256, 256, 10, 16, 16, 20000)
    assert off["status"] == 0 and off["total"] == sv1
    assert off["ranges"] < off["vals"] < off["slots"] < off["aux"] < off["total"]
    assert all(v % 256 == 0 for v in off.values())
    # slots hold K uint16 per pixel
    assert off["aux"] - off["slots"] >= 10 * 256 * 256 * 2


@pytest.mark.parametrize("args,code", [
    ((-1, 3, 16, 16, 10, 16, 16, 100), -1),
    ((10, 0, 16, 16, 10, 16, 16, 100), -1),
    ((10, 33, 16, 16, 10, 16, 16, 100), -1),
    ((10, 3, 0, 16, 10, 16, 16, 100), -1),
    ((10, 3, 16, 16, 0, 16, 16, 100), -1),
    ((10, 3, 16, 16, 33, 16, 16, 100), -1),
    ((10, 3, 16, 16, 10, 16, 16, 0), -1),
    ((10, 3, 16, 16, 10, 16, 16, 1 << 31), -1),
    ((10, 3, 16, 16, 10, 8, 8, 100), -4),
    ((10, 3, 16, 16, 10, 32, 16, 100), -4),
])
def test_size_query_rejects_bad_arguments(nat, args, code):
    with pytest.raises(nat.IGSError) as e:
        nat.igs_render_buffer_sizes(*args)
    assert e.value.status == code


def test_render_validates_before_device_work(nat):
    L = nat.lib()
    # NULL image / workspace: rejected synchronously, no HIP call is made
    assert L.igs_render(None, 0, 3, 16, 16, 10, 16, 16, 100, None, None, 0, None, 0, None) == -1
    assert L.igs_render(None, 0, 3, 16, 16, 10, 8, 8, 100, None, None, 0, None, 0, None) == -4
    assert L.igs_render_backward(None, 5, 3, 16, 16, 10, 16, 16, 100, None, None, None, 0, None,
                                 None, 0, None) == -1
    assert L.igs_l1_loss_grad(None, None, 3, 4, 4, None, None, None, 0, None) == -1
    assert L.igs_adam_step(None, None, None, None, None, None, None, 4, 3, 8, 8, 1e-3, 1e-3, 1e-3,
                           1e-3, 0.9, 0.999, 1e-8, 0.1, 4.0, None) == -1
    assert L.igs_fit_to_render(None, None, 4, 0, 8, 8, None) == -1
    assert L.igs_grad_to_fit(None, None, None, 4, 3, 8, 8, None) == -1
    assert L.igs_grad_to_fit(None, None, None, 4, 0, 8, 8, None) == -1
    # fused render + L1: saved state and target are required, n is limited to 16 channels
    assert L.igs_render_l1(None, 0, 3, 16, 16, 10, 16, 16, 100, None, None, None, None, 0, None, 0,
                           None) == -1
    assert L.igs_render_l1(None, 0, 17, 16, 16, 10, 16, 16, 100, None, None, None, None, 0, None,
                           0, None) == -4
    assert L.igs_render_backward_l1(None, 5, 3, 16, 16, 10, 16, 16, 100, None, 0, None, None, 0,
                                    None) == -1
    assert L.igs_render_backward_l1(None, 5, 17, 16, 16, 10, 16, 16, 100, None, 0, None, None, 0,
                                    None) == -4
    # single-pass L1 evaluation: target, loss, gradient, saved state and workspace are required,
    # n is limited to 16 channels, and a batch must describe itself consistently
    assert L.igs_render_l1_grad(None, 0, 3, 16, 16, 10, 16, 16, 100, None, None, None, None, 0,
                                None, 0, None) == -1
    assert L.igs_render_l1_grad(None, 5, 3, 16, 16, 10, 16, 16, 100, None, None, None, None, 0,
                                None, 0, None) == -1
    assert L.igs_render_l1_grad(None, 0, 17, 16, 16, 10, 16, 16, 100, None, None, None, None, 0,
                                None, 0, None) == -4
    assert L.igs_render_l1_grad(None, 0, 3, 16, 16, 10, 8, 8, 100, None, None, None, None, 0,
                                None, 0, None) == -4
    descs = (nat.ImageDesc * 2)()
    tot = (ctypes.c_int64 * 4)()
    Hs, Ws, Ns = ((ctypes.c_int32 * 2)(*v) for v in ((16, 40), (16, 24), (5, 9)))
    assert L.igs_batch_describe(2, 3, Hs, Ws, Ns, descs, tot) == 0
    assert L.igs_render_l1_grad_batched(None, descs, None, 2, 3, 10, 100, None, None, None, None,
                                        0, None, 0, None) == -1
    assert L.igs_render_l1_grad_batched(None, descs, None, 2, 17, 10, 100, None, None, None, None,
                                        0, None, 0, None) == -4
    descs[1].pix_off += 1
    assert L.igs_render_l1_grad_batched(None, descs, None, 2, 3, 10, 100, None, None, None, None,
                                        0, None, 0, None) == -1
    sz = ctypes.c_size_t(0)
    assert L.igs_l1_workspace_size(0, ctypes.byref(sz)) == -1
    assert L.igs_l1_workspace_size(1000, ctypes.byref(sz)) == 0 and sz.value >= 16


def test_noalloc_single_pass_validates_before_device_work(nat):
    """The no-allocation single-pass call rejects bad arguments, and a problem whose workspace
    would not fit its static array, before any HIP call (the fake pointers are never
    dereferenced)."""
    L = nat.lib()
    fake = ctypes.c_void_p(0x1000)
    args = lambda n=3, tile=16, cap=100, tgt=fake, saved=fake: (
        fake, 10, n, 64, 64, 10, tile, tile, cap, tgt, fake, fake, saved, 1 << 20, None)
    assert L.igs_render_l1_grad_noalloc(*args(tgt=None)) == -1
    assert L.igs_render_l1_grad_noalloc(*args(saved=None)) == -1
    assert L.igs_render_l1_grad_noalloc(*args(tile=8)) == -4
    assert L.igs_render_l1_grad_noalloc(*args(n=17)) == -4
    ws_fit, _ = nat.igs_render_buffer_sizes(10, 3, 64, 64, 10, 16, 16, 100)
    assert ws_fit <= nat.IGS_NOALLOC_SCRATCH_BYTES
    big = 1 << 24
    ws_big, _ = nat.igs_render_buffer_sizes(10, 3, 64, 64, 10, 16, 16, big)
    assert ws_big > nat.IGS_NOALLOC_SCRATCH_BYTES
    assert L.igs_render_l1_grad_noalloc(*args(cap=big)) == -2


def test_l1_ssim_validates_before_device_work(nat):
    L = nat.lib()
    sz = ctypes.c_size_t(0)
    assert L.igs_l1_ssim_workspace_size(0, 8, 8, ctypes.byref(sz)) == -1
    assert L.igs_l1_ssim_workspace_size(3, 100, 70, ctypes.byref(sz)) == 0
    # three fp32 maps of the image and the per-block sums
    assert sz.value >= 3 * 3 * 100 * 70 * 4 + 3 * 8
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation
    assert L.igs_l1_ssim_loss_grad(None, fake, 3, 8, 8, 0.1, fake, fake, fake, 1 << 20, None) == -1
    assert L.igs_l1_ssim_loss_grad(fake, fake, 3, 8, 8, -0.1, fake, fake, fake, 1 << 20,
                                   None) == -1
    assert L.igs_l1_ssim_loss_grad(fake, fake, 3, 8, 8, float("nan"), fake, fake, fake, 1 << 20,
                                   None) == -1
    assert L.igs_l1_ssim_loss_grad(fake, fake, 0, 8, 8, 0.1, fake, fake, fake, 1 << 20, None) == -1
    assert L.igs_l1_ssim_loss_grad(fake, fake, 3, 8, 8, 0.1, fake, fake, fake, 16, None) == -2


def test_placement_validates_before_device_work(nat):
    L = nat.lib()
    sz = ctypes.c_size_t(0)
    assert L.igs_place_workspace_size(0, 8, ctypes.byref(sz)) == -1
    assert L.igs_place_workspace_size(100, 70, ctypes.byref(sz)) == 0 and sz.value >= 2 * 7000 * 8
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation
    big = 1 << 30
    # first + count beyond N_total, negative count, bad lambda, bad scale, no target
    assert L.igs_init_gaussians(fake, 3, 8, 8, 0.3, fake, 10, 5.0, fake, None, 15, 6, fake, big,
                                None) == -1
    assert L.igs_init_gaussians(fake, 3, 8, 8, 0.3, fake, -1, 5.0, fake, None, 15, 0, fake, big,
                                None) == -1
    assert L.igs_init_gaussians(fake, 3, 8, 8, 1.5, fake, 10, 5.0, fake, None, 15, 0, fake, big,
                                None) == -1
    assert L.igs_init_gaussians(fake, 3, 8, 8, 0.3, fake, 10, 0.0, fake, None, 15, 0, fake, big,
                                None) == -1
    assert L.igs_init_gaussians(None, 3, 8, 8, 0.3, fake, 10, 5.0, fake, None, 15, 0, fake, big,
                                None) == -1
    assert L.igs_init_gaussians(fake, 3, 8, 8, 0.3, fake, 10, 5.0, fake, None, 15, 0, fake, 8,
                                None) == -2
    assert L.igs_add_gaussians(None, fake, 3, 8, 8, fake, 10, 5.0, fake, None, 15, 0, fake, big,
                               None) == -1


def test_decoding_validates_before_device_work(nat):
    L = nat.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation
    assert L.igs_bin(fake, 10, 3, 16, 16, 10, 16, 16, 100, None, 0, fake, 1 << 30, None) == -1
    assert L.igs_bin(fake, 10, 3, 16, 16, 10, 8, 8, 100, fake, 1 << 30, fake, 1 << 30, None) == -4
    assert L.igs_query(fake, 10, 3, 16, 16, 10, 16, 16, 100, fake, 1 << 30, None, 5, fake,
                       None, 0, None) == -1
    assert L.igs_query(fake, 10, 3, 16, 16, 10, 16, 16, 100, fake, 1 << 30, fake, -1, fake,
                       None, 0, None) == -1
    assert L.igs_query(fake, 10, 3, 16, 16, 10, 16, 16, 100, fake, 64, fake, 5, fake, None, 0,
                       None) == -2
    # a sorting workspace that is too small
    assert L.igs_query(fake, 10, 3, 16, 16, 10, 16, 16, 100, fake, 1 << 30, fake, 5, fake, fake,
                       8, None) == -2
    sz = ctypes.c_size_t(0)
    assert L.igs_query_workspace_size(1000, 500, 3, 64, 64, ctypes.byref(sz)) == 0
    assert sz.value >= 16000 + 500 * 128  # the point sort and one 128-byte record per Gaussian
    assert L.igs_query_workspace_size(-1, 500, 3, 64, 64, ctypes.byref(sz)) == -1
    assert L.igs_query_workspace_size(1000, 500, 0, 64, 64, ctypes.byref(sz)) == -1
    assert L.igs_params_to_fp16(None, 10, 3, fake, None) == -1
    assert L.igs_decode_fp16(fake, 10, 3, 11, 16, 16, fake, None) == -1
    assert L.igs_decode_fp16(fake, 10, 3, 5, 0, 16, fake, None) == -1


def test_launch_config_roundtrip_and_validation(nat):
    L = nat.lib()
    try:
        nat.igs_set_launch_config(1, 6, 0, 128, 16)
        assert nat.igs_get_launch_config().as_tuple() == (1, 6, 0, 128, 16)
        for bad in ((2, 0, 1), (0, -1, 1), (0, 65, 1), (0, 0, 2), (0, 0, 1, 32), (0, 0, 1, 288),
                    (0, 0, 1, 100), (0, 0, 1, 0, -1), (0, 0, 1, 0, 33)):
            with pytest.raises(nat.IGSError) as e:
                nat.igs_set_launch_config(*bad)
            assert e.value.status == -1
        assert nat.igs_get_launch_config().as_tuple() == (1, 6, 0, 128, 16)
        assert L.igs_set_launch_config(None) == -1 and L.igs_get_launch_config(None) == -1
    finally:
        nat.igs_set_launch_config(0, 0, 1)
    assert nat.igs_get_launch_config().as_tuple() == (0, 0, 1, 0, 0)


def test_launch_config_is_per_host_thread(nat):
    """A setting made on one thread leaves every other thread's settings alone, and a new thread
    starts from the defaults."""
    import threading
    seen = {}

    def worker():
        seen["start"] = nat.igs_get_launch_config().as_tuple()
        nat.igs_set_launch_config(1, 5, 0)
        seen["set"] = nat.igs_get_launch_config().as_tuple()

    try:
        nat.igs_set_launch_config(1, 8, 1)
        t = threading.Thread(target=worker)
        t.start()
        t.join()
        assert seen == {"start": (0, 0, 1, 0, 0), "set": (1, 5, 0, 0, 0)}
        assert nat.igs_get_launch_config().as_tuple() == (1, 8, 1, 0, 0)
    finally:
        nat.igs_set_launch_config(0, 0, 1)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2407_01866_amd import _native
    monkeypatch.setattr(_native, "_lib", None)
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        _native.lib()
