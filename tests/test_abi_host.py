"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/disc.h, and rejects invalid arguments
and out-of-order calls before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "disc.h")


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    if not os.path.exists(d.LIB_PATH):
        from paper_1204_6295_amd import build

        build.build()
    d.lib()
    return d


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(disc_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(disc):
    names = declared_functions()
    assert len(names) >= 20
    raw = ctypes.CDLL(disc.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    bound = {s[0] for s in disc._SIGS}
    assert set(names) == bound


def test_params_struct_layout(disc):
    # int[3], float, int, int[8], int, float, float, int, float, int,
    # int, float, float, float, float, int[3], int, int
    assert ctypes.sizeof(disc.Params) == 4 * (3 + 1 + 1 + 8 + 1 + 1 + 1 + 1 + 1 + 1 + 1 + 4 + 3 + 1 + 1)


def test_defaults(disc):
    p = disc.Params()
    assert disc.lib().disc_params_default(ctypes.byref(p)) == 0
    assert list(p.patch) == [11, 11, 11] and p.sigma == 2.0 and p.levels == 3
    assert list(p.iters)[:3] == [100, 100, 100] and p.global_shift == 1
    assert p.force_mode == 0 and p.stop_eps == 0.0 and p.stop_lag == 10


@pytest.mark.parametrize("kw,msg", [
    (dict(patch=(4, 5, 5)), "odd"),
    (dict(patch=(33, 5, 5)), "odd"),
    (dict(patch=(5, 5, 17)), "pz"),
    (dict(sigma=0.0), "sigma"),
    (dict(sigma=2.7), "sigma"),
    (dict(levels=9, iters=(1,) * 8), None),
    (dict(levels=0, iters=()), "levels"),
    (dict(iters=(10, -1, 10)), "negative"),
    (dict(var_floor=float("nan")), "var_floor"),
    (dict(diff_floor=-1.0), "diff_floor"),
    (dict(force_mode=2), "force_mode"),
    (dict(stop_eps=-1e-4), "stop_eps"),
    (dict(stop_eps=1e-4, stop_lag=0), "stop_lag"),
    (dict(mask_mode=1, fill_t=(7, 6, 3)), "fill_t"),
    (dict(mask_mode=1, fill_passes=0), "fill_passes"),
    (dict(mask_mode=1, a_lo=1.5, a_hi=0.5), "a_lo"),
])
def test_create_rejects_invalid_params(disc, kw, msg):
    base = dict(patch=(11, 11, 11), sigma=2.0, levels=3, iters=(100, 100, 100))
    base.update(kw)
    p = disc.Params()
    disc.lib().disc_params_default(ctypes.byref(p))
    for d in range(3):
        p.patch[d] = base["patch"][d]
    p.sigma = base["sigma"]
    p.levels = base["levels"]
    for i, k in enumerate(base["iters"]):
        p.iters[i] = k
    p.var_floor = base.get("var_floor", 1e-2)
    p.diff_floor = base.get("diff_floor", 1e-3)
    p.force_mode = base.get("force_mode", 0)
    p.stop_eps = base.get("stop_eps", 0.0)
    p.stop_lag = base.get("stop_lag", 10)
    p.mask_mode = base.get("mask_mode", 0)
    for d, v in enumerate(base.get("fill_t", (7, 7, 3))):
        p.fill_t[d] = v
    p.fill_passes = base.get("fill_passes", 10)
    p.a_lo = base.get("a_lo", 0.5)
    p.a_hi = base.get("a_hi", 1.5)
    h = ctypes.c_void_p(1)
    rc = disc.lib().disc_create(ctypes.byref(p), ctypes.byref(h))
    assert rc == disc.DISC_EINVAL and not h.value
    if msg:
        assert msg in disc.lib().disc_last_error(None).decode()


def test_workspace_bytes(disc):
    p = disc.make_params()
    nb = disc.lib().disc_workspace_bytes(ctypes.byref(p), 256, 256, 96)
    n = 256 * 256 * 96
    # per level: shifted CBCT, standardised CBCT (+ CT below the finest); fields, m, f;
    # plus FP64 partial sums (global shift; two per z-pass workgroup for the
    # stopping rule) and the l^(k) history
    expect = 4 * (2 * n + 3 * (n // 8) + 3 * (n // 64)) + 4 * (6 * n + 2 * n)
    assert expect <= nb <= expect + 512 * 1024
    assert disc.lib().disc_workspace_bytes(ctypes.byref(p), 0, 5, 5) == 0
    assert disc.lib().disc_workspace_bytes(None, 5, 5, 5) == 0


def test_state_errors_without_gpu(disc):
    L = disc.lib()
    p = disc.make_params()
    h = ctypes.c_void_p()
    assert L.disc_create(ctypes.byref(p), ctypes.byref(h)) == 0
    try:
        assert L.disc_iterate(h, 1, None) == disc.DISC_ESTATE
        assert L.disc_run(h, None) == disc.DISC_ESTATE
        assert L.disc_get_corrected(h, ctypes.c_void_p(4096), None) == disc.DISC_ESTATE
        assert L.disc_state(h, None, None, None) == disc.DISC_ESTATE
        fake = ctypes.c_void_p(1 << 20)
        # argument errors are caught on the host before any HIP call
        assert L.disc_set_volumes(h, None, fake, 8, 8, 8, fake, 1 << 30, None) == disc.DISC_EINVAL
        assert L.disc_set_volumes(h, fake, fake, 0, 8, 8, fake, 1 << 30, None) == disc.DISC_EINVAL
        assert L.disc_set_volumes(h, fake, fake, 8, 8, 8, ctypes.c_void_p((1 << 20) + 16), 1 << 30,
                                  None) == disc.DISC_EINVAL
        assert L.disc_set_volumes(h, fake, fake, 64, 64, 64, fake, 1000, None) == disc.DISC_ENOMEM
        assert b"needs" in L.disc_last_error(h)
        assert L.disc_iterate(h, -1, None) == disc.DISC_ESTATE
        assert L.disc_timing_read(h, 9, -1, None, None, None) == disc.DISC_EINVAL
        assert L.disc_timing_enable(h, -1) == disc.DISC_EINVAL
        assert L.disc_get_stats(h, 0, None, None, 0, None) == disc.DISC_ESTATE
    finally:
        L.disc_destroy(h)
    L.disc_destroy(None)


def test_step_argument_errors_without_gpu(disc):
    L = disc.lib()
    fake = ctypes.c_void_p(1 << 20)
    patch = (ctypes.c_int * 3)(3, 3, 3)
    bad = (ctypes.c_int * 3)(3, 2, 3)
    assert L.disc_step_warp(None, fake, 4, 4, 4, fake, None) == disc.DISC_EINVAL
    assert L.disc_step_warp(fake, fake, 4, 4, 70000, fake, None) == disc.DISC_EINVAL
    assert L.disc_step_correct(fake, fake, 4, 4, 4, bad, fake, None) == disc.DISC_EINVAL
    assert L.disc_step_static_stats(fake, 4, 4, 4, patch, -1.0, fake, None) == disc.DISC_EINVAL
    assert L.disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0, float("inf"), 0, fake, fake, None,
                                    None, None, None) == disc.DISC_EINVAL
    assert L.disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0, 1e-3, 0, None, fake, None,
                                    None, None, None) == disc.DISC_EINVAL
    assert L.disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0, 1e-3, 2, fake, fake, None,
                                    None, None, None) == disc.DISC_EINVAL
    # the next iteration's warp needs both the CT and the output
    assert L.disc_step_force_smooth(fake, fake, fake, 4, 4, 4, 2.0, 1e-3, 0, fake, fake, None,
                                    fake, None, None) == disc.DISC_EINVAL
    assert L.disc_step_smooth(fake, 4, 4, 4, 3.0, fake, fake, None) == disc.DISC_EINVAL
    assert L.disc_step_shift(fake, fake, 0, fake, None, fake, 1 << 20, None) == disc.DISC_EINVAL
    assert L.disc_step_shift(fake, fake, 10, fake, None, fake, 8, None) == disc.DISC_ENOMEM
    assert L.disc_step_upsample_field(fake, 0, 1, 1, fake, 2, 2, 2, None) == disc.DISC_EINVAL
    assert L.disc_copy_kernel(fake, fake, 10, None) == disc.DISC_EINVAL
    assert L.disc_step_shift_scratch_bytes() >= 16 * 1024


def test_ssd_argument_errors_without_gpu(disc):
    L = disc.lib()
    fake = ctypes.c_void_p(1 << 20)
    loss = ctypes.c_void_p(1 << 21)
    patch = (ctypes.c_int * 3)(5, 5, 5)
    bad = (ctypes.c_int * 3)(5, 4, 5)
    need = L.disc_ssd_scratch_bytes(16, 16, 16)
    # m, D (4 B), two double2 buffers (16 B) per voxel, plus the partial sums
    assert need >= 40 * 16 ** 3
    assert L.disc_ssd_scratch_bytes(16, 16, 0) == 0
    args = (fake, fake, fake, 16, 16, 16)
    assert L.disc_ssd_loss(*args, bad, loss, fake, need, None) == disc.DISC_EINVAL
    assert L.disc_ssd_loss(*args, patch, None, fake, need, None) == disc.DISC_EINVAL
    assert L.disc_ssd_loss(*args, patch, loss, fake, need - 1, None) == disc.DISC_ENOMEM
    assert L.disc_ssd_loss(*args, patch, loss, ctypes.c_void_p((1 << 20) + 8), need, None) == disc.DISC_EINVAL
    assert L.disc_ssd_grad(*args, patch, None, None, None, fake, need, None) == disc.DISC_EINVAL
    assert L.disc_ssd_grad(None, fake, fake, 16, 16, 16, patch, None, fake, None, fake, need,
                           None) == disc.DISC_EINVAL
    assert L.disc_ssd_grad(*args, patch, None, fake, None, fake, 100, None) == disc.DISC_ENOMEM


def test_batch_host_checks(disc):
    L = disc.lib()
    p = disc.make_params(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(10,))
    dims = (ctypes.c_int * 6)(40, 30, 20, 33, 17, 9)
    h = ctypes.c_void_p()
    assert L.disc_batch_create(ctypes.byref(p), 2, dims, ctypes.byref(h)) == disc.DISC_OK
    try:
        ws = L.disc_batch_workspace_bytes(h)
        assert ws >= 40 * (40 * 30 * 20 + 33 * 17 * 9)
        assert L.disc_batch_set_tiles(h, 24, 256, 512, 2048) == disc.DISC_EINVAL
        assert L.disc_batch_set_tiles(h, 16, 64, 64, 64) == disc.DISC_OK
        assert L.disc_batch_iterate(h, 1, 1, None) == disc.DISC_ESTATE
        assert L.disc_batch_get_field(h, 0, ctypes.c_void_p(1 << 20), None) == disc.DISC_ESTATE
        fake = (ctypes.c_void_p * 2)(1 << 20, 1 << 21)
        assert L.disc_batch_set_volumes(h, fake, fake, ctypes.c_void_p(1 << 22), ws - 1, None) == disc.DISC_ENOMEM
        assert L.disc_batch_set_volumes(h, fake, fake, ctypes.c_void_p((1 << 22) + 4), ws, None) == disc.DISC_EINVAL
        assert b"aligned" in L.disc_batch_last_error(h)
    finally:
        L.disc_batch_destroy(h)
    p3 = disc.make_params(patch=(5, 5, 5), sigma=1.5, levels=2, iters=(10, 10))
    assert L.disc_batch_create(ctypes.byref(p3), 2, dims, ctypes.byref(h)) == disc.DISC_ENOTSUP
    assert L.disc_batch_create(ctypes.byref(p), 17, dims, ctypes.byref(h)) == disc.DISC_EINVAL
    bad = (ctypes.c_int * 3)(0, 4, 4)
    assert L.disc_batch_create(ctypes.byref(p), 1, bad, ctypes.byref(h)) == disc.DISC_EINVAL
    L.disc_batch_destroy(None)


def test_autotune_key_is_order_free(disc):
    a = disc.autotune_key([(64, 128, 128), (80, 192, 192)], (11, 11, 11), 2.0)
    b = disc.autotune_key([(80, 192, 192), (64, 128, 128)], (11, 11, 11), 2.0)
    assert a == b and "p11x11x11" in a


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1204_6295_amd as d

    monkeypatch.setattr(d, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(d, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        d.lib()
