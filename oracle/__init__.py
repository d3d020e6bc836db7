"""FP64 CPU oracle of DISC (arXiv 1204.6295) -- TEST INFRASTRUCTURE ONLY.

This package is the checker the HIP library is compared against. Only the
test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product package never does, and the two
share no code. The arithmetic lives in ``disc_oracle.c`` (plain C, FP64,
OpenMP over z-slices); this module only marshals numpy arrays.

Array conventions: volumes are numpy arrays of shape (nz, ny, nx) (x fastest);
fields have shape (3, nz, ny, nx) with components (x, y, z) in voxels.
Functions named ``*_pts`` read FP32 state and evaluate single voxels, for
sampled checks at sizes where whole-volume oracle runs take too long.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "disc_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_HDR = os.path.join(_HERE, "disc_oracle.h")

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_L = ctypes.POINTER(ctypes.c_long)
_IP = ctypes.POINTER(ctypes.c_int)
_I = ctypes.c_int


class Params(ctypes.Structure):
    """Mirror of ``orc_params`` (disc_oracle.h)."""

    _fields_ = [
        ("patch", ctypes.c_int * 3),
        ("sigma", ctypes.c_double),
        ("levels", ctypes.c_int),
        ("iters", ctypes.c_int * 8),
        ("global_shift", ctypes.c_int),
        ("var_floor", ctypes.c_double),
        ("diff_floor", ctypes.c_double),
        ("force_mode", ctypes.c_int),
        ("stop_eps", ctypes.c_double),
        ("stop_lag", ctypes.c_int),
        ("mask_mode", ctypes.c_int),
        ("hu0", ctypes.c_double),
        ("a_lo", ctypes.c_double),
        ("a_hi", ctypes.c_double),
        ("fill_h", ctypes.c_double),
        ("fill_t", ctypes.c_int * 3),
        ("fill_passes", ctypes.c_int),
    ]


def make_params(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(20,), global_shift=True,
                var_floor=1e-2, diff_floor=1e-3, force_mode=0, stop_eps=0.0, stop_lag=10, mask_mode=0,
                hu0=0.0, a_lo=0.5, a_hi=1.5, fill_h=0.0, fill_t=(7, 7, 3), fill_passes=10):
    p = Params()
    for d in range(3):
        p.patch[d] = int(patch[d])
    p.sigma = float(sigma)
    p.levels = int(levels)
    for i, k in enumerate(iters):
        p.iters[i] = int(k)
    p.global_shift = 1 if global_shift else 0
    p.var_floor = float(var_floor)
    p.diff_floor = float(diff_floor)
    p.force_mode = int(force_mode)
    p.stop_eps = float(stop_eps)
    p.stop_lag = int(stop_lag)
    p.mask_mode = int(mask_mode)
    p.hu0 = float(hu0)
    p.a_lo = float(a_lo)
    p.a_hi = float(a_hi)
    p.fill_h = float(fill_h)
    for d in range(3):
        p.fill_t[d] = int(fill_t[d])
    p.fill_passes = int(fill_passes)
    return p


def build():
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    subprocess.check_call([
        "gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
        "-Wall", "-Wextra", "-o", _SO, _SRC, "-lm",
    ])


_lib = None


def lib():
    global _lib
    if _lib is None:
        # build when missing or older than the C source
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_threads.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_mean.restype = ctypes.c_double
        L.orc_mean.argtypes = [_D, ctypes.c_long]
        L.orc_global_shift.restype = ctypes.c_double
        L.orc_global_shift.argtypes = [_D, _D, ctypes.c_long, _D]
        L.orc_downsample2.argtypes = [_D, _I, _I, _I, _D]
        L.orc_upsample_field.argtypes = [_D, _I, _I, _I, _D, _I, _I, _I]
        L.orc_warp.argtypes = [_D, _D, _I, _I, _I, _D]
        L.orc_patch_moments.argtypes = [_D, _I, _I, _I, _I, _I, _I, _D, _D]
        L.orc_correct.argtypes = [_D, _D, _D, _D, _D, ctypes.c_long, ctypes.c_double, _D, _D, _D]
        L.orc_force.argtypes = [_D, _D, _I, _I, _I, ctypes.c_double, _D]
        L.orc_gauss_taps.restype = ctypes.c_int
        L.orc_gauss_taps.argtypes = [ctypes.c_double, _D]
        L.orc_gauss.argtypes = [_D, _I, _I, _I, ctypes.c_double, _D]
        L.orc_iterate.argtypes = [_D, _D, _D, _D, _D, _I, _I, _I, ctypes.POINTER(Params), _D, _D, _D]
        L.orc_register.restype = ctypes.c_int
        L.orc_register.argtypes = [_D, _D, _I, _I, _I, ctypes.POINTER(Params), _D, _D]
        L.orc_warp_pts.argtypes = [_F, _F, _I, _I, _I, _L, ctypes.c_long, _D]
        L.orc_correct_pts.argtypes = [_F, _F, _I, _I, _I, _I, _I, _I, ctypes.c_double, _L, ctypes.c_long, _D]
        L.orc_force_pts.argtypes = [_F, _F, _F, _I, _I, _I, ctypes.c_double, _L, ctypes.c_long, _D]
        L.orc_gauss_pts.argtypes = [_F, _I, _I, _I, ctypes.c_double, _L, ctypes.c_long, _D]
        L.orc_force_double.argtypes = [_D, _D, _I, _I, _I, ctypes.c_double, _D]
        _U8 = ctypes.POINTER(ctypes.c_ubyte)
        L.orc_fill.restype = ctypes.c_int
        L.orc_fill.argtypes = [_D, _D, _U8, _D, _I, _I, _I, ctypes.c_double, _IP, _I, _D, _D]
        L.orc_fill_ex.restype = ctypes.c_int
        L.orc_fill_ex.argtypes = [_D, _D, _U8, _D, _I, _I, _I, ctypes.c_double, _IP, _I, _D, _D, _U8]
        L.orc_mask_fill.restype = ctypes.c_int
        L.orc_mask_fill.argtypes = [_D, _D, _D, _D, _D, _D, _I, _I, _I, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, _IP, _I, _D, _D, _U8]
        L.orc_a_median.restype = ctypes.c_double
        L.orc_a_median.argtypes = [_D, _D, _I, _I, _I, _I, _I, _I, ctypes.c_double]
        L.orc_register_ex.restype = ctypes.c_int
        L.orc_register_ex.argtypes = [_D, _D, _I, _I, _I, ctypes.POINTER(Params), _D, _D, _IP, _D, _I]
        L.orc_ssd_loss.restype = ctypes.c_double
        L.orc_ssd_loss.argtypes = [_D, _D, _D, _I, _I, _I, _I, _I, _I, ctypes.c_double]
        L.orc_ssd_grad.argtypes = [_D, _D, _D, _I, _I, _I, _I, _I, _I, ctypes.c_double, _D]
        L.orc_ssd_grad_pts.argtypes = [_F, _F, _F, _I, _I, _I, _I, _I, _I, ctypes.c_double, _L,
                                       ctypes.c_long, _D]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_F)


def _dims(v):
    nz, ny, nx = v.shape[-3:]
    return int(nx), int(ny), int(nz)


def threads():
    return int(lib().orc_threads())


def set_threads(n):
    """OpenMP threads of later oracle calls (n >= 1)."""
    lib().orc_set_threads(int(n))


def mean(v):
    v, p = _d(v)
    return lib().orc_mean(p, v.size)


def global_shift(ct, cbct0):
    """Returns (Delta HU, shifted CBCT)."""
    ct, pc = _d(ct)
    cb, pb = _d(cbct0)
    out = np.empty_like(cb)
    dhu = lib().orc_global_shift(pc, pb, ct.size, out.ctypes.data_as(_D))
    return dhu, out


def downsample2(v):
    v, p = _d(v)
    nx, ny, nz = _dims(v)
    out = np.empty(((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2))
    lib().orc_downsample2(p, nx, ny, nz, out.ctypes.data_as(_D))
    return out


def upsample_field(rc, fine_shape):
    rc, p = _d(rc)
    cnx, cny, cnz = _dims(rc)
    fnz, fny, fnx = fine_shape
    out = np.empty((3, fnz, fny, fnx))
    lib().orc_upsample_field(p, cnx, cny, cnz, out.ctypes.data_as(_D), fnx, fny, fnz)
    return out


def warp(ct, r):
    ct, pc = _d(ct)
    r, pr = _d(r)
    nx, ny, nz = _dims(ct)
    assert r.shape == (3,) + ct.shape
    out = np.empty_like(ct)
    lib().orc_warp(pc, pr, nx, ny, nz, out.ctypes.data_as(_D))
    return out


def patch_moments(img, patch):
    img, p = _d(img)
    nx, ny, nz = _dims(img)
    mu = np.empty_like(img)
    var = np.empty_like(img)
    lib().orc_patch_moments(p, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]),
                            mu.ctypes.data_as(_D), var.ctypes.data_as(_D))
    return mu, var


def correct(mu_m, var_m, mu_s, var_s, s, tau=1e-2):
    arrs = [_d(a) for a in (mu_m, var_m, mu_s, var_s, s)]
    n = arrs[0][0].size
    a = np.empty_like(arrs[0][0])
    b = np.empty_like(a)
    f = np.empty_like(a)
    lib().orc_correct(*[q for _, q in arrs], n, float(tau), a.ctypes.data_as(_D),
                      b.ctypes.data_as(_D), f.ctypes.data_as(_D))
    return a, b, f


def force(m, f, eps_d=1e-3):
    m, pm = _d(m)
    f, pf = _d(f)
    nx, ny, nz = _dims(m)
    u = np.empty((3,) + m.shape)
    lib().orc_force(pm, pf, nx, ny, nz, float(eps_d), u.ctypes.data_as(_D))
    return u


def force_double(m, f, eps_d=1e-3):
    """Both terms of Eq. 1 (double force)."""
    m, pm = _d(m)
    f, pf = _d(f)
    nx, ny, nz = _dims(m)
    u = np.empty((3,) + m.shape)
    lib().orc_force_double(pm, pf, nx, ny, nz, float(eps_d), u.ctypes.data_as(_D))
    return u


def gauss_taps(sigma):
    w = np.zeros(129)
    R = lib().orc_gauss_taps(float(sigma), w.ctypes.data_as(_D))
    if R < 0:
        raise ValueError("sigma must be positive with ceil(3 sigma) <= 64")
    return w[: 2 * R + 1].copy()


def gauss(v, sigma):
    v, p = _d(v)
    nx, ny, nz = _dims(v)
    out = np.empty_like(v)
    lib().orc_gauss(p, nx, ny, nz, float(sigma), out.ctypes.data_as(_D))
    return out


def iterate(ct, s, r, params, n=1, mu_s=None, var_s=None):
    """Run ``n`` DISC iterations at one level. Returns (r, m, f, rt) of the last one."""
    ct, pc = _d(ct)
    s, ps = _d(s)
    if mu_s is None:
        mu_s, var_s = patch_moments(s, params.patch)
    mu_s, pmu = _d(mu_s)
    var_s, pvar = _d(var_s)
    r = np.array(r, dtype=np.float64, copy=True)
    nx, ny, nz = _dims(ct)
    m = np.empty_like(ct)
    f = np.empty_like(ct)
    rt = np.empty_like(r)
    for _ in range(n):
        lib().orc_iterate(pc, ps, pmu, pvar, r.ctypes.data_as(_D), nx, ny, nz, ctypes.byref(params),
                          m.ctypes.data_as(_D), f.ctypes.data_as(_D), rt.ctypes.data_as(_D))
    return r, m, f, rt


def register(ct, cbct, params):
    """Whole Algorithm A1. Returns (r at the finest level, I'_s of the last iteration)."""
    ct, pc = _d(ct)
    cb, pb = _d(cbct)
    nx, ny, nz = _dims(ct)
    r = np.empty((3,) + ct.shape)
    f = np.empty_like(ct)
    rc = lib().orc_register(pc, pb, nx, ny, nz, ctypes.byref(params), r.ctypes.data_as(_D),
                            f.ctypes.data_as(_D))
    if rc != 0:
        raise ValueError("orc_register rejected its arguments")
    return r, f


def register_ex(ct, cbct, params):
    """Algorithm A1 with the Sec. 2.3 stopping rule (params.stop_eps > 0).
    Returns (r, I'_s, iterations run per level, l^(k) per level)."""
    ct, pc = _d(ct)
    cb, pb = _d(cbct)
    nx, ny, nz = _dims(ct)
    r = np.empty((3,) + ct.shape)
    f = np.empty_like(ct)
    done = (ctypes.c_int * 8)()
    stride = max(1, max(int(params.iters[l]) for l in range(params.levels)))
    hist = np.full((params.levels, stride), np.nan)
    rc = lib().orc_register_ex(pc, pb, nx, ny, nz, ctypes.byref(params), r.ctypes.data_as(_D),
                               f.ctypes.data_as(_D), done, hist.ctypes.data_as(_D), stride)
    if rc != 0:
        raise ValueError("orc_register_ex rejected its arguments")
    n = [int(done[l]) for l in range(params.levels)]
    return r, f, n, [hist[l, :n[l]].copy() for l in range(params.levels)]


def _pts(pts):
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    return pts, pts.ctypes.data_as(_L)


def warp_pts(ct, r, pts):
    ct, pc = _f(ct)
    r, pr = _f(r)
    pts, pp = _pts(pts)
    nx, ny, nz = _dims(ct)
    out = np.empty(pts.size)
    lib().orc_warp_pts(pc, pr, nx, ny, nz, pp, pts.size, out.ctypes.data_as(_D))
    return out


def correct_pts(m, s, patch, pts, tau=1e-2):
    m, pm = _f(m)
    s, ps = _f(s)
    pts, pp = _pts(pts)
    nx, ny, nz = _dims(m)
    out = np.empty(pts.size)
    lib().orc_correct_pts(pm, ps, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]),
                          float(tau), pp, pts.size, out.ctypes.data_as(_D))
    return out


def force_pts(m, f, r, pts, eps_d=1e-3):
    m, pm = _f(m)
    f, pf = _f(f)
    r, pr = _f(r)
    pts, pp = _pts(pts)
    nx, ny, nz = _dims(m)
    out = np.empty((pts.size, 3))
    lib().orc_force_pts(pm, pf, pr, nx, ny, nz, float(eps_d), pp, pts.size, out.ctypes.data_as(_D))
    return out


def gauss_pts(rt, sigma, pts):
    rt, pr = _f(rt)
    pts, pp = _pts(pts)
    nx, ny, nz = _dims(rt)
    out = np.empty((pts.size, 3))
    lib().orc_gauss_pts(pr, nx, ny, nz, float(sigma), pp, pts.size, out.ctypes.data_as(_D))
    return out


def ssd_loss(ct, s, r, patch, tau=1e-2):
    """L = sum (m - I'_s)^2 with m = warp(ct, r) (FP64)."""
    ct, pc = _d(ct)
    s, ps = _d(s)
    r, pr = _d(r)
    nx, ny, nz = _dims(ct)
    return lib().orc_ssd_loss(pc, ps, pr, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]),
                              float(tau))


def ssd_grad(ct, s, r, patch, tau=1e-2):
    """Analytic dL/dr, shape (3, nz, ny, nx)."""
    ct, pc = _d(ct)
    s, ps = _d(s)
    r, pr = _d(r)
    nx, ny, nz = _dims(ct)
    out = np.empty((3,) + ct.shape)
    lib().orc_ssd_grad(pc, ps, pr, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]),
                       float(tau), out.ctypes.data_as(_D))
    return out


def ssd_grad_pts(ct, s, r, patch, pts, tau=1e-2):
    """dL/dr at linear voxel indices pts from FP32 state; returns (npts, 3)."""
    ct, pc = _f(ct)
    s, ps = _f(s)
    r, pr = _f(r)
    nx, ny, nz = _dims(ct)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty((len(pts), 3))
    lib().orc_ssd_grad_pts(pc, ps, pr, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]),
                           float(tau), pts.ctypes.data_as(_L), len(pts), out.ctypes.data_as(_D))
    return out


def fill(a0, b0, valid0, s, h, t=(7, 7, 3), passes=10):
    """Eq. 8-10 fill from (a0, b0) with initial validity valid0 (bool).
    Returns (A, B, passes that filled something)."""
    a0, pa = _d(a0)
    b0, pb = _d(b0)
    s, ps = _d(s)
    v = np.ascontiguousarray(valid0, dtype=np.uint8)
    nx, ny, nz = _dims(s)
    A = np.empty_like(s)
    B = np.empty_like(s)
    tt = (ctypes.c_int * 3)(*[int(x) for x in t])
    used = lib().orc_fill(pa, pb, v.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), ps, nx, ny, nz, float(h), tt,
                          int(passes), A.ctypes.data_as(_D), B.ctypes.data_as(_D))
    return A, B, used


def fill_ex(a0, b0, valid0, s, h, t=(7, 7, 3), passes=10):
    """orc_fill with the pass that filled each voxel: returns (A, B, passes
    used, pass_of) with pass_of 0 = valid from the start, p = filled by pass
    p (1-based), 255 = never filled."""
    a0, pa = _d(a0)
    b0, pb = _d(b0)
    s, ps = _d(s)
    v = np.ascontiguousarray(valid0, dtype=np.uint8)
    nx, ny, nz = _dims(s)
    A = np.empty_like(s)
    B = np.empty_like(s)
    pass_of = np.empty(s.shape, dtype=np.uint8)
    tt = (ctypes.c_int * 3)(*[int(x) for x in t])
    _U8 = ctypes.POINTER(ctypes.c_ubyte)
    used = lib().orc_fill_ex(pa, pb, v.ctypes.data_as(_U8), ps, nx, ny, nz, float(h), tt, int(passes),
                             A.ctypes.data_as(_D), B.ctypes.data_as(_D), pass_of.ctypes.data_as(_U8))
    return A, B, used, pass_of


def mask_fill(m, s, patch, tau, hu0, a_min, a_max, h, t=(7, 7, 3), passes=10):
    """Eq. 5-10 at one level: returns (A, B, xi, passes used)."""
    m, pm = _d(m)
    s, ps = _d(s)
    nx, ny, nz = _dims(m)
    mu_m, var_m = patch_moments(m, patch)
    mu_s, var_s = patch_moments(s, patch)
    A = np.empty_like(m)
    B = np.empty_like(m)
    xi = np.empty(m.shape, dtype=np.uint8)
    tt = (ctypes.c_int * 3)(*[int(x) for x in t])
    used = lib().orc_mask_fill(pm, ps, _d(mu_m)[1], _d(var_m)[1], _d(mu_s)[1], _d(var_s)[1], nx, ny, nz,
                               float(tau), float(hu0), float(a_min), float(a_max), float(h), tt, int(passes),
                               A.ctypes.data_as(_D), B.ctypes.data_as(_D),
                               xi.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    return A, B, xi.astype(bool), used


def a_median(ct, s, patch, tau=1e-2):
    ct, pc = _d(ct)
    s, ps = _d(s)
    nx, ny, nz = _dims(ct)
    return lib().orc_a_median(pc, ps, nx, ny, nz, int(patch[0]), int(patch[1]), int(patch[2]), float(tau))


def register_steps(ct, cbct, params, chunk=10, on_chunk=None):
    """Algorithm A1 (Sec. 2.3) with fixed iteration counts, run from the same
    C steps as ``register`` but in chunks of ``chunk`` iterations, so a
    caller can follow a long run: ``on_chunk(level, k, r, f)`` is called
    after every chunk with the level's iteration count k and the current
    field and corrected image. The order of operations is that of
    ``register`` (shift, pyramid, per-level static moments, iterations,
    up-sampling), so the result is bitwise the same."""
    if params.mask_mode != 0 or params.stop_eps > 0.0:
        raise ValueError("register_steps covers the fixed-count, unmasked schedule")
    ct = np.ascontiguousarray(ct, dtype=np.float64)
    cb = np.ascontiguousarray(cbct, dtype=np.float64)
    if params.global_shift:
        _, s = global_shift(ct, cb)
    else:
        s = cb.copy()
    L = int(params.levels)
    cts, ss = [ct], [s]
    for _ in range(L - 1):
        cts.insert(0, downsample2(cts[0]))
        ss.insert(0, downsample2(ss[0]))
    r = np.zeros((3,) + cts[0].shape)
    f = None
    for l in range(L):
        if l > 0:
            r = upsample_field(r, cts[l].shape)
        patch = tuple(int(params.patch[d]) for d in range(3))
        mu_s, var_s = patch_moments(ss[l], patch)
        f = ss[l].copy()
        k = 0
        while k < int(params.iters[l]):
            n = min(int(chunk), int(params.iters[l]) - k)
            r, _, f, _ = iterate(cts[l], ss[l], r, params, n=n, mu_s=mu_s, var_s=var_s)
            k += n
            if on_chunk is not None:
                on_chunk(l, k, r, f)
    return r, f
