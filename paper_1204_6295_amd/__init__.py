"""MI355X DISC: demons CT-to-CBCT registration with simultaneous intensity
correction (Zhen et al., arXiv 1204.6295), as hand-written gfx950 HIP
kernels behind the C ABI of ``include/disc.h``.

This module only marshals arguments: torch supplies device memory and the
stream, every step runs in ``libdisc.so``. If the library is missing the
import of any entry point raises -- there is no fallback.

Array conventions: volumes are float32 CUDA(HIP) tensors of shape
(nz, ny, nx); fields have shape (3, nz, ny, nx), components (x, y, z) in
voxels, with m(x) = CT(x + r(x)).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdisc.so")

DISC_OK, DISC_EINVAL, DISC_ENOMEM, DISC_EHIP, DISC_ESTATE, DISC_ENOTSUP = 0, -1, -2, -3, -4, -5
MAX_LEVELS = 8
KERNELS = {"warp": 0, "correct": 1, "force_xy": 2, "smooth_z": 3, "upsample": 4}

_V = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float
_IP = ctypes.POINTER(ctypes.c_int)


class Params(ctypes.Structure):
    """Mirror of ``disc_params``."""

    _fields_ = [
        ("patch", ctypes.c_int * 3),
        ("sigma", ctypes.c_float),
        ("levels", ctypes.c_int),
        ("iters", ctypes.c_int * MAX_LEVELS),
        ("global_shift", ctypes.c_int),
        ("var_floor", ctypes.c_float),
        ("diff_floor", ctypes.c_float),
    ]


class DiscError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("disc error %d: %s" % (code, msg))
        self.code = code


_lib = None

# (name, restype, argtypes) of every exported entry point
_SIGS = [
    ("disc_params_default", _I, [ctypes.POINTER(Params)]),
    ("disc_create", _I, [ctypes.POINTER(Params), ctypes.POINTER(_V)]),
    ("disc_destroy", None, [_V]),
    ("disc_last_error", ctypes.c_char_p, [_V]),
    ("disc_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Params), _I, _I, _I]),
    ("disc_set_volumes", _I, [_V, _V, _V, _I, _I, _I, _V, ctypes.c_size_t, _V]),
    ("disc_iterate", _I, [_V, _I, _V]),
    ("disc_run", _I, [_V, _V]),
    ("disc_state", _I, [_V, _IP, _IP, _IP]),
    ("disc_get_field", _I, [_V, _V, _IP, _V]),
    ("disc_set_field", _I, [_V, _V, _V]),
    ("disc_get_corrected", _I, [_V, _V, _V]),
    ("disc_step_warp", _I, [_V, _V, _I, _I, _I, _V, _V]),
    ("disc_step_static_stats", _I, [_V, _I, _I, _I, _IP, _F, _V, _V]),
    ("disc_step_correct", _I, [_V, _V, _I, _I, _I, _IP, _V, _V]),
    ("disc_step_force_smooth", _I, [_V, _V, _V, _I, _I, _I, _F, _F, _V, _V, _V, _V]),
    ("disc_step_smooth", _I, [_V, _I, _I, _I, _F, _V, _V, _V]),
    ("disc_step_shift_scratch_bytes", ctypes.c_size_t, []),
    ("disc_step_shift", _I, [_V, _V, ctypes.c_long, _V, _V, _V, ctypes.c_size_t, _V]),
    ("disc_step_downsample", _I, [_V, _I, _I, _I, _V, _V]),
    ("disc_step_upsample_field", _I, [_V, _I, _I, _I, _V, _I, _I, _I, _V]),
    ("disc_copy_kernel", _I, [_V, _V, ctypes.c_size_t, _V]),
    ("disc_timing_enable", _I, [_V, _I]),
    ("disc_timing_read", _I, [_V, _I, _I, _IP, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]),
]


def lib():
    """The loaded libdisc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdisc.so is not built (run __graft_entry__.build() or "
                               "python -m paper_1204_6295_amd.build); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _err(ctx=None):
    m = lib().disc_last_error(ctx)
    return m.decode() if m else ""


def _check(rc, ctx=None):
    if rc != DISC_OK:
        raise DiscError(rc, _err(ctx))


def _dev(t, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA(HIP) tensor" % name)
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float32" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return _V(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _V(s.cuda_stream)


def _vol_dims(t):
    if t.dim() != 3:
        raise ValueError("volume must have shape (nz, ny, nx)")
    nz, ny, nx = t.shape
    return int(nx), int(ny), int(nz)


def make_params(patch=(11, 11, 11), sigma=2.0, levels=3, iters=(100, 100, 100), global_shift=True,
                var_floor=1e-2, diff_floor=1e-3):
    p = Params()
    lib().disc_params_default(ctypes.byref(p))
    for d in range(3):
        p.patch[d] = int(patch[d])
    p.sigma = float(sigma)
    p.levels = int(levels)
    iters = list(iters)
    if len(iters) != levels:
        raise ValueError("iters needs one count per level")
    for i in range(MAX_LEVELS):
        p.iters[i] = int(iters[i]) if i < len(iters) else 0
    p.global_shift = 1 if global_shift else 0
    p.var_floor = float(var_floor)
    p.diff_floor = float(diff_floor)
    return p


class Registration:
    """One DISC registration context (disc_create ... disc_destroy).

    The workspace is a torch uint8 tensor sized by disc_workspace_bytes; the
    context keeps references to it and to the CT, which the library borrows.
    """

    def __init__(self, patch=(11, 11, 11), sigma=2.0, levels=3, iters=(100, 100, 100),
                 global_shift=True, var_floor=1e-2, diff_floor=1e-3):
        self.params = make_params(patch, sigma, levels, iters, global_shift, var_floor, diff_floor)
        h = _V()
        _check(lib().disc_create(ctypes.byref(self.params), ctypes.byref(h)))
        self._h = h
        self._keep = ()

    def close(self):
        if getattr(self, "_h", None):
            lib().disc_destroy(self._h)
            self._h = None
            self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, shape):
        nz, ny, nx = shape
        return int(lib().disc_workspace_bytes(ctypes.byref(self.params), nx, ny, nz))

    def set_volumes(self, ct, cbct, stream=None):
        nx, ny, nz = _vol_dims(ct)
        nbytes = self.workspace_bytes(ct.shape)
        if nbytes == 0:
            raise DiscError(DISC_EINVAL, "invalid dims or parameters for shape %s" % (tuple(ct.shape),))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=ct.device)
        if ws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        _check(lib().disc_set_volumes(self._h, _dev(ct, name="ct"), _dev(cbct, ct.shape, "cbct"),
                                      nx, ny, nz, _V(ws.data_ptr()), nbytes, _stream(stream)), self._h)
        self._keep = (ct, ws)
        self.device = ct.device
        return self

    def iterate(self, n=1, stream=None):
        _check(lib().disc_iterate(self._h, int(n), _stream(stream)), self._h)

    def run(self, stream=None):
        _check(lib().disc_run(self._h, _stream(stream)), self._h)

    def state(self):
        lv, it = ctypes.c_int(), ctypes.c_int()
        dims = (ctypes.c_int * 3)()
        _check(lib().disc_state(self._h, ctypes.byref(lv), ctypes.byref(it), dims), self._h)
        return lv.value, it.value, (dims[2], dims[1], dims[0])

    def field(self, stream=None):
        _, _, shape = self.state()
        out = torch.empty((3,) + shape, dtype=torch.float32, device=self.device)
        _check(lib().disc_get_field(self._h, _dev(out), None, _stream(stream)), self._h)
        return out

    def set_field(self, r, stream=None):
        _, _, shape = self.state()
        _check(lib().disc_set_field(self._h, _dev(r, (3,) + shape, "r"), _stream(stream)), self._h)

    def corrected(self, stream=None):
        _, _, shape = self.state()
        out = torch.empty(shape, dtype=torch.float32, device=self.device)
        _check(lib().disc_get_corrected(self._h, _dev(out), _stream(stream)), self._h)
        return out

    def timing_enable(self, max_records):
        _check(lib().disc_timing_enable(self._h, int(max_records)), self._h)

    def timing_read(self, kernel, level=-1):
        """(launches, total ms, total voxels) of one kernel, at one level or all (-1)."""
        kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        n = ctypes.c_int()
        ms = ctypes.c_double()
        vox = ctypes.c_double()
        _check(lib().disc_timing_read(self._h, kid, int(level), ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(vox)), self._h)
        return n.value, ms.value, vox.value


# ---- single steps (same kernels as Registration.iterate) ----------------------

def _patch(patch):
    return (ctypes.c_int * 3)(*[int(p) for p in patch])


def warp(ct, r, stream=None):
    nx, ny, nz = _vol_dims(ct)
    m = torch.empty_like(ct)
    _check(lib().disc_step_warp(_dev(ct, name="ct"), _dev(r, (3,) + tuple(ct.shape), "r"), nx, ny, nz,
                                _dev(m), _stream(stream)))
    return m


def static_stats(s, patch, var_floor=1e-2, stream=None):
    nx, ny, nz = _vol_dims(s)
    ys = torch.empty_like(s)
    _check(lib().disc_step_static_stats(_dev(s, name="s"), nx, ny, nz, _patch(patch), float(var_floor),
                                        _dev(ys), _stream(stream)))
    return ys


def correct(m, ys, patch, stream=None):
    nx, ny, nz = _vol_dims(m)
    f = torch.empty_like(m)
    _check(lib().disc_step_correct(_dev(m, name="m"), _dev(ys, m.shape, "ys"), nx, ny, nz, _patch(patch),
                                   _dev(f), _stream(stream)))
    return f


def force_smooth(m, f, r, sigma, diff_floor=1e-3, want_rt=False, stream=None):
    """Eq. 1 force, update and Gaussian. Returns r_out, or (r_out, r - u)."""
    nx, ny, nz = _vol_dims(m)
    q = torch.empty_like(r)
    out = torch.empty_like(r)
    rt = torch.empty_like(r) if want_rt else None
    _check(lib().disc_step_force_smooth(_dev(m, name="m"), _dev(f, m.shape, "f"),
                                        _dev(r, (3,) + tuple(m.shape), "r"), nx, ny, nz, float(sigma),
                                        float(diff_floor), _dev(q), _dev(out),
                                        _dev(rt) if want_rt else None, _stream(stream)))
    return (out, rt) if want_rt else out


def smooth(rt, sigma, stream=None):
    if rt.dim() != 4 or rt.shape[0] != 3:
        raise ValueError("field must have shape (3, nz, ny, nx)")
    nz, ny, nx = rt.shape[1:]
    q = torch.empty_like(rt)
    r = torch.empty_like(rt)
    _check(lib().disc_step_smooth(_dev(rt, name="rt"), nx, ny, nz, float(sigma), _dev(q), _dev(r),
                                  _stream(stream)))
    return r


def shift(ct, cbct, stream=None):
    """Returns (shifted CBCT, Delta HU as a 1-element float64 device tensor)."""
    n = ct.numel()
    nb = int(lib().disc_step_shift_scratch_bytes())
    scratch = torch.empty(nb, dtype=torch.uint8, device=ct.device)
    s = torch.empty_like(cbct)
    dhu = torch.empty(1, dtype=torch.float64, device=ct.device)
    _check(lib().disc_step_shift(_dev(ct, name="ct"), _dev(cbct, ct.shape, "cbct"), n, _dev(s),
                                 _V(dhu.data_ptr()), _V(scratch.data_ptr()), nb, _stream(stream)))
    return s, dhu


def downsample(v, stream=None):
    nx, ny, nz = _vol_dims(v)
    out = torch.empty(((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2), dtype=torch.float32, device=v.device)
    _check(lib().disc_step_downsample(_dev(v), nx, ny, nz, _dev(out), _stream(stream)))
    return out


def upsample_field(rc, fine_shape, stream=None):
    cnz, cny, cnx = rc.shape[1:]
    fnz, fny, fnx = fine_shape
    rf = torch.empty((3, fnz, fny, fnx), dtype=torch.float32, device=rc.device)
    _check(lib().disc_step_upsample_field(_dev(rc), cnx, cny, cnz, _dev(rf), fnx, fny, fnz, _stream(stream)))
    return rf


def copy_kernel(src, dst, stream=None):
    nbytes = src.numel() * src.element_size()
    _check(lib().disc_copy_kernel(_V(src.data_ptr()), _V(dst.data_ptr()), nbytes, _stream(stream)))
