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

DISC_OK, DISC_EINVAL, DISC_ENOMEM, DISC_EHIP, DISC_ESTATE, DISC_ENOTSUP, DISC_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MAX_LEVELS = 8
KERNELS = {"warp": 0, "correct": 1, "force_xy": 2, "smooth_z": 3, "upsample": 4, "fill": 5}

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
        ("force_mode", ctypes.c_int),
        ("stop_eps", ctypes.c_float),
        ("stop_lag", ctypes.c_int),
        ("mask_mode", ctypes.c_int),
        ("hu0", ctypes.c_float),
        ("a_lo", ctypes.c_float),
        ("a_hi", ctypes.c_float),
        ("fill_h", ctypes.c_float),
        ("fill_t", ctypes.c_int * 3),
        ("fill_passes", ctypes.c_int),
        ("check_finite", ctypes.c_int),
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
    ("disc_step_force_smooth", _I, [_V, _V, _V, _I, _I, _I, _F, _F, _I, _V, _V, _V, _V, _V, _V]),
    ("disc_get_mask", _I, [_V, _V, _V]),
    ("disc_get_stats", _I, [_V, _I, _IP, ctypes.POINTER(ctypes.c_double), _I, _V]),
    ("disc_get_mask_params", _I, [_V, ctypes.POINTER(ctypes.c_float), _V]),
    ("disc_step_smooth", _I, [_V, _I, _I, _I, _F, _V, _V, _V]),
    ("disc_step_shift_scratch_bytes", ctypes.c_size_t, []),
    ("disc_step_shift", _I, [_V, _V, ctypes.c_long, _V, _V, _V, ctypes.c_size_t, _V]),
    ("disc_step_downsample", _I, [_V, _I, _I, _I, _V, _V]),
    ("disc_step_upsample_field", _I, [_V, _I, _I, _I, _V, _I, _I, _I, _V]),
    ("disc_ssd_scratch_bytes", ctypes.c_size_t, [_I, _I, _I]),
    ("disc_ssd_loss", _I, [_V, _V, _V, _I, _I, _I, _IP, _V, _V, ctypes.c_size_t, _V]),
    ("disc_ssd_grad", _I, [_V, _V, _V, _I, _I, _I, _IP, _V, _V, _V, _V, ctypes.c_size_t, _V]),
    ("disc_ssd_loss_noalloc", _I, [_V, _V, _V, _I, _I, _I, _IP, _V, _V]),
    ("disc_batch_create", _I, [ctypes.POINTER(Params), _I, _IP, ctypes.POINTER(_V)]),
    ("disc_batch_destroy", None, [_V]),
    ("disc_batch_last_error", ctypes.c_char_p, [_V]),
    ("disc_batch_workspace_bytes", ctypes.c_size_t, [_V]),
    ("disc_batch_set_tiles", _I, [_V, _I, _I, _I, _I]),
    ("disc_batch_set_volumes", _I, [_V, ctypes.POINTER(_V), ctypes.POINTER(_V), _V, ctypes.c_size_t, _V]),
    ("disc_batch_iterate", _I, [_V, _I, _I, _V]),
    ("disc_batch_run", _I, [_V, _I, _V]),
    ("disc_batch_get_field", _I, [_V, _I, _V, _V]),
    ("disc_batch_get_corrected", _I, [_V, _I, _V, _V]),
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
                var_floor=1e-2, diff_floor=1e-3, force_mode=0, stop_eps=0.0, stop_lag=10, mask_mode=0,
                hu0=0.0, a_lo=0.5, a_hi=1.5, fill_h=0.0, fill_t=(7, 7, 3), fill_passes=10, check_finite=False):
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
    p.check_finite = 1 if check_finite else 0
    return p


class Registration:
    """One DISC registration context (disc_create ... disc_destroy).

    The workspace is a torch uint8 tensor sized by disc_workspace_bytes; the
    context keeps references to it and to the CT, which the library borrows.
    """

    def __init__(self, patch=(11, 11, 11), sigma=2.0, levels=3, iters=(100, 100, 100),
                 global_shift=True, var_floor=1e-2, diff_floor=1e-3, force_mode=0, stop_eps=0.0,
                 stop_lag=10, mask_mode=0, hu0=0.0, a_lo=0.5, a_hi=1.5, fill_h=0.0, fill_t=(7, 7, 3),
                 fill_passes=10, check_finite=False):
        self.params = make_params(patch, sigma, levels, iters, global_shift, var_floor, diff_floor,
                                  force_mode, stop_eps, stop_lag, mask_mode, hu0, a_lo, a_hi, fill_h, fill_t,
                                  fill_passes, check_finite)
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

    def stats(self, level, max_k=None, stream=None):
        """Stopping-rule state of a level: (iterations run, l^(k) for k < that)."""
        k = int(max_k if max_k is not None else max(self.params.iters[i] for i in range(self.params.levels)))
        hist = (ctypes.c_double * max(k, 1))()
        done = ctypes.c_int()
        _check(lib().disc_get_stats(self._h, int(level), ctypes.byref(done), hist, k, _stream(stream)), self._h)
        n = int(done.value)
        return n, [hist[i] for i in range(min(n, k))]

    def mask_params(self, stream=None):
        """Mask mode: {hu0, a_min, a_max, h, a_m} as resolved at set-up."""
        out = (ctypes.c_float * 5)()
        _check(lib().disc_get_mask_params(self._h, out, _stream(stream)), self._h)
        return dict(zip(("hu0", "a_min", "a_max", "h", "a_m"), [float(v) for v in out]))

    def mask(self, stream=None):
        """Mask mode: uint8 map of the latest iteration (0 = not masked,
        p = filled by fill pass p, 255 = masked and never filled)."""
        _, _, shape = self.state()
        out = torch.empty(shape, dtype=torch.uint8, device=self.device)
        _check(lib().disc_get_mask(self._h, _V(out.data_ptr()), _stream(stream)), self._h)
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


def force_smooth(m, f, r, sigma, diff_floor=1e-3, want_rt=False, force_mode=0, ct=None, stream=None):
    """Eq. 1 force (static-gradient term, or both terms with force_mode=1),
    update and Gaussian. Returns r_out, or (r_out, r - u); with ct given,
    the z pass also warps ct by r_out (the next iteration's m, as in a
    registration) and m_next is appended to the result."""
    nx, ny, nz = _vol_dims(m)
    q = torch.empty_like(r)
    out = torch.empty_like(r)
    rt = torch.empty_like(r) if want_rt else None
    m_next = torch.empty_like(m) if ct is not None else None
    _check(lib().disc_step_force_smooth(_dev(m, name="m"), _dev(f, m.shape, "f"),
                                        _dev(r, (3,) + tuple(m.shape), "r"), nx, ny, nz, float(sigma),
                                        float(diff_floor), int(force_mode), _dev(q), _dev(out),
                                        _dev(rt) if want_rt else None,
                                        _dev(ct, m.shape, "ct") if ct is not None else None,
                                        _dev(m_next) if ct is not None else None, _stream(stream)))
    res = (out,) + ((rt,) if want_rt else ()) + ((m_next,) if ct is not None else ())
    return res[0] if len(res) == 1 else res


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


# ---- differentiable DISC ---------------------------------------------------

def _ssd_scratch(ct):
    nx, ny, nz = _vol_dims(ct)
    nb = int(lib().disc_ssd_scratch_bytes(nx, ny, nz))
    if nb == 0:
        raise ValueError("invalid volume dims for the SSD loss")
    return torch.empty(nb, dtype=torch.uint8, device=ct.device), nb


def ssd_loss(ct, ys, r, patch, stream=None):
    """L = sum (m - I'_s)^2 (float64 0-d device tensor); ys from static_stats."""
    nx, ny, nz = _vol_dims(ct)
    scratch, nb = _ssd_scratch(ct)
    loss = torch.empty((), dtype=torch.float64, device=ct.device)
    _check(lib().disc_ssd_loss(_dev(ct, name="ct"), _dev(ys, ct.shape, "ys"), _dev(r, (3,) + tuple(ct.shape), "r"),
                               nx, ny, nz, _patch(patch), _V(loss.data_ptr()), _V(scratch.data_ptr()), nb,
                               _stream(stream)))
    return loss


def ssd_loss_noalloc(ct, ys, r, patch, out=None, stream=None):
    """ssd_loss without device allocation in the library (its scratch is a
    fixed device array; out: an optional preallocated float64 0-d tensor)."""
    nx, ny, nz = _vol_dims(ct)
    loss = out if out is not None else torch.empty((), dtype=torch.float64, device=ct.device)
    if loss.dtype != torch.float64 or loss.numel() != 1 or not loss.is_cuda:
        raise TypeError("out must be a one-element float64 device tensor")
    _check(lib().disc_ssd_loss_noalloc(_dev(ct, name="ct"), _dev(ys, ct.shape, "ys"),
                                       _dev(r, (3,) + tuple(ct.shape), "r"), nx, ny, nz, _patch(patch),
                                       _V(loss.data_ptr()), _stream(stream)))
    return loss


def ssd_grad(ct, ys, r, patch, scale=None, want_loss=False, stream=None):
    """dL/dr (3, nz, ny, nx), times scale (1-element float32 device tensor)."""
    nx, ny, nz = _vol_dims(ct)
    scratch, nb = _ssd_scratch(ct)
    grad = torch.empty_like(r)
    loss = torch.empty((), dtype=torch.float64, device=ct.device) if want_loss else None
    if scale is not None and (scale.dtype != torch.float32 or scale.numel() != 1 or not scale.is_cuda):
        raise TypeError("scale must be a 1-element float32 device tensor")
    _check(lib().disc_ssd_grad(_dev(ct, name="ct"), _dev(ys, ct.shape, "ys"), _dev(r, (3,) + tuple(ct.shape), "r"),
                               nx, ny, nz, _patch(patch), _V(scale.data_ptr()) if scale is not None else None,
                               _dev(grad), _V(loss.data_ptr()) if want_loss else None, _V(scratch.data_ptr()),
                               nb, _stream(stream)))
    return (grad, loss) if want_loss else grad


class SSDLoss(torch.autograd.Function):
    """L(r) = sum (m - I'_s)^2 with its hand-written backward (the patch
    moments are recomputed in the backward pass)."""

    @staticmethod
    def forward(ctx, r, ct, ys, patch):
        ctx.save_for_backward(r, ct, ys)
        ctx.patch = tuple(int(p) for p in patch)
        return ssd_loss(ct, ys, r, ctx.patch)

    @staticmethod
    def backward(ctx, g):
        r, ct, ys = ctx.saved_tensors
        scale = g.detach().to(torch.float32).reshape(1).contiguous()
        return ssd_grad(ct, ys, r, ctx.patch, scale=scale), None, None, None


def ssd(r, ct, ys, patch):
    """Differentiable SSD loss of the field r (see SSDLoss)."""
    return SSDLoss.apply(r, ct, ys, patch)


# ---- batches of volumes ------------------------------------------------------

MAX_BATCH = 16


class Batch:
    """Independent CT/CBCT pairs of uneven sizes advanced together (one
    resolution level): three batched launches per iteration (the CT is
    warped once after set-up, then by each iteration's z pass), optionally
    replayed from a captured HIP graph. force_mode 1 takes both Eq. 1 terms."""

    def __init__(self, shapes, patch=(11, 11, 11), sigma=2.0, iters=100, global_shift=True,
                 var_floor=1e-2, diff_floor=1e-3, force_mode=0):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.params = make_params(patch=patch, sigma=sigma, levels=1, iters=(iters,), global_shift=global_shift,
                                  var_floor=var_floor, diff_floor=diff_floor, force_mode=force_mode)
        n = len(self.shapes)
        dims = (ctypes.c_int * (3 * n))(*[d for (nz, ny, nx) in self.shapes for d in (nx, ny, nz)])
        h = _V()
        _check(lib().disc_batch_create(ctypes.byref(self.params), n, dims, ctypes.byref(h)))
        self._h = h
        self._ws = None
        self._inputs = None

    def close(self):
        if getattr(self, "_h", None):
            lib().disc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != DISC_OK:
            m = lib().disc_batch_last_error(self._h)
            raise DiscError(rc, m.decode() if m else "")

    def set_tiles(self, mom_ts=32, mom_target=256, plane_target=256, z_target=8192):
        self._check(lib().disc_batch_set_tiles(self._h, int(mom_ts), int(mom_target), int(plane_target),
                                               int(z_target)))

    def set_volumes(self, cts, cbcts, stream=None):
        if len(cts) != len(self.shapes) or len(cbcts) != len(self.shapes):
            raise ValueError("one ct and one cbct per pair")
        for ct, cb, shp in zip(cts, cbcts, self.shapes):
            _dev(ct, shp, "ct")
            _dev(cb, shp, "cbct")
        nb = int(lib().disc_batch_workspace_bytes(self._h))
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=cts[0].device)
        n = len(self.shapes)
        pc = (_V * n)(*[t.data_ptr() for t in cts])
        pb = (_V * n)(*[t.data_ptr() for t in cbcts])
        self._inputs = (cts, cbcts)  # the CTs are borrowed by the library
        self._check(lib().disc_batch_set_volumes(self._h, pc, pb, _V(self._ws.data_ptr()), nb, _stream(stream)))

    def iterate(self, n=1, use_graph=True, stream=None):
        self._check(lib().disc_batch_iterate(self._h, int(n), 1 if use_graph else 0, _stream(stream)))

    def run(self, use_graph=True, stream=None):
        self._check(lib().disc_batch_run(self._h, 1 if use_graph else 0, _stream(stream)))

    def field(self, v, stream=None):
        out = torch.empty((3,) + self.shapes[v], dtype=torch.float32, device=self._ws.device)
        self._check(lib().disc_batch_get_field(self._h, int(v), _dev(out), _stream(stream)))
        return out

    def corrected(self, v, stream=None):
        out = torch.empty(self.shapes[v], dtype=torch.float32, device=self._ws.device)
        self._check(lib().disc_batch_get_corrected(self._h, int(v), _dev(out), _stream(stream)))
        return out


# Launch-knob candidates of the batched iteration, tried by the autotuner.
TILE_CANDIDATES = [
    dict(mom_ts=32, mom_target=256, plane_target=256, z_target=8192),
    dict(mom_ts=32, mom_target=256, plane_target=512, z_target=2048),
    dict(mom_ts=32, mom_target=128, plane_target=256, z_target=1024),
    dict(mom_ts=32, mom_target=512, plane_target=1024, z_target=4096),
    dict(mom_ts=16, mom_target=256, plane_target=512, z_target=2048),
    dict(mom_ts=16, mom_target=1024, plane_target=1024, z_target=8192),
]


def autotune_key(shapes, patch, sigma):
    sh = ";".join("x".join(str(v) for v in s) for s in sorted(tuple(s) for s in shapes))
    return "%s|p%s|s%g" % (sh, "x".join(str(int(p)) for p in patch), float(sigma))


def autotune(batch, cts, cbcts, cache_path=None, iters=5, candidates=None):
    """Times each candidate tile setting on this batch (eager launches, after
    one warm-up iteration) and keeps the fastest; results are cached in a
    JSON file keyed by the sorted shapes, patch and sigma. Leaves the batch
    set to the chosen tiles and re-initialised (set_volumes). Returns
    (tiles, ms per iteration, whether it came from the cache)."""
    import json
    import time

    key = autotune_key(batch.shapes, batch.params.patch, batch.params.sigma)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        best = cache[key]
        batch.set_tiles(**best["tiles"])
        batch.set_volumes(cts, cbcts)
        return best["tiles"], best["ms_per_iteration"], True
    results = []
    for cand in (candidates or TILE_CANDIDATES):
        batch.set_tiles(**cand)
        batch.set_volumes(cts, cbcts)
        batch.iterate(1, use_graph=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.iterate(iters, use_graph=False)
        torch.cuda.synchronize()
        results.append(((time.perf_counter() - t0) * 1000.0 / iters, cand))
    ms, best = min(results, key=lambda r: r[0])
    batch.set_tiles(**best)
    batch.set_volumes(cts, cbcts)
    if cache_path:
        cache[key] = {"tiles": best, "ms_per_iteration": ms,
                      "all": [{"tiles": c, "ms_per_iteration": t} for t, c in results]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, ms, False
