"""Analytic CT phantoms, known smooth deformations and a CBCT artifact model.

The paper evaluates on a simulated head-and-neck CBCT (MC scatter + FDK) and on
six clinical head-and-neck CT/CBCT pairs (Sec. 2.4.1, 2.4.2); neither dataset
is available, so these seeded phantoms stand in for them, with the paper's HU
ranges and artifact types (scatter cupping, streaks, bow-tie crescent, noise;
Sec. 1 and Sec. 2.3 "Delta HU is about 100 HU").

Construction (all in FP64, cast to FP32 at the end):
  * CT(x): painter's-order analytic scene (ellipsoids, shells, tubes), averaged
    over 2x2x2 sub-voxel samples (partial volume), so no voxel is an exact
    trilinear sample of another.
  * r_true(x): sum of Gaussian bumps with random vector amplitudes, scaled so
    that max |r_true| equals the configured value (mm), returned in voxels.
  * CBCT(x) = g(x) * (scene(x + r_true(x)) + 1000) - 1000 + artifacts + 100 + noise,
    with g a radial quadratic cupping gain acting on attenuation (HU + 1000).
Under the model I_m(x + v(x)) = I_s(x) (Sec. 2.1), the field that registers the
CT onto this CBCT is r_true itself.

Arrays: volumes (nz, ny, nx) float32, x fastest; r_true (3, nz, ny, nx) float32
with components (x, y, z) in voxels. Random numbers come from
``numpy.random.default_rng([12046295, config_id, pair])``.
"""
from dataclasses import dataclass, field

import numpy as np
import torch

SEED_BASE = 12046295

# Workloads. shape is (nz, ny, nx); spacing is (dz, dy, dx) in mm.
CONFIGS = {
    # 48^3 ellipsoid phantom, single resolution.
    "ellipsoid48": dict(cid=1, kind="ellipsoid", shape=(48, 48, 48), spacing=(1.0, 1.0, 1.0),
               max_def_mm=3.0, patch=(5, 5, 5), sigma=1.5, levels=1, iters=(20,)),
    # head-and-neck-like 256 x 256 x 96, 1.95 x 1.95 x 2.5 mm.
    "hn256x256x96": dict(cid=2, kind="hn", shape=(96, 256, 256), spacing=(2.5, 1.953125, 1.953125),
               max_def_mm=8.0, patch=(11, 11, 11), sigma=2.0, levels=3, iters=(100, 100, 100)),
    # clinical size 512 x 512 x 160, same field of view.
    "hn512x512x160": dict(cid=3, kind="hn", shape=(160, 512, 512), spacing=(1.5, 0.9765625, 0.9765625),
               max_def_mm=12.0, patch=(15, 15, 15), sigma=2.0, levels=3, iters=(200, 200, 200)),
}

# Field of view of the head-and-neck scene (mm): 500 x 500 x 240.
HN_FOV = (240.0, 500.0, 500.0)
BATCH_SHAPES = [(64, 128, 128), (80, 192, 192), (96, 256, 256), (128, 384, 384)]


@dataclass
class Case:
    name: str
    ct: np.ndarray
    cbct: np.ndarray
    r_true: np.ndarray
    spacing: tuple
    params: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# scene primitives (evaluated on torch float64 coordinate tensors, in mm)
# --------------------------------------------------------------------------

def _rand_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def _ell_q(px, py, pz, c, ax, rot):
    """Quadratic form of an ellipsoid (<= 1 inside). Points (px, py, pz) in mm."""
    dx, dy, dz = px - c[0], py - c[1], pz - c[2]
    if rot is None:
        u, v, w = dx, dy, dz
    else:
        # body coordinates: rot^T (p - c)
        u = rot[0, 0] * dx + rot[1, 0] * dy + rot[2, 0] * dz
        v = rot[0, 1] * dx + rot[1, 1] * dy + rot[2, 1] * dz
        w = rot[0, 2] * dx + rot[1, 2] * dy + rot[2, 2] * dz
    return (u / ax[0]) ** 2 + (v / ax[1]) ** 2 + (w / ax[2]) ** 2


class Scene:
    """Painter's-order list of objects; later objects overwrite earlier ones."""

    def __init__(self, background=-1000.0):
        self.background = background
        self.objs = []
        self.body = None  # (center, axes) of the body ellipsoid / cylinder

    def ellipsoid(self, c, ax, value, rot=None):
        self.objs.append(("ell", (np.asarray(c, float), np.asarray(ax, float), rot), float(value)))

    def shell(self, c, ax, thick, value, half=None):
        """Ellipsoidal shell; ``half`` = (axis, sign) keeps one half-space."""
        self.objs.append(("shell", (np.asarray(c, float), np.asarray(ax, float), float(thick), half),
                          float(value)))

    def tube(self, cxy, axy, zr, value):
        self.objs.append(("tube", (np.asarray(cxy, float), np.asarray(axy, float), zr), float(value)))

    def inside(self, kind, prm, px, py, pz):
        if kind == "ell":
            c, ax, rot = prm
            return _ell_q(px, py, pz, c, ax, rot) <= 1.0
        if kind == "shell":
            c, ax, th, half = prm
            m = (_ell_q(px, py, pz, c, ax, None) <= 1.0) & (_ell_q(px, py, pz, c, ax - th, None) > 1.0)
            if half is not None:
                axis, sign = half
                coord = (px, py, pz)[axis] - c[axis]
                m = m & (coord * sign > 0)
            return m
        if kind == "tube":
            cxy, axy, (z0, z1) = prm
            return ((((px - cxy[0]) / axy[0]) ** 2 + ((py - cxy[1]) / axy[1]) ** 2) <= 1.0) & (pz >= z0) & (pz <= z1)
        raise ValueError(kind)

    def eval(self, px, py, pz):
        img = torch.full_like(px, self.background)
        for kind, prm, val in self.objs:
            img = torch.where(self.inside(kind, prm, px, py, pz), torch.full_like(px, val), img)
        return img

    def in_body(self, px, py, pz):
        c, ax = self.body
        return _ell_q(px, py, pz, c, ax, None) <= 1.0


def _ellipsoid_scene(rng, extent_mm):
    """Random ellipsoid phantom: body 0-80 HU, 6 soft ellipsoids 0-80 HU,
    3 bone ellipsoids 700-1500 HU, background -1000 HU."""
    s = Scene()
    body_ax = rng.uniform(16.0, 21.0, size=3)
    body_c = rng.uniform(-1.0, 1.0, size=3)
    s.ellipsoid(body_c, body_ax, rng.uniform(0.0, 80.0))
    s.body = (body_c, body_ax)
    for _ in range(6):
        c = body_c + rng.uniform(-0.55, 0.55, size=3) * body_ax
        s.ellipsoid(c, rng.uniform(3.0, 8.0, size=3), rng.uniform(0.0, 80.0), _rand_rotation(rng))
    for _ in range(3):
        c = body_c + rng.uniform(-0.5, 0.5, size=3) * body_ax
        s.ellipsoid(c, rng.uniform(2.0, 6.0, size=3), rng.uniform(700.0, 1500.0), _rand_rotation(rng))
    return s


def _hn_scene(rng):
    """Head-and-neck-like scene in mm (origin at the volume centre, z up):
    soft tissue ~40 HU, fat/muscle pockets, skull shell 1000-1500 HU, brain
    ~35 HU, airway tube -1000 HU, mandible half-shell 700-1200 HU, vertebral
    column ~800 HU."""
    s = Scene()
    jit = lambda a: a * rng.uniform(0.95, 1.05)  # noqa: E731
    body_c = np.array([0.0, 0.0, 0.0])
    body_ax = np.array([jit(95.0), jit(115.0), 400.0])
    s.ellipsoid(body_c, body_ax, 40.0 + rng.uniform(-5, 5))
    s.body = (body_c, body_ax)
    # fat and muscle pockets in the neck
    for _ in range(8):
        c = np.array([rng.uniform(-60, 60), rng.uniform(-70, 70), rng.uniform(-110, 0)])
        val = rng.choice([rng.uniform(-120, -60), rng.uniform(50, 75)])
        s.ellipsoid(c, rng.uniform([10, 10, 20], [25, 25, 50]), val, _rand_rotation(rng))
    # skull: shell around the brain, upper part of the field of view
    sk_c = np.array([0.0, jit(5.0), 55.0])
    sk_ax = np.array([jit(82.0), jit(100.0), jit(95.0)])
    s.shell(sk_c, sk_ax, 6.0, rng.uniform(1000.0, 1500.0))
    s.ellipsoid(sk_c, sk_ax - 6.0, 35.0 + rng.uniform(-3, 3))
    # a few brain structures for texture
    for _ in range(4):
        c = sk_c + np.array([rng.uniform(-40, 40), rng.uniform(-50, 50), rng.uniform(-20, 40)])
        s.ellipsoid(c, rng.uniform([8, 8, 8], [20, 20, 20]), rng.uniform(20, 45), _rand_rotation(rng))
    # mandible: anterior half of an ellipsoidal shell
    s.shell(np.array([0.0, 15.0, -25.0]), np.array([jit(62.0), jit(72.0), jit(28.0)]), 9.0,
            rng.uniform(700.0, 1200.0), half=(1, +1))
    # airway: elliptic tube along z
    s.tube(np.array([0.0, jit(22.0)]), np.array([jit(9.0), jit(13.0)]), (-130.0, 15.0), -1000.0)
    # vertebral column with discs
    s.tube(np.array([0.0, -48.0]), np.array([jit(14.0), jit(13.0)]), (-130.0, 10.0), 800.0 + rng.uniform(-50, 50))
    for zc in np.arange(-115.0, 5.0, 24.0):
        s.ellipsoid(np.array([0.0, -48.0, zc]), np.array([15.0, 14.0, 2.5]), 90.0)
    return s


def _coords(shape, spacing, z0, z1, device):
    """mm coordinates of voxel centres for planes z0..z1-1 (origin at the volume centre)."""
    nz, ny, nx = shape
    dz, dy, dx = spacing
    zs = (torch.arange(z0, z1, dtype=torch.float64, device=device) - (nz - 1) / 2.0) * dz
    ys = (torch.arange(ny, dtype=torch.float64, device=device) - (ny - 1) / 2.0) * dy
    xs = (torch.arange(nx, dtype=torch.float64, device=device) - (nx - 1) / 2.0) * dx
    pz, py, px = torch.meshgrid(zs, ys, xs, indexing="ij")
    return px, py, pz


def _bumps(rng, scene, n, sigma_mm):
    c0, ax = scene.body
    cs, amps = [], []
    for _ in range(n):
        cs.append(c0 + rng.uniform(-0.6, 0.6, size=3) * np.minimum(ax, [120, 120, 100]))
        v = rng.normal(size=3)
        amps.append(v / np.linalg.norm(v) * rng.uniform(0.5, 1.0))
    return np.array(cs), np.array(amps), sigma_mm


def _field_mm(bumps, px, py, pz):
    cs, amps, sig = bumps
    out = [torch.zeros_like(px) for _ in range(3)]
    for c, a in zip(cs, amps):
        g = torch.exp(-((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2) / (2.0 * sig * sig))
        for k in range(3):
            out[k] = out[k] + a[k] * g
    return out


def _synthesize(name, cid, pair, shape, spacing, scene_fn, n_bumps, bump_sigma_mm, max_def_mm,
                gain_min, noise_sd, streak_amp, crescent_amp, device, slab):
    rng = np.random.default_rng([SEED_BASE, cid, pair])
    scene = scene_fn(rng)
    bumps = _bumps(rng, scene, n_bumps, bump_sigma_mm)
    phi0 = rng.uniform(0.0, 2.0 * np.pi)
    cres_off = rng.uniform(8.0, 14.0) * np.array([np.cos(phi0 * 1.7), np.sin(phi0 * 1.7)])
    nz, ny, nx = shape
    dz, dy, dx = spacing

    # deformation scale: max |r_true| over the grid equals max_def_mm
    peak = 0.0
    for z0 in range(0, nz, slab):
        px, py, pz = _coords(shape, spacing, z0, min(nz, z0 + slab), device)
        f = _field_mm(bumps, px, py, pz)
        peak = max(peak, float(torch.sqrt(f[0] ** 2 + f[1] ** 2 + f[2] ** 2).max()))
    scale = max_def_mm / peak

    half_diag = float(np.hypot((nx - 1) / 2.0 * dx, (ny - 1) / 2.0 * dy))
    offs = [(ox, oy, oz) for oz in (-0.25, 0.25) for oy in (-0.25, 0.25) for ox in (-0.25, 0.25)]
    ct = np.empty(shape, np.float32)
    cb = np.empty(shape, np.float32)
    rt = np.empty((3,) + shape, np.float32)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        px, py, pz = _coords(shape, spacing, z0, z1, device)
        fx, fy, fz = (scale * f for f in _field_mm(bumps, px, py, pz))
        acc_ct = torch.zeros_like(px)
        acc_cb = torch.zeros_like(px)
        for ox, oy, oz in offs:
            qx, qy, qz = px + ox * dx, py + oy * dy, pz + oz * dz
            acc_ct += scene.eval(qx, qy, qz)
            acc_cb += scene.eval(qx + fx, qy + fy, qz + fz)
        acc_ct /= len(offs)
        acc_cb /= len(offs)
        # cupping: radial quadratic gain on attenuation
        rho = torch.sqrt(px ** 2 + py ** 2) / half_diag
        gain = gain_min + (1.0 - gain_min) * torch.clamp(rho, max=1.0) ** 2
        cbv = gain * (acc_cb + 1000.0) - 1000.0
        body = scene.in_body(px + fx, py + fy, pz + fz)
        if streak_amp:
            theta = torch.atan2(py, px)
            cbv = cbv + torch.where(body, streak_amp * torch.sin(8.0 * theta + phi0), torch.zeros_like(px))
        if crescent_amp:
            c0, ax = scene.body
            rr = 0.85 * min(ax[0], ax[1])
            d1 = (px ** 2 + py ** 2) <= rr * rr
            d2 = ((px - cres_off[0]) ** 2 + (py - cres_off[1]) ** 2) <= rr * rr
            cres = torch.where(d1 & ~d2, torch.full_like(px, crescent_amp), torch.zeros_like(px))
            cres = torch.where(d2 & ~d1, torch.full_like(px, -crescent_amp), cres)
            cbv = cbv + torch.where(body, cres, torch.zeros_like(px))
        cbv = cbv + 100.0
        ct[z0:z1] = acc_ct.cpu().numpy()
        cb[z0:z1] = cbv.cpu().numpy()
        rt[0, z0:z1] = (fx / dx).cpu().numpy()
        rt[1, z0:z1] = (fy / dy).cpu().numpy()
        rt[2, z0:z1] = (fz / dz).cpu().numpy()
    noise = rng.standard_normal(size=shape, dtype=np.float32) * np.float32(noise_sd)
    cb += noise
    return Case(name=name, ct=ct, cbct=cb, r_true=rt, spacing=tuple(spacing))


def make_ellipsoid_pair(shape=(48, 48, 48), pair=0, cid=1, device="cpu", max_def_vox=3.0,
                        noise_sd=20.0, gain_min=0.85):
    """48^3-style ellipsoid phantom (1 mm voxels): body 0-80 HU, soft 0-80 HU,
    bone 700-1500 HU; CBCT = CT warped by 4 Gaussian bumps (sigma 6 voxels,
    max 3 voxels), cupping gain 0.85-1.0, +100 HU, N(0, 20^2) noise."""
    return _synthesize("ellipsoid%dx%dx%d" % (shape[2], shape[1], shape[0]), cid, pair, shape,
                       (1.0, 1.0, 1.0), lambda rng: _ellipsoid_scene(rng, shape), 4, 6.0,
                       max_def_vox, gain_min, noise_sd, 0.0, 0.0, device, slab=64)


def make_hn_pair(shape, pair=0, cid=2, max_def_mm=8.0, device="cpu", fov=HN_FOV):
    """Head-and-neck-like pair on a grid of ``shape`` covering ``fov`` mm:
    6 deformation bumps (sigma 20 mm) scaled to ``max_def_mm``; CBCT with
    cupping gain 0.75-1.0, 8-fold sinusoidal streaks of +-150 HU, a +-80 HU
    crescent, +100 HU and N(0, 30^2) noise."""
    spacing = tuple(fov[i] / shape[i] for i in range(3))
    slab = max(1, int(4_000_000 // (shape[1] * shape[2])))
    return _synthesize("hn%dx%dx%d" % (shape[2], shape[1], shape[0]), cid, pair, shape, spacing,
                       _hn_scene, 6, 20.0, max_def_mm, 0.75, 30.0, 150.0, 80.0, device, slab)


def make_case(name, pair=0, device="cpu"):
    """Inputs of a named workload ('ellipsoid48', 'hn256x256x96', 'hn512x512x160')."""
    cfg = CONFIGS[name]
    if cfg["kind"] == "ellipsoid":
        case = make_ellipsoid_pair(cfg["shape"], pair=pair, cid=cfg["cid"], device=device,
                                   max_def_vox=cfg["max_def_mm"])
    else:
        case = make_hn_pair(cfg["shape"], pair=pair, cid=cfg["cid"], max_def_mm=cfg["max_def_mm"],
                            device=device)
    case.name = name
    case.params = {k: cfg[k] for k in ("patch", "sigma", "levels", "iters")}
    return case


def make_batch(n=16, seed_pair0=0, device="cpu"):
    """Uneven batch of head-and-neck pairs, sizes drawn uniformly from BATCH_SHAPES."""
    rng = np.random.default_rng([SEED_BASE, 4, 10_000])
    picks = rng.integers(0, len(BATCH_SHAPES), size=n)
    return [make_hn_pair(BATCH_SHAPES[k], pair=seed_pair0 + i, cid=4, device=device)
            for i, k in enumerate(picks)]


def smooth_blob_pair(shape, shift, pair=0, n_blobs=40, device="cpu"):
    """Smooth analytic image (sum of Gaussian blobs, evaluated exactly) and its
    copy translated by ``shift`` = (tx, ty, tz) voxels: CBCT(x) = CT(x + t).
    Used for the known-translation check."""
    rng = np.random.default_rng([SEED_BASE, 90, pair])
    nz, ny, nx = shape
    cs = rng.uniform([4, 4, 4], [nx - 5, ny - 5, nz - 5], size=(n_blobs, 3))
    amps = rng.uniform(-400.0, 600.0, size=n_blobs)
    sig = rng.uniform(2.0, 4.0, size=n_blobs)

    def ev(tx, ty, tz):
        pz, py, px = torch.meshgrid(torch.arange(nz, dtype=torch.float64, device=device) + tz,
                                    torch.arange(ny, dtype=torch.float64, device=device) + ty,
                                    torch.arange(nx, dtype=torch.float64, device=device) + tx,
                                    indexing="ij")
        img = torch.zeros_like(px)
        for c, a, s in zip(cs, amps, sig):
            img += a * torch.exp(-((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2) / (2 * s * s))
        return img.cpu().numpy().astype(np.float32)

    return ev(0.0, 0.0, 0.0), ev(*shift)
