"""Shared helpers for the GPU parity tests (tolerances, tensors, sampling)."""
import numpy as np

# Per-step parity bar: max|gpu - ref| / max|ref| per output array.
STEP_RTOL = 1e-4
# Final field after a whole registration: per-voxel Euclidean error (voxels).
FIELD_MAX = 0.05
FIELD_RMS = 0.01


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(gpu - ref).max() / (scale if scale > 0 else 1.0))


def field_err(r_gpu, r_ref):
    e = np.sqrt(((np.asarray(r_gpu, np.float64) - np.asarray(r_ref, np.float64)) ** 2).sum(0))
    return float(e.max()), float(np.sqrt((e ** 2).mean()))


def to_dev(a, dev="cuda:0"):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def to_np(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def sample_points(shape, n, seed, include_corners=True):
    """Linear voxel indices: n random voxels plus every corner and a few
    voxels on each face (the clamped-stencil cases)."""
    nz, ny, nx = shape
    g = np.random.default_rng([99, seed])
    pts = list(g.integers(0, nz * ny * nx, size=n))
    if include_corners:
        for z in (0, nz - 1):
            for y in (0, ny - 1):
                for x in (0, nx - 1):
                    pts.append((z * ny + y) * nx + x)
        for _ in range(4):
            x, y, z = g.integers(0, nx), g.integers(0, ny), g.integers(0, nz)
            for zz, yy, xx in ((0, y, x), (nz - 1, y, x), (z, 0, x), (z, ny - 1, x), (z, y, 0), (z, y, nx - 1)):
                pts.append((zz * ny + yy) * nx + xx)
    return np.unique(np.array(pts, dtype=np.int64))
