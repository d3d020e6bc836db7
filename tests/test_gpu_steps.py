"""Per-step parity of the HIP kernels against the FP64 oracle.

Every step runs through the C ABI (disc_step_*), i.e. the same kernels as
disc_iterate, on identical FP32 inputs; the oracle promotes them to FP64.
Shapes span several 32 x 32 (and 16 x 16) tiles with ragged tails in x, y
and z, plus degenerate volumes (single voxel, single row, dims below the
patch size).
Bar: max|gpu - ref| / max|ref| <= 1e-4 per output array.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import STEP_RTOL, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(29, 37, 150), (9, 17, 70), (1, 1, 1), (2, 3, 1), (1, 1, 67), (5, 1, 3), (3, 70, 2)]


def rng(seed):
    return np.random.default_rng([31, seed])


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


@pytest.mark.parametrize("shape", SHAPES)
def test_warp(disc, shape):
    g = rng(1)
    ct = (g.normal(size=shape) * 400).astype(np.float32)
    r = g.uniform(-6, 6, size=(3,) + shape).astype(np.float32)
    m = to_np(disc.warp(to_dev(ct), to_dev(r)))
    ref = oracle.warp(ct, r)
    assert rel_err(m, ref) <= STEP_RTOL


def test_warp_zero_and_integer_fields_are_exact(disc):
    shape = (7, 9, 70)
    ct = (rng(2).normal(size=shape) * 400).astype(np.float32)
    m = to_np(disc.warp(to_dev(ct), to_dev(np.zeros((3,) + shape))))
    assert np.array_equal(m, ct)
    r = np.stack([np.full(shape, 2.0), np.full(shape, -1.0), np.full(shape, 1.0)]).astype(np.float32)
    m = to_np(disc.warp(to_dev(ct), to_dev(r)))
    assert np.array_equal(m[:-1, 1:, :-2], ct[1:, :-1, 2:])


PATCHES = [(3, 3, 3), (5, 3, 1), (11, 11, 11), (7, 9, 15), (31, 31, 1), (1, 1, 1), (15, 15, 15)]


@pytest.mark.parametrize("patch", PATCHES)
@pytest.mark.parametrize("shape", [(29, 37, 150), (3, 2, 5)])
def test_correct(disc, shape, patch):
    g = rng(3)
    m = (g.normal(size=shape) * 300 + 40).astype(np.float32)
    s = (0.8 * m + g.normal(size=shape) * 50 - 60).astype(np.float32)
    ys = disc.static_stats(to_dev(s), patch, 1e-2)
    f = to_np(disc.correct(to_dev(m), ys, patch))
    mu_m, var_m = oracle.patch_moments(m, patch)
    mu_s, var_s = oracle.patch_moments(s, patch)
    _, _, ref = oracle.correct(mu_m, var_m, mu_s, var_s, s, 1e-2)
    assert rel_err(f, ref) <= STEP_RTOL


def test_correct_on_phantom_with_flat_regions(disc):
    """Ellipsoid phantom: exactly flat CT patches (var_M = 0), flat static
    patches (var_S = 0 in a constant-CBCT block) and strong edges."""
    from synth.phantom import make_ellipsoid_pair

    c = make_ellipsoid_pair((40, 44, 48), pair=5)
    s = c.cbct.copy()
    s[:8, :10, :12] = 250.0  # a flat static region: mean-only matching there
    for patch in [(5, 5, 5), (11, 11, 11)]:
        ys = disc.static_stats(to_dev(s), patch, 1e-2)
        f = to_np(disc.correct(to_dev(c.ct), ys, patch))
        mu_m, var_m = oracle.patch_moments(c.ct, patch)
        mu_s, var_s = oracle.patch_moments(s, patch)
        _, _, ref = oracle.correct(mu_m, var_m, mu_s, var_s, s, 1e-2)
        assert rel_err(f, ref) <= STEP_RTOL
        assert (var_s <= 1e-2).sum() > 0


@pytest.mark.parametrize("shape", SHAPES + [(40, 70, 66)])
@pytest.mark.parametrize("sigma", [1.5, 2.0])
def test_force_and_smooth(disc, shape, sigma):
    """Production force + Gaussian kernels: r - u against the oracle's Eq. 1
    force, and the smoothed field against the oracle Gaussian of the GPU's
    own r - u (identical FP32 input)."""
    g = rng(4)
    m = (g.normal(size=shape) * 300).astype(np.float32)
    f = (m + g.normal(size=shape) * 40).astype(np.float32)
    f.flat[:: 7] = m.flat[:: 7]  # d = 0 exactly: zero force
    r = g.uniform(-2, 2, size=(3,) + shape).astype(np.float32)
    out, rt = disc.force_smooth(to_dev(m), to_dev(f), to_dev(r), sigma, 1e-3, want_rt=True)
    out, rt = to_np(out), to_np(rt)
    u_ref = oracle.force(m, f, 1e-3)
    ref = r.astype(np.float64) - u_ref
    assert rel_err(rt, ref) <= STEP_RTOL
    u_gpu = r.astype(np.float64) - rt.astype(np.float64)
    assert np.abs(u_gpu - u_ref).max() <= 1e-5
    assert np.sqrt((u_gpu ** 2).sum(0)).max() <= 0.5 + 1e-6
    sref = np.stack([oracle.gauss(rt[c], sigma) for c in range(3)])
    assert rel_err(out, sref) <= STEP_RTOL


@pytest.mark.parametrize("sigma", [0.3, 0.7, 1.5, 2.0, 2.6])
@pytest.mark.parametrize("shape", [(29, 37, 150), (4, 3, 2), (1, 1, 1)])
def test_smooth(disc, shape, sigma):
    g = rng(5)
    rt = g.normal(size=(3,) + shape).astype(np.float32)
    r = to_np(disc.smooth(to_dev(rt), sigma))
    ref = np.stack([oracle.gauss(rt[c], sigma) for c in range(3)])
    assert rel_err(r, ref) <= STEP_RTOL


def test_shift(disc):
    g = rng(6)
    shape = (29, 37, 150)
    ct = (g.normal(size=shape) * 300 + 20).astype(np.float32)
    cb = (g.normal(size=shape) * 300 - 180).astype(np.float32)
    s, dhu = disc.shift(to_dev(ct), to_dev(cb))
    dref, sref = oracle.global_shift(ct, cb)
    assert abs(float(to_np(dhu)[0]) - dref) <= 1e-9 * abs(dref)
    assert rel_err(to_np(s), sref) <= 1e-6


@pytest.mark.parametrize("shape", [(29, 37, 150), (5, 3, 7), (1, 1, 1), (2, 2, 2)])
def test_downsample(disc, shape):
    v = (rng(7).normal(size=shape) * 500).astype(np.float32)
    out = to_np(disc.downsample(to_dev(v)))
    assert rel_err(out, oracle.downsample2(v)) <= STEP_RTOL


@pytest.mark.parametrize("coarse,fine", [((15, 19, 75), (29, 37, 150)), ((3, 2, 4), (6, 4, 8)), ((1, 1, 1), (2, 1, 2))])
def test_upsample_field(disc, coarse, fine):
    rc = rng(8).normal(size=(3,) + coarse).astype(np.float32)
    rf = to_np(disc.upsample_field(to_dev(rc), fine))
    assert rel_err(rf, oracle.upsample_field(rc, fine)) <= STEP_RTOL


def test_copy_kernel(disc):
    import torch

    a = torch.randn(1 << 20, device="cuda:0")
    b = torch.empty_like(a)
    disc.copy_kernel(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_invalid_arguments_raise(disc):
    import torch

    x = torch.zeros((4, 4, 4), device="cuda:0")
    with pytest.raises(disc.DiscError):
        disc.correct(x, x, (4, 3, 3))
    with pytest.raises(disc.DiscError):
        disc.smooth(torch.zeros((3, 4, 4, 4), device="cuda:0"), 0.0)
    with pytest.raises(disc.DiscError):
        disc.static_stats(x, (3, 3, 17))
