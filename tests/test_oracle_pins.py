"""Pins of the FP64 oracle against things other than itself.

Each test checks one oracle function against an independent reference: a
library routine (scipy.ndimage), a closed form, an invariant that follows
from the paper's equations, a hand-worked example, or brute force. A planted
mistake in any oracle step (dropped term, wrong sign, transposed axis, wrong
clamp) fails at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from synth.phantom import make_case, smooth_blob_pair

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.default_rng([7, seed])


# --------------------------------------------------------------------------
# Eq. 3 patch moments
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(11, 10, 9), (7, 6, 5), (2, 4, 3)])
@pytest.mark.parametrize("patch", [(3, 3, 3), (5, 3, 1), (5, 5, 5), (1, 1, 1), (7, 9, 3), (13, 1, 5)])
def test_patch_moments_vs_uniform_filter(shape, patch):
    """Clamped box mean == scipy uniform_filter(mode='nearest'); the variance
    equals E[x^2] - E[x]^2 from the same library filter."""
    img = rng(1).normal(size=shape) * 300.0 + 40.0
    mu, var = oracle.patch_moments(img, patch)
    size = (patch[2], patch[1], patch[0])  # array axes are (z, y, x)
    mu_ref = ndi.uniform_filter(img, size=size, mode="nearest")
    m2_ref = ndi.uniform_filter(img * img, size=size, mode="nearest")
    np.testing.assert_allclose(mu, mu_ref, rtol=0, atol=1e-10 * np.abs(img).max())
    np.testing.assert_allclose(var, m2_ref - mu_ref ** 2, rtol=0, atol=1e-9 * (img ** 2).max())


def test_patch_moments_brute_force():
    """Per-voxel loops over an explicitly clamped patch, numpy mean/var."""
    nz, ny, nx = 4, 5, 6
    img = rng(2).uniform(-1000, 1500, size=(nz, ny, nx))
    px, py, pz = 3, 5, 1
    mu, var = oracle.patch_moments(img, (px, py, pz))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                vals = []
                for k in range(-(pz // 2), pz // 2 + 1):
                    for j in range(-(py // 2), py // 2 + 1):
                        for i in range(-(px // 2), px // 2 + 1):
                            vals.append(img[min(max(z + k, 0), nz - 1), min(max(y + j, 0), ny - 1),
                                            min(max(x + i, 0), nx - 1)])
                assert len(vals) == px * py * pz
                assert abs(mu[z, y, x] - np.mean(vals)) < 1e-10
                assert abs(var[z, y, x] - np.var(vals)) < 1e-8


def test_patch_moments_linear_closed_form():
    """For m = ax + by + cz + e, away from the border the patch mean is the
    centre value and the variance is sum a_d^2 (p_d^2 - 1)/12."""
    nz, ny, nx = 20, 21, 22
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c, e = 3.5, -2.0, 7.25, -400.0
    img = a * x + b * y + c * z + e
    patch = (5, 7, 3)
    mu, var = oracle.patch_moments(img, patch)
    R = [p // 2 for p in patch]
    sl = (slice(R[2], nz - R[2]), slice(R[1], ny - R[1]), slice(R[0], nx - R[0]))
    np.testing.assert_allclose(mu[sl], img[sl], atol=1e-9)
    expect = a * a * (patch[0] ** 2 - 1) / 12 + b * b * (patch[1] ** 2 - 1) / 12 + c * c * (patch[2] ** 2 - 1) / 12
    np.testing.assert_allclose(var[sl], expect, rtol=1e-11)
    # at the x = 0 border of a 1-D ramp with a 3-patch the clamped values are {0, 0, 1}
    mu1, var1 = oracle.patch_moments(np.arange(5.0).reshape(1, 1, 5), (3, 1, 1))
    assert abs(mu1[0, 0, 0] - 1 / 3) < 1e-15 and abs(var1[0, 0, 0] - 2 / 9) < 1e-15


# --------------------------------------------------------------------------
# Eq. 5-6 and I'_s: hand-worked example and the Appendix identity
# --------------------------------------------------------------------------

def test_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "moment_match_3voxel.json")))
    m = np.array(g["m"]).reshape(1, 1, 3)
    s = np.array(g["s"]).reshape(1, 1, 3)
    mu_m, var_m = oracle.patch_moments(m, g["patch"])
    mu_s, var_s = oracle.patch_moments(s, g["patch"])
    for k in range(3):
        assert Fraction(g["mu_m"][k]) == Fraction(mu_m.flat[k]).limit_denominator(1000)
        assert Fraction(g["var_m"][k]) == Fraction(var_m.flat[k]).limit_denominator(1000)
        assert Fraction(g["mu_s"][k]) == Fraction(mu_s.flat[k]).limit_denominator(1000)
        assert Fraction(g["var_s"][k]) == Fraction(var_s.flat[k]).limit_denominator(1000)
    a, b, f = oracle.correct(mu_m, var_m, mu_s, var_s, s)
    np.testing.assert_allclose(a.ravel(), g["a_value"], rtol=1e-13)
    np.testing.assert_allclose(b.ravel(), g["b_value"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(f.ravel(), g["f_value"], rtol=1e-13)
    u = oracle.force(m, f)
    np.testing.assert_allclose(u[0].ravel(), g["u_x_value"], rtol=1e-12, atol=1e-15)
    assert np.all(u[1] == 0) and np.all(u[2] == 0)


def test_appendix_identity_moments_matched():
    """Appendix A.2-A.3: the transformed patch a S_P + b has mean E(M) and
    variance var(M) at every voxel whose static patch is not flat."""
    shape = (6, 7, 8)
    patch = (3, 5, 3)
    m = rng(3).normal(size=shape) * 200.0 + 50.0
    s = rng(4).normal(size=shape) * 30.0 - 100.0
    mu_m, var_m = oracle.patch_moments(m, patch)
    mu_s, var_s = oracle.patch_moments(s, patch)
    a, b, f = oracle.correct(mu_m, var_m, mu_s, var_s, s)
    nz, ny, nx = shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                zi = np.clip(np.arange(z - 1, z + 2), 0, nz - 1)
                yi = np.clip(np.arange(y - 2, y + 3), 0, ny - 1)
                xi = np.clip(np.arange(x - 1, x + 2), 0, nx - 1)
                SP = s[np.ix_(zi, yi, xi)].ravel()
                MP = m[np.ix_(zi, yi, xi)].ravel()
                SPc = a[z, y, x] * SP + b[z, y, x]
                assert abs(SPc.mean() - MP.mean()) < 1e-9
                assert abs(SPc.var() - MP.var()) < 1e-7 * MP.var()
                assert a[z, y, x] > 0


def test_flat_static_patch_matches_mean_only():
    shape = (5, 5, 5)
    m = rng(5).normal(size=shape) * 10
    s = np.full(shape, 123.0)
    mu_m, var_m = oracle.patch_moments(m, (3, 3, 3))
    mu_s, var_s = oracle.patch_moments(s, (3, 3, 3))
    a, b, f = oracle.correct(mu_m, var_m, mu_s, var_s, s)
    assert np.all(a == 1.0)
    np.testing.assert_allclose(f, mu_m, atol=1e-12)


# --------------------------------------------------------------------------
# Eq. 1 force
# --------------------------------------------------------------------------

def test_force_bounded_by_half():
    """AM-GM on Eq. 1's single term: |u| = |d| |g| / (|g|^2 + d^2) <= 1/2."""
    shape = (9, 10, 11)
    m = rng(6).normal(size=shape) * 500
    f = rng(7).normal(size=shape) * 500
    u = oracle.force(m, f)
    mag = np.sqrt((u ** 2).sum(0))
    assert mag.max() <= 0.5 + 1e-15
    assert mag.max() > 0.3


def test_force_direction_and_floor():
    """On f = ramp along x and m = f + d: u = d g / (g^2 + d^2) along x only;
    |d| below eps_d gives u = 0 exactly."""
    nx = 12
    f = np.tile(np.arange(nx, dtype=float) * 4.0, (3, 5, 1))
    for d, expect in [(2.0, 2 * 4 / (16 + 4)), (-8.0, -8 * 4 / (16 + 64)), (5e-4, 0.0)]:
        u = oracle.force(f + d, f, eps_d=1e-3)
        np.testing.assert_allclose(u[0][:, :, 1:-1], expect, rtol=1e-14)
        assert np.all(u[1] == 0) and np.all(u[2] == 0)
    # clamped border: the central difference becomes (f1 - f0) / 2
    u = oracle.force(f + 2.0, f)
    assert abs(u[0][0, 0, 0] - 2 * 2 / (4 + 4)) < 1e-14


# --------------------------------------------------------------------------
# Gaussian regularisation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.7, 1.1, 1.5, 2.0])
def test_gauss_vs_scipy(sigma):
    v = rng(8).normal(size=(9, 14, 17))
    R = int(np.ceil(3 * sigma))
    ref = ndi.gaussian_filter(v, sigma=sigma, mode="nearest", radius=R)
    np.testing.assert_allclose(oracle.gauss(v, sigma), ref, atol=1e-13)
    w = oracle.gauss_taps(sigma)
    assert len(w) == 2 * R + 1 and abs(w.sum() - 1) < 1e-15


def test_gauss_direct_3d_and_invariants():
    sigma = 1.5
    v = rng(9).normal(size=(7, 8, 9))
    w = oracle.gauss_taps(sigma)
    k3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    ref = ndi.correlate(v, k3, mode="nearest")
    np.testing.assert_allclose(oracle.gauss(v, sigma), ref, atol=1e-13)
    # constants are preserved
    c = np.full((6, 7, 8), -3.25)
    np.testing.assert_allclose(oracle.gauss(c, 2.0), c, atol=1e-14)
    # linear fields are preserved away from the border
    z, y, x = np.meshgrid(np.arange(20), np.arange(20), np.arange(20), indexing="ij")
    lin = 0.3 * x - 0.2 * y + 0.1 * z
    g = oracle.gauss(lin.astype(float), 1.5)
    np.testing.assert_allclose(g[5:-5, 5:-5, 5:-5], lin[5:-5, 5:-5, 5:-5], atol=1e-13)


# --------------------------------------------------------------------------
# warp (Sec. 2.1 model), pyramid and up-sampling (Sec. 2.3, A1)
# --------------------------------------------------------------------------

def test_warp_vs_map_coordinates():
    shape = (8, 9, 10)
    ct = rng(10).normal(size=shape) * 400
    r = rng(11).uniform(-3.5, 3.5, size=(3,) + shape)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([z + r[2], y + r[1], x + r[0]])
    ref = ndi.map_coordinates(ct, coords, order=1, mode="nearest")
    np.testing.assert_allclose(oracle.warp(ct, r), ref, atol=1e-10)


def test_warp_special_cases():
    shape = (6, 7, 8)
    ct = rng(12).normal(size=shape) * 400
    assert np.array_equal(oracle.warp(ct, np.zeros((3,) + shape)), ct)
    # integer shift (2, -1, 1): interior equals the shifted image bitwise
    r = np.stack([np.full(shape, 2.0), np.full(shape, -1.0), np.full(shape, 1.0)])
    m = oracle.warp(ct, r)
    assert np.array_equal(m[:-1, 1:, :-2], ct[1:, :-1, 2:])
    # trilinear reproduces linear functions exactly inside the volume
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    lin = 2 * x - 3 * y + 5 * z + 1.0
    rr = rng(13).uniform(-0.4, 0.4, size=(3,) + shape)
    ml = oracle.warp(lin, rr)
    expect = 2 * (x + rr[0]) - 3 * (y + rr[1]) + 5 * (z + rr[2]) + 1
    sl = (slice(1, -1),) * 3
    np.testing.assert_allclose(ml[sl], expect[sl], atol=1e-12)


def test_global_shift_matches_means():
    """Sec. 2.3: the shifted CBCT has the CT's mean; Delta HU has the CT-minus-CBCT sign."""
    ct = rng(20).normal(size=(5, 6, 7)) * 100 + 30.0
    cb = rng(21).normal(size=(5, 6, 7)) * 100 - 170.0
    dhu, s = oracle.global_shift(ct, cb)
    assert abs(dhu - (ct.mean() - cb.mean())) < 1e-10 and dhu > 150
    assert abs(s.mean() - ct.mean()) < 1e-10
    np.testing.assert_allclose(s - cb, dhu, atol=1e-12)


def test_downsample_and_upsample():
    v = rng(14).normal(size=(6, 8, 10))
    ref = v.reshape(3, 2, 4, 2, 5, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(oracle.downsample2(v), ref, atol=1e-14)
    # odd sizes: the last block repeats the edge plane
    w = rng(15).normal(size=(5, 3, 7))
    pad = np.pad(w, ((0, 1), (0, 1), (0, 1)), mode="edge")
    ref = pad.reshape(3, 2, 2, 2, 4, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(oracle.downsample2(w), ref, atol=1e-14)
    assert np.all(oracle.downsample2(np.full((5, 5, 5), 7.5)) == 7.5)
    # up-sampling: 2 * trilinear at (x + 1/2)/2 - 1/2
    rc = rng(16).normal(size=(3, 4, 5, 6))
    fine = (8, 10, 11)
    up = oracle.upsample_field(rc, fine)
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) / 2 - 0.5 for n in fine], indexing="ij")
    for c in range(3):
        ref = 2 * ndi.map_coordinates(rc[c], np.stack([z, y, x]), order=1, mode="nearest")
        np.testing.assert_allclose(up[c], ref, atol=1e-12)
    const = np.full((3, 4, 4, 4), 1.25)
    assert np.allclose(oracle.upsample_field(const, (8, 8, 8)), 2.5, atol=0)


# --------------------------------------------------------------------------
# invariants of the whole iteration
# --------------------------------------------------------------------------

def test_identical_images_give_zero_update():
    """S = CT: Delta HU = 0, a = 1, b = 0, I'_s = CT, u = 0, r stays 0 exactly."""
    c = make_case("ellipsoid48")
    ct = c.ct.astype(np.float64)
    p = oracle.make_params(patch=(5, 5, 5), sigma=1.5, levels=2, iters=(3, 3))
    r, f = oracle.register(ct, ct, p)
    assert np.all(r == 0.0)
    assert np.array_equal(f, ct)


@pytest.mark.parametrize("kind", ["noise", "labels"])
def test_affine_cbct_is_corrected_back(kind):
    """S = alpha CT + beta inside every patch: I'_s = CT (a = 1/alpha), the
    force vanishes and r stays exactly 0. Images with no near-flat patches:
    textured noise, or a label image with values at least 50 HU apart."""
    g = rng(17)
    shape = (12, 13, 14)
    if kind == "noise":
        ct = g.normal(size=shape) * 200 + 30
    else:
        ct = g.choice([-1000.0, -50.0, 0.0, 60.0, 700.0, 1300.0], size=shape)
        ct = ndi.zoom(ct, 1, order=0)
    for alpha, beta in [(0.8, 120.0), (1.3, -250.0)]:
        s = alpha * ct + beta
        p = oracle.make_params(patch=(3, 3, 3), sigma=1.5, levels=1, iters=(4,))
        r, f = oracle.register(ct, s, p)
        assert np.all(r == 0.0)
        np.testing.assert_allclose(f, ct, atol=1e-9 * 1500)


def test_known_translation():
    """CBCT(x) = CT(x + t) for a smooth analytic image (sign and limit).
    (i) one iteration moves r towards t; (ii) r = t is a fixed point of DISC;
    (iii) the warp/force/Gaussian composition without correction (plain
    demons) converges to t; (iv) DISC from r = 0 removes most of the shift
    (moment matching absorbs part of a translation of a locally near-affine
    image, so the DISC limit from zero is only approached)."""
    t = np.array([0.7, -0.4, 0.3])
    shape = (48, 48, 48)
    ct, cb = smooth_blob_pair(shape, tuple(t))
    ct = ct.astype(np.float64)
    cb = cb.astype(np.float64)
    gm = np.sqrt(sum(q ** 2 for q in np.gradient(ct)))
    mask = gm > np.percentile(gm, 70)
    med = lambda r: np.array([np.median(r[c][mask]) for c in range(3)])  # noqa: E731

    p1 = oracle.make_params(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(1,))
    r1, _ = oracle.register(ct, cb, p1)
    assert float(np.sum([r1[c][mask].mean() * t[c] for c in range(3)])) > 0

    r0 = np.stack([np.full(shape, v) for v in t])
    rfix, _, _, _ = oracle.iterate(ct, cb, r0, oracle.make_params(patch=(5, 5, 5), sigma=1.5), n=20)
    assert np.abs(med(rfix) - t).max() < 0.02

    r = np.zeros((3,) + shape)
    for _ in range(50):
        m = oracle.warp(ct, r)
        r = r - oracle.force(m, cb)
        r = np.stack([oracle.gauss(r[c], 1.5) for c in range(3)])
    assert np.abs(med(r) - t).max() < 0.05

    p = oracle.make_params(patch=(7, 7, 7), sigma=1.5, levels=2, iters=(50, 50))
    rd, _ = oracle.register(ct, cb, p)
    assert np.linalg.norm(med(rd) - t) < 0.25 * np.linalg.norm(t)


def _box_moments(v, patch):
    """Patch mean and population variance over the clamped patch (scipy)."""
    size = (patch[2], patch[1], patch[0])
    mu = ndi.uniform_filter(v, size=size, mode="nearest")
    return mu, ndi.uniform_filter(v * v, size=size, mode="nearest") - mu * mu


def _literal_iteration(ct, s, mu_s, var_s, r, patch, sigma, tau=1e-2, eps=1e-3):
    """One DISC iteration (Algorithm A1 steps 1, 3-6) composed from library
    routines: map_coordinates warp, uniform_filter moments, Eq. 5-6,
    clipped central differences for Eq. 1, gaussian_filter. Returns (r, m, f)."""
    shape = ct.shape
    R = int(np.ceil(3 * sigma))
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    m = ndi.map_coordinates(ct, np.stack([z + r[2], y + r[1], x + r[0]]), order=1, mode="nearest")
    mu_m, var_m = _box_moments(m, patch)
    a = np.where(var_s > tau, np.sqrt(np.maximum(var_m, 0) / np.where(var_s > tau, var_s, 1.0)), 1.0)
    f = a * s + (mu_m - a * mu_s)
    grads = []
    for ax in (2, 1, 0):
        n = shape[ax]
        up = np.take(f, np.clip(np.arange(n) + 1, 0, n - 1), axis=ax)
        dn = np.take(f, np.clip(np.arange(n) - 1, 0, n - 1), axis=ax)
        grads.append((up - dn) / 2)
    d = m - f
    den = grads[0] ** 2 + grads[1] ** 2 + grads[2] ** 2 + d * d
    ok = (den > 0) & (np.abs(d) >= eps)
    u = np.stack([np.where(ok, d * gq / np.where(den > 0, den, 1), 0.0) for gq in grads])
    rt = r - u
    r = np.stack([ndi.gaussian_filter(rt[c], sigma, mode="nearest", radius=R) for c in range(3)])
    return r, m, f


def test_literal_iteration_matches_oracle():
    """An independent composition of library routines (map_coordinates,
    uniform_filter, clipped central differences, gaussian_filter) equals
    three oracle iterations on a 12^3 volume."""
    g = rng(18)
    shape = (12, 12, 12)
    ct = g.normal(size=shape) * 300
    s = 0.9 * ndi.shift(ct, (0.3, -0.6, 0.8), order=1, mode="nearest") + 40 + g.normal(size=shape) * 10
    patch, sigma = (3, 5, 3), 1.5
    mu_s, var_s = _box_moments(s, patch)
    r = np.zeros((3,) + shape)
    for _ in range(3):
        r, m, f = _literal_iteration(ct, s, mu_s, var_s, r, patch, sigma)
    ro, mo, fo, _ = oracle.iterate(ct, s, np.zeros((3,) + shape), oracle.make_params(patch=patch, sigma=sigma), n=3)
    np.testing.assert_allclose(mo, m, atol=1e-9)
    np.testing.assert_allclose(fo, f, atol=1e-8)
    np.testing.assert_allclose(ro, r, atol=1e-9)


def _block_mean2(v):
    """2x2x2 block mean with the last plane repeated on odd extents (numpy)."""
    pad = np.pad(v, [(0, n % 2) for n in v.shape], mode="edge")
    nz, ny, nx = pad.shape
    return pad.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def _upsample2(rc, fine):
    """r_fine = 2 trilinear(r_coarse, (x + 1/2)/2 - 1/2), edge replicated (scipy)."""
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) / 2 - 0.5 for n in fine], indexing="ij")
    return np.stack([2 * ndi.map_coordinates(rc[c], np.stack([z, y, x]), order=1, mode="nearest")
                     for c in range(3)])


@pytest.mark.parametrize("shape,levels,iters,shift", [
    ((10, 13, 16), 3, (3, 2, 2), True),
    ((9, 12, 11), 2, (4, 3), False),
])
def test_level_schedule_matches_composition(shape, levels, iters, shift):
    """The whole Algorithm A1 schedule (Sec. 2.3): global shift, block-mean
    pyramid, r = 0 at the coarsest level, the per-level iteration with the
    static moments of that level, and the x2 trilinear up-sampling of the
    field at every level switch -- composed independently from numpy/scipy
    on odd and even dims -- equals orc_register. A dropped up-sampling, a
    field restarted at zero, a missing factor 2 or a level run with the
    wrong static image each changes the final field."""
    g = rng(40)
    ct = ndi.gaussian_filter(g.normal(size=shape), 1.0) * 900 + 50
    s0 = 0.8 * ndi.shift(ct, (0.4, -0.7, 0.5), order=1, mode="nearest") - 130 + g.normal(size=shape) * 15
    patch, sigma = (3, 3, 3), 1.0
    s = s0 + (ct.mean() - s0.mean()) if shift else s0.copy()
    cts, ss = [ct], [s]
    for _ in range(levels - 1):
        cts.insert(0, _block_mean2(cts[0]))
        ss.insert(0, _block_mean2(ss[0]))
    r = np.zeros((3,) + cts[0].shape)
    for lv in range(levels):
        if lv > 0:
            r = _upsample2(r, cts[lv].shape)
        mu_s, var_s = _box_moments(ss[lv], patch)
        for _ in range(iters[lv]):
            r, m, f = _literal_iteration(cts[lv], ss[lv], mu_s, var_s, r, patch, sigma)
    p = oracle.make_params(patch=patch, sigma=sigma, levels=levels, iters=iters, global_shift=shift)
    ro, fo = oracle.register(ct, s0, p)
    assert np.abs(r).max() > 0.05  # the schedule moved the field
    np.testing.assert_allclose(ro, r, atol=1e-9)
    np.testing.assert_allclose(fo, f, atol=1e-8 * np.abs(f).max())


def test_point_evaluators_agree_with_whole_volume():
    """The *_pts functions (FP32 inputs) equal the whole-volume oracle steps."""
    g = rng(19)
    shape = (9, 10, 11)
    ct = (g.normal(size=shape) * 300).astype(np.float32)
    s = (g.normal(size=shape) * 300).astype(np.float32)
    r = g.uniform(-2, 2, size=(3,) + shape).astype(np.float32)
    pts = g.choice(ct.size, 60, replace=False)
    m = oracle.warp(ct, r)
    np.testing.assert_allclose(oracle.warp_pts(ct, r, pts), m.ravel()[pts], rtol=1e-14, atol=1e-12)
    m32 = m.astype(np.float32)
    patch = (3, 5, 7)
    mu_m, var_m = oracle.patch_moments(m32, patch)
    mu_s, var_s = oracle.patch_moments(s, patch)
    _, _, f = oracle.correct(mu_m, var_m, mu_s, var_s, s)
    np.testing.assert_allclose(oracle.correct_pts(m32, s, patch, pts), f.ravel()[pts], rtol=1e-12, atol=1e-9)
    f32 = f.astype(np.float32)
    u = oracle.force(m32, f32)
    rt = r.astype(np.float64) - u
    got = oracle.force_pts(m32, f32, r, pts)
    for c in range(3):
        np.testing.assert_allclose(got[:, c], rt[c].ravel()[pts], rtol=1e-13, atol=1e-13)
    rt32 = rt.astype(np.float32)
    gs = np.stack([oracle.gauss(rt32[c], 1.5) for c in range(3)])
    got = oracle.gauss_pts(rt32, 1.5, pts)
    for c in range(3):
        np.testing.assert_allclose(got[:, c], gs[c].ravel()[pts], atol=1e-12)


# --------------------------------------------------------------------------
# Differentiable DISC: SSD between m = warp(CT, r) and I'_s (Eq. 3-6)
# --------------------------------------------------------------------------

def _ssd_case(shape, seed):
    g = rng(seed)
    ct = g.normal(0.0, 100.0, shape).cumsum(axis=2)
    s = 0.8 * ct + g.normal(0.0, 20.0, shape) + 50.0
    # fractional parts kept away from 0 and 1 so that +-eps never crosses a
    # cell of the piecewise-trilinear warp
    r = np.floor(g.uniform(-1.5, 1.5, (3,) + shape)) + g.uniform(0.2, 0.8, (3,) + shape)
    return ct, s, r


@pytest.mark.parametrize("patch", [(3, 3, 3), (5, 3, 1), (9, 9, 9), (1, 3, 5)])
def test_ssd_gradient_vs_finite_differences(patch):
    """The analytic dL/dr equals central differences of the oracle's own loss
    at every coordinate of a small, edge-dominated volume (every patch is
    clamped somewhere), and the FD error falls as eps^2 (so it is truncation,
    not a wrong term)."""
    ct, s, r = _ssd_case((5, 6, 7), 3)
    g = oracle.ssd_grad(ct, s, r, patch)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = np.zeros_like(r)
        for idx in np.ndindex(r.shape):
            rp = r.copy()
            rm = r.copy()
            rp[idx] += eps
            rm[idx] -= eps
            fd[idx] = (oracle.ssd_loss(ct, s, rp, patch) - oracle.ssd_loss(ct, s, rm, patch)) / (2 * eps)
        errs.append(np.abs(g - fd).max() / np.abs(fd).max())
    assert errs[0] < 1e-5
    assert errs[1] < errs[0] / 30.0


def test_ssd_minimum_at_consistent_images():
    """S = CT or S = alpha CT + beta at r = 0: I'_s = m everywhere, so L = 0
    and the gradient vanishes (a minimum)."""
    g = rng(4)
    ct = g.normal(0.0, 200.0, (6, 7, 8)).cumsum(axis=1)
    r = np.zeros((3,) + ct.shape)
    for s in (ct.copy(), 1.7 * ct - 300.0):
        assert oracle.ssd_loss(ct, s, r, (3, 3, 3)) < 1e-16 * (ct * ct).sum()
        gr = oracle.ssd_grad(ct, s, r, (3, 3, 3))
        assert np.abs(gr).max() < 1e-9 * np.abs(ct).max()


def test_ssd_flat_patches_and_unit_patch():
    """A 1x1x1 patch makes every static patch flat (a = 1, I'_s = m): L = 0
    and gradient 0 up to rounding. A constant static image makes I'_s = E(M): L is the sum of
    squared deviations of m from its patch mean, checked against scipy."""
    ct, s, r = _ssd_case((4, 5, 6), 5)
    # I'_s = s + (m - s) equals m up to one rounding
    scale = np.abs(ct).max()
    assert oracle.ssd_loss(ct, s, r, (1, 1, 1)) <= ct.size * (1e-15 * scale) ** 2
    assert np.abs(oracle.ssd_grad(ct, s, r, (1, 1, 1))).max() <= 1e-12 * scale * scale
    flat = np.full(ct.shape, 40.0)
    m = oracle.warp(ct, r)
    mu = ndi.uniform_filter(m, size=(3, 3, 3), mode="nearest")
    ref = ((m - mu) ** 2).sum()
    assert abs(oracle.ssd_loss(ct, flat, r, (3, 3, 3)) - ref) <= 1e-10 * ref


def test_ssd_gradient_point_evaluator():
    """The point evaluator (FP32 state, local recomputation of moments)
    equals the whole-volume gradient on the same FP32-rounded inputs."""
    ct, s, r = _ssd_case((6, 7, 9), 6)
    ct32, s32, r32 = (a.astype(np.float32) for a in (ct, s, r))
    for patch in ((3, 3, 3), (5, 3, 1), (9, 9, 9)):
        g = oracle.ssd_grad(ct32.astype(np.float64), s32.astype(np.float64), r32.astype(np.float64), patch)
        pts = np.arange(ct.size)
        gp = oracle.ssd_grad_pts(ct32, s32, r32, patch, pts)
        assert np.abs(gp.T.reshape(g.shape) - g).max() <= 1e-12 * np.abs(g).max()


# --------------------------------------------------------------------------
# Eq. 1 double force and the Sec. 2.3 stopping rule
# --------------------------------------------------------------------------

def test_double_force_closed_form_on_linear_images():
    """f = alpha x, m = beta x + c: both gradients are constant along x in the
    interior, so u_x = d alpha / (alpha^2 + d^2) + d beta / (beta^2 + d^2)
    with d = m - f, and u_y = u_z = 0 there."""
    shape = (5, 6, 12)
    x = np.broadcast_to(np.arange(shape[2], dtype=np.float64), shape)
    for alpha, beta, c in ((3.0, 2.0, 7.0), (-1.5, 4.0, -2.0), (2.0, 2.0, 0.5)):
        f = alpha * x
        m = beta * x + c
        u = oracle.force_double(m, f, 0.0)
        d = m - f
        ref = d * alpha / (alpha ** 2 + d ** 2) + d * beta / (beta ** 2 + d ** 2)
        inner = (slice(None), slice(None), slice(1, -1))
        assert np.allclose(u[0][inner], ref[inner], rtol=1e-13, atol=1e-15)
        assert np.abs(u[1:]).max() == 0.0


def test_double_force_is_static_term_minus_swapped_term():
    """The moving-gradient term of Eq. 1 is the static-gradient term with the
    images' roles swapped and the sign of d reversed, so
    force_double(m, f) = force(m, f) - force(f, m) voxel by voxel; and both
    vanish on identical images."""
    g = rng(8)
    m = g.normal(0.0, 200.0, (7, 8, 9)).cumsum(axis=0)
    f = m + g.normal(0.0, 30.0, m.shape)
    for eps in (0.0, 1e-3, 5.0):
        u = oracle.force_double(m, f, eps)
        ref = oracle.force(m, f, eps) - oracle.force(f, m, eps)
        assert np.allclose(u, ref, rtol=1e-12, atol=1e-14)
    assert np.abs(oracle.force_double(m, m.copy(), 1e-3)).max() == 0.0


def test_stopping_rule():
    """l^(k) is the definition written out (two fixed-count runs of the
    oracle give r^(k) and r^(k+1)); the level ends at the first k >= lag with
    l^(k-lag) - l^(k) <= eps; identical images stop right at k = lag; a
    non-positive eps keeps the fixed counts."""
    from synth.phantom import make_ellipsoid_pair

    c = make_ellipsoid_pair((20, 22, 24), pair=5)
    ct, cb = c.ct.astype(np.float64), c.cbct.astype(np.float64)
    lag, K = 3, 14
    # full history with a rule that never fires
    p_all = oracle.make_params(patch=(3, 3, 3), iters=(K,), stop_eps=1e-300, stop_lag=lag)
    _, _, n_all, h_all = oracle.register_ex(ct, cb, p_all)
    h = h_all[0]
    assert n_all == [K] and np.isinf(h[0])
    for k in (1, 5, 9):
        rk, _ = oracle.register(ct, cb, oracle.make_params(patch=(3, 3, 3), iters=(k,)))
        rk1, _ = oracle.register(ct, cb, oracle.make_params(patch=(3, 3, 3), iters=(k + 1,)))
        num = np.sqrt(((rk1 - rk) ** 2).sum(axis=0)).sum()
        den = np.sqrt((rk ** 2).sum(axis=0)).sum()
        assert abs(h[k] - num / den) <= 1e-12 * num / den
    drops = h[:-lag] - h[lag:]  # l^(k - lag) - l^(k) for k = lag .. K-1
    eps = float(np.median(drops[np.isfinite(drops)]))
    first = next(k for k in range(lag, K) if h[k - lag] - h[k] <= eps)
    _, _, n, hh = oracle.register_ex(ct, cb, oracle.make_params(patch=(3, 3, 3), iters=(K,), stop_eps=eps,
                                                                 stop_lag=lag))
    assert n == [first + 1] and np.array_equal(hh[0], h[:first + 1])
    _, _, n_id, h_id = oracle.register_ex(ct, ct.copy(), oracle.make_params(
        patch=(3, 3, 3), iters=(K,), stop_eps=1e-4, stop_lag=lag))
    assert n_id == [lag + 1] and np.all(h_id[0] == 0.0)
    _, _, n_off, _ = oracle.register_ex(ct, cb, oracle.make_params(patch=(3, 3, 3), iters=(K,), stop_eps=0.0))
    assert n_off == [K]


# --------------------------------------------------------------------------
# Eq. 7-10: mask and weighted fill of a, b
# --------------------------------------------------------------------------

def test_fill_weighted_average_hand_worked():
    """A 3-voxel line, middle voxel masked: Eq. 8-10 by hand,
    a = (w0 a0 + w2 a2) / (w0 + w2) with w = exp(-(s_i - s_x)^2 / h^2)."""
    s = np.array([0.0, 10.0, 30.0]).reshape(1, 1, 3)
    a0 = np.array([1.0, 9.0, 3.0]).reshape(s.shape)
    b0 = np.array([-5.0, 9.0, 7.0]).reshape(s.shape)
    valid = np.array([1, 0, 1], bool).reshape(s.shape)
    A, B, used = oracle.fill(a0, b0, valid, s, h=20.0, t=(3, 1, 1), passes=4)
    w0, w2 = np.exp(-100.0 / 400.0), np.exp(-400.0 / 400.0)
    assert used == 1
    assert abs(A[0, 0, 1] - (w0 * 1.0 + w2 * 3.0) / (w0 + w2)) < 1e-15
    assert abs(B[0, 0, 1] - (w0 * -5.0 + w2 * 7.0) / (w0 + w2)) < 1e-14
    assert A[0, 0, 0] == 1.0 and A[0, 0, 2] == 3.0  # unmasked voxels unchanged


def test_fill_passes_jacobi_reach_and_leftover():
    """A line valid only at x = 0, T of radius 1: pass p fills x = p (a voxel
    filled in a pass is not used in that same pass), every filled value is
    a0[0], and voxels beyond the last pass keep their Eq. 5-6 values."""
    n = 8
    s = np.zeros((1, 1, n))
    a0 = np.arange(n, dtype=float).reshape(s.shape) + 2.0
    b0 = -a0
    valid = np.zeros(s.shape, bool)
    valid[0, 0, 0] = True
    A, B, used = oracle.fill(a0, b0, valid, s, h=50.0, t=(3, 1, 1), passes=3)
    assert used == 3
    assert np.array_equal(A[0, 0, :4], [2.0] * 4) and np.array_equal(B[0, 0, :4], [-2.0] * 4)
    assert np.array_equal(A[0, 0, 4:], a0[0, 0, 4:]) and np.array_equal(B[0, 0, 4:], b0[0, 0, 4:])
    A, _, used = oracle.fill(a0, b0, valid, s, h=50.0, t=(3, 1, 1), passes=20)
    assert used == n - 1 and np.all(A == 2.0)
    # the pass that filled each voxel: x = p in pass p, 255 past the last pass
    A2, B2, used2, pass_of = oracle.fill_ex(a0, b0, valid, s, h=50.0, t=(3, 1, 1), passes=3)
    assert used2 == 3 and np.array_equal(pass_of[0, 0], [0, 1, 2, 3, 255, 255, 255, 255])
    ref_a, ref_b, _ = oracle.fill(a0, b0, valid, s, h=50.0, t=(3, 1, 1), passes=3)
    assert np.array_equal(A2, ref_a) and np.array_equal(B2, ref_b)


def test_fill_far_intensities_still_fill():
    """Every Eq. 10 weight is positive, so a masked voxel with valid
    neighbours is always filled, however far their intensities are: with
    dS = 40 h and 41 h (exp(-1600) underflows in FP64) the fill is the Eq. 9
    average whose weight ratio is exp(-(41^2 - 40^2)) = exp(-81); with a
    single neighbour at dS = 50 h it is that neighbour's (a, b) exactly."""
    h = 10.0
    s = np.array([400.0, 0.0, -410.0]).reshape(1, 1, 3)
    a0 = np.array([2.0, 0.0, 5.0]).reshape(s.shape)
    b0 = np.array([-3.0, 0.0, 11.0]).reshape(s.shape)
    valid = np.array([1, 0, 1], bool).reshape(s.shape)
    A, B, used = oracle.fill(a0, b0, valid, s, h=h, t=(3, 1, 1), passes=1)
    r = np.exp(-81.0)
    assert used == 1
    assert abs(A[0, 0, 1] - (2.0 + r * 5.0) / (1.0 + r)) < 1e-15
    assert abs(B[0, 0, 1] - (-3.0 + r * 11.0) / (1.0 + r)) < 1e-14
    s1 = np.array([500.0, 0.0]).reshape(1, 1, 2)
    A, B, _ = oracle.fill(a0[..., :2], b0[..., :2], valid[..., :2], s1, h=h, t=(3, 1, 1), passes=1)
    assert A[0, 0, 1] == 2.0 and B[0, 0, 1] == -3.0


def test_fill_region_stays_inside_the_volume():
    """T counts only voxels inside the volume (no edge replication): with
    uniform s, x = 1 masked and radius 2 along x, the fill is the plain mean
    over x = 0, 2, 3; a replicated edge would count x = 0 twice."""
    s = np.zeros((1, 1, 5))
    a0 = np.array([1.0, 0.0, 4.0, 7.0, 100.0]).reshape(s.shape)
    valid = np.array([1, 0, 1, 1, 1], bool).reshape(s.shape)
    A, _, _ = oracle.fill(a0, a0, valid, s, h=10.0, t=(5, 1, 1), passes=1)
    assert abs(A[0, 0, 1] - (1.0 + 4.0 + 7.0) / 3.0) < 1e-15


def test_mask_and_median_against_library_moments():
    """xi = |m - s| > HU0 or a outside [a_min, a_max] (Eq. 7), with a from
    scipy box moments; a_m = numpy median over voxels where neither patch is
    flat; the unmasked voxels keep Eq. 5-6 values."""
    g = rng(9)
    shape = (6, 9, 11)
    m = g.normal(0.0, 100.0, shape).cumsum(axis=2)
    s = 0.9 * m + g.normal(0.0, 40.0, shape)
    size = (3, 3, 3)

    def mom(v):
        mu = ndi.uniform_filter(v, size=size, mode="nearest")
        return mu, np.maximum(ndi.uniform_filter(v * v, size=size, mode="nearest") - mu * mu, 0.0)

    mu_m, var_m = mom(m)
    mu_s, var_s = mom(s)
    a = np.where(var_s > 1e-2, np.sqrt(var_m / var_s), 1.0)
    b = mu_m - a * mu_s
    both = (var_s > 1e-2) & (var_m > 1e-2)
    am = oracle.a_median(m, s, (3, 3, 3))
    assert abs(am - np.median(np.sqrt(var_m[both] / var_s[both]))) < 1e-9
    hu0, lo, hi = 60.0, 0.5 * am, 1.5 * am
    A, B, xi, _ = oracle.mask_fill(m, s, (3, 3, 3), 1e-2, hu0, lo, hi, h=hu0, passes=10)
    ref = (np.abs(m - s) > hu0) | (a < lo) | (a > hi)
    near = (np.abs(np.abs(m - s) - hu0) < 1e-6) | (np.abs(a - lo) < 1e-9) | (np.abs(a - hi) < 1e-9)
    assert np.array_equal(xi[~near], ref[~near]) and 0.05 < xi.mean() < 0.95
    keep = ~xi
    assert np.allclose(A[keep], a[keep], rtol=1e-9) and np.allclose(B[keep], b[keep], rtol=1e-9, atol=1e-6)


def test_mask_off_limits_and_identical_images():
    """A mask that never fires (huge HU0, a range [0, inf)) gives the hot
    path bitwise; identical images stay an exact fixed point with the mask
    on (a = 1 everywhere, nothing masked)."""
    from synth.phantom import make_case

    c = make_case("ellipsoid48")
    ct, cb = c.ct.astype(np.float64), c.cbct.astype(np.float64)
    base = dict(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(4,))
    r0, f0 = oracle.register(ct, cb, oracle.make_params(**base))
    r1, f1 = oracle.register(ct, cb, oracle.make_params(mask_mode=1, hu0=1e9, a_lo=0.0, a_hi=1e300, **base))
    assert np.array_equal(r0, r1) and np.array_equal(f0, f1)
    r2, f2 = oracle.register(ct, ct.copy(), oracle.make_params(mask_mode=1, **base))
    assert np.abs(r2).max() == 0.0


def test_chunked_schedule_equals_register():
    """oracle.register_steps (the schedule in chunks, for long runs that
    report progress) runs the same C steps in the same order as
    orc_register: bitwise equal field and corrected image, and every chunk
    reported once per level in order."""
    g = rng(41)
    shape = (11, 14, 17)
    ct = ndi.gaussian_filter(g.normal(size=shape), 1.0) * 900 + 50
    s0 = 0.9 * ndi.shift(ct, (0.3, 0.6, -0.4), order=1, mode="nearest") + 70 + g.normal(size=shape) * 10
    p = oracle.make_params(patch=(3, 3, 5), sigma=1.2, levels=2, iters=(5, 7))
    seen = []
    rs, fs = oracle.register_steps(ct, s0, p, chunk=3, on_chunk=lambda l, k, r, f: seen.append((l, k)))
    ro, fo = oracle.register(ct, s0, p)
    assert seen == [(0, 3), (0, 5), (1, 3), (1, 6), (1, 7)]
    assert np.abs(ro).max() > 0.05
    assert np.array_equal(rs, ro) and np.array_equal(fs, fo)
