"""Whole-volume parity at the benchmarked size and launch geometry.

The 256x256x96 head-and-neck pair with patch 11^3 and sigma 2 is the shape
the timed registration runs at its finest level, so every kernel here takes
the launch geometry it takes there: the 32 x 32 moments tile with 24-plane
z chunks (correction and the Eq. 7 mask sweep), the force + xy pipeline with
24-plane chunks, and the ring z pass with 6-plane chunks and the fused warp
of the next iteration. Each step runs through the C ABI on identical FP32
inputs and is compared with the FP64 oracle at every voxel (not samples).

Bars: per output array max|gpu - ref| / max|ref| <= 1e-4; the force also per
voxel to 1e-5 voxel absolute. The Eq. 7 mask is a threshold decision: voxels
whose oracle margin to HU_0 or to a_min / a_max lies within FP32 rounding
may take either side; every other voxel must take the oracle's side, and the
fill is then compared from the GPU's own mask.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import FIELD_MAX, FIELD_RMS, STEP_RTOL, field_err, rel_err, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

NAME = "hn256x256x96"


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


@pytest.fixture(scope="module")
def case():
    from synth.phantom import make_case

    return make_case(NAME)


@pytest.fixture(scope="module")
def mid_state(disc, case):
    """A mid-registration state: a few finest-level iterations from a
    partial version of the known deformation."""
    from synth.phantom import CONFIGS

    cfg = CONFIGS[NAME]
    ct, cb = to_dev(case.ct), to_dev(case.cbct)
    reg = disc.Registration(patch=cfg["patch"], sigma=cfg["sigma"], levels=1, iters=(3,))
    reg.set_volumes(ct, cb)
    reg.set_field(to_dev(0.6 * case.r_true))
    reg.run()
    r = reg.field()
    s, _ = disc.shift(ct, cb)
    return dict(ct=ct, cb=cb, r=r, s=s, patch=cfg["patch"], sigma=cfg["sigma"])


def test_steps_whole_volume(disc, mid_state):
    st = mid_state
    ct, r, s, patch, sigma = st["ct"], st["r"], st["s"], st["patch"], st["sigma"]
    m = disc.warp(ct, r)
    ys = disc.static_stats(s, patch)
    f = disc.correct(m, ys, patch)
    out, rt, m_next = disc.force_smooth(m, f, r, sigma, want_rt=True, ct=ct)
    ct_h, r_h, s_h, m_h, f_h, out_h, rt_h, mn_h = (to_np(x) for x in (ct, r, s, m, f, out, rt, m_next))
    assert np.abs(r_h).max() > 0.5

    e_w = rel_err(m_h, oracle.warp(ct_h, r_h))
    mu_m, var_m = oracle.patch_moments(m_h, patch)
    mu_s, var_s = oracle.patch_moments(s_h, patch)
    _, _, f_ref = oracle.correct(mu_m, var_m, mu_s, var_s, s_h)
    e_c = rel_err(f_h, f_ref)
    u_ref = oracle.force(m_h, f_h)
    rt_ref = r_h.astype(np.float64) - u_ref
    e_f = max(rel_err(rt_h[c], rt_ref[c]) for c in range(3))
    u_err = float(np.abs((r_h.astype(np.float64) - rt_h) - u_ref).max())
    g_ref = np.stack([oracle.gauss(rt_h[c], sigma) for c in range(3)])
    e_g = max(rel_err(out_h[c], g_ref[c]) for c in range(3))
    e_n = rel_err(mn_h, oracle.warp(ct_h, out_h))
    print("256x256x96 whole-volume rel errors: warp %.2g correct %.2g force %.2g (u abs %.2g) gauss %.2g "
          "next warp %.2g" % (e_w, e_c, e_f, u_err, e_g, e_n))
    assert max(e_w, e_c, e_f, e_g, e_n) <= STEP_RTOL
    assert u_err <= 1e-5


def test_registration_iterations_whole_volume(disc, case, mid_state):
    """Two iterations of disc_iterate itself from the mid-registration field
    (the second one uses the m made by the first one's z pass), against two
    oracle iterations from the same FP32 state.

    The steps match at about 1e-7 on identical inputs (above), but here the
    oracle keeps m and I'_s in FP64 while the GPU stores them in FP32. Where
    the two images agree to a fraction of an HU and the gradient of I'_s is
    as small, the Eq. 1 force is ill-conditioned in d = m - I'_s: with |d|
    and |grad| near eps_d = 1e-3 HU, the FP32 rounding of m and I'_s (at
    most 1.2e-4 HU below 2048 HU) moves u by up to about 0.06 voxel at that
    voxel, and the sigma-2 Gaussian (peak weight 0.0079) spreads it as at
    most about 5e-4 voxel of field. So the corrected image is held to the
    per-step bar, the field to 1e-3 voxel after one iteration and to the
    final-field bars after two (where the first iteration's difference has
    gone through the warp)."""
    st = mid_state
    reg = disc.Registration(patch=st["patch"], sigma=st["sigma"], levels=1, iters=(2,))
    reg.set_volumes(st["ct"], st["cb"])
    reg.set_field(st["r"])
    ct_h, r0_h, s_h = to_np(st["ct"]), to_np(st["r"]), to_np(st["s"])
    p = oracle.make_params(patch=st["patch"], sigma=st["sigma"], levels=1, iters=(1,))
    mu_s, var_s = oracle.patch_moments(s_h, st["patch"])
    r_ref = r0_h
    for k in range(2):
        reg.iterate(1)
        r_ref, _, f_ref, _ = oracle.iterate(ct_h, s_h, r_ref, p, n=1, mu_s=mu_s, var_s=var_s)
        r_g, f_g = to_np(reg.field()), to_np(reg.corrected())
        e_r = max(rel_err(r_g[c], r_ref[c]) for c in range(3))
        e_abs = float(np.abs(r_g - r_ref).max())
        e_f = rel_err(f_g, f_ref)
        emax, erms = field_err(r_g, r_ref)
        print("iteration %d: field rel %.2g (abs %.2g vox; per-voxel max %.2g rms %.2g), corrected rel %.2g"
              % (k + 1, e_r, e_abs, emax, erms, e_f))
        assert e_f <= STEP_RTOL
        assert emax <= (1e-3 if k == 0 else FIELD_MAX) and erms <= FIELD_RMS


def test_masked_iteration_whole_volume(disc, case):
    """The first masked iteration at the benchmarked size (m = CT at r = 0):
    the Eq. 5-6 pair and the Eq. 7 mask from the finest-level 11^3 mask
    sweep, then every Eq. 8-10 fill pass, against the oracle at every voxel.
    The pass map (which pass filled each voxel) must equal the oracle's
    exactly when the oracle fills from the GPU's mask."""
    from synth.phantom import CONFIGS

    cfg = CONFIGS[NAME]
    patch = cfg["patch"]
    reg = disc.Registration(patch=patch, sigma=cfg["sigma"], levels=1, iters=(1,), mask_mode=1)
    ct, cb = to_dev(case.ct), to_dev(case.cbct)
    reg.set_volumes(ct, cb)
    reg.run()
    f_g = to_np(reg.corrected())
    stamp = to_np(reg.mask())
    mp = reg.mask_params()
    s, _ = disc.shift(ct, cb)
    s_h = to_np(s).astype(np.float64)
    m_h = case.ct.astype(np.float64)
    mu_m, var_m = oracle.patch_moments(m_h, patch)
    mu_s, var_s = oracle.patch_moments(s_h, patch)
    a0, b0, _ = oracle.correct(mu_m, var_m, mu_s, var_s, s_h)
    # Eq. 7 on the oracle's values, with the margin of each decision
    dm = np.abs(m_h - s_h) - mp["hu0"]
    xi_ref = (dm > 0) | (a0 < mp["a_min"]) | (a0 > mp["a_max"])
    near = (np.abs(dm) <= 1e-3) | (np.abs(a0 - mp["a_min"]) <= 1e-5 * mp["a_min"]) | \
        (np.abs(a0 - mp["a_max"]) <= 1e-5 * mp["a_max"])
    xi_gpu = stamp != 0
    wrong = (xi_gpu != xi_ref) & ~near
    print("masked %.3f of the voxels, %d within rounding of a threshold (%d decided the other way), "
          "%d decided wrongly" % (xi_gpu.mean(), int(near.sum()), int(((xi_gpu != xi_ref) & near).sum()),
                                  int(wrong.sum())))
    assert not wrong.any()
    assert 0.05 < xi_gpu.mean() < 0.999
    A, B, used, pass_of = oracle.fill_ex(a0, b0, ~xi_gpu, s_h, mp["h"], t=(7, 7, 3), passes=10)
    mism = int((pass_of != stamp).sum())
    f_ref = A * s_h + B
    print("fill: %d passes used, pass map mismatches %d, corrected rel %.2g" % (used, mism, rel_err(f_g, f_ref)))
    assert used >= 2
    assert mism == 0
    assert rel_err(f_g, f_ref) <= STEP_RTOL


@pytest.mark.parametrize("patch", [(3, 3, 3), (11, 11, 11), (13, 13, 13), (15, 15, 15)])
def test_correction_sweep_on_ragged_large_volume(disc, patch):
    """The large-volume correction sweeps (the z-first sweep for isotropic
    patches up to 13^3, the x -> y -> z sweep beyond; 32 x 32 tiles times
    nz >= 4096 planes-tiles) on a volume ragged in x, y and z
    (230 x 250 x 70: partial tiles on two sides, a short last z chunk), every
    voxel against Eq. 3-6 in FP64, with a static image whose patches include
    flat ones (constant blocks), so both epilogue branches run."""
    g = np.random.default_rng([57, patch[0]])
    shape = (70, 250, 230)
    m = (g.normal(size=shape) * 200 + 40).astype(np.float32)
    s = (0.8 * m + g.normal(size=shape) * 30 - 60).astype(np.float32)
    s[10:40, 50:120, 60:150] = 35.0  # flat static region
    md, sd = to_dev(m), to_dev(s)
    ys = disc.static_stats(sd, patch)
    f = to_np(disc.correct(md, ys, patch))
    mu_m, var_m = oracle.patch_moments(m, patch)
    mu_s, var_s = oracle.patch_moments(s, patch)
    _, _, f_ref = oracle.correct(mu_m, var_m, mu_s, var_s, s)
    e = rel_err(f, f_ref)
    print("%s ragged 230x250x70: correction rel err %.3g" % (patch, e))
    assert e <= STEP_RTOL
