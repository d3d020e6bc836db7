"""Eq. 7-10 mask and fill on the GPU against the FP64 oracle.

At set-up the device resolves the Sec. 2.3 rules (a_m, HU_0, h); one
iteration from r = 0 then exercises the mask and every fill pass on known
inputs (m = CT exactly), and whole registrations compare fields. Mask
decisions are taken on FP32 data on the GPU and in FP64 by the oracle: the
per-region fill cases accept either decision for voxels within FP32
rounding of HU_0 or of a_min / a_max, require the oracle's decision
everywhere else, and then compare the fill pass by pass from the GPU's own
mask; the whole-registration cases use inputs whose |m - S| and a stay far
from the thresholds.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import FIELD_MAX, FIELD_RMS, field_err, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


def _ellipsoid48():
    from synth.phantom import make_case

    c = make_case("ellipsoid48")
    return c.ct, c.cbct


def test_mask_parameters_match_the_rules(disc):
    ct, cb = _ellipsoid48()
    reg = disc.Registration(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(1,), mask_mode=1)
    reg.set_volumes(to_dev(ct), to_dev(cb))
    mp = reg.mask_params()
    dhu, s = oracle.global_shift(ct, cb)
    am = oracle.a_median(ct, s, (5, 5, 5))
    print("GPU %s; oracle a_m %.6f, HU0 %.4f" % (mp, am, 2 * abs(dhu)))
    assert abs(mp["a_m"] - am) <= 1e-6 * am
    assert abs(mp["hu0"] - 2 * abs(dhu)) <= 1e-5 * abs(dhu)
    assert abs(mp["a_min"] - 0.5 * am) <= 1e-6 * am and abs(mp["a_max"] - 1.5 * am) <= 1e-6 * am
    assert mp["h"] == mp["hu0"]


def test_first_iteration_mask_and_fill(disc):
    """At r = 0 the deformed image is the CT itself, so the corrected image
    of the first iteration is Eq. 5-10 on known inputs: GPU vs oracle."""
    ct, cb = _ellipsoid48()
    reg = disc.Registration(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(1,), mask_mode=1)
    reg.set_volumes(to_dev(ct), to_dev(cb))
    reg.run()
    f = to_np(reg.corrected())
    mp = reg.mask_params()
    _, s = oracle.global_shift(ct, cb)
    s32 = s.astype(np.float32).astype(np.float64)
    A, B, xi, used = oracle.mask_fill(ct, s32, (5, 5, 5), 1e-2, mp["hu0"], mp["a_min"], mp["a_max"], mp["h"],
                                      t=(7, 7, 3), passes=10)
    f_ref = A * s32 + B
    err = np.abs(f - f_ref)
    print("masked %.3f, passes %d, max |f - ref| %.3g HU, rel %.3g" % (xi.mean(), used, err.max(),
                                                                       rel_err(f, f_ref)))
    assert 0.05 < xi.mean() < 0.95 and used >= 2
    assert rel_err(f, f_ref) <= 1e-4


@pytest.mark.parametrize("shape,t,passes", [
    ((48, 48, 48), (3, 3, 1), 10),
    ((48, 48, 48), (7, 7, 3), 1),
    ((20, 45, 70), (7, 7, 3), 10),
    ((20, 45, 70), (5, 9, 5), 4),
    ((20, 45, 70), (1, 1, 1), 2),  # T is the voxel itself: nothing can be filled
    ((20, 45, 70), (13, 13, 3), 3),  # generic work-list kernel, reach of one tile in x
    ((12, 40, 36), (15, 15, 9), 3),  # T region too large for LDS: gathers from cache
    ((48, 128, 128), (7, 7, 3), 10),  # 3072 fill tiles
    ((40, 256, 256), (7, 7, 3), 10),  # 10240 fill tiles, more than the workgroups of a pass
    ((20, 45, 70), (13, 7, 5), 4),  # work-list kernel with its LDS just under the 64 KiB limit
    ((20, 45, 70), (13, 9, 5), 4),  # just over it: the cache-gather kernel
])
def test_fill_passes_and_regions(disc, shape, t, passes):
    """One iteration from r = 0 for several T regions and pass counts, on
    volumes with ragged tiles: the pass structure (which voxels each pass
    fills, and from what) must equal the oracle's. The GPU's Eq. 7 mask is
    checked against the oracle's decision (voxels within FP32 rounding of a
    threshold may take either side), then the oracle fills from the GPU's
    mask and the pass map (disc_get_mask: 0 valid, p filled by pass p, 255
    never filled) must be identical voxel for voxel."""
    from synth.phantom import make_hn_pair

    if shape == (48, 48, 48):
        ct, cb = _ellipsoid48()
    else:
        # pairs whose |m - S| and a stay at least 4e-5 (relative) from the
        # Eq. 7 thresholds, far beyond the FP32 rounding of |m - S| (3e-8)
        c = make_hn_pair(shape, pair={(20, 45, 70): 0, (12, 40, 36): 3, (48, 128, 128): 5,
                                       (40, 256, 256): 3}[shape])
        ct, cb = c.ct, c.cbct
    kw = dict(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(1,), mask_mode=1, fill_t=t, fill_passes=passes)
    reg = disc.Registration(**kw)
    reg.set_volumes(to_dev(ct), to_dev(cb))
    reg.run()
    f = to_np(reg.corrected())
    mp = reg.mask_params()
    _, s = oracle.global_shift(ct, cb)
    s32 = s.astype(np.float32).astype(np.float64)
    A, B, xi, used = oracle.mask_fill(ct, s32, (5, 5, 5), 1e-2, mp["hu0"], mp["a_min"], mp["a_max"], mp["h"],
                                      t=t, passes=passes)
    f_ref = A * s32 + B
    print("%s T %s passes %d: masked %.3f, used %d, rel %.3g" % (shape, t, passes, xi.mean(), used,
                                                                 rel_err(f, f_ref)))
    assert xi.any() and (~xi).any()
    if t == (1, 1, 1):
        assert used == 0
    assert rel_err(f, f_ref) <= 1e-4
    # the pass map, filled by the oracle from the GPU's own mask
    stamp = to_np(reg.mask())
    ctd = ct.astype(np.float64)
    mu_m, var_m = oracle.patch_moments(ctd, (5, 5, 5))
    mu_s, var_s = oracle.patch_moments(s32, (5, 5, 5))
    a0, b0, _ = oracle.correct(mu_m, var_m, mu_s, var_s, s32)
    dm = np.abs(ctd - s32) - mp["hu0"]
    near = (np.abs(dm) <= 1e-3) | (np.abs(a0 - mp["a_min"]) <= 1e-5 * mp["a_min"]) | \
        (np.abs(a0 - mp["a_max"]) <= 1e-5 * mp["a_max"])
    xi_gpu = stamp != 0
    assert not ((xi_gpu != xi) & ~near).any()
    _, _, used2, pass_of = oracle.fill_ex(a0, b0, ~xi_gpu, s32, mp["h"], t=t, passes=passes)
    assert np.array_equal(pass_of, stamp), "pass maps differ at %d voxels" % int((pass_of != stamp).sum())


def test_masked_registration_matches_oracle(disc):
    ct, cb = _ellipsoid48()
    kw = dict(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(20,), mask_mode=1)
    reg = disc.Registration(**kw)
    reg.set_volumes(to_dev(ct), to_dev(cb))
    reg.run()
    r_ref, f_ref = oracle.register(ct, cb, oracle.make_params(**kw))
    emax, erms = field_err(to_np(reg.field()), r_ref)
    print("masked 48^3: field err max %.3g rms %.3g; |r| max %.3g" % (emax, erms, np.abs(r_ref).max()))
    assert emax <= FIELD_MAX and erms <= FIELD_RMS
    assert rel_err(to_np(reg.corrected()), f_ref) <= 1e-3


def test_masked_pyramid_and_determinism(disc):
    from synth.phantom import make_hn_pair

    c = make_hn_pair((24, 64, 64), pair=2)
    kw = dict(patch=(7, 7, 5), sigma=2.0, levels=2, iters=(8, 6), mask_mode=1, fill_passes=6)
    outs = []
    for _ in range(2):
        reg = disc.Registration(**kw)
        reg.set_volumes(to_dev(c.ct), to_dev(c.cbct))
        reg.run()
        outs.append((to_np(reg.field()), to_np(reg.corrected())))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    r_ref, f_ref = oracle.register(c.ct, c.cbct, oracle.make_params(**kw))
    emax, erms = field_err(outs[0][0], r_ref)
    print("masked pyramid: field err max %.3g rms %.3g" % (emax, erms))
    assert emax <= FIELD_MAX and erms <= FIELD_RMS
