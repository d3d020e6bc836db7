"""Parity at the full workload sizes, on sampled voxels.

The 256x256x96 (patch 11^3, sigma 2) and 512x512x160 (patch 15^3, sigma 2)
pairs are too large for whole-volume oracle runs in a test, so each step
runs on the GPU through the C ABI -- the same kernels and launch
configuration as the timed registration -- and the oracle recomputes a few
hundred voxels (random, every corner, and voxels on every face) from the
same FP32 state. Bar per step: max|gpu - ref| / max|ref| <= 1e-4 with the
scale taken over the whole GPU output array.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import STEP_RTOL, sample_points, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


def scaled_err(gpu_pts, ref_pts, gpu_full):
    scale = float(np.abs(gpu_full).max())
    return float(np.abs(np.asarray(gpu_pts, np.float64) - ref_pts).max()) / (scale if scale > 0 else 1.0)


@pytest.mark.parametrize("name", ["hn256x256x96", "hn512x512x160"])
def test_steps_sampled_at_full_size(disc, name):
    from synth.phantom import CONFIGS, make_case

    cfg = CONFIGS[name]
    case = make_case(name, device="cuda")
    patch, sigma = cfg["patch"], cfg["sigma"]
    ct = to_dev(case.ct)
    cb = to_dev(case.cbct)
    # a realistic mid-registration field: a few finest-level iterations from
    # a partial version of the known deformation
    reg = disc.Registration(patch=patch, sigma=sigma, levels=1, iters=(3,))
    reg.set_volumes(ct, cb)
    reg.set_field(to_dev(0.6 * case.r_true))
    reg.run()
    r = reg.field()
    s, _ = disc.shift(ct, cb)
    m = disc.warp(ct, r)
    ys = disc.static_stats(s, patch)
    f = disc.correct(m, ys, patch)
    out, rt = disc.force_smooth(m, f, r, sigma, want_rt=True)
    ct_h, r_h, s_h, m_h, f_h, out_h, rt_h = (to_np(x) for x in (ct, r, s, m, f, out, rt))
    assert np.isfinite(out_h).all() and np.abs(r_h).max() > 0.5
    pts = sample_points(case.ct.shape, 300, seed=7)
    e_w = scaled_err(m_h.ravel()[pts], oracle.warp_pts(ct_h, r_h, pts), m_h)
    e_c = scaled_err(f_h.ravel()[pts], oracle.correct_pts(m_h, s_h, patch, pts), f_h)
    rt_ref = oracle.force_pts(m_h, f_h, r_h, pts)
    e_f = max(scaled_err(rt_h[c].ravel()[pts], rt_ref[:, c], rt_h[c]) for c in range(3))
    u_err = max(float(np.abs((r_h[c].ravel()[pts].astype(np.float64) - rt_h[c].ravel()[pts])
                             - (r_h[c].ravel()[pts].astype(np.float64) - rt_ref[:, c])).max()) for c in range(3))
    g_ref = oracle.gauss_pts(rt_h, sigma, pts)
    e_g = max(scaled_err(out_h[c].ravel()[pts], g_ref[:, c], out_h[c]) for c in range(3))
    print("%s sampled rel errors: warp %.2g correct %.2g force %.2g (u abs %.2g) gauss %.2g"
          % (name, e_w, e_c, e_f, u_err, e_g))
    assert max(e_w, e_c, e_f, e_g) <= STEP_RTOL
    assert u_err <= 1e-5


def test_full_schedule_c2_deterministic_and_sane(disc):
    """The benchmarked registration (3 levels x 100 iterations at 256x256x96):
    bitwise reproducible and finite, and its corrected CBCT matches the
    deformed CT far better than the raw (shifted) CBCT does, in voxel values
    and in histogram (the intensity-consistency property of Sec. 3.2,
    Fig. 7). Field accuracy against the known deformation is not asserted:
    with these artifact strengths and fixed iteration counts, and without the
    Eq. 7-10 mask, both plain demons and DISC add spurious deformation."""
    from synth.phantom import CONFIGS, make_case

    cfg = CONFIGS["hn256x256x96"]
    case = make_case("hn256x256x96", device="cuda")
    ct, cb = to_dev(case.ct), to_dev(case.cbct)
    outs = []
    for _ in range(2):
        reg = disc.Registration(patch=cfg["patch"], sigma=cfg["sigma"], levels=cfg["levels"], iters=cfg["iters"])
        reg.set_volumes(ct, cb)
        reg.run()
        outs.append((reg.field(), reg.corrected()))
    r, f = outs[0]
    assert bool((r == outs[1][0]).all()) and bool((f == outs[1][1]).all())
    s, _ = disc.shift(ct, cb)
    m = disc.warp(ct, r)
    r_h, f_h, m_h, s_h = (to_np(x) for x in (r, f, m, s))
    assert np.isfinite(r_h).all() and np.isfinite(f_h).all()
    body = case.ct > -500
    e_raw = np.abs(s_h - m_h)[body].mean()
    e_cor = np.abs(f_h - m_h)[body].mean()
    bins = np.linspace(-1100, 1600, 271)
    hist = lambda v: np.histogram(v[body], bins=bins)[0] / body.sum()  # noqa: E731
    h_raw = np.abs(hist(s_h) - hist(m_h)).sum()
    h_cor = np.abs(hist(f_h) - hist(m_h)).sum()
    print("256x256x96 mean |S - m| %.1f HU, mean |I's - m| %.1f HU; histogram L1 %.3f -> %.3f"
          % (e_raw, e_cor, h_raw, h_cor))
    assert e_cor < 0.5 * e_raw
    assert h_cor < h_raw
