"""Whole-volume parity of one iteration's steps at the clinical size.

The 512x512x160 head-and-neck pair with patch 15^3 and sigma 2 runs the
finest level of that registration with its own launch geometry: the
z-first moments sweep with 768-thread workgroups (the 15^3 variant), the
force + xy pipeline and the ring z pass with the fused next warp, each on
32 x 32-column tiles (16 x 16 per plane) with the z chunks this size
selects. Each step runs through the C ABI on identical FP32 inputs
from a mid-registration state and is compared with the FP64 oracle at every
voxel: max|gpu - ref| / max|ref| <= 1e-4 per output array, and the force per
voxel to 1e-5 voxel absolute.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import STEP_RTOL, rel_err, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NAME = "hn512x512x160"


def test_steps_whole_volume_clinical_size():
    import paper_1204_6295_amd as disc
    from synth.phantom import CONFIGS, make_case

    cfg = CONFIGS[NAME]
    patch, sigma = cfg["patch"], cfg["sigma"]
    assert tuple(patch) == (15, 15, 15)
    case = make_case(NAME)
    ct, cb = to_dev(case.ct), to_dev(case.cbct)
    reg = disc.Registration(patch=patch, sigma=sigma, levels=1, iters=(2,))
    reg.set_volumes(ct, cb)
    reg.set_field(to_dev(0.6 * case.r_true))
    reg.run()
    r = reg.field()
    reg.close()
    s, _ = disc.shift(ct, cb)
    m = disc.warp(ct, r)
    ys = disc.static_stats(s, patch)
    f = disc.correct(m, ys, patch)
    out, rt, m_next = disc.force_smooth(m, f, r, sigma, want_rt=True, ct=ct)
    ct_h, r_h, s_h, m_h, f_h, out_h, rt_h, mn_h = (to_np(x) for x in (ct, r, s, m, f, out, rt, m_next))
    del m, f, out, rt, m_next
    assert np.abs(r_h).max() > 1.0

    e_w = rel_err(m_h, oracle.warp(ct_h, r_h))
    mu_m, var_m = oracle.patch_moments(m_h, patch)
    mu_s, var_s = oracle.patch_moments(s_h, patch)
    _, _, f_ref = oracle.correct(mu_m, var_m, mu_s, var_s, s_h)
    del mu_m, var_m, mu_s, var_s
    e_c = rel_err(f_h, f_ref)
    del f_ref
    u_ref = oracle.force(m_h, f_h)
    rt_ref = r_h.astype(np.float64) - u_ref
    e_f = max(rel_err(rt_h[c], rt_ref[c]) for c in range(3))
    u_err = float(np.abs((r_h.astype(np.float64) - rt_h) - u_ref).max())
    del u_ref, rt_ref
    e_g = max(rel_err(out_h[c], oracle.gauss(rt_h[c], sigma)) for c in range(3))
    e_n = rel_err(mn_h, oracle.warp(ct_h, out_h))
    print("512x512x160 whole-volume rel errors: warp %.2g correct %.2g force %.2g (u abs %.2g) gauss %.2g "
          "next warp %.2g" % (e_w, e_c, e_f, u_err, e_g, e_n))
    assert max(e_w, e_c, e_f, e_g, e_n) <= STEP_RTOL
    assert u_err <= 1e-5
