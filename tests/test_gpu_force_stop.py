"""Eq. 1 double force and the Sec. 2.3 stopping rule on the GPU.

The double-force kernel path is compared with the oracle per step (r - u and
the smoothed field) and over whole registrations; the device-side stopping
rule must run the oracle's iteration count per level, record l^(k) to
1e-3 relative, and leave the oracle's field to the final-field bar. The
tolerance used for the rule is chosen from the oracle's own history with a
wide margin around the first crossing, so that FP32 against FP64 cannot
change the decision.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import FIELD_MAX, FIELD_RMS, STEP_RTOL, field_err, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


def rng(seed):
    return np.random.default_rng([1204, 44, seed])


@pytest.mark.parametrize("shape,sigma", [((21, 37, 70), 1.5), ((33, 64, 41), 2.0), ((3, 5, 2), 1.0)])
def test_double_force_step(disc, shape, sigma):
    g = rng(1)
    m = (g.normal(size=shape) * 300).astype(np.float32)
    f = (m + g.normal(size=shape) * 40).astype(np.float32)
    f.flat[::7] = m.flat[::7]  # d = 0 exactly: zero force
    r = g.uniform(-2, 2, size=(3,) + shape).astype(np.float32)
    out, rt = disc.force_smooth(to_dev(m), to_dev(f), to_dev(r), sigma, 1e-3, want_rt=True, force_mode=1)
    out, rt = to_np(out), to_np(rt)
    u_ref = oracle.force_double(m, f, 1e-3)
    assert rel_err(rt, r.astype(np.float64) - u_ref) <= STEP_RTOL
    u_gpu = r.astype(np.float64) - rt.astype(np.float64)
    assert np.abs(u_gpu - u_ref).max() <= 2e-5
    # each Eq. 1 term is at most 1/2 voxel long (AM-GM), so the sum at most 1
    assert np.sqrt((u_gpu ** 2).sum(0)).max() <= 1.0 + 1e-6
    sref = np.stack([oracle.gauss(rt[c], sigma) for c in range(3)])
    assert rel_err(out, sref) <= STEP_RTOL


def test_double_force_registration(disc):
    from synth.phantom import make_case

    c = make_case("ellipsoid48")
    kw = dict(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(20,), force_mode=1)
    reg = disc.Registration(**kw)
    reg.set_volumes(to_dev(c.ct), to_dev(c.cbct))
    reg.run()
    r = to_np(reg.field())
    r_ref, f_ref = oracle.register(c.ct, c.cbct, oracle.make_params(**kw))
    emax, erms = field_err(r, r_ref)
    print("double force 48^3: field err max %.3g rms %.3g; |r| max %.3g" % (emax, erms, np.abs(r_ref).max()))
    assert emax <= FIELD_MAX and erms <= FIELD_RMS
    assert rel_err(to_np(reg.corrected()), f_ref) <= 1e-3
    # the two forces give different fields
    r_static, _ = oracle.register(c.ct, c.cbct, oracle.make_params(patch=(5, 5, 5), sigma=1.5, levels=1,
                                                                     iters=(20,)))
    assert np.abs(r_ref - r_static).max() > 0.05


def _clear_margin(hists, counts, caps, eps, lag, margin=0.02):
    """True when every level's decision is far from eps: each drop
    l^(k-lag) - l^(k) before the level's last iteration exceeds (1 + margin)
    eps, and a level that stopped early did so with a drop below
    (1 - margin) eps."""
    for h, n, cap in zip(hists, counts, caps):
        for k in range(lag, n):
            d = h[k - lag] - h[k]
            last = k == n - 1
            if last and n < cap:
                if not d <= (1 - margin) * eps:
                    return False
            elif not (d > (1 + margin) * eps):
                return False
    return True


def _pick_eps(ct, cb, base, lag):
    """Candidates: geometric midpoints of consecutive drops of a run without
    the rule (the drops shrink by 5-10 % per iteration, while FP32 moves a
    drop by about 1e-4 relative); the first whose own oracle run decides
    every level with a 2 % margin and stops at least one level early."""
    _, _, _, h_all = oracle.register_ex(ct, cb, oracle.make_params(stop_eps=1e-300, stop_lag=lag, **base))
    h = h_all[-1]
    drops = [h[k - lag] - h[k] for k in range(lag, len(h))]
    mids = [float(np.sqrt(a * b)) for a, b in zip(drops, drops[1:]) if np.isfinite(a) and a > b > 0]
    for eps in (mids[len(mids) // 2:] + mids[:len(mids) // 2][::-1]):
        r, f, n, hh = oracle.register_ex(ct, cb, oracle.make_params(stop_eps=eps, stop_lag=lag, **base))
        caps = [base["iters"][lv] for lv in range(base["levels"])]
        if any(nn < cap for nn, cap in zip(n, caps)) and _clear_margin(hh, n, caps, eps, lag):
            return eps, (r, f, n, hh)
    return None, None


@pytest.mark.parametrize("levels,iters,shape", [(1, (40,), None), (2, (25, 30), (28, 40, 44))])
def test_stopping_rule_matches_oracle(disc, levels, iters, shape):
    from synth.phantom import make_case, make_ellipsoid_pair

    c = make_case("ellipsoid48") if shape is None else make_ellipsoid_pair(shape, pair=3)
    lag = 4
    base = dict(patch=(5, 5, 5), sigma=1.5, levels=levels, iters=iters)
    eps, ref = _pick_eps(c.ct, c.cbct, base, lag)
    assert eps is not None, "no eps with a clear decision margin"
    r_ref, f_ref, n_ref, h_ref = ref
    kw = dict(base, stop_eps=eps, stop_lag=lag)
    reg = disc.Registration(**kw)
    reg.set_volumes(to_dev(c.ct), to_dev(c.cbct))
    reg.run()
    for lv in range(levels):
        n, h = reg.stats(lv)
        print("level %d: GPU %d iterations, oracle %d (cap %d, eps %.3g); l[:4] %s"
              % (lv, n, n_ref[lv], iters[lv], eps, np.round(h[:4], 5)))
        assert n == n_ref[lv]
        h, hr = np.array(h), np.array(h_ref[lv])
        fin = np.isfinite(hr)
        assert np.array_equal(np.isfinite(h), fin)
        assert np.abs(h[fin] - hr[fin]).max() <= 1e-3 * np.abs(hr[fin]).max()
    emax, erms = field_err(to_np(reg.field()), r_ref)
    print("stopped field err max %.3g rms %.3g" % (emax, erms))
    assert emax <= FIELD_MAX and erms <= FIELD_RMS
    assert rel_err(to_np(reg.corrected()), f_ref) <= 1e-3


def test_stopping_rule_identical_images(disc):
    """S = CT: dr = 0 and r = 0, so l^(k) = 0 and the level stops at k = lag;
    the field stays exactly zero."""
    from synth.phantom import make_case

    c = make_case("ellipsoid48")
    reg = disc.Registration(patch=(5, 5, 5), sigma=1.5, levels=1, iters=(30,), stop_eps=1e-4, stop_lag=6)
    reg.set_volumes(to_dev(c.ct), to_dev(c.ct))
    reg.run()
    n, h = reg.stats(0)
    assert n == 7 and all(v == 0.0 for v in h)
    assert float(reg.field().abs().max()) == 0.0
    assert reg.state()[1] == 30  # scheduled iterations keep counting
