"""Differentiable DISC on the GPU: SSD loss and its hand-written gradient.

L(r) = sum (m - I'_s)^2, m = CT(x + r), I'_s moment-matched to m (Eq. 3-6).
The HIP path (warp, moments sweep in SSD mode, box adjoint, gradient kernel)
is compared with the FP64 oracle: the loss to 1e-4 relative, the gradient to
1e-3 relative (max-scaled), at sizes that span several tiles with ragged
tails, at the full 256x256x96 size on sampled voxels, and along random
directions against central finite differences of the oracle's loss.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.helpers import sample_points, to_dev, to_np

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3
LOSS_RTOL = 1e-4


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


def _case(shape, seed, amp=1.5):
    g = np.random.default_rng([1204, seed])
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ct = (400.0 * np.sin(xx / 3.1) * np.cos(yy / 4.3) + 300.0 * np.sin(zz / 2.7 + xx / 5.0)
          + g.normal(0.0, 20.0, shape))
    s = 0.85 * ct + 60.0 + 40.0 * np.sin(yy / 9.0) + g.normal(0.0, 15.0, shape)
    r = g.uniform(-amp, amp, (3,) + shape)
    return ct.astype(np.float32), s.astype(np.float32), r.astype(np.float32)


def _max_rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("shape,patch", [
    ((23, 29, 37), (5, 5, 5)),
    ((17, 45, 70), (5, 3, 3)),
    ((9, 33, 40), (3, 7, 1)),
    ((20, 20, 20), (11, 11, 11)),
])
def test_loss_and_grad_match_oracle(disc, shape, patch):
    ct, s, r = _case(shape, sum(shape))
    ct_d, s_d, r_d = to_dev(ct), to_dev(s), to_dev(r)
    ys = disc.static_stats(s_d, patch)
    grad, loss = disc.ssd_grad(ct_d, ys, r_d, patch, want_loss=True)
    loss_only = disc.ssd_loss(ct_d, ys, r_d, patch)
    ref_l = oracle.ssd_loss(ct.astype(np.float64), s.astype(np.float64), r.astype(np.float64), patch)
    ref_g = oracle.ssd_grad(ct.astype(np.float64), s.astype(np.float64), r.astype(np.float64), patch)
    e_l = abs(float(loss) - ref_l) / ref_l
    e_g = _max_rel(to_np(grad), ref_g)
    print("%s patch %s: loss rel %.2g, grad rel %.2g" % (shape, patch, e_l, e_g))
    assert float(loss) == float(loss_only)
    assert e_l <= LOSS_RTOL
    assert e_g <= GRAD_RTOL


def test_grad_vs_finite_differences(disc):
    """<grad, v> on the GPU equals the FP64 central difference of the oracle
    loss along v, for random directions confined to random 32^3 sub-blocks
    (eps = 1e-3 voxel; the field keeps its fractional parts away from cell
    edges so that no sample crosses a trilinear cell)."""
    shape, patch = (40, 48, 48), (5, 5, 5)
    ct, s, _ = _case(shape, 11)
    g = np.random.default_rng([1204, 12])
    r = (np.floor(g.uniform(-1.5, 1.5, (3,) + shape)) + g.uniform(0.1, 0.9, (3,) + shape)).astype(np.float32)
    ys = disc.static_stats(to_dev(s), patch)
    grad = to_np(disc.ssd_grad(to_dev(ct), ys, to_dev(r), patch)).astype(np.float64)
    ct64, s64, r64 = (a.astype(np.float64) for a in (ct, s, r))
    eps = 1e-3
    for k in range(3):
        v = np.zeros_like(r64)
        z0, y0, x0 = (int(g.integers(0, n - 32 + 1)) for n in shape)
        v[:, z0:z0 + 32, y0:y0 + 32, x0:x0 + 32] = g.normal(size=(3, 32, 32, 32))
        fd = (oracle.ssd_loss(ct64, s64, r64 + eps * v, patch)
              - oracle.ssd_loss(ct64, s64, r64 - eps * v, patch)) / (2 * eps)
        dd = float((grad * v).sum())
        print("direction %d: FD %.6e  <grad,v> %.6e" % (k, fd, dd))
        assert abs(dd - fd) <= GRAD_RTOL * abs(fd)


def test_sampled_grad_at_full_size(disc):
    """256x256x96, patch 11^3: the gradient at sampled voxels (random,
    corners, faces) against the oracle's point evaluator on the same FP32
    state, from a realistic mid-registration field."""
    from synth.phantom import CONFIGS, make_case

    cfg = CONFIGS["hn256x256x96"]
    case = make_case("hn256x256x96", device="cuda")
    patch = cfg["patch"]
    ct, cb = to_dev(case.ct), to_dev(case.cbct)
    r = to_dev(0.6 * case.r_true)
    ys = disc.static_stats(cb, patch)
    grad = to_np(disc.ssd_grad(ct, ys, r, patch))
    pts = sample_points(case.ct.shape, 150, seed=3)
    ref = oracle.ssd_grad_pts(to_np(ct), to_np(cb), to_np(r), patch, pts)
    scale = np.abs(grad).max()
    err = max(float(np.abs(grad[c].ravel()[pts].astype(np.float64) - ref[:, c]).max()) for c in range(3)) / scale
    print("256x256x96 sampled gradient rel error %.2g (scale %.3g)" % (err, scale))
    assert err <= GRAD_RTOL


def test_autograd_function_and_determinism(disc):
    shape, patch = (16, 24, 40), (5, 5, 3)
    ct, s, r = _case(shape, 21)
    ct_d, ys = to_dev(ct), disc.static_stats(to_dev(s), patch)
    r_d = to_dev(r).requires_grad_(True)
    loss = disc.ssd(r_d, ct_d, ys, patch)
    (g_auto,) = torch.autograd.grad(3.0 * loss, r_d)
    g1 = disc.ssd_grad(ct_d, ys, r_d.detach(), patch)
    g2 = disc.ssd_grad(ct_d, ys, r_d.detach(), patch)
    assert bool((g1 == g2).all())
    assert torch.allclose(g_auto, 3.0 * g1, rtol=1e-6, atol=0.0)
    assert float(loss.detach()) == float(disc.ssd_loss(ct_d, ys, r_d.detach(), patch))


def test_consistent_images_are_a_minimum(disc):
    """S = 1.3 CT - 200 at r = 0: I'_s = m, so L ~ 0 and the gradient ~ 0
    relative to the gradient of a perturbed field."""
    shape, patch = (12, 20, 33), (3, 3, 3)
    ct, _, r = _case(shape, 31)
    s = (1.3 * ct.astype(np.float64) - 200.0).astype(np.float32)
    ct_d, ys = to_dev(ct), disc.static_stats(to_dev(s), patch)
    g0, l0 = disc.ssd_grad(ct_d, ys, torch.zeros((3,) + shape, device="cuda"), patch, want_loss=True)
    g1, l1 = disc.ssd_grad(ct_d, ys, to_dev(0.5 * r), patch, want_loss=True)
    assert float(l0) <= 1e-6 * float(l1)
    assert float(g0.abs().max()) <= 1e-3 * float(g1.abs().max())


def test_gradient_descent_lowers_the_loss(disc):
    """A few steps of plain gradient descent on r from a perturbed start
    lower L monotonically (sanity of sign and scale)."""
    shape, patch = (20, 32, 32), (5, 5, 5)
    ct, s, _ = _case(shape, 41)
    ct_d = to_dev(ct)
    r = torch.zeros((3,) + shape, device="cuda")
    ys = disc.static_stats(to_dev(s), patch)
    losses = []
    for _ in range(5):
        g, loss = disc.ssd_grad(ct_d, ys, r, patch, want_loss=True)
        losses.append(float(loss))
        step = 0.2 / max(float(g.abs().max()), 1e-30)
        r = (r - step * g).contiguous()
    print("GD losses", losses)
    assert all(b < a for a, b in zip(losses, losses[1:]))


def test_invalid_arguments(disc):
    ct = torch.zeros((8, 8, 8), device="cuda")
    r = torch.zeros((3, 8, 8, 8), device="cuda")
    with pytest.raises(disc.DiscError):
        disc.ssd_loss(ct, ct, r, (4, 3, 3))
    lib = disc.lib()
    assert lib.disc_ssd_scratch_bytes(0, 8, 8) == 0
