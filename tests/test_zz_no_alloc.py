"""The allocation-free SSD loss (disc_ssd_loss_noalloc) against disc_ssd_loss.

Both run the same kernels in the same launch geometry, so the loss must be
bitwise equal. Two calls in a row, the second on a smaller volume, check
that the fixed scratch array is reused correctly (the second call must not
see the first call's contents); volumes beyond the array are rejected on the
host before any device work.
"""
import ctypes

import numpy as np
import pytest

from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    import paper_1204_6295_amd as d

    d.lib()
    return d


def _case(shape, seed):
    from synth.phantom import make_hn_pair

    c = make_hn_pair(shape, pair=seed)
    g = np.random.default_rng([77, seed])
    r = (0.7 * c.r_true + g.normal(scale=0.3, size=c.r_true.shape)).astype(np.float32)
    return to_dev(c.ct), to_dev(c.cbct), to_dev(r)


def test_noalloc_loss_equals_workspace_loss(disc):
    import torch

    patch = (11, 11, 11)
    results = []
    for shape, seed in (((96, 256, 256), 1), ((40, 72, 88), 2)):
        ct, cb, r = _case(shape, seed)
        s, _ = disc.shift(ct, cb)
        ys = disc.static_stats(s, patch)
        ref = disc.ssd_loss(ct, ys, r, patch)
        got = disc.ssd_loss_noalloc(ct, ys, r, patch)
        torch.cuda.synchronize()
        print("%s: loss %.17g (workspace) %.17g (allocation-free)" % (shape, ref.item(), got.item()))
        assert ref.item() > 0.0
        assert got.item() == ref.item()
        results.append(got.item())
    assert results[0] != results[1]


def test_noalloc_loss_rejects_oversize_volumes(disc):
    L = disc.lib()
    fake = ctypes.c_void_p(1 << 20)
    patch = (ctypes.c_int * 3)(11, 11, 11)
    # 512 x 512 x 160 needs 168 MB of scratch, beyond the 32 MiB array
    assert L.disc_ssd_loss_noalloc(fake, fake, fake, 512, 512, 160, patch, fake, None) == disc.DISC_ENOMEM
    assert b"32 MiB" in L.disc_last_error(None) or b"holds" in L.disc_last_error(None)
