"""The allocation-free entry point woi_estimate_noalloc against woi_estimate, through the C ABI.

Two calls in a row on one device (the second with fewer points) must each match woi_estimate
with the same query: per-walk values are the same, only the chunking of the per-point sums
differs, so means, SEs and gradients agree to rounding.  A call on a problem that is not yet
on the device is refused (the entry point allocates nothing)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2508_16767_amd import woi  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


def _close(a, b, scale):
    return np.all(np.abs(a - b) <= 1e-9 * (np.abs(b) + scale))


@pytest.mark.parametrize("precision,estimator", [(woi.FP64, woi.PLAIN), (woi.FP32, woi.PLAIN), (woi.FP32, woi.VR)])
def test_noalloc_matches_estimate_twice(precision, estimator):
    p, xs = W.star_tree_2d(n_points=700)
    gp = woi.Problem(p)
    woi.upload(gp)
    for pts, walks in ((xs, 20000), (xs[:130], 6000)):   # second call: a smaller input
        kw = dict(seed=77, precision=precision, estimator=estimator, schedule_mode=woi.SCHED_SHARED)
        ref = [_np(t) for t in woi.estimate(gp, pts, walks, 4, **kw)]
        got = [_np(t) for t in woi.estimate_noalloc(gp, pts, walks, 4, **kw)]
        torch.cuda.synchronize()
        sd = ref[1] * np.sqrt(walks)                       # sample sd per point
        assert _close(got[0], ref[0], sd.max())
        assert np.allclose(got[1], ref[1], rtol=1e-7)
        gsd = ref[3] * np.sqrt(walks)
        assert _close(got[2], ref[2], gsd.max())
        assert np.allclose(got[3], ref[3], rtol=1e-7)


def test_noalloc_large_walk_count_and_refusals():
    """More samples than the fixed array holds as 2^20-lane chunks: the chunks grow instead; a
    problem that was never uploaded, a shared-trajectory query and too many points are refused."""
    p, xs = W.concentric_disk_2d()
    gp = woi.Problem(p)
    with pytest.raises(woi.WoiError, match="INVALID_ARG"):
        woi.estimate_noalloc(gp, xs, 100, 4)                # not uploaded: the call would allocate
    woi.upload(gp)
    ref = [_np(t) for t in woi.estimate(gp, xs, 300000, 4, seed=3)]
    got = [_np(t) for t in woi.estimate_noalloc(gp, xs, 300000, 4, seed=3)]
    assert _close(got[0], ref[0], (ref[1] * np.sqrt(300000)).max())
    assert np.allclose(got[1], ref[1], rtol=1e-7)
    with pytest.raises(woi.WoiError, match="UNSUPPORTED"):
        q = woi.make_query(100, 4, batch_share=4)
        import ctypes as C
        x = torch.as_tensor(xs, device="cuda")
        out = [torch.empty(len(xs), dtype=torch.float64, device="cuda") for _ in range(2)]
        woi._check(woi._lib.woi_estimate_noalloc(gp.handle, C.c_void_p(x.data_ptr()), len(xs), C.byref(q),
                                                 C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr()),
                                                 None, None, None, None))
    big = np.zeros((400000, 2))
    with pytest.raises(woi.WoiError, match="INVALID_ARG"):
        woi.estimate_noalloc(gp, big, 10, 2)                # 400000 x 48 B > 16 MiB
