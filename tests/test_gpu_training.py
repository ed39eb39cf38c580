"""GPU parity of the surrogate training data (Sec. 5, Eq. MLP_loss) made by woi_training_points:
the interior grid points, boundary points, normals and flux targets against the oracle's own
construction, and the WoI estimates at the interior points against the oracle on identical
random streams."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_2508_16767_amd import woi  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


CASES = [("bower_ex3_2d", lambda: W.bower_ex3_2d(), 100, 0.0, 500),
         ("star_tree_2d", lambda: W.star_tree_2d(n_points=8)[0], 64, 0.01, 256),
         ("zheng_ex3_3d", lambda: W.zheng_ex3_3d(), 25, 0.0, 51),
         ("ellipsoid_tree_3d", lambda: W.ellipsoid_tree_3d(n_points=8)[0], 20, 0.02, 12),
         ("single_ellipsoid_3d", lambda: W.single_ellipsoid_linear(3, [0.9, 0.6, 0.4], sigma=2.0)[0], 18, 0.0, 10)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_training_points_match_oracle(case):
    name, make, n, margin, bc = CASES[case]
    p = make()
    x, yb, nb, fb, cnt = woi.training_points(woi.Problem(p), n, margin=margin, bc_n=bc)
    xo, ybo, nbo, fbo = O.OracleProblem(p).training_points(n, margin=margin, bc_n=bc)
    assert cnt == len(xo) > 0, (name, cnt, len(xo))
    assert np.allclose(_np(x), xo, rtol=0, atol=1e-14)
    assert np.allclose(_np(yb), ybo, rtol=0, atol=1e-13)
    assert np.allclose(_np(nb), nbo, rtol=0, atol=1e-12)
    assert np.allclose(_np(fb), fbo, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(fbo).max()))


def test_training_interior_estimates_and_capacity():
    """WoI at the generated interior points (the surrogate's targets): FP64 against the oracle on
    the same streams; a capacity below the count writes the first `cap` points and reports all."""
    p = W.bower_ex3_2d()
    gp = woi.Problem(p)
    x, _, _, _, cnt = woi.training_points(gp, 100)
    assert cnt == len(x)
    idx = np.array([0, 1, cnt // 2, cnt - 1])
    mean, se, g, gse = [_np(t) for t in woi.estimate(gp, x, 20000, 4, seed=3, schedule_mode=woi.SCHED_SHARED)]
    mo, so, go, _, _ = O.estimate(O.OracleProblem(p), _np(x)[idx], 20000, 4, seed=3, schedule_mode=1, groups=idx)
    assert np.allclose(mean[idx], mo, rtol=1e-9, atol=1e-9 * so.max())
    assert np.allclose(g[idx], go, rtol=1e-9, atol=1e-9 * np.abs(go).max())
    x2, _, _, _, cnt2 = woi.training_points(gp, 100, cap=1000)
    assert cnt2 == cnt and len(x2) == 1000 and np.array_equal(_np(x2), _np(x)[:1000])
