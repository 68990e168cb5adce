"""The baseline lifting as a special case of the method (Prop. 2): a data term given only at
the labels (sampled costs with tau == gamma), so every interval's convex piece is the chord
between its end labels. GPU only, through the C-ABI.

* one iteration from a random state against the oracle, for every launch configuration;
* a run to a small certified gap whose interval contains the optimum of an independent
  primal-dual solve of the baseline lifting with the ordered-box projection.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from tests import checkers as ck

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402
from tests.test_gpu_parity import _gpu_state, _load_same_state  # noqa: E402

from tests.gpu_tilings import TILING_IDS, TILINGS, use_tiling  # noqa: E402
CASES = [("tq_L6", W.baseline_lifting(W.truncated_quadratic(L=6, H=9, W=131, seed=41))),
         ("tq_L16", W.baseline_lifting(W.truncated_quadratic(L=16, H=7, W=70, seed=42)))]


@pytest.mark.parametrize("tiling", TILINGS, ids=TILING_IDS)
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_single_iteration_from_random_state(orc, name, wl, tiling):
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    if not use_tiling(g, tiling, wl.W, wl.k):
        return
    st = W.random_state(31, wl.k, wl.H, wl.W)
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got, ref = _gpu_state(g), o.get_state()
    for n in S.STATE_ORDER:
        err = np.abs(got[n].astype(np.float64) - ref[n])
        bound = 2e-5 * (1.0 + np.abs(ref[n]))
        assert np.all(err <= bound), (name, n, err.max())


def test_run_to_gap_brackets_independent_baseline_solve():
    rng = np.random.default_rng(43)
    H, Wd, L = 12, 70, 5
    gamma = np.array([0.0, 0.2, 0.45, 0.7, 1.0])
    costs = rng.uniform(0, 1, size=(L, H, Wd)).astype(np.float32)
    lam = 0.15
    wl = W.Workload("p2", H, Wd, gamma, W.SAMPLED, lam, tau=gamma.copy(), samples=costs)
    g = S.Problem.from_workload(wl, adaptive=False)
    g.run_to_gap(1e-5, 60000)
    rep = g.energy()
    Pb, Db = ck.baseline_lifting(costs.astype(np.float64), gamma, lam, iters=40000, tol=1e-9)
    assert Pb - Db <= 1e-7 * abs(Pb)
    assert rep["rel_gap"] <= 1e-4
    assert rep["dual_lb"] <= Pb * (1 + 1e-7) and Db <= rep["primal_ub"] * (1 + 1e-7)
