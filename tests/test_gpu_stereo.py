"""The stereo matching-cost builder (sl_stereo_costs, Sec. 5.4) against the oracle, and a
stereo solve on the GPU-built volume against the oracle's solve on its own volume. GPU
only. The costs are FP32 sums of 32 absolute differences of FP32 gradients: held to
1e-5 (1 + |oracle|) per entry; a truncation decision can only move an entry by that
rounding.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _pair(seed, H, Wd):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, 1, (H, Wd)).astype(np.float32),
            rng.uniform(0, 1, (H, Wd)).astype(np.float32))


@pytest.mark.parametrize("H,Wd,D,trunc", [(13, 150, 7, 0.8), (1, 1, 3, np.inf), (5, 64, 64, 1.5),
                                          (70, 1, 2, 0.3), (9, 129, 1, np.inf), (33, 70, 130, 2.0)])
def test_costs_match_oracle(orc, H, Wd, D, trunc):
    left, right = _pair(H * 1000 + Wd, H, Wd)
    print(f"stereo costs {H}x{Wd} D={D} trunc={trunc}", flush=True)
    got = S.stereo_costs(left, right, D, trunc).cpu().numpy().astype(np.float64)
    ref = orc.stereo_costs(left, right, D, trunc)
    err = np.abs(got - ref)
    assert np.all(err <= 1e-5 * (1.0 + np.abs(ref))), err.max()


def test_full_size_pair(orc):
    wl = W.stereo()
    left, right = wl.pair
    got = S.stereo_costs(left, right, 64, 1.0).cpu().numpy().astype(np.float64)
    ref = orc.stereo_costs(left, right, 64, 1.0)
    err = np.abs(got - ref)
    assert np.all(err <= 1e-5 * (1.0 + np.abs(ref))), err.max()


def test_solve_on_built_volume(orc):
    """A sampled stereo problem on the GPU-built costs against the oracle on its own."""
    base = W.stereo(H=24, W=90, n_disp=33, L=5)     # labels 0, 8, .., 32 on the samples
    left, right = base.pair
    vol_g = S.stereo_costs(left, right, 33, 1.0)
    vol_o = orc.stereo_costs(left, right, 33, 1.0).astype(np.float32)
    wl_o = W.Workload("st", 24, 90, base.gamma, W.SAMPLED, 0.5, tau=base.tau, samples=vol_o)
    g = S.Problem(24, 90, base.gamma, W.SAMPLED, 0.5, tau=base.tau, samples=vol_g)
    o = orc.Problem(wl_o)
    g.run(200)
    o.run(200)
    eg, eo = g.energy(), o.monitor()
    for a, b in ((eg["primal_ub"], eo["primal"]), (eg["dual_lb"], eo["dual"])):
        assert abs(a - b) <= 1e-5 * abs(b), (a, b)


def test_largest_disparity_count_and_zero_truncation(orc):
    """D at its documented maximum (1024, far beyond the image width) and trunc = 0."""
    left, right = _pair(11, 9, 70)
    got = S.stereo_costs(left, right, 1024, 2.0).cpu().numpy().astype(np.float64)
    ref = orc.stereo_costs(left, right, 1024, 2.0)
    assert np.all(np.abs(got - ref) <= 1e-5 * (1.0 + np.abs(ref)))
    # beyond the width every disparity reads column 0 of the right image: identical planes
    assert np.array_equal(got[70], got[1023])
    zero = S.stereo_costs(left, right, 5, 0.0).cpu().numpy()
    assert np.all(zero == 0.0)
