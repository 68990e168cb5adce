"""The periodic quadratic data term (phase unwrapping, Sec. 5.5) on the HIP path against the
FP64 oracle, through the C-ABI. GPU only. Tolerances as for the other data terms: one
iteration within 2e-5 (1 + |oracle|) per entry for every launch configuration; the
monitor on an identical state within 1e-9 relative; bounds after a fixed number of
iterations within 1e-5; batch members bitwise equal to lone solves; the reverse pass
within 1e-3 relative L2 (lambda 1e-4).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402
from tests.test_gpu_parity import _gpu_state, _load_same_state, _rel  # noqa: E402

from tests.gpu_tilings import TILING_IDS, TILINGS, use_tiling  # noqa: E402
CASES = [("L8", W.phase_unwrapping(seed=51, H=9, W=131, L=8)),
         ("L5_lam", W.phase_unwrapping(seed=52, H=13, W=70, L=5, lam=0.2)),
         ("L16", W.phase_unwrapping(seed=53, H=6, W=64, L=16, lam=0.05))]


@pytest.mark.parametrize("tiling", TILINGS, ids=TILING_IDS)
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_single_iteration_from_random_state(orc, name, wl, tiling):
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    if not use_tiling(g, tiling, wl.W, wl.k):
        return
    st = W.random_state(41, wl.k, wl.H, wl.W)
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got, ref = _gpu_state(g), o.get_state()
    for n in S.STATE_ORDER:
        err = np.abs(got[n].astype(np.float64) - ref[n])
        bound = 2e-5 * (1.0 + np.abs(ref[n]))
        assert np.all(err <= bound), (name, n, err.max())


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_monitor_on_identical_state(orc, name, wl):
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    st = W.random_state(42, wl.k, wl.H, wl.W, scale=0.3)
    _load_same_state(g, o, st)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) < 1e-9
    assert _rel(eg["dual_lb"], eo["dual"]) < 1e-9
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) < 1e-9


def test_fixed_iterations(orc):
    wl = W.phase_unwrapping(seed=54, H=40, W=72, L=8, lam=0.05)
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    g.run(300)
    o.run(300)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) <= 1e-5
    assert _rel(eg["dual_lb"], eo["dual"]) <= 1e-5
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) <= 1e-5


def test_batch_member_equals_lone_solve():
    wls = [W.phase_unwrapping(seed=60 + j, H=H, W=Wd, L=L)
           for j, (H, Wd, L) in enumerate([(9, 131, 8), (33, 64, 5), (1, 70, 2)])]
    b = S.BatchProblem(wls)
    b.run(13)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        s = S.Problem.from_workload(wl)
        s.set_tiling(*b.get_tiling())
        s.run(13)
        ul_s, _ = s.read_u()
        ul, _ = b.read_u_of(i)
        rep, rep_s = b.energy_of(i), s.energy()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ul.cpu().numpy(), ul_s.cpu().numpy())
        for key in ("primal_ub", "dual_lb", "e_nonconvex"):
            assert rep[key] == rep_s[key], (i, key)
        s.close()
    b.close()


def test_gradients_match_oracle_reverse_pass(orc):
    from tests.test_gpu_adjoint import _check_close, _gpu_grads
    wl = W.phase_unwrapping(seed=55, H=30, W=70, L=6, lam=0.1)
    K, C = 40, 7
    g = np.random.default_rng(56).uniform(0, 4 * np.pi, (wl.H, wl.W))
    o = orc.Problem(wl)
    o.unrolled_forward(K)
    _, uo = o.read_u()
    u, gf, gl, gw = _gpu_grads(wl, K, C, g)
    assert np.abs(u - uo).max() <= 1e-4
    gfo, glo, _ = o.unrolled_backward(2.0 * (u.astype(np.float64) - g))
    _check_close(gf, gfo, "grad f")
    assert abs(gl - glo) <= 1e-4 * abs(glo), (gl, glo)
    assert gw is None


def test_bf16_single_iteration(orc):
    """BF16 storage of the duals with periodic pieces: one iteration from a state already
    representable in BF16 (duals to BF16 rounding, the rest to FP32 accuracy)."""
    from tests.test_gpu_parity import _bf16_round
    name, wl = CASES[0]
    g = S.Problem.from_workload(wl, storage="bf16")
    o = orc.Problem(wl)
    st = W.random_state(43, wl.k, wl.H, wl.W)
    for n in ("v", "z", "px", "py"):
        st[n] = _bf16_round(st[n])
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got, ref = _gpu_state(g), o.get_state()
    for n in S.STATE_ORDER:
        tol = 4e-3 if n in ("v", "z", "px", "py") else 2e-5
        err = np.abs(got[n].astype(np.float64) - ref[n])
        assert np.all(err <= tol * (1.0 + np.abs(ref[n]))), (n, err.max())


def test_adaptive_run_unwraps():
    """The phase workload at a reduced size solved to a 1e-3 gap with adaptive steps: the
    read-out lies on the generating phase's branch almost everywhere."""
    wl = W.phase_unwrapping(H=64, W=64, L=8)
    g = S.Problem.from_workload(wl, adaptive=True)
    g.run_to_gap(1e-3, 30000)
    assert g.energy()["rel_gap"] <= 1e-3
    _, u = g.read_u()
    err = u.cpu().numpy().astype(np.float64) - wl.target
    assert np.mean(np.abs(err) < np.pi) > 0.95


@pytest.mark.parametrize("tiling", [(1, 4, 64), (4, 4, 128)], ids=["g1t4c64", "g4t4c128"])
def test_periodic_with_anisotropic_tv(orc, tiling):
    """Both options together: periodic pieces and the l-inf box projection."""
    wl = W.phase_unwrapping(seed=57, H=10, W=100, L=6, lam=0.3)
    wl.tv = 1
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    g.set_tiling(*tiling)
    st = W.random_state(44, wl.k, wl.H, wl.W)
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got, ref = _gpu_state(g), o.get_state()
    for n in S.STATE_ORDER:
        err = np.abs(got[n].astype(np.float64) - ref[n])
        assert np.all(err <= 2e-5 * (1.0 + np.abs(ref[n]))), (n, err.max())
    # the monitor on an identical state (both sides load the same FP32 values)
    st2 = W.random_state(45, wl.k, wl.H, wl.W, scale=0.3)
    _load_same_state(g, o, st2)
    eg, eo = g.energy(), o.monitor()
    for a_, b_ in ((eg["primal_ub"], eo["primal"]), (eg["dual_lb"], eo["dual"]),
                   (eg["e_nonconvex"], eo["e_nc"])):
        assert _rel(a_, b_) < 1e-9, (a_, b_)
