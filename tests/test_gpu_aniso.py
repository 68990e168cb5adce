"""The anisotropic TV (l1 norm of the gradient; K a product of l-inf boxes) on the HIP path
against the FP64 oracle, through the C-ABI. GPU only.

Tolerances as for the isotropic TV: one iteration from a random state within
2e-5 (1 + |oracle|) per entry, for every launch configuration of the fused kernel; the
monitor on an identical state within 1e-9 relative; bounds after a fixed number of
iterations within 1e-5 relative; batched members bitwise equal to lone solves; the
reverse pass within 1e-3 relative L2 (lambda 1e-4).
"""
import copy

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from tests import checkers as ck

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402
from tests.test_gpu_parity import (_bf16_round, _gpu_state, _load_same_state,  # noqa: E402
                                   _rel, _sampled_workload)

from tests.gpu_tilings import TILING_IDS, TILINGS, use_tiling  # noqa: E402


def _aniso(wl):
    wl = copy.copy(wl)
    wl.tv = 1
    return wl


def _cases():
    rng = np.random.default_rng(300)
    out = []
    f = rng.uniform(-0.1, 1.1, size=(13, 150)).astype(np.float32)
    out.append(("quad_L6_offset", W.Workload("q6", 13, 150, np.array([-1.0, -0.4, 0.1, 0.9, 1.3, 2.0]),
                                             W.QUAD, 0.3, f=2 * f, a=3.0)))
    out.append(("tq_L10", W.truncated_quadratic(L=10, H=9, W=131, seed=31)))
    wl = W.truncated_quadratic(L=8, H=11, W=70, seed=32)
    wl.tau = wl.gamma.copy()
    wl.samples = rng.normal(0, 0.05, size=(8, 11, 70)).astype(np.float32)
    out.append(("tq_add_L8", wl))
    out.append(("sampled_L8", _sampled_workload(10, 97, 33)))
    out.append(("one_row", W.truncated_quadratic(L=6, H=1, W=200, seed=34)))
    out.append(("one_col", W.truncated_quadratic(L=6, H=77, W=1, seed=35)))
    out.append(("w64", W.truncated_quadratic(L=5, H=6, W=64, seed=36)))
    return [(n, _aniso(w)) for n, w in out]


CASES = _cases()


def _pair(wl, orc, storage="fp32"):
    return S.Problem.from_workload(wl, storage=storage), orc.Problem(wl)


@pytest.mark.parametrize("tiling", TILINGS, ids=TILING_IDS)
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_single_iteration_from_random_state(orc, name, wl, tiling):
    g, o = _pair(wl, orc)
    if not use_tiling(g, tiling, wl.W, wl.k):
        return
    st = W.random_state(21, wl.k, wl.H, wl.W)
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got, ref = _gpu_state(g), o.get_state()
    for n in S.STATE_ORDER:
        err = np.abs(got[n].astype(np.float64) - ref[n])
        bound = 2e-5 * (1.0 + np.abs(ref[n]))
        worst = np.unravel_index(np.argmax(err - bound), err.shape)
        assert np.all(err <= bound), f"{name}/{n}: err {err[worst]:.3e} at {worst}"
    # the box is active somewhere (the sampled case, on labels 0..63, has a radius beyond
    # the random p)
    rad = o.normalized()[1] * np.diff(o.normalized()[0])
    on_face = np.isclose(np.abs(ref["px"]), rad[:, None, None], rtol=0, atol=1e-12)
    assert wl.rho == W.SAMPLED or on_face.any()


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_monitor_on_identical_state(orc, name, wl):
    g, o = _pair(wl, orc)
    st = W.random_state(22, wl.k, wl.H, wl.W, scale=0.3)
    _load_same_state(g, o, st)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) < 1e-9
    assert _rel(eg["dual_lb"], eo["dual"]) < 1e-9
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) < 1e-9


def test_truncated_quadratic_fixed_iterations(orc):
    wl = _aniso(W.truncated_quadratic(L=10, H=40, W=72, seed=37))
    g, o = _pair(wl, orc)
    g.run(300)
    o.run(300)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) <= 1e-5
    assert _rel(eg["dual_lb"], eo["dual"]) <= 1e-5
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) <= 1e-5


def test_convex_run_to_gap_brackets_unlifted_optimum():
    """Quadratic data, L = 5: the relaxation with the l1 norm is exact, so the certified
    interval of the GPU run contains the optimum of the unlifted anisotropic ROF."""
    wl = _aniso(W.rof(H=48, W=56))
    wl.gamma = W.equispaced(5)
    g = S.Problem.from_workload(wl)
    g.run_to_gap(1e-4, 40000)
    rep = g.energy()
    _, Pf, Df = ck.fgp_box_rof(wl.f, wl.lam, aniso=True, tol=1e-9)
    assert rep["rel_gap"] <= 1e-4
    # both bounds are certified at every iterate (FP64 sums over an FP32 state)
    assert rep["dual_lb"] <= Pf * (1 + 1e-7) and Df <= rep["primal_ub"] * (1 + 1e-7)


def test_bf16_single_iteration(orc):
    name, wl = CASES[1]
    g, o = _pair(wl, orc, "bf16")
    st = W.random_state(23, wl.k, wl.H, wl.W)
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


@pytest.mark.parametrize("tiling", [(1, 4, 64), (2, 8, 64), (1, 4, 128)], ids=["g1t4c64", "g2t8c64", "g1t4c128"])
def test_batch_mixing_both_kinds_equals_lone_solves(tiling):
    shapes = [(9, 130, 5), (40, 90, 10), (1, 70, 2), (17, 200, 8)]
    wls = [W.truncated_quadratic(L=L, H=H, W=Wd, seed=60 + j) for j, (H, Wd, L) in enumerate(shapes)]
    wls = [_aniso(w) if j % 2 == 0 else w for j, w in enumerate(wls)]
    iters = 13
    b = S.BatchProblem(wls)
    b.set_tiling(*tiling)
    b.run(iters)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        print(f"batch member {i} tv={wl.tv} {wl.H}x{wl.W} L={wl.L} tiling={tiling}", flush=True)
        s = S.Problem.from_workload(wl)
        s.set_tiling(*tiling)
        s.run(iters)
        ul_s, u_s = s.read_u()
        rep_s = s.energy()
        ul, u = b.read_u_of(i)
        rep = b.energy_of(i)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ul.cpu().numpy(), ul_s.cpu().numpy())
        np.testing.assert_array_equal(u.cpu().numpy(), u_s.cpu().numpy())
        for key in ("primal_ub", "dual_lb", "e_nonconvex"):
            assert rep[key] == rep_s[key], (i, key)
        s.close()
    b.close()


def test_gradients_match_oracle_reverse_pass(orc):
    from tests.test_gpu_adjoint import _check_close, _gpu_grads, _tq_w
    rng = np.random.default_rng(305)
    wl = _aniso(_tq_w(6, 40, 70, 38, rng))
    K, C = 40, 7
    g = rng.uniform(0, 1, (wl.H, wl.W))
    o = orc.Problem(wl)
    o.unrolled_forward(K)
    _, uo = o.read_u()
    u, gf, gl, gw = _gpu_grads(wl, K, C, g)
    assert np.abs(u - uo).max() <= 1e-5
    gfo, glo, gwo = o.unrolled_backward(2.0 * (u.astype(np.float64) - g))
    _check_close(gf, gfo, "grad f")
    assert abs(gl - glo) <= 1e-4 * abs(glo), (gl, glo)
    _check_close(gw, gwo, "grad w")
