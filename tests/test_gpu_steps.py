"""Step control on the GPU: the balance of dual against primal steps, the residual norms of
one iteration (against the FP64 oracle's on the same pair of states) and the adaptive
balance of sl_run_to_gap. GPU only.

Tolerance of the residual norms: the per-entry terms are FP32 differences of FP32 states
(relative rounding about 1e-7 of the larger operand) summed in FP64, so the l1 sums agree
with the oracle's to 1e-5 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _state(g):
    t = g.save_state()
    torch.cuda.synchronize()
    return {n: a.astype(np.float64) for n, a in S.unpack_state(t, g.k, g.H, g.W).items()}


@pytest.mark.parametrize("c", [1.0, 0.25])
def test_residual_norms_match_oracle(orc, c):
    wl = W.truncated_quadratic(L=6, H=20, W=70, seed=31)
    g = S.Problem.from_workload(wl)
    g.set_step_balance(c)
    g.run(37)
    before = _state(g)
    rp, rd, kty, kx = g.residuals_full()
    after = _state(g)
    o = orc.Problem(wl, step_balance=c)
    rpo, rdo = o.residual_norms(before, after)
    # the scales of the scaled balancing rule: |y| and |x| (l1) at the new iterate
    kxo = sum(np.abs(after[n]).sum() for n in ("u", "s"))
    ktyo = sum(np.abs(after[n]).sum() for n in ("v", "z", "px", "py", "qd"))
    print(f"c={c}: gpu {rp:.9g} {rd:.9g} {kty:.9g} {kx:.9g} oracle {rpo:.9g} {rdo:.9g} {ktyo:.9g} {kxo:.9g}")
    assert abs(rp - rpo) <= 1e-5 * rpo and abs(rd - rdo) <= 1e-5 * rdo
    assert abs(kty - ktyo) <= 1e-5 * ktyo and abs(kx - kxo) <= 1e-5 * kxo


def test_balance_matches_oracle_iteration(orc):
    wl = W.truncated_quadratic(L=5, H=40, W=72, seed=25)
    g = S.Problem.from_workload(wl)
    g.set_step_balance(1 / 16)
    o = orc.Problem(wl, step_balance=1 / 16)
    g.run(300)
    o.run(300)
    eg, eo = g.energy(), o.monitor()
    assert abs(eg["primal_ub"] - eo["primal"]) <= 1e-5 * abs(eo["primal"])
    assert abs(eg["dual_lb"] - eo["dual"]) <= 1e-5 * abs(eo["dual"])


def test_balance_one_restores_default_steps():
    wl = W.truncated_quadratic(L=6, H=16, W=70, seed=4)
    a = S.Problem.from_workload(wl)
    b = S.Problem.from_workload(wl)
    b.set_step_balance(0.1)
    b.set_step_balance(1.0)
    a.run(25)
    b.run(25)
    assert torch.equal(a.read_u()[0], b.read_u()[0])
    with pytest.raises(S.SublabelError):
        b.set_step_balance(0.0)
    with pytest.raises(S.SublabelError):
        b.set_residual_target(-1.0)


def test_adaptive_run_reaches_gap_and_brackets_oracle(orc):
    wl = W.truncated_quadratic(L=8, H=48, W=64, seed=9)
    g = S.Problem.from_workload(wl, adaptive=True)
    n = g.run_to_gap(1e-3, 30000)
    e = g.energy()
    assert e["rel_gap"] <= 1e-3, (n, e)
    c = g.get_step_balance()
    assert 1 / 4096 <= c <= 4096 and c != 1.0
    # same problem, fixed steps: slower
    f = S.Problem.from_workload(wl, adaptive=False)
    nf = f.run_to_gap(1e-3, n)
    assert f.energy()["rel_gap"] > 1e-3 or nf >= n
    # the certified interval contains the relaxed optimum the oracle brackets
    o = orc.Problem(wl, step_balance=c)
    orc.run_to_gap(o, 1e-3, 60000)
    ro = o.monitor()
    assert e["best_dual"] <= ro["best_primal"] * (1 + 1e-6)
    assert ro["best_dual"] <= e["best_primal"] * (1 + 1e-6)
    # deterministic: the same run again gives the same balance and bounds
    g2 = S.Problem.from_workload(wl, adaptive=True)
    assert g2.run_to_gap(1e-3, 30000) == n
    assert g2.get_step_balance() == c and g2.energy()["best_primal"] == e["best_primal"]


@pytest.mark.parametrize("graphs", [True, False], ids=["graphs", "eager"])
def test_batch_adaptive_members_equal_lone_adaptive_runs(graphs):
    """Every batch member is rebalanced from its own residuals exactly as a lone adaptive
    solve with the same tiling and check interval: same iterations, same iterates, whether
    the iterations and the per-check work (saved duals, residuals, monitors) are replayed
    from graphs or launched eagerly."""
    wls = [W.truncated_quadratic(L=4, H=24, W=70, seed=61), W.truncated_quadratic(L=6, H=30, W=64, seed=62),
           W.truncated_quadratic(L=8, H=16, W=90, seed=63)]
    b = S.BatchProblem(wls, check_every=48, adaptive=True)
    b.set_graphs(graphs)
    tiling = b.get_tiling()
    b.run_to_gap(1e-3, 30000)
    for i, wl in enumerate(wls):
        g = S.Problem.from_workload(wl, check_every=48, adaptive=True)
        g.set_tiling(*tiling)
        n = g.run_to_gap(1e-3, 30000)
        nb, active = b.info_of(i)
        print(f"member {i} L={wl.L}: lone {n} iterations, batch {nb}, balance {g.get_step_balance():.4g}")
        assert nb == n and not active
        assert torch.equal(b.read_u_of(i)[0], g.read_u()[0])
        assert b.energy_of(i)["rel_gap"] <= 1e-3
        g.close()
    b.close()
