"""Auxiliary subsystems on the GPU: the SL_TRACE log of gap-controlled runs (one JSON object
per line) and the numeric-error path of the certified monitor. GPU only."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _lines(path):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def test_trace_of_a_single_solve(tmp_path, monkeypatch):
    trace = tmp_path / "trace.jsonl"
    monkeypatch.setenv("SL_TRACE", str(trace))
    wl = W.truncated_quadratic(L=6, H=40, W=70, seed=21)
    g = S.Problem.from_workload(wl, storage="bf16", check_every=50)
    n = g.run_to_gap(1e-3, 20000)
    rep = g.energy()
    rows = _lines(trace)
    checks = [r for r in rows if r["event"] == "check"]
    assert len(checks) == n // 50
    assert [r["iters"] for r in checks] == list(range(50, n + 1, 50))
    assert checks[-1]["rel_gap"] <= 1e-3 and all(r["rel_gap"] > 1e-3 for r in checks[:-1])
    assert checks[-1]["primal"] == rep["primal_ub"] and checks[-1]["dual"] == rep["dual_lb"]
    # the storage column follows the widening event, if any
    widen = [r for r in rows if r["event"] == "widen"]
    assert len(widen) <= 1
    for r in checks:
        assert r["storage"] == ("fp32" if widen and r["iters"] > widen[0]["iters"] else "bf16")
    g.close()
    monkeypatch.delenv("SL_TRACE")
    g = S.Problem.from_workload(wl, check_every=50)
    g.run_to_gap(1e-3, 200)
    assert len(_lines(trace)) == len(rows)        # nothing written without SL_TRACE
    g.close()


def test_trace_of_a_batch(tmp_path, monkeypatch):
    trace = tmp_path / "trace.jsonl"
    monkeypatch.setenv("SL_TRACE", str(trace))
    wls = [W.truncated_quadratic(L=L, H=24, W=64, seed=30 + L) for L in (2, 4, 8)]
    b = S.BatchProblem(wls, check_every=48)
    done = b.run_to_gap(1e-3, 30000)
    rows = _lines(trace)
    retired = {r["member"]: r for r in rows if r["event"] == "retire"}
    assert sorted(retired) == [0, 1, 2]
    for i in range(3):
        n, active = b.info_of(i)
        assert not active and retired[i]["iters"] == n and retired[i]["rel_gap"] <= 1e-3
    checks = [r for r in rows if r["event"] == "batch_check"]
    assert checks[-1]["batched_iters"] == done and checks[-1]["active"] >= 1
    assert [r["active"] for r in checks] == sorted((r["active"] for r in checks), reverse=True)
    b.close()


def _widen_check(checks, tol, stall_checks, progress, widen_gap):
    """The iteration count of the check at which the finishing rule widens a bf16 problem,
    recomputed from the bounds each check logged (None: it never widens)."""
    best_p, best_d, ref, stall = float("inf"), -float("inf"), None, 0
    for c in checks:
        best_p, best_d = min(best_p, c["primal"]), max(best_d, c["dual"])
        rel = (best_p - best_d) / max(abs(best_p), abs(best_d), 1e-30)
        if rel <= tol:
            return None
        if widen_gap > 0 and rel <= widen_gap:
            return c["iters"]
        if stall_checks <= 0:
            continue
        g = best_p - best_d
        if ref is None or g < ref * (1.0 - progress):
            ref, stall = g, 0
            continue
        stall += 1
        if stall >= stall_checks:
            return c["iters"]
    return None


@pytest.mark.parametrize("rule", [(4, 0.1, 0.05), (3, 0.2, 0.0), (4, 1e-3, 0.0), (0, 0.1, 0.2)],
                         ids=["default", "fast_stall", "slow_stall", "gap_only"])
def test_finishing_rule_matches_trace(tmp_path, monkeypatch, rule):
    """The check at which a bf16 solve widens its duals is the one the documented rule picks
    from the certified bounds of the checks before it (recomputed here from the trace)."""
    trace = tmp_path / "trace.jsonl"
    monkeypatch.setenv("SL_TRACE", str(trace))
    wl = W.truncated_quadratic(L=2, H=48, W=96, seed=17)
    g = S.Problem.from_workload(wl, storage="bf16", check_every=25)
    if rule != (4, 0.1, 0.05):
        g.set_finishing(*rule)
    g.run_to_gap(1e-3, 20000)
    rows = _lines(trace)
    checks = [r for r in rows if r["event"] == "check"]
    widen = [r["iters"] for r in rows if r["event"] == "widen"]
    want = _widen_check(checks, 1e-3, *rule)
    print(f"rule {rule}: widened at {widen}, rule gives {want}, {checks[-1]['iters']} iterations")
    assert widen == ([] if want is None else [want])
    assert g.storage_info() == (("fp32", want) if want is not None else ("bf16", checks[-1]["iters"]))
    if rule == (4, 0.1, 0.05):
        assert checks[-1]["rel_gap"] <= 1e-3
    g.close()


def test_finishing_arguments():
    g = S.Problem.from_workload(W.truncated_quadratic(L=3, H=8, W=64, seed=2), storage="bf16")
    for bad in [(-1, 0.1, 0.0), (4, 0.0, 0.0), (4, 1.0, 0.0), (4, 0.1, -1e-3), (4, 0.1, float("inf")),
                (4, float("nan"), 0.0)]:
        with pytest.raises(S.SublabelError) as e:
            g.set_finishing(*bad)
        assert e.value.status == 1, bad
    g.close()


def test_nonfinite_state_is_a_numeric_error():
    """A non-finite dual makes the certificate non-finite: sl_energy and sl_run_to_gap
    return SL_ERR_NUMERIC instead of a bound. (A non-finite primal value is clamped away by
    the repair of the primal point, whose bound stays valid.)"""
    wl = W.truncated_quadratic(L=5, H=9, W=70, seed=3)
    g = S.Problem.from_workload(wl)
    st = W.random_state(5, wl.k, wl.H, wl.W)
    st["px"][2, 4, 10] = np.nan
    g.load_state(S.pack_state(st))
    with pytest.raises(S.SublabelError) as e:
        g.energy()
    assert e.value.status == 5 and "non-finite" in str(e.value)
    with pytest.raises(S.SublabelError) as e:
        g.run_to_gap(1e-3, 100)
    assert e.value.status == 5
    g.close()
