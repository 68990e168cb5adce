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
