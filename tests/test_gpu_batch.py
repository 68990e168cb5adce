"""Batched solves (many independent problems per launch, hipGraph replay of the
iteration period, autotuned tiling) through the C-ABI. GPU only.

The batch kernel runs the same per-tile code as the single-instance kernel, so a batch
member must match a single-instance solve of the same problem with the same tiling bit for
bit, whatever mix of sizes and label counts shares the launch and whether the period is
replayed from a graph or launched eagerly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402

from tests.gpu_tilings import TILING_IDS, TILINGS, use_tiling  # noqa: E402


def _mixed_tq():
    # sizes that leave ragged 64 x 4 and 64 x 8 tiles, label counts 2 .. 28 (the maximum)
    shapes = [(9, 131, 5), (40, 90, 10), (1, 70, 2), (33, 64, 20), (17, 200, 8), (1, 1, 4), (5, 70, 28)]
    return [W.truncated_quadratic(L=L, H=H, W=Wd, seed=40 + j) for j, (H, Wd, L) in enumerate(shapes)]


def _mixed_tq_even():
    # a similar mix with even widths (pixel pairs need them) and at most 16 labels (the
    # largest label count whose LDS fits every pixel-pair tiling)
    shapes = [(9, 130, 5), (40, 90, 10), (1, 70, 2), (33, 64, 14), (17, 200, 8), (2, 2, 4), (5, 70, 16)]
    return [W.truncated_quadratic(L=L, H=H, W=Wd, seed=40 + j) for j, (H, Wd, L) in enumerate(shapes)]


def _mixed_sampled():
    out = []
    # the last member sits at both maxima (28 labels, 256 samples)
    for j, (H, Wd, L, M) in enumerate([(10, 97, 8, 64), (6, 65, 4, 13), (21, 30, 6, 40), (5, 70, 28, 256)]):
        rng = np.random.default_rng(70 + j)
        tau = np.arange(M, dtype=np.float64)
        idx = np.round(np.linspace(0, M - 1, L)).astype(int)
        base = rng.uniform(0, 1, size=(M, H, Wd))
        costs = np.abs(base - base[rng.integers(0, M)]).astype(np.float32)
        out.append(W.Workload(f"smp{j}", H, Wd, tau[idx], W.SAMPLED, 0.5, tau=tau, samples=costs))
    return out


def _single(wl, tiling, iters):
    g = S.Problem.from_workload(wl)
    g.set_tiling(*tiling)
    g.run(iters)
    ul, u = g.read_u()
    rep = g.energy()
    torch.cuda.synchronize()
    g.close()
    return ul.cpu().numpy(), u.cpu().numpy(), rep


def _assert_member_equals(b, i, ref):
    ul, u = b.read_u_of(i)
    rep = b.energy_of(i)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ul.cpu().numpy(), ref[0])
    np.testing.assert_array_equal(u.cpu().numpy(), ref[1])
    for key in ("primal_ub", "dual_lb", "e_nonconvex"):
        assert rep[key] == ref[2][key], (i, key, rep[key], ref[2][key])


@pytest.mark.parametrize("tiling", TILINGS, ids=TILING_IDS)
def test_batch_member_equals_single_solve(tiling):
    wls = _mixed_tq() if tiling[2] == 64 else _mixed_tq_even()
    iters = 13                     # two graph periods and a tail of eager launches
    b = S.BatchProblem(wls)
    b.set_tiling(*tiling)
    b.run(iters)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        print(f"batch member {i} {wl.H}x{wl.W} L={wl.L} tiling={tiling}", flush=True)
        _assert_member_equals(b, i, _single(wl, tiling, iters))
        assert b.info_of(i) == (iters, True)
    b.close()


def test_batch_sampled_member_equals_single_solve():
    wls = _mixed_sampled()
    b = S.BatchProblem(wls)
    tiling = b.get_tiling()
    b.run(20)
    for i, wl in enumerate(wls):
        _assert_member_equals(b, i, _single(wl, tiling, 20))
    b.close()


def test_batch_bf16_member_equals_single_solve():
    wls = _mixed_tq()[:4]
    b = S.BatchProblem(wls, storage="bf16")
    tiling = b.get_tiling()
    b.run(9)
    for i, wl in enumerate(wls):
        g = S.Problem.from_workload(wl, storage="bf16")
        g.set_tiling(*tiling)
        g.run(9)
        ul, u = g.read_u()
        rep = g.energy()
        torch.cuda.synchronize()
        _assert_member_equals(b, i, (ul.cpu().numpy(), u.cpu().numpy(), rep))
        g.close()
    b.close()


def test_graph_replay_equals_eager_launches():
    """Graph replays interleaved with the program's own eager work and synchronisations
    give the same iterates as eager launches after every replay."""
    wls = _mixed_tq()
    bg = S.BatchProblem(wls)
    be = S.BatchProblem(wls)
    be.set_graphs(False)
    x = torch.randn(1 << 20, device="cuda:0")
    for chunk in (6, 12, 5, 7, 18):
        bg.run(chunk)
        be.run(chunk)
        y = (x * 1.5).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for i in range(len(wls)):
            ug, _ = bg.read_u_of(i)
            ue, _ = be.read_u_of(i)
            torch.cuda.synchronize()
            assert torch.equal(ug, ue), (chunk, i)
    for i in range(len(wls)):
        assert bg.energy_of(i) == be.energy_of(i)
    bg.close()
    be.close()


def test_batch_member_matches_oracle(orc):
    wls = _mixed_tq()
    b = S.BatchProblem(wls)
    b.run(60)
    for i in (1, 3, 4, 6):
        o = orc.Problem(wls[i])
        o.run(60)
        rg, ro = b.energy_of(i), o.monitor()
        for kg, ko in (("primal_ub", "primal"), ("dual_lb", "dual"), ("e_nonconvex", "e_nc")):
            assert abs(rg[kg] - ro[ko]) <= 1e-5 * abs(ro[ko]), (i, kg, rg[kg], ro[ko])
    b.close()


def test_batch_run_to_gap_retires_members():
    wls = [W.truncated_quadratic(L=2, H=32, W=32, seed=1)]
    wls += [W.truncated_quadratic(L=L, H=24, W=70, seed=90 + L) for L in (4, 6)]
    b = S.BatchProblem(wls, check_every=48, adaptive=False)
    tol = 2e-2                     # the oracle reaches it after 576, 2304 and 5568 iterations
    done = b.run_to_gap(tol, 20000)
    assert done <= 20000
    for i in range(len(wls)):
        n, active = b.info_of(i)
        rep = b.energy_of(i)
        assert not active and rep["rel_gap"] <= tol, (i, n, rep)
        assert n % 48 == 0
    # retired members are frozen
    before = [b.read_u_of(i)[0].clone() for i in range(len(wls))]
    b.run(12)
    for i in range(len(wls)):
        assert torch.equal(b.read_u_of(i)[0], before[i])
    b.close()


def test_batch_finishing_rule_off_and_immediate():
    """With the finishing rule off (no stall count, widen gap 0) every member keeps bf16 duals
    through any number of checks (the throughput measurement relies on it); with a widen gap
    above every reachable gap each member widens at its first check, on its own, and keeps
    counting its bf16 iterations."""
    wls = _mixed_tq()[:5]
    b = S.BatchProblem(wls, storage="bf16", adaptive=True, check_every=12)
    b.set_finishing(0, widen_gap=0.0)
    for _ in range(6):
        b.run_to_gap(0.0, 12)            # a zero gap is never met: every member stays active
    for i in range(len(wls)):
        n, active = b.info_of(i)
        assert active and n == 72
        assert b.storage_info(i) == ("bf16", 72), i
    b.close()
    b = S.BatchProblem(wls, storage="bf16", adaptive=True, check_every=12)
    b.set_finishing(0, widen_gap=1e30)
    b.run_to_gap(0.0, 12)
    for i in range(len(wls)):
        assert b.storage_info(i) == ("fp32", 12), i
    b.run_to_gap(0.0, 12)
    for i in range(len(wls)):
        assert b.storage_info(i) == ("fp32", 12), i
        assert b.info_of(i)[0] == 24
    b.close()


def test_autotune_resets_state_and_uses_cache(tmp_path):
    wl = W.truncated_quadratic(L=10, H=64, W=128, seed=11)
    g = S.Problem.from_workload(wl)
    fresh = g.energy()
    g.run(30)
    cache = str(tmp_path / "tiling.cache")
    t1 = g.autotune(iters=10, cache=cache)
    assert t1 in TILINGS and g.get_tiling() == t1
    assert g.energy() == fresh                    # iteration state back at its start
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"|{TILINGS.index(t1)}")
    t2 = g.autotune(iters=10, cache=cache)        # served from the cache
    assert t2 == t1 and len(open(cache).read().splitlines()) == 1
    g.close()

    b = S.BatchProblem(_mixed_tq())
    tb = b.autotune(iters=6)
    assert tb in TILINGS
    for i in range(6):
        assert b.info_of(i) == (0, True)
    b.close()


def test_batch_rejects_mixed_kinds():
    wls = [_mixed_tq()[0], _mixed_sampled()[0]]
    with pytest.raises(S.SublabelError):
        S.BatchProblem(wls)


def test_batched_monitor_matches_each_members_monitor(tmp_path, monkeypatch):
    """The checks of a batch solve run every active member's certificate in one launch per
    stage (members with bf16 and with float duals, both TV kinds); each member's bounds must
    equal those of its own monitor on the same state, bit for bit. Every member retires at
    the first check (tolerance 10), where the trace records the batched bounds."""
    import json
    trace = tmp_path / "trace.jsonl"
    monkeypatch.setenv("SL_TRACE", str(trace))
    wls = [W.truncated_quadratic(L=2, H=24, W=64, seed=91), W.truncated_quadratic(L=4, H=40, W=70, seed=92),
           W.truncated_quadratic(L=6, H=17, W=130, seed=93), W.truncated_quadratic(L=3, H=64, W=64, seed=94)]
    wls[3].tv = S.TV_ANISO
    b = S.BatchProblem(wls, storage="bf16", check_every=48)
    b.widen(1)
    b.widen(3)
    b.run(30)
    b.run_to_gap(10.0, 48)
    rows = [json.loads(line) for line in open(trace) if line.strip()]
    retired = {r["member"]: r for r in rows if r["event"] == "retire"}
    assert sorted(retired) == [0, 1, 2, 3]
    for i in range(4):
        e = b.energy_of(i)
        assert e["primal_ub"] == retired[i]["primal"] and e["dual_lb"] == retired[i]["dual"], i
    assert [b.storage_info(i)[0] for i in range(4)] == ["bf16", "fp32", "bf16", "fp32"]
    b.close()
