"""BF16 dual storage with its FP32 finishing phase, through the C-ABI. GPU only.

Widening the duals is exact (every bf16 value is a float), so a problem widened after n
iterations must hold the same state as before, and continue bit for bit like a float
problem loaded with that state. In a batch every member widens on its own (its tiles move
from the bf16 work list to the float one), so a member must match a lone problem widened at
the same iteration. Gap-controlled solves with bf16 duals reach a 1e-3 certified gap, and
their certified intervals contain the FP64 oracle's optimum.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _sampled(H, Wd, seed, L=6, M=30):
    rng = np.random.default_rng(seed)
    tau = np.arange(M, dtype=np.float64)
    idx = np.round(np.linspace(0, M - 1, L)).astype(int)
    base = rng.uniform(0, 1, size=(M, H, Wd))
    costs = np.abs(base - base[rng.integers(0, M)]).astype(np.float32)
    return W.Workload(f"smp{seed}", H, Wd, tau[idx], W.SAMPLED, 0.5, tau=tau, samples=costs)


CASES = [("tq", W.truncated_quadratic(L=7, H=37, W=150, seed=61)),
         ("quad", W.rof(H=33, W=70)),
         ("sampled", _sampled(19, 77, 62))]


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n0", [1, 4])
def test_widen_keeps_state_and_continues_as_fp32(name, wl, n0):
    """After n0 bf16 iterations (both rotation parities of the double-buffered duals):
    the packed state is unchanged by widening, and the next iterations equal those of a
    float problem loaded with that state."""
    print(f"widen: {name} {wl.H}x{wl.W} L={wl.L} after {n0} iterations", flush=True)
    g = S.Problem.from_workload(wl, storage="bf16")
    g.run(n0)
    before = g.save_state().clone()
    assert g.storage_info() == ("bf16", n0)
    g.widen()
    assert g.storage_info() == ("fp32", n0)
    after = g.save_state().clone()
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    f = S.Problem.from_workload(wl, storage="fp32")
    f.set_tiling(*g.get_tiling())
    f.load_state(after)
    g.run(11)
    f.run(11)
    torch.cuda.synchronize()
    assert torch.equal(g.save_state(), f.save_state())
    ge, fe = g.energy(), f.energy()
    for key in ("primal_ub", "dual_lb", "e_nonconvex"):
        assert ge[key] == fe[key], key
    g.widen()                      # already float: no-op
    with pytest.raises(S.SublabelError) as e:      # float duals are never narrowed
        S._check(S.lib().sl_set_storage(f.h, -1, S.STORE_BF16_DUAL))
    assert e.value.status == 2
    g.close()
    f.close()


def test_batch_members_widen_independently():
    """Members 1 and 3 of a bf16 batch are widened after 7 iterations and the batch runs 17
    more (eager launches, then two graph replays, over two work lists); every member equals
    a lone problem treated the same way."""
    shapes = [(9, 131, 5), (40, 90, 10), (1, 70, 2), (33, 64, 20), (17, 200, 8)]
    wls = [W.truncated_quadratic(L=L, H=H, W=Wd, seed=80 + j) for j, (H, Wd, L) in enumerate(shapes)]
    b = S.BatchProblem(wls, storage="bf16")
    tiling = b.get_tiling()
    b.run(7)
    b.widen(1)
    b.widen(3)
    b.run(17)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        print(f"batch member {i} {wl.H}x{wl.W} L={wl.L}", flush=True)
        g = S.Problem.from_workload(wl, storage="bf16")
        g.set_tiling(*tiling)
        g.run(7)
        if i in (1, 3):
            g.widen()
        g.run(17)
        ul, u = g.read_u()
        rep = g.energy()
        bul, bu = b.read_u_of(i)
        brep = b.energy_of(i)
        torch.cuda.synchronize()
        assert torch.equal(bul, ul) and torch.equal(bu, u)
        for key in ("primal_ub", "dual_lb", "e_nonconvex"):
            assert brep[key] == rep[key], (i, key)
        assert b.storage_info(i) == (("fp32", 7) if i in (1, 3) else ("bf16", 24))
        g.close()
    b.close()


def test_batch_bf16_reaches_gap_and_brackets_oracle(orc):
    """Mixed sizes and label counts (2 to 16), bf16 duals, adaptive steps, every member run
    to a 1e-3 certified gap with the float finishing phase; each member's certified interval
    overlaps the FP64 oracle's (two certified intervals of one problem both contain its
    optimum), the oracle run to a 1e-2 gap or 20 000 iterations."""
    sizes = [(24, 24, 2), (16, 40, 4), (32, 32, 8), (20, 28, 16), (8, 64, 4), (30, 30, 2)]
    wls = [W.truncated_quadratic(L=L, H=H, W=Wd, seed=300 + j) for j, (H, Wd, L) in enumerate(sizes)]
    b = S.BatchProblem(wls, storage="bf16", adaptive=True, check_every=48)
    done = b.run_to_gap(1e-3, 60000)
    for i, wl in enumerate(wls):
        rep = b.energy_of(i)
        n, active = b.info_of(i)
        storage, n16 = b.storage_info(i)
        o = orc.Problem(wl)
        ro = None
        for _ in range(80):
            o.run(250)
            ro = o.monitor()
            if ro["rel_gap"] <= 1e-2:
                break
        print(f"member {i} {wl.H}x{wl.W} L={wl.L}: {n} its ({n16} bf16, now {storage}), rel gap "
              f"{rep['rel_gap']:.2e}; oracle [{ro['best_dual']:.6g}, {ro['best_primal']:.6g}] "
              f"gpu [{rep['best_dual']:.6g}, {rep['best_primal']:.6g}]", flush=True)
        assert not active and rep["rel_gap"] <= 1e-3, (i, rep)
        assert rep["best_dual"] <= ro["best_primal"] * (1 + 1e-9) + 1e-12
        assert ro["best_dual"] <= rep["best_primal"] * (1 + 1e-9) + 1e-12
    assert done <= 60000
    b.close()


def test_batch_widening_with_saturated_grids():
    """Regression: members widened one after another while both work lists have more tiles
    than the launch has blocks, so the grids (and the captured graph) do not change between
    widenings. The float list lives at a fixed place in the work table, so the graph's
    launches stay valid; every member equals a lone problem treated the same way."""
    wls = [W.truncated_quadratic(L=2, H=512, W=512, seed=500 + j) for j in range(8)]
    b = S.BatchProblem(wls, storage="bf16")
    tiling = b.get_tiling()
    plan = [(7, None), (12, 0), (12, 1), (12, 2), (12, 3)]   # (iterations, member widened before them)
    for n, m in plan:
        if m is not None:
            b.widen(m)
        b.run(n)
    torch.cuda.synchronize()
    for i, wl in enumerate(wls):
        print(f"saturated batch member {i}", flush=True)
        g = S.Problem.from_workload(wl, storage="bf16")
        g.set_tiling(*tiling)
        for n, m in plan:
            if m == i:
                g.widen()
            g.run(n)
        ul, _ = g.read_u()
        rep = g.energy()
        bul, _ = b.read_u_of(i)
        brep = b.energy_of(i)
        torch.cuda.synchronize()
        assert torch.equal(bul, ul), i
        for key in ("primal_ub", "dual_lb", "e_nonconvex"):
            assert brep[key] == rep[key], (i, key)
        g.close()
    b.close()


def _bf16_rne(a):
    """float32 -> bfloat16 by round to nearest, ties to even (finite values; a carry into
    the exponent field gives the next binade or infinity), returned as float32."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def test_storage_rounding_is_nearest_even():
    """Loading a state into bf16 storage rounds v, z and p to nearest even: exact ties with an
    even and an odd kept part, values just beside a tie, subnormals, negative values, and
    the largest finite values (which round to infinity). Compared bit for bit."""
    special = np.array([0x3F808000, 0x3F818000, 0x3F807FFF, 0x3F808001, 0xBF818000, 0x00008000,
                        0x00018000, 0x00017FFF, 0x80018000, 0x7F7F8000, 0x7F7F7FFF, 0x7F7FFFFF,
                        0x00000000, 0x80000000, 0x3F800000, 0x4049_0FDB], dtype=np.uint32).view(np.float32)
    wl = W.truncated_quadratic(L=4, H=5, W=70, seed=8)
    st = W.random_state(3, wl.k, wl.H, wl.W)
    rng = np.random.default_rng(4)
    for n in ("v", "z", "px", "py"):
        a = st[n].reshape(-1)
        a[:special.size] = special
        a[special.size:] = rng.standard_normal(a.size - special.size).astype(np.float32) * \
            np.float32(2.0) ** rng.integers(-30, 30, a.size - special.size)
    g = S.Problem.from_workload(wl, storage="bf16")
    g.load_state(S.pack_state(st))
    t = g.save_state()
    torch.cuda.synchronize()
    got = S.unpack_state(t, g.k, g.H, g.W)
    g.close()
    for n in S.STATE_ORDER:
        want = _bf16_rne(st[n]) if n in ("v", "z", "px", "py") else st[n]
        assert np.array_equal(got[n].view(np.uint32), np.asarray(want, np.float32).view(np.uint32)), n
    # the cases by name: ties go to the even neighbour, the largest floats to infinity
    v = got["v"].reshape(-1)[:special.size].view(np.uint32)
    assert list(v[:2]) == [0x3F800000, 0x3F820000] and v[9] == 0x7F800000 and v[11] == 0x7F800000
    assert v[5] == 0 and v[6] == 0x00020000
