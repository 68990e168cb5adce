"""Temporal blocking (two iterations per pass over the state, k <= 3) through the C-ABI.
GPU only.

The two-iteration kernel repeats the one-pass kernel's arithmetic with one label group in
the same order, so its iterates must be bitwise those of the one-pass kernel in a
one-group launch configuration, on every data term it covers, for both TV kinds, on image
shapes that leave ragged tiles in both directions, for iteration counts that mix
two-iteration passes with single iterations; gap-controlled solves then take the same
path to the same certificate. Against the FP64 oracle it inherits the one-pass kernel's
bounds (checked here once more after 200 iterations).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _aniso(wl):
    wl.tv = S.TV_ANISO
    return wl


def _periodic(L, H, Wd, seed):
    wl = W.phase_unwrapping(seed=seed, H=H, W=Wd, L=L)
    return wl


CASES = [("rof_k1", W.rof(H=37, W=150)),
         ("tq_k1", W.truncated_quadratic(L=2, H=61, W=61, seed=41)),
         ("tq_k2", W.truncated_quadratic(L=3, H=13, W=200, seed=42)),
         ("tq_k3", W.truncated_quadratic(L=4, H=40, W=70, seed=43)),
         ("tq_k3_aniso", _aniso(W.truncated_quadratic(L=4, H=25, W=121, seed=44))),
         ("rof_aniso", _aniso(W.rof(H=64, W=64, seed=45))),
         ("periodic_k3", _periodic(4, 30, 90, 46)),
         ("one_row", W.truncated_quadratic(L=4, H=1, W=70, seed=47)),
         ("one_column", W.truncated_quadratic(L=3, H=70, W=1, seed=48)),
         ("tiny", W.truncated_quadratic(L=2, H=2, W=3, seed=49))]


def _state(g):
    t = g.save_state()
    torch.cuda.synchronize()
    return S.unpack_state(t, g.k, g.H, g.W)


def _pair(wl, seed):
    st = S.pack_state(W.random_state(seed, wl.k, wl.H, wl.W))
    a = S.Problem.from_workload(wl)
    a.set_tiling(1, 4, 64)
    b = S.Problem.from_workload(wl)
    b.set_tiling(1, 4, 64)
    b.set_temporal(True)
    a.load_state(st)
    b.load_state(st)
    return a, b


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n", [4, 7, 12])
def test_two_iteration_passes_equal_single_iterations(name, wl, n):
    print(f"case {name}: {wl.H}x{wl.W} L={wl.L} n={n}", flush=True)
    a, b = _pair(wl, 7 + n)
    a.run(n)
    b.run(n)
    sa, sb = _state(a), _state(b)
    for key in S.STATE_ORDER:
        assert np.array_equal(sa[key].view(np.uint32), sb[key].view(np.uint32)), key
    a.close()
    b.close()


def test_gap_controlled_solve_is_unchanged():
    """run_to_gap with two-iteration passes: the same iterations, bounds and read-out."""
    wl = W.truncated_quadratic(L=3, H=96, W=160, seed=50)
    out = []
    for temporal in (False, True):
        g = S.Problem.from_workload(wl, check_every=50)
        g.set_tiling(1, 4, 64)
        if temporal:
            g.set_temporal(True)
        n = g.run_to_gap(1e-3, 20000)
        e = g.energy()
        _, u = g.read_u()
        out.append((n, e["best_primal"], e["best_dual"], u.cpu().numpy()))
        g.close()
    assert out[0][:3] == out[1][:3]
    assert np.array_equal(out[0][3], out[1][3])
    assert out[1][0] < 20000


def test_against_the_oracle(orc):
    wl = W.truncated_quadratic(L=4, H=40, W=70, seed=51)
    g = S.Problem.from_workload(wl)
    g.set_temporal(True)
    g.run(200)
    o = orc.Problem(wl)
    o.run(200)
    got, ref = _state(g), o.get_state()
    for key in S.STATE_ORDER:
        err = np.abs(got[key].astype(np.float64) - ref[key])
        assert np.all(err <= 1e-5 * (1.0 + np.abs(ref[key]))), (key, err.max())
    g.close()


def test_unrolled_pass_keeps_single_iterations():
    """The unrolled forward pass ignores the two-iteration passes (its replays run the
    one-pass kernel), so its gradients do not depend on the setting."""
    wl = W.truncated_quadratic(L=3, H=24, W=64, seed=52)
    gu = torch.ones((wl.H, wl.W), device="cuda:0")
    res = []
    for temporal in (False, True):
        g = S.Problem.from_workload(wl)
        if temporal:
            g.set_temporal(True)
        g.unrolled_forward(12, 4)
        gf, gl, _ = g.unrolled_backward(gu)
        torch.cuda.synchronize()
        res.append((gf.cpu().numpy(), gl))
        g.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]


def test_unsupported_cases():
    cases = [W.truncated_quadratic(L=5, H=8, W=64, seed=53)]                        # k = 4
    M = 9
    rng = np.random.default_rng(5)
    cases.append(W.Workload("s", 6, 7, np.array([0.0, 4.0, 8.0]), W.SAMPLED, 0.3, tau=np.arange(float(M)),
                            samples=rng.uniform(0, 1, (M, 6, 7)).astype(np.float32)))  # sampled
    for wl in cases:
        g = S.Problem.from_workload(wl)
        with pytest.raises(S.SublabelError) as e:
            g.set_temporal(True)
        assert e.value.status == 2
        g.close()
    g = S.Problem.from_workload(W.rof(H=8, W=8), storage="bf16")
    with pytest.raises(S.SublabelError) as e:
        g.set_temporal(True)
    assert e.value.status == 2
    g.close()
    b = S.BatchProblem([W.rof(H=8, W=8), W.rof(H=8, W=16, seed=3)])
    with pytest.raises(S.SublabelError) as e:
        b.set_temporal(True)
    assert e.value.status == 2
    b.close()
