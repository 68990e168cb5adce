"""Parity of the HIP path (through the C-ABI) with the FP64 oracle. GPU only.

Tolerances (FP32 arithmetic against FP64):
  * one iteration from a random state: |gpu - oracle| <= 2e-5 (1 + |oracle|) per entry
  * ROF 64x64, L = 2, 2000 iterations: max |u_gpu - u_oracle| <= 1e-4 and relative
    primal / dual bounds within 1e-5
  * fixed iteration counts on truncated-quadratic and sampled problems: relative bounds
    within 1e-5
  * the monitor on an identical state: relative 1e-9 (both evaluate in FP64 with the same
    double parameters; only the summation order differs)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _pair(wl, orc, storage="fp32", normalize=True):
    g = S.Problem.from_workload(wl, storage=storage, normalize=normalize)
    o = orc.Problem(wl, normalize=normalize)
    return g, o


def _load_same_state(g, o, st):
    g.load_state(S.pack_state(st))
    o.set_state({n: st[n].astype(np.float64) for n in st})


def _gpu_state(g):
    t = g.save_state()
    torch.cuda.synchronize()
    return S.unpack_state(t, g.k, g.H, g.W)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-30)


def _sampled_workload(H, Wd, seed, L=8, M=64, lam=0.5):
    rng = np.random.default_rng(seed)
    tau = np.arange(M, dtype=np.float64)
    idx = np.round(np.linspace(0, M - 1, L)).astype(int)
    gamma = tau[idx]
    base = rng.uniform(0, 1, size=(M, H, Wd))
    costs = np.abs(base - base[rng.integers(0, M)]).astype(np.float32)
    return W.Workload("smp", H, Wd, gamma, W.SAMPLED, lam, tau=tau, samples=costs)


def _cases():
    rng = np.random.default_rng(100)
    out = []
    # (name, workload) spanning several 64x4 tiles with ragged tails
    f = rng.uniform(-0.1, 1.1, size=(13, 150)).astype(np.float32)
    out.append(("quad_L2", W.Workload("q2", 13, 150, W.equispaced(2), W.QUAD, 0.2, f=f, a=1.0)))
    out.append(("quad_L6_offset", W.Workload("q6", 13, 150, np.array([-1.0, -0.4, 0.1, 0.9, 1.3, 2.0]),
                                             W.QUAD, 0.3, f=2 * f, a=3.0)))
    for L in (2, 5, 10, 20):
        wl = W.truncated_quadratic(L=L, H=9, W=131, seed=7 + L)
        out.append((f"tq_L{L}", wl))
    wl = W.truncated_quadratic(L=8, H=11, W=70, seed=5)
    wl.tau = wl.gamma.copy()
    wl.samples = rng.normal(0, 0.05, size=(8, 11, 70)).astype(np.float32)
    out.append(("tq_add_L8", wl))
    wq = W.Workload("qa", 7, 66, W.equispaced(4), W.QUAD, 0.2, f=f[:7, :66].copy(), a=1.0,
                    tau=W.equispaced(4), samples=rng.normal(0, 0.1, size=(4, 7, 66)).astype(np.float32))
    out.append(("quad_add_L4", wq))
    out.append(("sampled_L8", _sampled_workload(10, 97, 3)))
    out.append(("sampled_L4_M13", _sampled_workload(6, 65, 4, L=4, M=13)))
    # both documented maxima at once: 28 labels on 256 samples
    out.append(("sampled_max", _sampled_workload(5, 70, 21, L=28, M=256)))
    out.append(("one_pixel", W.Workload("px", 1, 1, W.equispaced(4), W.TRUNC_QUAD, 0.2,
                                        f=np.array([[0.3]], np.float32), a=2.0, nu=0.025)))
    out.append(("one_row", W.truncated_quadratic(L=6, H=1, W=200, seed=3)))
    out.append(("one_col", W.truncated_quadratic(L=6, H=77, W=1, seed=4)))
    out.append(("k27", W.truncated_quadratic(L=28, H=5, W=70, seed=9)))
    # widths that are whole tiles: the gathers beyond the right edge fall outside the image
    out.append(("w64", W.truncated_quadratic(L=5, H=6, W=64, seed=12)))
    out.append(("w128", W.truncated_quadratic(L=7, H=8, W=128, seed=13)))
    return out


CASES = _cases()


from tests.gpu_tilings import TILING_IDS, TILINGS, use_tiling  # noqa: E402


@pytest.mark.parametrize("tiling", TILINGS, ids=TILING_IDS)
@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_single_iteration_from_random_state(orc, name, wl, tiling):
    """One fused iteration from the same random state: every field of the new state, for
    every launch configuration of the fused kernel."""
    g, o = _pair(wl, orc, "fp32")
    if not use_tiling(g, tiling, wl.W, wl.k):
        return
    st = W.random_state(11, wl.k, wl.H, wl.W)
    _load_same_state(g, o, st)
    g.run(1)
    o.run(1)
    got = _gpu_state(g)
    ref = o.get_state()
    for n in S.STATE_ORDER:
        err = np.abs(got[n].astype(np.float64) - ref[n])
        bound = 2e-5 * (1.0 + np.abs(ref[n]))
        worst = np.unravel_index(np.argmax(err - bound), err.shape)
        assert np.all(err <= bound), f"{name}/{n}: err {err[worst]:.3e} at {worst}, ref {ref[n][worst]}"


MONITOR_CASES = CASES[:8] + [c for c in CASES if c[0] in ("sampled_L8", "sampled_L4_M13", "sampled_max", "k27")]


@pytest.mark.parametrize("name,wl", MONITOR_CASES, ids=[c[0] for c in MONITOR_CASES])
def test_monitor_on_identical_state(orc, name, wl):
    """The FP64 monitor of both sides on the same (FP32) state."""
    g, o = _pair(wl, orc)
    st = W.random_state(12, wl.k, wl.H, wl.W, scale=0.3)
    _load_same_state(g, o, st)
    eg = g.energy()
    eo = o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) < 1e-9
    assert _rel(eg["dual_lb"], eo["dual"]) < 1e-9
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) < 1e-9


# label counts at the monitor's chunk boundaries (a block covers 4, 2 or 1 groups of 64
# pixels for k <= 8, <= 16 and above), on sizes whose pixel count leaves the last block
# partly empty; truncated quadratics exercise the straddle pieces evaluated after the loops
CHUNK_CASES = [(f"tq_k{L - 1}_{H}x{Wd}", W.truncated_quadratic(L=L, H=H, W=Wd, seed=300 + L))
               for (L, H, Wd) in ((9, 7, 83), (10, 5, 131), (17, 9, 45), (18, 3, 101), (2, 1, 1), (28, 2, 70))]


@pytest.mark.parametrize("name,wl", CHUNK_CASES, ids=[c[0] for c in CHUNK_CASES])
def test_monitor_at_chunk_boundaries(orc, name, wl):
    g, o = _pair(wl, orc)
    st = W.random_state(13, wl.k, wl.H, wl.W, scale=0.3)
    _load_same_state(g, o, st)
    eg = g.energy()
    eo = o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) < 1e-9
    assert _rel(eg["dual_lb"], eo["dual"]) < 1e-9
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) < 1e-9
    g.close()


def test_rof_2000_iterations(orc):
    """ROF 64x64, L = 2, lambda = 0.2, 2000 iterations: max |du| <= 1e-4, energies 1e-5."""
    wl = W.rof()
    g, o = _pair(wl, orc)
    g.run(wl.iters)
    o.run(wl.iters)
    _, ug = g.read_u()
    _, uo = o.read_u()
    err = np.abs(ug.cpu().numpy().astype(np.float64) - uo).max()
    assert err <= 1e-4, err
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) <= 1e-5
    assert _rel(eg["dual_lb"], eo["dual"]) <= 1e-5
    assert eg["rel_gap"] < 1e-4


@pytest.mark.parametrize("L,iters", [(5, 400), (10, 300), (20, 200)])
def test_truncated_quadratic_fixed_iterations(orc, L, iters):
    wl = W.truncated_quadratic(L=L, H=40, W=72, seed=20 + L)
    g, o = _pair(wl, orc)
    g.run(iters)
    o.run(iters)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) <= 1e-5
    assert _rel(eg["dual_lb"], eo["dual"]) <= 1e-5
    assert _rel(eg["e_nonconvex"], eo["e_nc"]) <= 1e-5


def test_sampled_fixed_iterations(orc):
    wl = _sampled_workload(24, 90, 8)
    g, o = _pair(wl, orc)
    g.run(200)
    o.run(200)
    eg, eo = g.energy(), o.monitor()
    assert _rel(eg["primal_ub"], eo["primal"]) <= 1e-5
    assert _rel(eg["dual_lb"], eo["dual"]) <= 1e-5


def test_save_load_roundtrip_and_determinism(orc):
    wl = W.truncated_quadratic(L=6, H=30, W=100, seed=31)
    g1 = S.Problem.from_workload(wl)
    g1.run(37)
    st = g1.save_state().clone()
    g1.run(40)
    a = g1.save_state().clone()
    g2 = S.Problem.from_workload(wl)
    g2.load_state(st)
    g2.run(40)
    b = g2.save_state().clone()
    g3 = S.Problem.from_workload(wl)
    g3.run(77)
    c = g3.save_state().clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, c)
    e1, e3 = g1.energy(), g3.energy()
    assert e1["primal_ub"] == e3["primal_ub"] and e1["dual_lb"] == e3["dual_lb"]


def test_tilings_agree():
    """Tile height and pixels per lane do not change a single bit; the number of label
    groups changes only the FP32 rounding of the chunk partial sums."""
    wl = W.truncated_quadratic(L=11, H=37, W=130, seed=32)
    outs = {}
    for tl in TILINGS:
        g = S.Problem.from_workload(wl)
        g.set_tiling(*tl)
        assert g.get_tiling() == tl
        g.run(25)
        outs[tl] = g.save_state().clone()
    torch.cuda.synchronize()
    for tl in TILINGS:
        same = (tl[0], 4, 64)           # same label groups: bitwise equal
        assert torch.equal(outs[tl], outs[same]), tl
        d = (outs[tl] - outs[(1, 4, 64)]).abs()
        assert (d <= 1e-4 * (1 + outs[(1, 4, 64)].abs())).all(), (tl, d.max().item())


def test_invalid_arguments_gpu():
    f = np.zeros((3, 3), np.float32)
    with pytest.raises(S.SublabelError) as e:
        S.Problem(3, 3, [0.0, 0.0, 1.0], S.RHO_QUAD, 0.1, f=f)
    assert e.value.status == 1
    with pytest.raises(S.SublabelError) as e:
        S.Problem(3, 3, [0.0, 0.5, 1.0], S.RHO_QUAD, 0.1, f=np.full((3, 3), np.nan, np.float32))
    assert e.value.status == 1
    with pytest.raises(S.SublabelError) as e:
        S.Problem(0, 3, [0.0, 1.0], S.RHO_QUAD, 0.1, f=f)
    assert e.value.status == 1
    with pytest.raises(S.SublabelError) as e:
        S.Problem(3, 3, W.equispaced(40), S.RHO_QUAD, 0.1, f=f)
    assert e.value.status == 2
    with pytest.raises(S.SublabelError) as e:   # H*W = 2^29: a plane would reach 2 GiB
        S.Problem(1 << 15, 1 << 14, [0.0, 1.0], S.RHO_QUAD, 0.1)
    assert e.value.status == 2 and "2^29" in str(e.value)


def _bf16_round(a):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("name,wl", [CASES[0], CASES[4], CASES[7], CASES[8]],
                         ids=[CASES[i][0] for i in (0, 4, 7, 8)])
def test_bf16_single_iteration(orc, name, wl):
    """BF16 storage of v, z, p: from a state already representable in BF16, one
    iteration matches the oracle to FP32 accuracy in u, s, q and to BF16 rounding
    (2^-8 relative) in the stored duals."""
    g = S.Problem.from_workload(wl, storage="bf16")
    o = orc.Problem(wl)
    st = W.random_state(13, wl.k, wl.H, wl.W)
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


def test_bf16_energy_error_at_convergence(orc):
    """ROF 64x64 against the FP64 oracle. FP32 storage: 3000 iterations reach the optimum
    within 1e-5 relative. BF16 dual storage alone stalls at a rounding floor (a stored dual
    carries a relative error of up to 2^-9; measured on this problem: primal 1.17e-3 above
    the optimum, flat from 1000 to 24000 iterations), so the gap-controlled solve finishes
    in float: once the best gap stops improving, the duals are widened in place and the
    solve continues to the 1e-3 certified gap, which bounds the energy error by 1e-3. The
    errors and the iterations of each phase are printed per result."""
    wl = W.rof()
    o = orc.Problem(wl)
    o.run(6000)
    ro = o.monitor()
    g = S.Problem.from_workload(wl, storage="fp32")
    g.run(3000)
    e = g.energy()
    err_p, err_d = _rel(e["best_primal"], ro["best_primal"]), _rel(e["best_dual"], ro["best_dual"])
    print(f"fp32 3000 its: primal {err_p:.2e} dual {err_d:.2e} vs FP64 oracle (6000 its)")
    assert err_p < 1e-5 and err_d < 1e-5
    g = S.Problem.from_workload(wl, storage="bf16")
    done = g.run_to_gap(1e-3, 20000)
    e = g.energy()
    storage, n16 = g.storage_info()
    err_p, err_d = _rel(e["best_primal"], ro["best_primal"]), _rel(e["best_dual"], ro["best_dual"])
    print(f"bf16 + finishing: {done} its ({n16} with bf16 duals, now {storage}); rel gap "
          f"{e['rel_gap']:.2e}; vs FP64 oracle primal {err_p:.2e} dual {err_d:.2e}")
    assert e["rel_gap"] <= 1e-3
    assert err_p <= 1e-3 and err_d <= 1e-3
    assert 0 < n16 <= done
    # certified bounds stay bounds of the FP64 optimum (up to the FP64 oracle's gap)
    assert e["best_dual"] <= ro["best_primal"] * (1 + 1e-6)
    assert e["best_primal"] >= ro["best_dual"] * (1 - 1e-6)
