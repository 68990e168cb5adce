"""The allocation-free solve (sl_solve_static, for callers that cannot allocate) against
the handle-based calls it stands for (sl_create on a caller workspace, sl_run or
sl_run_to_gap, sl_read_u, sl_energy), called through the C-ABI on the same inputs: two
calls in a row on one GPU, the second on a smaller problem, so the second must not see the
first's state in the library's fixed array. The same kernels run on both paths, so the
results must agree bit for bit."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)


def _handle_solve(S, wl, rel_gap, max_iters, dev, adaptive, check_every):
    g = S.Problem.from_workload(wl, device=dev, adaptive=adaptive, check_every=check_every)
    if rel_gap > 0:
        g.run_to_gap(rel_gap, max_iters)
    else:
        g.run(max_iters)
    ul, u = g.read_u()
    rep = g.energy()
    g.close()
    return ul, u, rep


def test_static_solve_equals_handle_solve_twice_shrinking():
    import paper_1512_01383_amd as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cases = [
        # truncated quadratic on ragged tiles, fixed iteration count, no checks
        (W.truncated_quadratic(L=6, H=97, W=161, seed=31), 0.0, 150, False, 50),
        # smaller: ROF run to a certified gap with adaptive steps (monitor and residual
        # sums copied through the call's own host memory)
        (W.rof(H=40, W=51), 1e-3, 3000, True, 25),
    ]
    stream = torch.cuda.current_stream(dev)
    for wl, gap, iters, adaptive, every in cases:
        print(f"static solve: {wl.name} {wl.H}x{wl.W} L={wl.L} gap={gap} iters={iters}", flush=True)
        it = S._Inst()
        d = S._make_desc(it, wl.H, wl.W, wl.gamma, wl.rho, wl.lam, wl.f, wl.a, wl.nu, wl.tau,
                         wl.samples, "fp32", True, every, dev, adaptive)
        ul = torch.full((wl.k, wl.H, wl.W), float("nan"), dtype=torch.float32, device=dev)
        u = torch.full((wl.H, wl.W), float("nan"), dtype=torch.float32, device=dev)
        rep = S.Report()
        torch.cuda.synchronize()
        st = S.lib().sl_solve_static(C.byref(d), gap, iters, C.c_void_p(ul.data_ptr()),
                                     C.c_void_p(u.data_ptr()), C.byref(rep),
                                     C.c_void_p(stream.cuda_stream))
        assert st == 0, S.lib().sl_last_error().decode()
        ul_h, u_h, rep_h = _handle_solve(S, wl, gap, iters, dev, adaptive, every)
        assert torch.equal(ul, ul_h)
        assert torch.equal(u, u_h)
        r = rep.as_dict()
        for key in ("primal_ub", "dual_lb", "best_primal", "best_dual", "rel_gap", "e_nonconvex",
                    "iters"):
            assert r[key] == rep_h[key], (key, r[key], rep_h[key])
        if gap > 0:
            assert r["rel_gap"] <= gap
        assert np.isfinite(u.cpu().numpy()).all()
