"""Parity at the full sizes of the benchmark workloads, in the launch configuration the
benchmark times (the automatic tiling), against the FP64 oracle. GPU only.

* truncated-quadratic denoising 256x256, L = 5, 10, 20: 200 iterations; certified bounds
  and nonconvex energy within 1e-5 relative, the read-out u within 1e-4 everywhere;
* the same image with the anisotropic TV (L = 20) and the phase-unwrapping workload
  (256x256, L = 8 on [0, 4 pi]): the same bounds, u within 1e-4 of the label range;
* sampled-cost stereo 384x288, 64 samples, L = 8: the workload's 1000 iterations;
  bounds within 1e-5 relative;
* the 64-instance batch: eight members after 30 batched iterations, bounds within 1e-5
  of max(|P|, |D|) (this early the dual bound can be a near-cancelling sum close to 0);
* the monitor on an identical full-size state: 1e-9 relative.
Tolerances as derived for the small cases (the per-step FP32 error does not depend on
the image size; PDHG is non-expansive, so the trajectories separate at most linearly in
the accumulated rounding).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_01383_amd as S  # noqa: E402


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-30)


@pytest.fixture(autouse=True)
def _threads(orc):
    orc.set_threads(16)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("L", [5, 10, 20])
def test_truncated_quadratic_full_size(orc, L):
    wl = W.truncated_quadratic(L=L)
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    print(f"tq 256x256 L={L}: tiling {g.get_tiling()}", flush=True)
    g.run(200)
    o.run(200)
    eg, eo = g.energy(), o.monitor()
    for kg, ko in (("primal_ub", "primal"), ("dual_lb", "dual"), ("e_nonconvex", "e_nc")):
        print(f"  {kg}: gpu {eg[kg]:.10g} oracle {eo[ko]:.10g} rel {_rel(eg[kg], eo[ko]):.2e}")
        assert _rel(eg[kg], eo[ko]) <= 1e-5
    _, ug = g.read_u()
    _, uo = o.read_u()
    err = np.abs(ug.cpu().numpy() - uo).max()
    print(f"  max |u_gpu - u_oracle| = {err:.2e}")
    assert err <= 1e-4


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kind", ["aniso_tq20", "phase"])
def test_widened_workloads_full_size(orc, kind):
    """The anisotropic TV on the 256x256, L = 20 benchmark image and the 256x256, L = 8
    phase-unwrapping workload: 200 iterations in the benchmark's launch configuration."""
    if kind == "phase":
        wl = W.phase_unwrapping()
    else:
        wl = W.truncated_quadratic(L=20)
        wl.tv = 1
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    print(f"{kind}: tiling {g.get_tiling()}", flush=True)
    g.run(200)
    o.run(200)
    eg, eo = g.energy(), o.monitor()
    for kg, ko in (("primal_ub", "primal"), ("dual_lb", "dual"), ("e_nonconvex", "e_nc")):
        print(f"  {kg}: gpu {eg[kg]:.10g} oracle {eo[ko]:.10g} rel {_rel(eg[kg], eo[ko]):.2e}")
        assert _rel(eg[kg], eo[ko]) <= 1e-5
    _, ug = g.read_u()
    _, uo = o.read_u()
    err = np.abs(ug.cpu().numpy() - uo).max()
    print(f"  max |u_gpu - u_oracle| = {err:.2e}")
    assert err <= 1e-4 * max(1.0, float(wl.gamma[-1] - wl.gamma[0]))


@pytest.mark.timeout(300)
def test_stereo_full_size(orc):
    wl = W.stereo()
    g = S.Problem.from_workload(wl)
    o = orc.Problem(wl)
    g.run(wl.iters)
    o.run(wl.iters)
    eg, eo = g.energy(), o.monitor()
    for kg, ko in (("primal_ub", "primal"), ("dual_lb", "dual")):
        print(f"  {kg}: gpu {eg[kg]:.10g} oracle {eo[ko]:.10g} rel {_rel(eg[kg], eo[ko]):.2e}")
        assert _rel(eg[kg], eo[ko]) <= 1e-5


@pytest.mark.timeout(300)
def test_batch_members_full_size(orc):
    wls = W.batch()
    b = S.BatchProblem(wls)
    b.run(30)
    for i in range(0, 64, 8):
        o = orc.Problem(wls[i])
        o.run(30)
        eg, eo = b.energy_of(i), o.monitor()
        # early on the dual bound is a near-cancelling sum (it can sit close to 0): errors
        # are measured on the scale of the certificate, max(|P|, |D|), as the gap is
        scale = max(abs(eo["primal"]), abs(eo["dual"]))
        dp = abs(eg["primal_ub"] - eo["primal"]) / scale
        dd = abs(eg["dual_lb"] - eo["dual"]) / scale
        print(f"member {i} {wls[i].H}x{wls[i].W} L={wls[i].L}: primal {dp:.2e} dual {dd:.2e}", flush=True)
        assert dp <= 1e-5 and dd <= 1e-5
    b.close()


@pytest.mark.timeout(300)
def test_monitor_full_size_identical_state(orc):
    wl = W.truncated_quadratic(L=20)
    g = S.Problem.from_workload(wl)
    g.run(500)
    t = g.save_state()
    torch.cuda.synchronize()
    st = S.unpack_state(t, g.k, g.H, g.W)
    o = orc.Problem(wl)
    o.set_state({n: a.astype(np.float64) for n, a in st.items()})
    eg, eo = g.energy(), o.monitor()
    for kg, ko in (("primal_ub", "primal"), ("dual_lb", "dual"), ("e_nonconvex", "e_nc")):
        assert _rel(eg[kg], eo[ko]) <= 1e-9, (kg, eg[kg], eo[ko])
