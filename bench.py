"""Benchmark of the lifted primal-dual iteration on one MI355X.

Workload (default, --workload batch): 64 truncated-quadratic instances of mixed size
(U{64,128,256,512}^2) and label count (U{2,4,8,16}), lambda = 0.25, solved together by one
launch per iteration with the duals stored in bf16 (FP32 arithmetic, FP64
certificate). One step is one check interval of the gap-controlled batch solve: 48 batched
iterations followed by every member's FP64 certified-gap monitor and step balance, with
inputs and state resident in HBM.

Reported: pixel-label-iterations/s (k = L-1 labels counted per pixel), the HIP-event
average duration of the batched iteration kernel against its algorithmic bytes (roofline),
the time for every member to reach a 1e-3 certified relative gap (bf16 with the float
finishing phase, against the members solved one after another and the batch in float),
the FP64 CPU oracle timed on a bounded sample of the same members (baseline, not the
target), and single-instance kernel timings (256^2 cache-resident, 2048^2 in HBM).
Other workloads: tq (one truncated-quadratic instance), stereo, phase, diff, labels.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CHECK_EVERY = 50
CHECK_BATCH = 48      # check interval of batched solves (a multiple of the 6-iteration period)
KERNEL_SOURCES = ("paper_1512_01383_amd/csrc/pdhg_iter.hip", "paper_1512_01383_amd/csrc/device_math.hpp",
                  "paper_1512_01383_amd/csrc/internal.hpp")


def kernel_hash() -> str:
    """Hash of the code of the fused iteration kernel (ties counter data to a kernel):
    the sources with // comments and blank space removed, so comment edits keep it."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str, kernel: str = "pdhg_iter", tiling=None):
    """HBM bytes per launch from the committed counter profile of this workload, if it
    was taken on the current kernel sources and, when given, the same tiling (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_key}_traffic.json")
    try:
        with open(path) as f:
            prof = json.load(f)
    except OSError:
        return None
    if prof.get("kernel_hash") != kernel_hash():
        return None
    if tiling is not None and prof.get("tiling") is not None and list(prof["tiling"]) != list(tiling):
        return None
    return prof.get("hbm_bytes_per_launch")


def algorithmic_bytes_per_pixel(k: int, rho: int, M: int, bf16: bool, add: bool) -> int:
    """Bytes one fused iteration must move per pixel: read u, u_prev, s, s_prev, v, z,
    p (2 per label), q and the data plane(s); write u, s, v, z, p, q."""
    dual = 2 if bf16 else 4
    per_label = 4 * 6 + dual * 8          # u,u_prev,u_new,s,s_prev,s_new ; v,z,px,py r+w
    data = 4 * (M if rho == 2 else 1) + (4 * (k + 1) if add else 0)
    return k * per_label + 8 + data       # + q read and write


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--storage", default=None, choices=["fp32", "bf16"],
                    help="dual storage (default: bf16 for the batch, fp32 otherwise)")
    ap.add_argument("--tv", default="iso", choices=["iso", "aniso"],
                    help="regulariser: isotropic (l2) or anisotropic (l1) total variation")
    ap.add_argument("--kernel-iters", type=int, default=500)
    ap.add_argument("--gap-max-iters", type=int, default=60000)
    ap.add_argument("--no-gap", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--workload", default="batch",
                    choices=["tq", "stereo", "phase", "batch", "diff", "labels", "cpu", "temporal"],
                    help="batch: 64 mixed instances in one launch per iteration "
                         "(default); tq: one truncated-quadratic instance; diff: forward and "
                         "backward of 200 unrolled iterations (256x256, L=8)")
    ap.add_argument("--study", default="tq", choices=["tq", "phase", "stereo", "norm"],
                    help="data of the label-count study: truncated quadratic or phase unwrapping")
    ap.add_argument("--batch-iters", type=int, default=240)
    ap.add_argument("--tiling", default=None,
                    help="batch tiling 'groups,rows,cols' instead of the autotuned one (counter runs, "
                         "whose serialised dispatches skew the autotuner's timings)")
    ap.add_argument("--no-extra", action="store_true",
                    help="batch mode: skip the single-instance kernel timings")
    args = ap.parse_args()
    if args.storage is None:
        args.storage = "bf16" if args.workload == "batch" else "fp32"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the iteration would shard by image strips with one-row halos).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "diff":
        return bench_diff(args)
    if args.workload == "labels":
        return bench_labels(args)
    if args.workload == "cpu":
        return bench_cpu(args)
    if args.workload == "temporal":
        return bench_temporal(args)

    if args.workload == "stereo":
        wl = W.stereo()            # sampled costs, 384x288, 64 disparities, L = 8
    elif args.workload == "phase":
        wl = W.phase_unwrapping(H=args.size, W=args.size)   # periodic quadratic, L = 8
    else:
        wl = W.truncated_quadratic(L=args.L, H=args.size, W=args.size)
    wl.tv = 1 if args.tv == "aniso" else 0
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = S.Problem.from_workload(wl, storage=args.storage, check_every=CHECK_EVERY, device=dev,
                                adaptive=False)
    stream = g.stream
    k, N = wl.k, wl.H * wl.W

    def step():
        # one check interval of the library's own solve loop: CHECK_EVERY fused iterations,
        # the FP64 monitor and its result on the host (rel_gap 0 is never met early)
        g.run_to_gap(0.0, CHECK_EVERY)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = N * k * CHECK_EVERY * args.steps / dt

    # dominant kernel: HIP events around a run of fused iterations on the library's stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    g.run(20)
    ev0.record(stream)
    g.run(args.kernel_iters)
    ev1.record(stream)
    ev1.synchronize()
    kern_ms = ev0.elapsed_time(ev1) / args.kernel_iters
    bpp = algorithmic_bytes_per_pixel(k, wl.rho, wl.M, args.storage == "bf16", False)
    bytes_per_launch = bpp * N
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9

    # stereo: the matching-cost builder (Sec. 5.4 costs) on the same pair, timed alone
    cost_build = None
    if args.workload == "stereo":
        D = wl.M
        left_d = torch.as_tensor(wl.pair[0], device=dev)
        right_d = torch.as_tensor(wl.pair[1], device=dev)
        vol = torch.empty((D, wl.H, wl.W), dtype=torch.float32, device=dev)
        cur = torch.cuda.current_stream(dev)
        S.stereo_costs(left_d, right_d, D, 1.0, out=vol)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(cur)
        for _ in range(50):
            S.stereo_costs(left_d, right_d, D, 1.0, out=vol)
        c1.record(cur)
        c1.synchronize()
        cms = c0.elapsed_time(c1) / 50
        cbytes = 4 * N * (D + 2)            # write the volume once, read both images once
        cost_build = {"kernel": "k_stereo_costs", "kernel_ms": cms, "disparities": D,
                      "algorithmic_bytes_per_launch": cbytes,
                      "achieved_GBs": cbytes / (cms * 1e-3) / 1e9,
                      "frac": cbytes / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # time to a 1e-3 certified relative gap from a fresh start: adaptive step balance
    # (residual balancing at every check) and, for reference, the fixed default steps
    gap = None
    if not args.no_gap:
        gap = {}
        for mode in ("adaptive", "fixed"):
            g2 = S.Problem.from_workload(wl, storage=args.storage, check_every=CHECK_EVERY,
                                         device=dev, adaptive=(mode == "adaptive"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = g2.run_to_gap(1e-3, args.gap_max_iters)
            t_gap = time.perf_counter() - t0
            rep = g2.energy()
            gap[mode] = {"seconds": t_gap, "iterations": done, "rel_gap": rep["rel_gap"],
                         "reached": rep["rel_gap"] <= 1e-3, "primal_ub": rep["best_primal"],
                         "dual_lb": rep["best_dual"], "e_nonconvex": rep["e_nonconvex"],
                         "step_balance": g2.get_step_balance()}
            if args.workload == "phase":
                # unwrapping quality against the generating phase (host-side evaluation)
                _, ug = g2.read_u()
                err = ug.cpu().numpy().astype(np.float64) - wl.target.astype(np.float64)
                gap[mode]["unwrap_rmse"] = float(np.sqrt(np.mean(err ** 2)))
                gap[mode]["unwrap_branch_correct"] = float(np.mean(np.abs(err) < np.pi))
            g2.close()

    cpu = None
    if not args.no_cpu:
        import oracle
        ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        ncores = oracle.set_threads(ncores)
        o = oracle.Problem(wl)
        o.run(2)
        t0 = time.perf_counter()
        o.run(5)
        per_it = (time.perf_counter() - t0) / 5
        n_it = max(5, int(args.cpu_seconds / max(per_it, 1e-6)))
        t0 = time.perf_counter()
        o.run(n_it)
        dt_cpu = time.perf_counter() - t0
        # the same on one thread, over a shorter sample
        oracle.set_threads(1)
        t0 = time.perf_counter()
        o.run(2)
        per1 = (time.perf_counter() - t0) / 2
        n1 = max(2, int(args.cpu_seconds / 3 / max(per1, 1e-6)))
        t0 = time.perf_counter()
        o.run(n1)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(ncores)
        cpu = {"value": N * k * n_it / dt_cpu, "unit": "pixel-label-iter/s", "cores": ncores,
               "kind": "oracle",
               "sample": f"{n_it} FP64 iterations of the same {wl.H}x{wl.W} L={wl.L} problem "
                         f"({dt_cpu:.1f} s, monitor excluded)",
               "value_1_thread": N * k * n1 / dt1,
               "sample_1_thread": f"{n1} iterations ({dt1:.1f} s)"}

    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": value,
        "unit": "pixel-label-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "f32 (bf16 dual storage)",
        "data": "synthetic",
        "config": {"workload": (f"sampled-cost stereo {wl.W}x{wl.H}, {wl.M} disparity samples, "
                                f"L={wl.L}, lambda={wl.lam}" if args.workload == "stereo" else
                                f"phase unwrapping {wl.H}x{wl.W}, periodic quadratic pieces on "
                                f"[0, 4 pi], L={wl.L}, lambda={wl.lam}" if args.workload == "phase" else
                                f"truncated-quadratic denoising {wl.H}x{wl.W}, L={wl.L}, "
                                f"lambda={wl.lam}, nu=0.025") +
                               (", anisotropic TV" if wl.tv else "") +
                               f"; step = {CHECK_EVERY} fused iterations + FP64 gap monitor",
                   "H": wl.H, "W": wl.W, "L": wl.L, "storage": args.storage, "tv": args.tv},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(f"tq{wl.H}_L{wl.L}_{args.storage}" + ("_aniso" if wl.tv else ""),
                                                  tiling=g.get_tiling())
                                 if args.workload == "tq" else
                                 measured_traffic(f"stereo{wl.W}x{wl.H}_L{wl.L}_{args.storage}", tiling=g.get_tiling())
                                 if args.workload == "stereo" else None),
                     "kernel": "pdhg_iter_kernel", "kernel_ms": kern_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "kernel_hash": kernel_hash(), "tiling": list(g.get_tiling())},
        "cpu_baseline": cpu,
        "time_to_gap_1e-3": gap,
    }
    if cost_build is not None:
        out["stereo_cost_build"] = cost_build
    print(json.dumps(out))


def bench_labels(args):
    """Label-count study of Sec. 5 on the synthetic truncated-quadratic image: the proposed
    relaxation (per-interval convex envelopes of the data term) against the baseline
    lifting (the data term known only at the labels, the special case of Prop. 2), each
    solved from zero to a 1e-3 certified gap, with fixed and with adaptive steps. The
    quality measure is the energy (eq. 1) of the back-projected u with the true truncated
    quadratic, evaluated on the host after the solve."""
    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.study == "stereo":
        return bench_labels_stereo(args, dev)
    if args.study == "norm":
        return bench_label_normalisation(args, dev)
    rows = []
    pli = 0.0
    gpu_s = 0.0
    phase = args.study == "phase"
    for L in ((2, 4, 8, 16) if phase else (2, 4, 8, 16, 28)):
        tq = (W.phase_unwrapping(L=L, H=args.size, W=args.size) if phase else
              W.truncated_quadratic(L=L, H=args.size, W=args.size))
        f = tq.f.astype(np.float64)
        for method, wl in (("proposed", tq), ("baseline", W.baseline_lifting(tq))):
            for adaptive in (False, True):
                g = S.Problem.from_workload(wl, check_every=CHECK_EVERY, device=dev,
                                            adaptive=adaptive)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                done = g.run_to_gap(1e-3, args.gap_max_iters)
                dt = time.perf_counter() - t0
                rep = g.energy()
                _, u = g.read_u()
                u = u.cpu().numpy().astype(np.float64)
                gx = np.zeros_like(u)
                gy = np.zeros_like(u)
                gx[:, :-1] = np.diff(u, axis=1)
                gy[:-1, :] = np.diff(u, axis=0)
                if phase:
                    dist = np.abs(np.mod(u - f + np.pi, 2 * np.pi) - np.pi)
                    data = 0.5 * tq.a * dist ** 2
                else:
                    data = np.minimum(0.5 * tq.a * (u - f) ** 2, tq.nu)
                e_true = float(data.sum() + tq.lam * np.sqrt(gx * gx + gy * gy).sum())
                rows.append({"L": L, "method": method, "steps": "adaptive" if adaptive else "fixed",
                             "iterations": done, "seconds": dt, "rel_gap": rep["rel_gap"],
                             "reached": rep["rel_gap"] <= 1e-3,
                             "relaxed_lower_bound": rep["best_dual"],
                             "energy_true_rho": e_true})
                if phase:
                    err = u - tq.target.astype(np.float64)
                    rows[-1]["unwrap_rmse"] = float(np.sqrt(np.mean(err ** 2)))
                    rows[-1]["unwrap_branch_correct"] = float(np.mean(np.abs(err) < np.pi))
                pli += float(wl.H * wl.W * wl.k) * done
                gpu_s += dt
                g.close()
    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": pli / gpu_s,
        "unit": "pixel-label-iter/s",
        "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": gpu_s / len(rows) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"label-count study, phase unwrapping {args.size}x{args.size}, "
                                f"lambda=0.005, L in 2,4,8,16" if phase else
                                f"label-count study, truncated-quadratic denoising {args.size}x"
                                f"{args.size}, lambda=0.25, nu=0.025, L in 2,4,8,16,28") +
                               "; proposed relaxation vs baseline lifting, each solve to a 1e-3 gap",
                   "step": "one solve to the gap"},
        "labels_study": rows,
    }
    print(json.dumps(out))


def bench_labels_stereo(args, dev):
    """Label-count study on the synthetic stereo pair (Sec. 5.4): the cost volume of the
    paper's matching cost (truncated sum of absolute gradient differences over 4x4
    patches, truncation 1) is built on the GPU for 64 disparities; the proposed relaxation
    uses all 64 samples (per-interval envelopes), the baseline lifting only the samples at
    its labels. Fixed steps (adaptive steps do not suit sampled costs), at most 20 000
    iterations. Measures: disparity error against the generating disparity map, and the
    energy with the full volume (linear between disparities), both on the host."""
    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    base = W.stereo()
    H, Wd, D = base.H, base.W, 64
    vol = S.stereo_costs(base.pair[0], base.pair[1], D, 1.0, device=dev)
    vol_h = vol.cpu().numpy().astype(np.float64)
    tau = np.arange(D, dtype=np.float64)
    truth = base.target.astype(np.float64)
    rows = []
    pli = 0.0
    gpu_s = 0.0
    for lam in (0.5, 0.05):
        for L in (2, 4, 8):
            idx = np.round(np.linspace(0, D - 1, L)).astype(np.int64)
            gamma = tau[idx]
            for method in ("proposed", "baseline"):
                if method == "proposed":
                    g = S.Problem(H, Wd, gamma, S.RHO_SAMPLED, lam, tau=tau, samples=vol,
                                  check_every=CHECK_EVERY, device=dev)
                else:
                    sel = vol[torch.as_tensor(idx, device=dev)].contiguous()
                    g = S.Problem(H, Wd, gamma, S.RHO_SAMPLED, lam, tau=gamma.copy(), samples=sel,
                                  check_every=CHECK_EVERY, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                done = g.run_to_gap(1e-3, 20000)
                dt = time.perf_counter() - t0
                rep = g.energy()
                _, u = g.read_u()
                u = u.cpu().numpy().astype(np.float64)
                lo = np.clip(np.floor(u).astype(np.int64), 0, D - 2)
                a = u - lo
                rr, cc = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
                data = (1 - a) * vol_h[lo, rr, cc] + a * vol_h[lo + 1, rr, cc]
                gx = np.zeros_like(u)
                gy = np.zeros_like(u)
                gx[:, :-1] = np.diff(u, axis=1)
                gy[:-1, :] = np.diff(u, axis=0)
                err = np.abs(u - truth)
                rows.append({"lambda": lam, "L": L, "method": method, "iterations": done,
                             "seconds": dt, "rel_gap": rep["rel_gap"],
                             "energy_full_volume": float(data.sum() + lam * np.sqrt(gx * gx + gy * gy).sum()),
                             "disparity_mae": float(err.mean()),
                             "within_1": float((err <= 1.0).mean()),
                             "within_3": float((err <= 3.0).mean())})
                pli += float(H * Wd * (L - 1)) * done
                gpu_s += dt
                g.close()
    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": pli / gpu_s,
        "unit": "pixel-label-iter/s",
        "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": gpu_s / len(rows) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"label-count study, stereo {Wd}x{H}, 64 disparities, gradient "
                               f"costs built on the GPU, L in 2,4,8, lambda in 0.5,0.05; proposed "
                               f"relaxation vs baseline lifting, fixed steps",
                   "step": "one solve to the gap or 20000 iterations"},
        "labels_study": rows,
    }
    print(json.dumps(out))


def bench_label_normalisation(args, dev):
    """Label-normalisation study: the operator of the split problem contains |gamma_i|,
    so the diagonal preconditioning depends on where the labels lie; mapping them onto
    [0, 1] is an exact reparametrisation. Iterations to a 1e-3 certified gap (at most
    30 000) with and without it, fixed and adaptive steps, on three label ranges: the
    truncated-quadratic image moved to [5, 6] (L = 10), phase unwrapping on [0, 4 pi]
    (L = 8), absolute-difference stereo on [0, 63] (L = 8)."""
    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    tq = W.truncated_quadratic(L=10, H=args.size, W=args.size)
    tq.gamma = tq.gamma + 5.0
    tq.f = (tq.f + 5.0).astype(np.float32)
    cases = [("truncated quadratic on [5, 6]", tq),
             ("phase unwrapping on [0, 4 pi]", W.phase_unwrapping(H=args.size, W=args.size)),
             ("stereo on [0, 63]", W.stereo())]
    rows = []
    pli = 0.0
    gpu_s = 0.0
    for name, wl in cases:
        for normalize in (True, False):
            for adaptive in (False, True):
                g = S.Problem.from_workload(wl, check_every=CHECK_EVERY, device=dev,
                                            normalize=normalize, adaptive=adaptive)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                done = g.run_to_gap(1e-3, 30000)
                dt = time.perf_counter() - t0
                rep = g.energy()
                rows.append({"case": name, "normalize": normalize,
                             "steps": "adaptive" if adaptive else "fixed", "iterations": done,
                             "seconds": dt, "rel_gap": rep["rel_gap"],
                             "reached": rep["rel_gap"] <= 1e-3,
                             "best_primal": rep["best_primal"], "best_dual": rep["best_dual"]})
                pli += float(wl.H * wl.W * wl.k) * done
                gpu_s += dt
                g.close()
    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": pli / gpu_s,
        "unit": "pixel-label-iter/s",
        "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": gpu_s / len(rows) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "label-normalisation study: truncated quadratic on [5, 6], phase "
                               "unwrapping on [0, 4 pi], stereo on [0, 63]; with and without "
                               "mapping the labels onto [0, 1], fixed and adaptive steps",
                   "step": "one solve to a 1e-3 gap or 30000 iterations"},
        "normalisation_study": rows,
    }
    print(json.dumps(out))


def cpu_model() -> str:
    """The host CPU's model name (Linux), for the CPU baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_cores() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def single_kernel_timing(S, wl, storage, dev, iters=200):
    """HIP-event average duration of the fused iteration kernel of one instance (the
    library's stream, after a short warm-up) against its algorithmic bytes."""
    import torch
    g = S.Problem.from_workload(wl, storage=storage, device=dev)
    g.run(20)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(g.stream)
    g.run(iters)
    ev1.record(g.stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1) / iters
    tiling = g.get_tiling()
    g.close()
    nbytes = algorithmic_bytes_per_pixel(wl.k, wl.rho, wl.M, storage == "bf16", False) * wl.H * wl.W
    return {"H": wl.H, "W": wl.W, "L": wl.L, "storage": storage, "kernel_ms": ms,
            "pixel_label_iter_per_s": wl.H * wl.W * wl.k / (ms * 1e-3),
            "algorithmic_bytes_per_launch": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
            "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "tiling": list(tiling)}


def bench_batch(args):
    """Batched, mixed-precision solve: 64 truncated-quadratic instances of mixed size
    (U{64,128,256,512}^2) and label count (U{2,4,8,16}) advanced together by one
    launch per iteration (graph-replayed rotation period, autotuned tiling), duals stored in
    bf16 (FP32 arithmetic, FP64 certificate). One step is one check interval of the
    gap-controlled batch solve: CHECK_BATCH batched iterations, every member's FP64 monitor
    and its adaptive step balance. Also: the time for every member to reach a 1e-3
    certified gap (bf16 with the float finishing phase), against the same members solved
    one after another and against the batch in float; the FP64 CPU oracle on the same
    members (bounded sample)."""
    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    wls = W.batch()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    storage = args.storage
    pli_it = sum(w.H * w.W * w.k for w in wls)

    b = S.BatchProblem(wls, storage=storage, device=dev, adaptive=True, check_every=CHECK_BATCH)
    if args.tiling:
        tiling = tuple(int(x) for x in args.tiling.split(","))
        b.set_tiling(*tiling)
    else:
        tiling = b.autotune(iters=12)
    b.set_finishing(0, widen_gap=0.0)   # no widening: the throughput steps stay in the requested storage
    stream = b.stream

    def step():
        b.run_to_gap(0.0, CHECK_BATCH)   # rel_gap 0 is never met: no member retires

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = pli_it * CHECK_BATCH * args.steps / dt

    # dominant kernel: HIP events on the batch's stream around graph-replayed iterations
    n_k = (args.batch_iters + 5) // 6 * 6
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.run(n_k)
    ev1.record(stream)
    ev1.synchronize()
    kern_ms = ev0.elapsed_time(ev1) / n_k
    bytes_launch = sum(algorithmic_bytes_per_pixel(w.k, w.rho, w.M, storage == "bf16", False) * w.H * w.W
                       for w in wls)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    b.close()

    # the same iterations, one instance after another (single-instance path, same storage)
    t_seq = 0.0
    for w in wls:
        g = S.Problem.from_workload(w, storage=storage, device=dev)
        g.run(12)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.run(n_k)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t1
        g.close()

    gap = None
    if not args.no_gap:
        gap = {"tol": 1e-3, "max_iters": args.gap_max_iters}
        for mode in ("batch_" + storage, "batch_fp32") if storage == "bf16" else ("batch_fp32",):
            st = "bf16" if mode == "batch_bf16" else "fp32"
            b = S.BatchProblem(wls, storage=st, device=dev, adaptive=True, check_every=CHECK_BATCH)
            b.set_tiling(*tiling)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            done = b.run_to_gap(1e-3, args.gap_max_iters)
            t_b = time.perf_counter() - t1
            reached, worst, pli16, pli32 = 0, 0.0, 0, 0
            for i, w in enumerate(wls):
                n_i, active = b.info_of(i)
                _, n16 = b.storage_info(i)
                rep = b.energy_of(i)
                reached += (not active) and rep["rel_gap"] <= 1e-3
                worst = max(worst, rep["rel_gap"])
                pli16 += w.H * w.W * w.k * n16
                pli32 += w.H * w.W * w.k * (n_i - n16)
            b.close()
            gap[mode] = {"seconds": t_b, "batched_iterations": done, "members_reached": int(reached),
                         "worst_rel_gap": worst,
                         "pixel_label_iters_bf16": pli16, "pixel_label_iters_fp32": pli32}
        t_s, reached_s = 0.0, 0
        for w in wls:
            g = S.Problem.from_workload(w, storage=storage, device=dev, adaptive=True,
                                        check_every=CHECK_BATCH)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g.run_to_gap(1e-3, args.gap_max_iters)
            t_s += time.perf_counter() - t1
            reached_s += g.energy()["rel_gap"] <= 1e-3
            g.close()
        gap["sequential_" + storage] = {"seconds": t_s, "members_reached": int(reached_s)}

    cpu = None
    if not args.no_cpu:
        import oracle
        ncores = oracle.set_threads(host_cores())

        def oracle_pass(n_it, budget=None):
            """n_it FP64 iterations of each member (one more before the clock starts, so
            first touches of the state are not timed); stops after `budget` seconds."""
            pli, total, members = 0, 0.0, 0
            for w in wls:
                o = oracle.Problem(w)
                o.run(1)
                t1 = time.perf_counter()
                o.run(n_it)
                total += time.perf_counter() - t1
                pli += w.H * w.W * w.k * n_it
                members += 1
                del o
                if budget is not None and total >= budget:
                    break
            return pli, total, members

        # one iteration of the largest member sets the sample size
        big_m = max(wls, key=lambda w: w.H * w.W * w.k)
        o = oracle.Problem(big_m)
        o.run(1)
        t1 = time.perf_counter()
        o.run(1)
        rate_est = big_m.H * big_m.W * big_m.k / max(time.perf_counter() - t1, 1e-6)
        del o
        n_it = max(1, int(args.cpu_seconds * rate_est / pli_it))
        pli_c, dt_cpu, _ = oracle_pass(n_it)
        oracle.set_threads(1)
        pli_1, dt1, m1 = oracle_pass(1, budget=args.cpu_seconds / 3)
        oracle.set_threads(ncores)
        cpu = {"value": pli_c / dt_cpu, "unit": "pixel-label-iter/s", "cores": ncores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{n_it} FP64 iterations of each of the 64 instances ({dt_cpu:.1f} s; "
                         f"problems built and first touched outside the clock)",
               "value_1_thread": pli_1 / dt1,
               "sample_1_thread": f"1 iteration of each of the first {m1} instances ({dt1:.1f} s)"}

    if args.calibrate_copy:
        # a plain 256 MiB device-to-device copy: the counters' reading for known bytes
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c

    extra = None
    if not args.no_extra:
        big = W.roofline()
        extra = {"tq256_L20_cache_resident": single_kernel_timing(
                     S, W.truncated_quadratic(L=20, H=256, W=256), "fp32", dev),
                 "tq2048_L16_fp32": single_kernel_timing(S, big, "fp32", dev),
                 "tq2048_L16_bf16": single_kernel_timing(S, big, "bf16", dev)}

    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": value,
        "unit": "pixel-label-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == "fp32" else "f32 (bf16 dual storage)",
        "data": "synthetic",
        "config": {"workload": "batched mixed precision: 64 truncated-quadratic instances, sizes "
                               "U{64,128,256,512}^2, L U{2,4,8,16}, lambda=0.25, nu=0.025, in one "
                               f"launch per iteration; step = {CHECK_BATCH} batched "
                               "iterations + every member's FP64 gap monitor and step balance",
                   "instances": len(wls), "pixel_label_per_iter": pli_it, "storage": storage,
                   "tiling": list(tiling)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"batch64_{storage}", kernel="pdhg_batch", tiling=tiling),
                     "kernel": "pdhg_batch_kernel", "kernel_ms": kern_ms,
                     "algorithmic_bytes_per_launch": bytes_launch, "kernel_hash": kernel_hash()},
        "cpu_baseline": cpu,
        "batch": {"seconds": dt, "iterations_timed_for_kernel": n_k,
                  "kernel_seconds_batched": kern_ms * n_k * 1e-3, "sequential_seconds": t_seq,
                  "speedup_vs_sequential": t_seq / (kern_ms * n_k * 1e-3)},
        "time_to_gap_1e-3": gap,
        "single_instance": extra,
    }
    print(json.dumps(out))


def bench_cpu(args):
    """CPU baselines of the other workloads beside the GPU (the FP64 oracle on the host's
    cores, and on one thread; a baseline, not a target): ROF 64^2 L=2 for its 2000
    iterations, the sampled-cost stereo problem for its 1000 iterations (timed on a bounded
    sample), the differentiation workload (K = 200 forward and reverse), and the paper-style
    relative energy error (E - E*)/E* of the GPU solve at a 1e-3 certified gap on ROF, with
    E* the midpoint of the oracle's certified interval after up to 100 000 FP64 iterations
    (its relative width is reported; below 1e-7)."""
    import numpy as np
    import torch

    import oracle
    import paper_1512_01383_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ncores = oracle.set_threads(host_cores())
    rows = {}

    def gpu_iters(wl, n):
        g = S.Problem.from_workload(wl, device=dev)
        g.run(5)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(g.stream)
        g.run(n)
        ev1.record(g.stream)
        ev1.synchronize()
        g.close()
        return ev0.elapsed_time(ev1) * 1e-3

    def cpu_iters(wl, n, threads):
        oracle.set_threads(threads)
        o = oracle.Problem(wl)
        o.run(1)
        t0 = time.perf_counter()
        o.run(n)
        dt = time.perf_counter() - t0
        oracle.set_threads(ncores)
        return dt

    # ROF: the 2000 iterations, and the paper-style error at a 1e-3 certified gap
    rof = W.rof()
    pl = rof.H * rof.W * rof.k
    t_g = gpu_iters(rof, 2000)
    t_c = cpu_iters(rof, 2000, ncores)
    t_1 = cpu_iters(rof, 2000, 1)
    o = oracle.Problem(rof)
    rep_o = oracle.run_to_gap(o, 1e-9, 100000, check_every=500)   # E* known to its certified gap
    e_star = 0.5 * (rep_o["best_primal"] + rep_o["best_dual"])
    g = S.Problem.from_workload(rof, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_gap = g.run_to_gap(1e-3, 60000)
    t_gap = time.perf_counter() - t0
    e = g.energy()
    g.close()
    rows["rof64_L2_2000its"] = {
        "gpu_seconds": t_g, "gpu_pli_per_s": pl * 2000 / t_g,
        "cpu_seconds": t_c, "cpu_pli_per_s": pl * 2000 / t_c, "cpu_1thread_seconds": t_1,
        "e_star": e_star, "e_star_rel_gap": rep_o["rel_gap"], "e_star_iterations": rep_o["iters"],
        "gpu_to_1e-3": {"iterations": n_gap, "seconds": t_gap, "rel_gap": e["rel_gap"],
                        "primal_rel_error": (e["best_primal"] - e_star) / e_star,
                        "e_nonconvex_rel_error": (e["e_nonconvex"] - e_star) / e_star}}

    # stereo: 1000 iterations on the GPU; the oracle on a bounded sample
    st = W.stereo()
    pl = st.H * st.W * st.k
    t_g = gpu_iters(st, 1000)
    n_c = 60
    t_c = cpu_iters(st, n_c, ncores)
    t_1 = cpu_iters(st, 6, 1)
    rows["stereo384x288_L8_1000its"] = {
        "gpu_seconds": t_g, "gpu_pli_per_s": pl * 1000 / t_g,
        "cpu_pli_per_s": pl * n_c / t_c, "cpu_seconds_est_1000its": t_c / n_c * 1000,
        "cpu_sample": f"{n_c} iterations ({t_c:.1f} s)", "cpu_1thread_pli_per_s": pl * 6 / t_1}

    # differentiation: K = 200 unrolled iterations, checkpoint every 20 (GPU) / full tape (oracle)
    wl = W.differentiation()
    tgt = torch.as_tensor(wl.target, device=dev)
    p = S.Problem.from_workload(wl, device=dev)
    p.unrolled_forward(200, 20)     # warm-up: workspace, first launches of every kernel
    _, u = p.read_u()
    p.unrolled_backward(2.0 * (u - tgt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.unrolled_forward(200, 20)
    _, u = p.read_u()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p.unrolled_backward(2.0 * (u - tgt))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    p.close()
    o = oracle.Problem(wl)
    c0 = time.perf_counter()
    o.unrolled_forward(200)
    _, uo = o.read_u()
    c1 = time.perf_counter()
    o.unrolled_backward(2.0 * (uo - wl.target.astype(np.float64)))
    c2 = time.perf_counter()
    del o
    rows["diff256_L8_K200"] = {"gpu_forward_s": t1 - t0, "gpu_backward_s": t2 - t1,
                               "cpu_forward_s": c1 - c0, "cpu_backward_s": c2 - c1}

    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": rows["rof64_L2_2000its"]["gpu_pli_per_s"],
        "unit": "pixel-label-iter/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": rows["rof64_L2_2000its"]["gpu_seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "CPU baselines: ROF 64x64 L=2 2000 iterations, sampled stereo 384x288 "
                               "L=8 1000 iterations, unrolled differentiation 256x256 L=8 K=200",
                   "step": "one pass over the three workloads"},
        "cpu": {"cores": ncores, "cpu_model": cpu_model(), "kind": "oracle"},
        "workloads": rows,
    }
    print(json.dumps(out))


BAND_IX, BAND_IY, BAND_RING = 60, 12, 2   # interior and ring of the two-iteration kernel's tiles


def band_bytes_per_pass(wl) -> int:
    """Bytes one two-iteration pass reads and writes: every tile loads its interior plus the
    ring (clipped to the image) of the 8k+1 state planes and the data plane (and the
    straddle table for truncated quadratics), and writes the interior's 8k+1 planes."""
    H, Wd, k = wl.H, wl.W, wl.k
    loaded = 0
    for r0 in range(0, H, BAND_IY):
        rows = min(H, r0 + BAND_IY + BAND_RING) - max(0, r0 - BAND_RING)
        for c0 in range(0, Wd, BAND_IX):
            loaded += rows * (min(Wd, c0 + BAND_IX + BAND_RING) - max(0, c0 - BAND_RING))
    read_planes = 8 * k + 2 + (1 if wl.rho == 1 else 0)
    return 4 * (read_planes * loaded + (8 * k + 1) * H * Wd)


def bench_temporal(args):
    """Temporal blocking (two iterations per pass over the state, k <= 3) against the
    one-pass kernel on the same problems: HIP-event time per iteration of each (the
    one-pass kernel in its automatic and in its one-group configuration, the two-iteration
    passes in groups of four iterations), the one-pass algorithmic bytes per iteration and
    the bytes a two-iteration pass moves (reported apart: temporal blocking changes the
    accounting). Value: pixel-label-iterations/s of the two-iteration path on the largest
    instance."""
    import torch
    import paper_1512_01383_amd as S
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def timed(g, iters):
        g.run(8)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.run(iters)
        e1.record(g.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / iters

    cases = [("rof_64_L2", W.rof(), 2000),
             ("rof_2048_L2", W.rof(H=2048, W=2048, seed=11), 200),
             ("tq_2048_L2", W.truncated_quadratic(L=2, H=2048, W=2048, seed=12), 200),
             ("tq_2048_L3", W.truncated_quadratic(L=3, H=2048, W=2048, seed=13), 200),
             ("tq_2048_L4", W.truncated_quadratic(L=4, H=2048, W=2048, seed=14), 200),
             ("tq_512_L2", W.truncated_quadratic(L=2, H=512, W=512, seed=15), 1000),
             ("tq_512_L4", W.truncated_quadratic(L=4, H=512, W=512, seed=16), 1000)]
    rows = {}
    for name, wl, iters in cases:
        g = S.Problem.from_workload(wl, device=dev)
        auto_ms = timed(g, iters)
        auto_tiling = list(g.get_tiling())
        g.set_tiling(1, 4, 64)
        one_ms = timed(g, iters)
        g.set_temporal(True)
        band_ms = timed(g, iters)
        g.close()
        nb1 = algorithmic_bytes_per_pixel(wl.k, wl.rho, wl.M, False, False) * wl.H * wl.W
        nbb = band_bytes_per_pass(wl)
        rows[name] = {"H": wl.H, "W": wl.W, "L": wl.L, "iters": iters,
                      "one_pass_ms": auto_ms, "one_pass_tiling": auto_tiling, "one_group_ms": one_ms,
                      "two_iteration_ms": band_ms, "speedup": auto_ms / band_ms,
                      "one_pass_bytes_per_iteration": nb1, "two_iteration_bytes_per_pass": nbb,
                      "one_pass_GBs": nb1 / (auto_ms * 1e-3) / 1e9,
                      "two_iteration_GBs": nbb / (2 * band_ms * 1e-3) / 1e9}
        print(f"{name}: one-pass {auto_ms * 1e3:.1f} us, two-iteration {band_ms * 1e3:.1f} us per iteration",
              file=sys.stderr, flush=True)
    big = rows["tq_2048_L2"]
    out = {"metric": "lifted PDHG pixel-label-iter/s", "unit": "pixel-label-iter/s",
           "value": big["H"] * big["W"] * (big["L"] - 1) / (big["two_iteration_ms"] * 1e-3),
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": big["two_iteration_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "temporal blocking: two iterations per pass over the state against "
                                  "one per pass, k <= 3; value on truncated quadratic 2048x2048, L=2"},
           "roofline": None, "cpu_baseline": None, "cases": rows}
    print(json.dumps(out))


def bench_diff(args):
    """Unrolled differentiation: K = 200 iterations with a checkpoint every 20 on the
    256x256, L = 8 truncated-quadratic instance with per-label additive values; loss =
    squared error of the read-out against the clean image; gradients w.r.t. f, lambda and
    the 8 x 256 x 256 additive values. Compared with the plain solve of the same instance to
    a 1e-3 certified gap (adaptive steps) on the same GPU."""
    import numpy as np
    import torch

    import paper_1512_01383_amd as S
    import workloads as W

    wl = W.differentiation()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, C = 200, 20
    tgt = torch.as_tensor(wl.target, device=dev)

    def one():
        p = S.Problem.from_workload(wl, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.unrolled_forward(K, C)
        _, u = p.read_u()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gf, gl, gw = p.unrolled_backward(2.0 * (u - tgt))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p.close()
        return t1 - t0, t2 - t1, gl

    for _ in range(max(1, args.warmup)):
        one()
    fw, bw = [], []
    for _ in range(max(1, args.steps)):
        a, b, gl = one()
        fw.append(a)
        bw.append(b)
    t_f, t_b = float(np.median(fw)), float(np.median(bw))
    g2 = S.Problem.from_workload(wl, device=dev, adaptive=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_gap = g2.run_to_gap(1e-3, args.gap_max_iters)
    t_gap = time.perf_counter() - t0
    rep = g2.energy()
    g2.close()
    pli = wl.H * wl.W * wl.k * K
    out = {
        "metric": "lifted PDHG pixel-label-iter/s",
        "value": pli / (t_f + t_b),
        "unit": "pixel-label-iter/s",
        "n_gpus": 1,
        "steps": len(fw),
        "warmup": max(1, args.warmup),
        "ms_per_step": (t_f + t_b) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "unrolled differentiation, truncated quadratic 256x256, L=8, K=200 "
                               "iterations, checkpoint every 20; step = forward + backward",
                   "K": K, "C": C},
        "differentiation": {"forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3,
                            "backward_over_forward": t_b / t_f, "grad_lambda": gl,
                            "plain_solve_to_1e-3": {"seconds": t_gap, "iterations": n_gap,
                                                    "rel_gap": rep["rel_gap"]}},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
