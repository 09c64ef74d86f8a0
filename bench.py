#!/usr/bin/env python3
"""Benchmark: Q(f) evaluations per second on one MI355X.

The timed step is one classical RK4 step (four evaluations of Q plus the
stage updates) of the 2D N = 64, L = 10, (N_r, N_s, N_sig) = (4, 4, 4)
workload in plain double precision, from the seeded three-Gaussian initial
data, dt = 1e-3.  `value` is evaluations per second over exactly `--steps`
steps with the state resident in device memory.  The same JSON line carries
the float form, the 3D N = 32 shapes, the exact-Galerkin (de-aliased) form,
the discontinuous data of Examples 3 and 6, the Nyquist-zero real form, the
two batched workloads, the
roofline of the dominant kernel, and the CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q(f) evals/sec, 2D N=64 & 3D N=32, FP32 vs FP64 at rel-L2 ≤1e-5"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}     # MI355X vector peaks
KERNELS = ["column_forward", "slab_pass", "column_pass"]
KERNEL_SOURCE = os.path.join(ROOT, "paper_2503_12805_amd", "csrc", "wke_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for name in ("wke_kernels.hip", "wke_fft.hpp", "wke_internal.hpp", "wke_shape.hpp", "wke_types.hpp"):
        with open(os.path.join(ROOT, "paper_2503_12805_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they are missing or were taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != source_hash():
        return None
    ent = data.get("workloads", {}).get(workload_key, {}).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


# --column-form / --split: fix the column pass instead of keeping the
# autotuner's choice (profiler runs use the choice of an unprofiled run, since
# the profiler's own overhead can change the ranking)
FIXED = {"form": None, "split": None}


def run_rk4(torch, wke, descs, grids, precision, steps, warmup, dt, galerkin=False, real=False):
    plan = wke.Plan(descs, precision, stream=torch.cuda.current_stream(), galerkin=galerkin, real=real)
    f = plan.pack(grids)
    plan.tuned = plan.tune(f, torch.zeros_like(f), reps=20).tolist()
    if FIXED["form"] is not None:
        plan.set_column_kernel(FIXED["form"])
        for row in plan.tuned:
            row[0], row[2] = float(wke.COLUMN_KINDS[FIXED["form"]]), None
    if FIXED["split"] is not None:
        plan.set_split(FIXED["split"])
        for row in plan.tuned:
            row[1], row[2] = float(FIXED["split"]), None
    m0 = plan.moments(f)
    scratch = f.clone()
    if warmup:
        plan.step(scratch, dt, warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    plan.step(f, dt, steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = start.elapsed_time(stop) / 1000.0
    m1 = plan.moments(f)
    return plan, f, wall, gpu_s, m0, m1


def median_of_runs(torch, plan, f, dt, runs=5, steps=25):
    """Second view of the same pipeline: HIP events over `runs` separate
    blocks of `steps` RK4 steps (100 evaluations each) on the plan's stream,
    after the warm-up already done; the median block."""
    rates = []
    for _ in range(runs):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.step(f, dt, steps)
        b.record()
        torch.cuda.synchronize()
        rates.append(4 * steps / (a.elapsed_time(b) / 1000.0))
    return {"method": "HIP events, %d runs of %d evaluations, median" % (runs, 4 * steps),
            "evals_per_s": round(float(sorted(rates)[runs // 2]), 2), "runs": [round(r, 1) for r in rates]}


def drift(m0, m1):
    out = []
    for a, b in zip(m0, m1):
        out.append({"mass_rel": abs(b[0] - a[0]) / abs(a[0]), "energy_rel": abs(b[1] - a[1]) / abs(a[1])})
    return out


def eval_error(torch, wke, oracle, wl, grid, precision, galerkin=False):
    """rel-L2 of one GPU evaluation against the oracle on the same input."""
    plan = wke.Plan([wke.desc_from_workload(wl)], precision, stream=torch.cuda.current_stream(), galerkin=galerkin)
    f = plan.pack([grid])
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    (q,) = plan.unpack(Q)
    ref = oracle.Q_galerkin(grid, wl) if galerkin else oracle.Q_physical(grid, oracle.nodes_for(wl))
    plan.close()
    return oracle.rel_l2(q, ref)


def sampled_error(torch, wke, oracle, wl, grid, precision, npts=4, seed=3):
    """Largest error at sampled grid points (where |Q| is largest) against the
    oracle's point-wise evaluation, relative to the largest |Q| there: for
    shapes whose full oracle evaluation takes too long here."""
    import numpy as np
    plan = wke.Plan([wke.desc_from_workload(wl)], precision, stream=torch.cuda.current_stream())
    f = plan.pack([grid])
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    (q,) = plan.unpack(Q)
    plan.close()
    top = np.argsort(np.abs(q).ravel())[::-1][:100]
    pick = np.random.default_rng(seed).choice(top, npts, replace=False)
    ref = oracle.Q_points(grid, oracle.nodes_for(wl), pick)
    return float(np.max(np.abs(q.ravel()[pick] - ref)) / np.max(np.abs(ref)))


def drift_curve(torch, wke, wl, grid, precision, dt, checkpoints):
    """|rho(t) - rho(0)| and |E(t) - E(0)| at the given step counts (untimed)."""
    plan = wke.Plan([wke.desc_from_workload(wl)], precision, stream=torch.cuda.current_stream())
    f = plan.pack([grid])
    m0 = plan.moments(f)[0]
    out, done = [], 0
    for n in checkpoints:
        plan.step(f, dt, n - done)
        done = n
        m = plan.moments(f)[0]
        out.append([round(n * dt, 6), abs(m[0] - m0[0]), abs(m[1] - m0[1])])
    plan.close()
    return out


def kernel_symbol(plan, precision, role):
    """Name of the kernel that runs a pass of this plan (one N per plan)."""
    dsc = plan.descs[0]
    if role == "column_pass":
        form = int(plan.tuned[0][0])
        return {0: "k_passB", 1: "k_passB_fp", 2: "k_passB_fp (fused)", 3: "k_passB_fp (half rounds)",
                4: "k_passB_fp (fused, matrix cores)"}[form] + (
            " (real)" if getattr(plan, "real", False) else "")
    if dsc.d == 2:
        return "k_passA2d"
    return "k_passA3d_reg" if dsc.N <= (32 if precision == "f32" else 16) else "k_passA3d"


def method_work(dsc):
    """The method's operation count for one evaluation of Q, independent of
    this implementation's sharing of coincident shifts: 1 forward transform,
    one inverse transform per (p1, p2) item for a and one per triple for b
    (c(sigma) = b(-sigma) reused when the sigma rule is antipodal, two per
    triple otherwise), each 5 n log2 n flops on n = N^d points, plus about 40
    flops per grid point and triple for the product and the weighted sum
    (Alg. 1; the complexity count of Section 3.4).  Returned split by axis:
    the transforms' axis-0 part (5 n log2 N each) with the products, and the
    part over axes 1..d-1."""
    n = float(dsc.N ** dsc.d)
    M = dsc.N_r * dsc.N_s * dsc.N_sig
    antipodal = dsc.d == 3 or dsc.N_sig % 2 == 0
    T = 1 + dsc.N_r * dsc.N_s + M * (1 if antipodal else 2)
    axis0 = T * 5.0 * n * math.log2(dsc.N) + 40.0 * n * M
    rest = T * 5.0 * n * (dsc.d - 1) * math.log2(dsc.N)
    return {"transforms": T, "flops": axis0 + rest, "flops_axis0_and_products": axis0, "flops_other_axes": rest}


def roofline(torch, plan, grids, precision, workload_key, us_per_eval, reps=200):
    """Roofline of the dominant kernel of the RK4 pipeline.

    The device time per evaluation, us_per_eval, comes from HIP events
    around the timed region (on the stream the kernels run on).  One
    evaluation is one slab pass plus one column pass (RK4 stage form), or the
    fused column pass alone; the time is split between the two kernels in
    the ratio of their back-to-back batch timings (wke_time_kernels, warm
    caches, median of three batches), which gives each kernel's average
    launch duration inside the timed region.  us_per_eval None (the
    exact-Galerkin plans, whose stages also project between the passes and
    run the column pass in its Q form): the batch timings themselves are the
    durations.

    `achieved` counts the method's operations (method_work): all of them for
    a fused column pass (one launch per evaluation); for the column pass of
    the two-kernel pipeline the transforms' axis-0 part and the products, for
    the slab pass the part over the other axes.  Beside it: the work this
    implementation executes (its own work model, which transforms each
    coincident shift once), and the HBM rate of the counter-measured traffic."""
    import numpy as np
    f = plan.pack(grids)
    # [fwd, slab, column(Q), column(RK)]: the median of three batches, so
    # that one disturbed batch does not skew the split
    us = np.median(np.stack([plan.time_kernels(f, torch.zeros_like(f), reps) for _ in range(3)]), axis=0)
    flops, nbytes = plan.work_model()                      # per kernel of one evaluation
    form = int(plan.tuned[0][0])
    fused = form in (2, 4)
    if fused:
        us[1] = 0.0                                        # no slab pass runs
    share_b = us[3] / (us[1] + us[3])
    if us_per_eval is None:
        dur = {"slab_pass": float(us[1]), "column_pass": float(us[2])}
    else:
        dur = {"slab_pass": us_per_eval * (1.0 - share_b), "column_pass": us_per_eval * share_b}
    k = "column_pass" if share_b >= 0.5 else "slab_pass"
    idx = {"slab_pass": 1, "column_pass": 2}
    t = dur[k] * 1e-6
    # the method's count for the kernel's share, summed over the instances
    # (the exact-Galerkin form runs the method on the grid of 2N points)
    mw = [method_work(dataclasses.replace(dsc, N=2 * dsc.N) if plan.galerkin else dsc) for dsc in plan.descs]
    if k == "column_pass":
        m_fl = sum(w["flops"] if fused else w["flops_axis0_and_products"] for w in mw)
    else:
        m_fl = sum(w["flops_other_axes"] for w in mw)
    fl, by = flops[idx[k]], nbytes[idx[k]]
    col_batch = us[2] if us_per_eval is None else us[3]
    per_kernel = {n: {"avg_us": round(float(dur[n]), 3),
                      "batch_us": round(float(col_batch if n == "column_pass" else us[1]), 3),
                      "impl_gflop": round(flops[idx[n]] / 1e9, 5), "model_mbytes": round(nbytes[idx[n]] / 1e6, 4)}
                  for n in ("slab_pass", "column_pass") if not (fused and n == "slab_pass")}
    col_key = {0: "column_pass_slots", 1: "column_pass_fp", 2: "column_pass_fused", 3: "column_pass_fp",
               4: "column_pass_fused_mfma"}[form]
    if us_per_eval is None:
        col_key = col_key.replace("column_pass", "column_pass_eval")
    traffic = measured_traffic(workload_key, k if k == "slab_pass" else col_key)
    peak = PEAK_TFLOPS[precision]
    roof = {"bound": "alu", "achieved": round(m_fl / t / 1e12, 4), "peak": peak, "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / peak, 5)
    roof["traffic"] = traffic
    roof["method_mflop_per_launch"] = round(m_fl / 1e6, 3)
    roof["impl"] = {"mflop_per_launch": round(fl / 1e6, 3), "tflops": round(fl / t / 1e12, 4),
                    "frac": round(fl / t / 1e12 / peak, 5), "model_mbytes_per_launch": round(by / 1e6, 4),
                    "model_hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 5)}
    if traffic:
        roof["measured_hbm"] = {"achieved": round(traffic / t / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(traffic / t / 1e9 / HBM_PEAK_GBS, 5)}
    roof["kernel"] = kernel_symbol(plan, precision, k) + (
        "" if k != "column_pass" else " (Q form)" if us_per_eval is None else " (RK4 stage form)")
    roof["avg_us"] = round(float(dur[k]), 3)
    roof["per_kernel"] = per_kernel
    roof["timing"] = ("back-to-back batch time of each kernel (wke_time_kernels)" if us_per_eval is None else
                      "device time per evaluation from HIP events over the timed region (%.3f us), split by "
                      "the kernels' back-to-back batch times" % us_per_eval)
    return roof


def cpu_baseline(oracle, wl, grid, dt, budget_s):
    """The oracle's RK4 (physical form: products of direct-sum interpolants)
    timed on the host on a bounded number of steps of the same workload."""
    nd = oracle.nodes_for(wl)
    oracle.Q_physical(grid, nd)          # the first call also starts the thread pool
    t0 = time.perf_counter()
    oracle.Q_physical(grid, nd)
    one = time.perf_counter() - t0
    nsteps = max(1, min(200, int(budget_s / max(4 * one, 1e-6))))
    t0 = time.perf_counter()
    oracle.rk4(grid, nd, dt, nsteps)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the Fourier form (the double convolution summed directly), one evaluation
    t0 = time.perf_counter()
    oracle.Q_fourier(grid, nd)
    fourier = time.perf_counter() - t0
    # one thread: the grid form once more, in a child process limited to one
    # OpenMP thread
    one_thread = None
    try:
        import dataclasses
        import subprocess
        import tempfile
        import numpy as np
        with tempfile.TemporaryDirectory() as tmp:
            path = os.path.join(tmp, "grid.npy")
            np.save(path, np.asarray(grid))
            code = ("import sys, time; sys.path.insert(0, %r); import numpy as np, oracle, wke_inputs as wi; "
                    "g = np.load(%r); nd = oracle.nodes_for(wi.Workload(*%r)); "
                    "t = time.perf_counter(); oracle.Q_physical(g, nd); print(time.perf_counter() - t)"
                    % (ROOT, path, dataclasses.astuple(wl)))
            r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                               env=dict(os.environ, OMP_NUM_THREADS="1"))
        one_thread = round(1.0 / float(r.stdout.strip().splitlines()[-1]), 4)
    except Exception:
        one_thread = None
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(4 * nsteps / el, 4), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": "%d RK4 steps (%d evaluations) of the same workload with the oracle's grid form "
                      "(direct-sum interpolants, no FFT), %.1f s" % (nsteps, 4 * nsteps, el),
            "fourier_form_evals_per_s": round(1.0 / fourier, 4),
            "grid_form_one_thread_evals_per_s": one_thread, "nproc": os.cpu_count(), "cpu_model": model}


# ---- secondary workloads ----------------------------------------------------
# Each returns one dict for the "variants" list of the JSON line; --only NAME
# runs one of them alone (its own process, e.g. for a profiler run).

class Ctx:
    def __init__(self, torch, wke, oracle, wi, args):
        self.torch, self.wke, self.oracle, self.wi, self.args = torch, wke, oracle, wi, args


def copy_probe(torch):
    """A plain 256 MiB device-to-device copy (calibrates HBM byte counters)."""
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 2 * src.numel() * 8


def v_c2_f32(c):
    wl = c.wi.workload("c2_2d_n64")
    g0 = c.wi.three_bumps_2d(wl.N, wl.L, 0)
    a = c.args
    log("[bench] 2D N=64 f32 RK4")
    p, fs, w, gs, m0, m1 = run_rk4(c.torch, c.wke, [c.wke.desc_from_workload(wl)], [g0], "f32", a.steps, a.warmup, a.dt)
    res = {"workload": "2D N=64 M=64 RK4", "precision": "f32", "evals_per_s": round(4 * a.steps / w, 2),
           "events_evals_per_s": round(4 * a.steps / gs, 2),
           "median_of_runs": median_of_runs(c.torch, p, fs, a.dt), "tuned_split": p.tuned,
           "rel_l2_vs_oracle": eval_error(c.torch, c.wke, c.oracle, wl, g0, "f32"), "drift": drift(m0, m1)[0],
           "roofline": roofline(c.torch, p, [g0], "f32", "c2_2d_n64_f32", 1e6 * gs / (4 * a.steps), a.reps)}
    p.close()
    return res


def _c3(c, prec):
    wl3 = c.wi.workload("c3_3d_n32")
    g3 = c.wi.aniso_gaussian_3d(wl3.N, wl3.L)
    a = c.args
    steps3 = a.steps
    log("[bench] 3D N=32 %s RK4: %d steps" % (prec, steps3))
    p3, f3, w3, gs3, b0, b1 = run_rk4(c.torch, c.wke, [c.wke.desc_from_workload(wl3)], [g3], prec, steps3,
                                      min(a.warmup, 3), a.dt)
    res = {"workload": "3D N=32 M=128 (2,8,8) cube RK4", "precision": prec,
           "evals_per_s": round(4 * steps3 / w3, 2), "events_evals_per_s": round(4 * steps3 / gs3, 2),
           "median_of_runs": median_of_runs(c.torch, p3, f3, a.dt), "tuned_split": p3.tuned,
           "rel_l2_vs_oracle": eval_error(c.torch, c.wke, c.oracle, wl3, g3, prec),
           "rj_profile_err_over_sum_K": rj_error(c, wl3, prec),
           "drift": drift(b0, b1)[0],
           "roofline": roofline(c.torch, p3, [g3], prec, "c3_3d_n32_" + prec, 1e6 * gs3 / (4 * steps3), a.reps)}
    p3.close()
    return res


def rj_error(c, wl, prec):
    """The 1/(1+|k|^2) check profile: Q nearly vanishes, so the error against
    the oracle is measured relative to the sum of the four term norms."""
    import numpy as np
    g = c.wi.rj_profile(wl.d, wl.N, wl.L)
    plan = c.wke.Plan([c.wke.desc_from_workload(wl)], prec, stream=c.torch.cuda.current_stream())
    f = plan.pack([g])
    Q = c.torch.zeros_like(f)
    plan.eval_Q(f, Q)
    c.torch.cuda.synchronize()
    (q,) = plan.unpack(Q)
    plan.close()
    ref, K = c.oracle.Q_physical(g, c.oracle.nodes_for(wl), return_terms=True)
    scale = sum(np.linalg.norm(k) for k in K) * 2.0 ** (1 - wl.d)
    return float(np.linalg.norm(q - ref) / scale)


def v_c2_galerkin_f64(c):
    """Exact-Galerkin (de-aliased) form of the headline shape: the operator on
    128 points per axis, the state and its projection kept there."""
    wl = c.wi.workload("c2_2d_n64")
    g0 = c.wi.three_bumps_2d(wl.N, wl.L, 0)
    a = c.args
    steps_g = max(1, a.steps // 4)
    log("[bench] 2D N=64 f64 RK4, exact-Galerkin form: %d steps" % steps_g)
    pg, _, wg, gsg, e0, e1 = run_rk4(c.torch, c.wke, [c.wke.desc_from_workload(wl)], [g0], "f64", steps_g,
                                     min(a.warmup, 3), a.dt, galerkin=True)
    res = {"workload": "2D N=64 M=64 RK4, exact-Galerkin (de-aliased, operator on 128 points)",
           "precision": "f64", "evals_per_s": round(4 * steps_g / wg, 2), "tuned_split": pg.tuned,
           "events_evals_per_s": round(4 * steps_g / gsg, 2),
           "rel_l2_vs_oracle": eval_error(c.torch, c.wke, c.oracle, wl, g0, "f64", galerkin=True),
           "drift": drift(e0, e1)[0],
           "roofline": roofline(c.torch, pg, [g0], "f64", "c2_2d_n64_f64_galerkin", None, a.reps)}
    pg.close()
    return res


def _example(c, key, prec):
    """The discontinuous data of Examples 3 (2D) and 6 (3D) at their own
    quadrature sizes and time step dt = 0.1."""
    label = {"ex3_2d_n64": "Example 3: 2D N=64, N_r=64, N_s=N_sig=12 (M=9216), S=3, discontinuous data, RK4 dt=0.1",
             "ex6_3d_n32": "Example 6: 3D N=32, N_r=32, 12-point design (M=4608), S=0.33, discontinuous data, "
                           "RK4 dt=0.1"}[key]
    wlx = c.wi.workload(key)
    gx = c.wi.discontinuous_ex3(wlx.d, wlx.N, wlx.L)
    steps_x = max(1, c.args.steps // (10 if wlx.d == 2 else 40))
    log("[bench] %s %s: %d steps" % (key, prec, steps_x))
    px, _, wx, gsx, x0, x1 = run_rk4(c.torch, c.wke, [c.wke.desc_from_workload(wlx)], [gx], prec, steps_x, 1, 0.1)
    roof = roofline(c.torch, px, [gx], prec, key + "_" + prec, 1e6 * gsx / (4 * steps_x), min(c.args.reps, 50))
    px.close()
    return {"workload": label, "precision": prec, "evals_per_s": round(4 * steps_x / wx, 2), "tuned_split": px.tuned,
            "events_evals_per_s": round(4 * steps_x / gsx, 2), "roofline": roof,
            "sampled_err_vs_oracle": sampled_error(c.torch, c.wke, c.oracle, wlx, gx, prec),
            "drift": drift(x0, x1)[0],
            "drift_curve_t_mass_energy": drift_curve(c.torch, c.wke, wlx, gx, prec, 0.1,
                                                     [10, 20, 50] if wlx.d == 2 else [5, 10, 20])}


def _real(c, key, prec):
    """The Nyquist-zero real form (modes with a -N/2 component dropped from
    the operator's input; real fields packed two per transform)."""
    wlx = c.wi.workload(key)
    if key.startswith("ex"):
        gx, dt = c.wi.discontinuous_ex3(wlx.d, wlx.N, wlx.L), 0.1
        steps = max(1, c.args.steps // (10 if wlx.d == 2 else 40))
    else:
        gx = c.wi.three_bumps_2d(wlx.N, wlx.L, 0) if wlx.d == 2 else c.wi.aniso_gaussian_3d(wlx.N, wlx.L)
        dt, steps = c.args.dt, max(1, c.args.steps // (1 if wlx.d == 2 else 4))
    log("[bench] %s %s real form: %d steps" % (key, prec, steps))
    px, _, wx, gsx, x0, x1 = run_rk4(c.torch, c.wke, [c.wke.desc_from_workload(wlx)], [gx], prec, steps,
                                     min(c.args.warmup, 3), dt, real=True)
    res = {"workload": "real form: " + key, "precision": prec, "evals_per_s": round(4 * steps / wx, 2),
           "events_evals_per_s": round(4 * steps / gsx, 2), "tuned_split": px.tuned, "drift": drift(x0, x1)[0]}
    f = px.pack([gx])
    Q = c.torch.zeros_like(f)
    px.eval_Q(f, Q)
    c.torch.cuda.synchronize()
    (q,) = px.unpack(Q)
    nd = c.oracle.nodes_for(wlx)
    if wlx.M <= 128:
        res["rel_l2_vs_oracle"] = c.oracle.rel_l2(q, c.oracle.Q_zero(gx, nd))
    else:
        import numpy as np
        top = np.argsort(np.abs(q).ravel())[::-1][:100]
        pick = np.random.default_rng(3).choice(top, 4, replace=False)
        ref = c.oracle.Q_points(c.oracle.nyquist_zero(np.real(gx), wlx.L), nd, pick)
        res["sampled_err_vs_oracle"] = float(np.max(np.abs(q.ravel()[pick] - ref)) / np.max(np.abs(ref)))
    res["roofline"] = roofline(c.torch, px, [gx], prec, key + "_" + prec + "_real", 1e6 * gsx / (4 * steps),
                               c.args.reps if wlx.M <= 128 else min(c.args.reps, 50))
    px.close()
    return res


def v_exact_f64(c):
    """The exact-weight reference system (2D N=16, the C1 data): its time, and
    the quadrature error of the fast method with the exact constraint
    against it as N_r, N_s = N_sigma grow."""
    import numpy as np
    torch, wke = c.torch, c.wke
    wl = c.wi.workload("c1_2d_n16")
    g = c.wi.two_gaussians_c1()
    desc = wke.Desc(2, 16, wl.L, 1, 1, 1)
    ft = torch.from_numpy(np.ascontiguousarray(g).ravel()).cuda()
    Q = torch.zeros_like(ft)
    wke.wke_exact_system(desc, ft, Q)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        wke.wke_exact_system(desc, ft, Q)
    el = (time.perf_counter() - t0) / reps
    ref = Q.cpu().numpy().reshape(16, 16)
    errs = []
    for nr, ns in [(2, 4), (4, 8), (8, 16), (16, 32)]:
        plan = wke.Plan([wke.Desc(2, 16, wl.L, nr, ns, ns)], "f64", galerkin=True)
        f = plan.pack([g])
        q = torch.zeros_like(f)
        plan.eval_Q(f, q)
        torch.cuda.synchronize()
        errs.append([nr, ns, ns, c.oracle.rel_l2(plan.unpack(q)[0], ref)])
        plan.close()
    t0 = time.perf_counter()
    oref = c.oracle.Q_exact(g, 2, 16, wl.L)
    cpu_s = time.perf_counter() - t0
    return {"workload": "exact-weight reference system, 2D N=16, L=8 (O(N^6) sums, 256-point radial rule)",
            "precision": "f64", "evals_per_s": round(1.0 / el, 2), "cpu_oracle_evals_per_s": round(1.0 / cpu_s, 3),
            "rel_l2_vs_oracle": c.oracle.rel_l2(ref, oref),
            "fast_method_quadrature_error_Nr_Ns_Nsig_relL2": errs}


def v_c4_f32(c):
    """Batched uneven 2D (16 each of N = 32, 48, 64, 96), float: RK4 steps
    timed with the N groups on concurrent streams (the plan's default), in
    order on one stream, and with graph replay; the launches one RK4 stage
    takes per group; and every instance against the oracle."""
    import numpy as np
    log("[bench] batch of 64 uneven 2D instances f32")
    c4 = c.wi.c4_batch()
    descs = [c.wke.desc_from_workload(w) for w, _ in c4]
    grids = [g for _, g in c4]
    steps4 = max(20, c.args.steps)
    p4, f4, w4, gs4, c0, c1 = run_rk4(c.torch, c.wke, descs, grids, "f32", steps4, min(c.args.warmup, 2), c.args.dt)
    med = median_of_runs(c.torch, p4, p4.pack(grids), c.args.dt)
    med = {"method": med["method"] + " (of the batch; x64 instances)",
           "instance_evals_per_s": round(64 * med["evals_per_s"], 2)}

    def rate(graphs, concurrent):
        p4.set_concurrency(concurrent)
        p4.set_graphs(graphs)
        g4 = p4.pack(grids)
        p4.step(g4, c.args.dt, 1)                  # (capture)
        c.torch.cuda.synchronize()
        a, b = c.torch.cuda.Event(enable_timing=True), c.torch.cuda.Event(enable_timing=True)
        a.record()
        p4.step(g4, c.args.dt, steps4)
        b.record()
        c.torch.cuda.synchronize()
        return round(64 * 4 * steps4 / (a.elapsed_time(b) / 1000.0), 2)
    in_order = rate(False, False)
    graph_conc = rate(True, True)
    graph_in_order = rate(True, False)
    p4.set_graphs(False)
    p4.set_concurrency(True)
    lps = [1 if int(row[0]) in (2, 4) else 2 for row in p4.tuned]      # fused: no slab pass
    Q = c.torch.zeros_like(f4)
    f0 = p4.pack(grids)
    p4.eval_Q(f0, Q)
    c.torch.cuda.synchronize()
    errs = [c.oracle.rel_l2(q, c.oracle.Q_physical(g, c.oracle.nodes_for(w)))
            for (w, g), q in zip(c4, p4.unpack(Q))]
    p4.close()
    return {"workload": "64 instances 2D N in {32,48,64,96} M=64 RK4", "precision": "f32",
            "instance_evals_per_s": round(64 * 4 * steps4 / w4, 2),
            "events_instance_evals_per_s": round(64 * 4 * steps4 / gs4, 2),
            "median_of_runs": med,
            "n_groups_on_concurrent_streams": len(p4.tuned),
            "events_instance_evals_per_s_groups_in_order": in_order,
            "events_instance_evals_per_s_graph_replay": graph_conc,
            "events_instance_evals_per_s_graph_replay_in_order": graph_in_order,
            "launches_per_rk4_stage_per_group": lps, "tuned_split": p4.tuned,
            "per_instance_rel_l2_vs_oracle": {"max": max(errs), "median": float(np.median(errs)),
                                              "instances": len(errs)},
            "drift_max": {k: max(d[k] for d in drift(c0, c1)) for k in ("mass_rel", "energy_rel")}}


def v_c5_f32(c):
    """3D N=64, L=12, (4,8,8), batch of 8, float with double state: 100 RK4
    steps timed, then the same steps in plain double (the reference path):
    relative L2 of the float state and the mass and energy drift of both,
    per instance."""
    import numpy as np
    c5 = c.wi.c5_batch()
    descs = [c.wke.desc_from_workload(w) for w, _ in c5]
    grids = [g for _, g in c5]
    # 100 steps of dt = 2e-4 (t = 0.02): with dt = 1e-3 this data's explicit
    # RK4 run turns non-finite between t = 0.02 and 0.05, in both precisions
    steps5, dt5 = 100, 2e-4
    log("[bench] batch of 8 3D N=64 f32: %d RK4 steps" % steps5)
    p5, f5, w5, gs5, d0, d1 = run_rk4(c.torch, c.wke, descs, grids, "f32", steps5, 1, dt5)
    res = {"workload": "8 instances 3D N=64 L=12 M=256 (4,8,8) cube, %d RK4 steps dt=%g" % (steps5, dt5),
           "precision": "f32", "instance_evals_per_s": round(8 * 4 * steps5 / w5, 2),
           "events_instance_evals_per_s": round(8 * 4 * steps5 / gs5, 2), "tuned_split": p5.tuned,
           "roofline": roofline(c.torch, p5, grids, "f32", "c5_3d_n64_f32",
                                1e6 * gs5 / (4 * steps5), max(1, c.args.reps // 40))}
    y32 = p5.unpack(f5)
    p5.close()
    log("[bench] batch of 8 3D N=64 f64 reference path: %d RK4 steps" % steps5)
    p6, f6, w6, _, e0, e1 = run_rk4(c.torch, c.wke, descs, grids, "f64", steps5, 1, dt5)
    y64 = p6.unpack(f6)
    p6.close()
    rel = [c.oracle.rel_l2(a, b) for a, b in zip(y32, y64)]
    rel_inc = [c.oracle.rel_l2(a - g, b - g) for a, b, g in zip(y32, y64, grids)]
    dm32, dm64 = drift(d0, d1), drift(e0, e1)
    res["vs_f64_gpu_path"] = {
        "f64_instance_evals_per_s": round(8 * 4 * steps5 / w6, 2),
        "state_rel_l2_max": max(rel), "increment_rel_l2_max": max(rel_inc),
        "mass_drift_f32_max": max(d["mass_rel"] for d in dm32), "mass_drift_f64_max": max(d["mass_rel"] for d in dm64),
        "energy_drift_f32_max": max(d["energy_rel"] for d in dm32),
        "energy_drift_f64_max": max(d["energy_rel"] for d in dm64),
        "mass_f32_minus_f64_rel_max": max(abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(d1, e1)),
        "energy_f32_minus_f64_rel_max": max(abs(a[1] - b[1]) / abs(b[1]) for a, b in zip(d1, e1))}
    return res


VARIANTS = {
    "c2_f32": v_c2_f32,
    "c3_f64": lambda c: _c3(c, "f64"),
    "c3_f32": lambda c: _c3(c, "f32"),
    "c2_galerkin_f64": v_c2_galerkin_f64,
    "ex3_f64": lambda c: _example(c, "ex3_2d_n64", "f64"),
    "ex3_f32": lambda c: _example(c, "ex3_2d_n64", "f32"),
    "ex6_f64": lambda c: _example(c, "ex6_3d_n32", "f64"),
    "ex6_f32": lambda c: _example(c, "ex6_3d_n32", "f32"),
    "c3_real_f64": lambda c: _real(c, "c3_3d_n32", "f64"),
    "c3_real_f32": lambda c: _real(c, "c3_3d_n32", "f32"),
    "ex6_real_f64": lambda c: _real(c, "ex6_3d_n32", "f64"),
    "exact_f64": v_exact_f64,
    "c4_f32": v_c4_f32,
    "c5_f32": v_c5_f32,
}



def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--cpu-budget", type=float, default=16.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", default="", help="run only this secondary workload and print its line: " +
                    ", ".join(VARIANTS))
    ap.add_argument("--reps", type=int, default=200, help="launches per kernel for the batch-time split")
    ap.add_argument("--column-form", choices=["slots", "fields", "fused", "fields_half", "fused_mfma"], default=None,
                    help="fix the column-pass form after autotuning (for profiler runs)")
    ap.add_argument("--split", type=int, default=None, help="fix the quadrature-sum split after autotuning")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    FIXED["form"], FIXED["split"] = args.column_form, args.split
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    import paper_2503_12805_amd as wke
    import wke_inputs as wi

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    wke.load_library()

    ctx = Ctx(torch, wke, oracle, wi, args)
    if args.only:
        if args.only not in VARIANTS:
            print("--only takes one of: %s" % ", ".join(VARIANTS), file=sys.stderr)
            sys.exit(2)
        res = VARIANTS[args.only](ctx)
        if args.copy_probe:
            res["copy_probe_bytes"] = copy_probe(torch)
        print(json.dumps(res), flush=True)
        return

    # ---- headline: 2D N=64, plain double, RK4 --------------------------------
    wl = wi.workload("c2_2d_n64")
    g0 = wi.three_bumps_2d(wl.N, wl.L, 0)
    desc = wke.desc_from_workload(wl)
    log("[bench] 2D N=64 f64 RK4: %d steps (%d warmup)" % (args.steps, args.warmup))
    plan, f, wall, gpu_s, m0, m1 = run_rk4(torch, wke, [desc], [g0], "f64", args.steps, args.warmup, args.dt)
    evals = 4 * args.steps
    value = evals / wall
    log("[bench]   %.1f evals/s (wall), %.1f evals/s (events)" % (value, evals / gpu_s))
    roof = roofline(torch, plan, [g0], "f64", "c2_2d_n64_f64", 1e6 * gpu_s / evals, args.reps)
    err64 = eval_error(torch, wke, oracle, wl, g0, "f64")
    log("[bench]   rel-L2 vs oracle %.2e; dominant kernel %s %.2f us" % (err64, roof["kernel"], roof["avg_us"]))
    med = median_of_runs(torch, plan, f, args.dt)
    plan.close()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000.0 * wall / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D N=64, L=10, (N_r,N_s,N_sig)=(4,4,4) M=64, classical RK4 dt=1e-3, "
                               "three seeded Gaussians (seed 0), plain double form; one step = 4 Q evaluations",
                   "d": 2, "N": 64, "L": 10.0, "M": 64, "dt": args.dt, "precision": "f64"},
        "rel_l2_vs_oracle": err64,
        "drift": drift(m0, m1)[0],
        "events_evals_per_s": round(evals / gpu_s, 2),
        "median_of_runs": med,
        "tuned_split": plan.tuned,
        "roofline": roof,
    }

    if not args.no_variants:
        res = {name: fn(ctx) for name, fn in VARIANTS.items()}
        out["variants"] = list(res.values())
        # the metric's four numbers, also at the top level
        legs = {"2d_n64_f64": out, "2d_n64_f32": res["c2_f32"], "3d_n32_f64": res["c3_f64"],
                "3d_n32_f32": res["c3_f32"]}
        out["metric_legs"] = {
            k: {"evals_per_s_wall": v["evals_per_s"] if k != "2d_n64_f64" else out["value"],
                "evals_per_s_events_median": v["median_of_runs"]["evals_per_s"],
                "rel_l2_vs_oracle": v["rel_l2_vs_oracle"],
                "dominant_kernel_roofline_frac": v["roofline"]["frac"]} for k, v in legs.items()}
        log("[bench] metric legs: " + ", ".join("%s %.0f evals/s wall, %.0f events median (rel-L2 %.1e)" % (
            k, v["evals_per_s_wall"], v["evals_per_s_events_median"], v["rel_l2_vs_oracle"])
            for k, v in out["metric_legs"].items()))

    if args.copy_probe:
        out["copy_probe_bytes"] = copy_probe(torch)

    if not args.no_cpu:
        log("[bench] CPU oracle baseline (about %.0f s of RK4 steps, one Fourier-form and one "
            "single-thread evaluation)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(oracle, wl, g0, args.dt, args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
