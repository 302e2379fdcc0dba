"""Benchmark: MGRIT solves of periodic linear advection on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole solve: FCF-MGRIT from the seeded U[0,1) initial
iterate to a space-time residual <= 1e-10 (discrete L2 norm), every level
of the hierarchy, with u0 and the initial iterate already resident in HBM.
The default workload is ERK3+U3, n_x = 4096, n_t = 16384, m = 8, 4-level
F-cycles, FP64.  value = n_x * n_t / (seconds per solve) in fine-step DOF/s.

The JSON line also carries:
  roofline      the fine-level relaxation kernel (the dominant one): its
                algorithmic HBM bytes per launch divided by its mean launch
                time from HIP events recorded on the plan's stream;
  cpu_baseline  the CPU oracle's sequential time-stepping (the plain
                definition of the result), timed on a bounded sample of the
                same workload on the host;
  workloads     the other solver forms (the 64 x 256 ERK1, the SDIRK3 and
                the ERK5 FP32-relaxation/FP64 pair), with time to tolerance;
  gpu_sequential  sequential time-stepping on the GPU (one workgroup,
                n_t steps) and MGRIT's speed-up over it.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time to ‖r‖≤1e-10 & fine-step DOF/s (FP32-relax vs FP64); "
          "serve p50/p99")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
MAIN = "erk3_u3_nx4096_nt16384_m8_fcycle"
TOL = 1e-10


def _plan(w, precision=None):
    from paper_1910_03726_amd import mgrit as M
    from paper_1910_03726_amd import inputs
    psi, mi = M.workload_psi(w)
    inflow = inputs.workload_inflow(w) if w.get("boundary") == "inflow" else None
    P = M.Plan(w["nx"], w["nt"], w["cfl"], w["scheme"], w["m"], w["levels"], psi,
               cycle=w["cycle"], precision=precision or w["precision"], inflow=inflow)
    return P, psi


def _inputs(w, torch):
    from paper_1910_03726_amd import inputs
    u0 = torch.tensor(inputs.workload_u0(w), dtype=torch.float64, device="cuda")
    nc = w["nt"] // w["m"]
    uinit = torch.tensor(inputs.random_iterate(nc + 1, w["nx"], w["init_seed"]),
                         dtype=torch.float64, device="cuda")
    return u0, uinit


def _timed_solves(P, u0, uinit, steps, warmup, torch, each=None):
    """Mean seconds per solve over `steps` timed solves (after `warmup`);
    each solve returns only once its GPU work is done, so `each` (a list)
    receives the per-solve times too."""
    out = torch.empty((1, P.nx), dtype=torch.float64, device="cuda")
    res = None
    for _ in range(warmup):
        res = P.solve(u0, uinit, tol=TOL, maxit=100, out="final", u_out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        res = P.solve(u0, uinit, tol=TOL, maxit=100, out="final", u_out=out)
        if each is not None:
            each.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    return dt, res


def _fine_nnz(w):
    from paper_1910_03726_amd import mgrit as M
    if w["scheme"].startswith("SDIRK"):
        return None
    off, _ = M.phi_taps(w["scheme"], w["cfl"], w["nx"])
    return len(off)


def measured_traffic(workload, source="relax_kernels.h"):
    """HBM bytes per launch of the fine relaxation kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel source
    changed since the counters were taken (hash recorded in the summary)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_counters.txt")
    src = os.path.join(ROOT, "paper_1910_03726_amd", "csrc", source)
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    rec, val = None, None
    for line in open(path):
        if line.startswith(f"kernel source ({source}) sha256[:16]:"):
            rec = line.rsplit(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch:"):
            val = float(line.split(":", 1)[1])
    return val if rec == sha else None


def roofline(P, w, u0, uinit, torch, workload):
    """Fine relaxation kernel: algorithmic bytes and flops over its launches."""
    P.set_profiling(True)
    r = P.solve(u0, uinit, tol=TOL, maxit=100, out="none")
    prof = P.profile()
    P.set_profiling(False)
    nx, m = w["nx"], w["m"]
    inflow = w.get("boundary") == "inflow"
    nc = w["nt"] // m
    it = r.iters
    # FC passes read the start C-point (and the correction after the first
    # iteration) and write one C-point; residual passes read two C-points and
    # write one: 8 bytes each, per interval and point.
    arrays = (2 + 3 * it) + 3 * (it + 1)
    launches = prof["launches"]["relax_fine"]
    bytes_total = arrays * nc * nx * 8.0
    ms = prof["ms"]["relax_fine"]
    avg_ms = ms / max(launches, 1)
    nnz = _fine_nnz(w)
    flops_total = 2.0 * nnz * prof["fine_dof_steps"] if nnz else None
    achieved_gbs = bytes_total / launches / (avg_ms * 1e-3) / 1e9
    t_hbm = bytes_total / (HBM_PEAK_GBS * 1e9)
    t_alu = flops_total / (FP64_PEAK_TFS * 1e12) if flops_total else 0.0
    out = {"bound": "hbm" if t_hbm >= t_alu else "alu",
           "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(workload, "bounded_kernels.h" if inflow else
                                       "relax_kernels.h"),
           "kernel": ("k_bounded_tiled" if inflow else "k_stencil") +
                     " (fine-level FC and residual passes)",
           "launches": launches, "avg_launch_ms": round(avg_ms, 5),
           "bytes_per_launch": bytes_total / launches,
           "fp64_tflops_achieved": (round(flops_total / (ms * 1e-3) / 1e12, 2)
                                    if flops_total else None),
           "fp64_tflops_peak": FP64_PEAK_TFS,
           "relaxation_dof_steps_per_s": prof["fine_dof_steps"] / (ms * 1e-3),
           "ms_by_class": {k: round(v, 4) for k, v in prof["ms"].items()},
           "launches_by_class": prof["launches"]}
    if out["bound"] == "alu":
        a = flops_total / launches / (avg_ms * 1e-3) / 1e12
        out.update({"achieved": round(a, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": round(a / FP64_PEAK_TFS, 4)})
    return out


def cpu_baseline(w, seconds=10.0):
    """The oracle's sequential time-stepping on a bounded sample of steps."""
    from oracle import rk
    from paper_1910_03726_amd import inputs
    d = rk.Discretization(w["scheme"], w["nx"], w["cfl"])
    u = inputs.workload_u0(w)
    t0 = time.perf_counter()
    u = d.step(u)
    one = max(time.perf_counter() - t0, 1e-6)
    n = int(max(8, min(w["nt"], seconds / one)))
    t0 = time.perf_counter()
    d.propagate(u, n)
    t = time.perf_counter() - t0
    return {"value": w["nx"] * n / t, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} of the {w['nt']} sequential time steps of the oracle "
                      f"(numpy, staged {w['scheme']}), n_x = {w['nx']}, {t:.1f} s"}


def gpu_sequential(P, w, u0, torch):
    """Sequential stepping on the GPU: one workgroup, n_t steps."""
    out = torch.empty((1, w["nx"]), dtype=torch.float64, device="cuda")
    P.phi_apply_batch(u0.view(1, -1), out, w["nt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.phi_apply_batch(u0.view(1, -1), out, w["nt"])
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _serve_run(reqs, u0s, arrivals, slots, setup_threads, budget):
    """Submit reqs at their arrival times (seconds after start); return
    (results, makespan seconds, server stats)."""
    import threading
    from paper_1910_03726_amd import mgrit as M
    S = M.Server(budget, slots=slots, setup_threads=setup_threads, max_bypass=8)
    ids = [None] * len(reqs)
    t0 = time.perf_counter()

    def submitter():
        for k, q in enumerate(reqs):
            if arrivals is not None:
                dt = arrivals[k] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            ids[k] = S.submit(q["nx"], q["nt"], q["scheme"], q["cfl"], q["m"], u0s[k],
                              precision=q["precision"], seed=q["init_seed"])

    th = threading.Thread(target=submitter)
    th.start()
    res = []
    for k, q in enumerate(reqs):
        while ids[k] is None:
            time.sleep(0.0005)
        r, _ = S.wait(ids[k], q["nx"])
        res.append(r)
    th.join()
    makespan = time.perf_counter() - t0
    st = S.stats()
    S.close()
    return res, makespan, st


def serving(n, torch, slots=8, setup_threads=8, budget_gib=128):
    """The serving mix: saturated throughput, then Poisson arrivals at 80% of
    it (p50/p99 latency); the plain FP64 per-solve form on a 10% sample."""
    import numpy as np
    from paper_1910_03726_amd import inputs, mgrit as M
    reqs = inputs.serving_requests(n, seed=7)
    u0s = [inputs.request_u0(q) for q in reqs]
    dof = sum(q["nx"] * q["nt"] for q in reqs)
    budget = budget_gib << 30
    res, span, st = _serve_run(reqs, u0s, None, slots, setup_threads, budget)
    ok = sum(r.status == M.OK for r in res)
    rate = n / span
    arr = inputs.poisson_arrivals(n, 0.8 * rate, seed=7)
    res2, span2, st2 = _serve_run(reqs, u0s, arr, slots, setup_threads, budget)
    lat = np.array([r.latency_ms for r in res2])
    lat_sat = np.array([r.latency_ms for r in res])
    # plain per-solve FP64: the same setup and plan path, one request at a
    # time (submit, wait, next) with one setup thread and one slot
    sample = [dict(q, precision="fp64") for q in reqs[::10]]
    t0 = time.perf_counter()
    sdof = 0
    with M.Server(budget, slots=1, setup_threads=1) as S1:
        for q in sample:
            r, _ = S1.wait(S1.submit(q["nx"], q["nt"], q["scheme"], q["cfl"], q["m"],
                                     inputs.request_u0(q), precision="fp64",
                                     seed=q["init_seed"]), q["nx"])
            sdof += q["nx"] * q["nt"]
    tb = time.perf_counter() - t0
    return {"requests": n, "completed_ok": ok, "slots": slots,
            "setup_threads": setup_threads, "hbm_budget_gib": budget_gib,
            "hbm_peak_gib": round(st.hbm_peak / (1 << 30), 3),
            "psi_cache_hits": st.psi_cache_hits, "psi_cache_misses": st.psi_cache_misses,
            "batches": st.batches, "batched_requests": st.batched_requests,
            "saturated": {"makespan_s": round(span, 3), "requests_per_s": round(rate, 2),
                          "dof_per_s": dof / span,
                          "p50_ms": round(float(np.percentile(lat_sat, 50)), 3),
                          "p99_ms": round(float(np.percentile(lat_sat, 99)), 3)},
            "poisson_80pct": {"rate_per_s": round(0.8 * rate, 2),
                              "makespan_s": round(span2, 3),
                              "dof_per_s": dof / span2,
                              "p50_ms": round(float(np.percentile(lat, 50)), 3),
                              "p99_ms": round(float(np.percentile(lat, 99)), 3)},
            "per_solve_fp64": {"sample": f"{len(sample)} of {n} requests (every 10th), "
                                         "FP64, one at a time: setup, plan, solve, release",
                               "dof_per_s": sdof / tb,
                               "ms_per_request": round(1e3 * tb / len(sample), 3)},
            "serving_speedup_vs_per_solve": round((dof / span) / (sdof / tb), 2)}


def _auto_levels(nt, m):
    L, span = 2, m * m
    while nt % span == 0 and nt // span >= 8:
        L += 1
        span *= m
    return L


def workload_line(name, steps, warmup, torch, precision=None, psi_rule=None):
    from paper_1910_03726_amd import inputs
    w = dict(inputs.WORKLOADS[name])
    if psi_rule:
        w["psi_rule"] = psi_rule
    P, psi = _plan(w, precision)
    u0, uinit = _inputs(w, torch)
    dt, r = _timed_solves(P, u0, uinit, steps, warmup, torch)
    st = r.stats
    d = {"precision": precision or w["precision"], "psi_rule": w["psi_rule"],
         "ms_to_tol": round(dt * 1e3, 3),
         "dof_per_s": w["nx"] * w["nt"] / dt, "iterations": r.iters,
         "outer_iterations": st.outer_iterations, "final_residual": r.hist[-1],
         "fine_passes_fp64": st.fine_passes_fp64, "fine_passes_fp32": st.fine_passes_fp32,
         "psi_nnz": [len(o) for o, _ in psi], "kernels": P.describe()}
    oc = P.operator_complexity()
    if oc == oc:
        d["operator_complexity"] = round(oc, 4)
    # fine relaxation passes of one profiled solve (HIP events per launch):
    # ERK passes do 2 nnz(Phi) flops per fine DOF-step; FP32 passes run at
    # the FP64 vector rate (packed FP32 is not used), so both are priced
    # against the FP64 vector peak
    P.set_profiling(True)
    P.solve(u0, uinit, tol=TOL, maxit=100, out="none")
    prof = P.profile()
    P.set_profiling(False)
    nnz = _fine_nnz(w)
    ms, n = prof["ms"]["relax_fine"], prof["launches"]["relax_fine"]
    fp = {"launches": n, "avg_ms": round(ms / max(n, 1), 4)}
    if nnz and ms > 0:
        tf = 2.0 * nnz * prof["fine_dof_steps"] / (ms * 1e-3) / 1e12
        fp.update({"tflops": round(tf, 2), "frac_of_fp64_vector_peak": round(tf / FP64_PEAK_TFS, 4)})
    d["fine_pass"] = fp
    d["ms_by_class"] = {k: round(v, 4) for k, v in prof["ms"].items()}
    P.close()
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=MAIN)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--serve", type=int, default=2000, metavar="N",
                    help="requests in the serving measurement (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times "
                         "(reference for HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(time-parallel sharding across GPUs is described in DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1910_03726_amd import inputs
    torch.cuda.init()
    w = dict(inputs.WORKLOADS[a.workload])
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P, psi = _plan(w)
    u0, uinit = _inputs(w, torch)
    each = []
    dt, r = _timed_solves(P, u0, uinit, a.steps, a.warmup, torch, each)
    line = {"metric": METRIC, "value": w["nx"] * w["nt"] / dt, "unit": "DOF/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if w["precision"] == "fp64" else "f32+f64",
            "data": "synthetic",
            "config": {"workload": a.workload, "scheme": w["scheme"], "nx": w["nx"],
                       "nt": w["nt"], "cfl": w["cfl"], "m": w["m"],
                       "levels": w["levels"], "cycle": w["cycle"], "tol": TOL,
                       "psi_rule": w["psi_rule"], "psi_nnz": [len(o) for o, _ in psi]},
            "iterations": r.iters, "final_residual": r.hist[-1],
            "step_ms": {"median": round(1e3 * float(np.median(each)), 4),
                        "p95": round(1e3 * float(np.percentile(each, 95)), 4),
                        "min": round(1e3 * min(each), 4)},
            "kernels": P.describe()}
    line["roofline"] = roofline(P, w, u0, uinit, torch, a.workload)
    tseq = gpu_sequential(P, w, u0, torch)
    line["gpu_sequential"] = {"ms": round(tseq * 1e3, 3),
                              "dof_per_s": w["nx"] * w["nt"] / tseq,
                              "mgrit_speedup": round(tseq / dt, 2)}
    P.close()
    if not a.no_extra:
        extra = {}
        if w["psi_rule"] == "bound":  # the same solve with the Sec. 4.4 width rule
            extra[a.workload + "@window_rule"] = workload_line(a.workload, 3, 1, torch,
                                                               psi_rule="window")
        for name in inputs.WORKLOADS:
            if name == a.workload:
                continue
            try:
                extra[name] = workload_line(name, 3, 1, torch)
                if inputs.WORKLOADS[name]["precision"] == "fp32":
                    extra[name + "@fp64"] = workload_line(name, 3, 1, torch, "fp64")
            except Exception as e:  # report, keep the main line
                extra[name] = {"error": str(e)}
        line["workloads"] = extra
    if a.serve > 0 and not a.no_extra:
        line["serving"] = serving(a.serve, torch)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
