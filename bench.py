"""Benchmark: MGRIT solves of periodic linear advection on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole solve: FCF-MGRIT from the seeded U[0,1) initial
iterate to a space-time residual <= 1e-10 (discrete L2 norm), every level
of the hierarchy, with u0 and the initial iterate already resident in HBM.
The default workload is the largest single-GPU configuration and the one
the precision comparison is quoted on: ERK5+U5, n_x = 8192, n_t = 65536,
m = 8, 5-level V-cycles, FP32 relaxation of FP64 iterates (residual of the
relaxed iterate, coarse levels and norms in FP64); value = n_x * n_t /
(seconds per solve) in fine-step DOF/s.  The same solve in plain FP64 is
timed next to it over the same number of steps.

The JSON line also carries:
  roofline      the fine-level relaxation kernel (the dominant one): its
                algorithmic work per launch (flops for VALU-bound stencils,
                HBM bytes for bandwidth-bound ones) divided by its mean
                launch time from HIP events recorded on the plan's stream;
  by_pass       every (level, pass, precision) of one profiled solve with its
                time per solve and its achieved HBM bandwidth and flop rate
                from the library's algorithmic byte and flop counts;
  error         the relative error of the returned C-points against a plain
                FP64 solve to 1e-14 of the same workload (which the GPU tests
                hold within 1e-12 of the oracle's exact discrete solution);
  cpu_baseline  the CPU oracle's sequential time-stepping (the plain
                definition of the result), timed on a bounded sample of the
                same workload on the host;
  workloads     the other configurations (ERK3 F-cycles, SDIRK3, the 64 x 256
                ERK1 check, inflow boundaries, the Sec. 4.4 width rule), each
                timed over at least 5 solves with its own roofline and error;
  gpu_sequential  sequential time-stepping on the GPU (one workgroup,
                n_t steps) and MGRIT's speed-up over it;
  serving       the request mix of the serving form (p50/p99 latency).
"""

import argparse
import hashlib
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
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (one FMA per lane
# per clock) x 2.4 GHz.  Non-packed FP32 FMAs issue at the same rate (the
# 157.3 TFLOP/s FP32 figure needs packed FP32, which this build disables),
# so FP32 passes are priced against the same peak.
VALU_PEAK_TFS = 78.6
MAIN = "erk5_u5_nx8192_nt65536_m8_fp32relax"
TOL = 1e-10
REF_TOL = 1e-14


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


def _timed_solves(P, u0, uinit, steps, warmup, torch):
    """(mean seconds per solve, per-solve seconds, last result) over `steps`
    timed solves after `warmup`; every solve returns once its GPU work is
    done, and the whole timed region is bracketed by synchronisations."""
    out = torch.empty((1, P.nx), dtype=torch.float64, device="cuda")
    res = None
    for _ in range(warmup):
        res = P.solve(u0, uinit, tol=TOL, maxit=100, out="final", u_out=out)
    torch.cuda.synchronize()
    each = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        res = P.solve(u0, uinit, tol=TOL, maxit=100, out="final", u_out=out)
        each.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    return dt, each, res


def _stats_ms(each):
    a = 1e3 * np.asarray(each)
    return {"median": round(float(np.median(a)), 4), "p95": round(float(np.percentile(a, 95)), 4),
            "min": round(float(a.min()), 4), "n": int(a.size)}


def _cpoint_error(P, u0, uinit, ref, torch):
    """Max relative error of the C-points of a solve to TOL against `ref`
    (C-points of the FP64 solve to REF_TOL), on the device."""
    r = P.solve(u0, uinit, tol=TOL, maxit=100, out="cpoints")
    err = float((r.out - ref).abs().max() / ref.abs().max())
    return err


def _reference(w, u0, uinit, torch):
    """C-points of the plain FP64 solve of the same workload to REF_TOL."""
    P, _ = _plan(w, "fp64")
    r = P.solve(u0, uinit, tol=REF_TOL, maxit=100, out="cpoints")
    P.close()
    return r.out, r.hist[-1]


def measured_traffic(workload, source):
    """HBM bytes per launch of the fine relaxation kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel source
    changed since the counters were taken (hash recorded in the summary)."""
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


def _kernel_source(w):
    if w.get("boundary") == "inflow":
        return "bounded_kernels.h", "k_bounded_reg"
    if w["scheme"].startswith("SDIRK"):
        return "sdirk_pf_kernels.h", "k_sdirk_pf"
    return "relax_kernels.h", "k_stencil"


def profiled(P, u0, uinit):
    """One profiled solve: the per-class split and the (level, pass,
    precision) table with achieved rates from algorithmic bytes and flops."""
    P.set_profiling(True)
    r = P.solve(u0, uinit, tol=TOL, maxit=100, out="none")
    prof = P.profile()
    detail = P.profile_detail()
    P.set_profiling(False)
    rows = []
    for e in detail:
        s = e["ms"] * 1e-3
        gbs = e["bytes"] / s / 1e9 if s > 0 else 0.0
        tfs = e["flops"] / s / 1e12 if s > 0 else 0.0
        rows.append({"level": e["level"] + 1, "pass": e["pass"], "precision": e["precision"],
                     "launches": e["launches"], "ms": round(e["ms"], 4),
                     "avg_us": round(1e3 * e["ms"] / max(e["launches"], 1), 2),
                     "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "TFLOP/s": round(tfs, 2), "valu_frac": round(tfs / VALU_PEAK_TFS, 4)})
    return r, prof, detail, rows


def roofline(w, detail, workload):
    """The fine relaxation passes (level 1, passes fc and res, both
    precisions): algorithmic work per launch over the mean launch time.
    The bound is the resource whose peak the algorithmic work would take
    longer to saturate."""
    fine = [e for e in detail if e["level"] == 0 and e["pass"] in ("fc", "res")]
    launches = sum(e["launches"] for e in fine)
    ms = sum(e["ms"] for e in fine)
    by = sum(e["bytes"] for e in fine)
    fl = sum(e["flops"] for e in fine)
    src, kname = _kernel_source(w)
    avg_s = ms * 1e-3 / max(launches, 1)
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (VALU_PEAK_TFS * 1e12)
    gbs = by / launches / avg_s / 1e9
    tfs = fl / launches / avg_s / 1e12
    out = {"kernel": kname + " (fine-level FC and residual passes)",
           "launches": launches, "avg_launch_ms": round(avg_s * 1e3, 5),
           "bytes_per_launch": by / launches, "flops_per_launch": fl / launches,
           "hbm_gbs": round(gbs, 1), "valu_tflops": round(tfs, 2),
           "traffic": measured_traffic(workload, src)}
    if t_hbm >= t_alu:
        out.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)})
    else:
        out.update({"bound": "alu", "achieved": round(tfs, 2), "peak": VALU_PEAK_TFS,
                    "unit": "TFLOP/s", "frac": round(tfs / VALU_PEAK_TFS, 4)})
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
    cpus = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": w["nx"] * n / t, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "host_cpus": cpus,
            "sample": f"{n} of the {w['nt']} sequential time steps of the oracle "
                      f"(numpy, staged {w['scheme']}, one thread), n_x = {w['nx']}, "
                      f"{t:.1f} s"}


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
            "saturated": {"note": "all requests submitted at t = 0: latency is queueing",
                          "makespan_s": round(span, 3), "requests_per_s": round(rate, 2),
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


def solve_record(name, w, steps, warmup, torch, precision=None, ref=None):
    """Time `steps` solves of workload w (after `warmup`), profile one, and
    measure the error of its C-points against the FP64 reference."""
    P, psi = _plan(w, precision)
    u0, uinit = _inputs(w, torch)
    dt, each, r = _timed_solves(P, u0, uinit, steps, warmup, torch)
    st = r.stats
    rec = {"precision": precision or w["precision"], "psi_rule": w["psi_rule"],
           "ms_to_tol": round(dt * 1e3, 4), "step_ms": _stats_ms(each),
           "dof_per_s": w["nx"] * w["nt"] / dt, "iterations": r.iters,
           "outer_iterations": st.outer_iterations, "final_residual": r.hist[-1],
           "fine_passes_fp64": st.fine_passes_fp64, "fine_passes_fp32": st.fine_passes_fp32,
           "psi_nnz": [len(o) for o, _ in psi], "kernels": P.describe()}
    oc = P.operator_complexity()
    if oc == oc:
        rec["operator_complexity"] = round(oc, 4)
    _, prof, detail, rows = profiled(P, u0, uinit)
    rec["roofline"] = roofline(w, detail, name)
    rec["ms_by_class"] = {k: round(v, 4) for k, v in prof["ms"].items()}
    rec["by_pass"] = rows
    if ref is None:
        ref, rres = _reference(w, u0, uinit, torch)
        rec["reference_residual"] = rres
    rec["error_vs_fp64_reference"] = _cpoint_error(P, u0, uinit, ref, torch)
    return P, u0, uinit, rec, ref, dt, each


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=MAIN)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline solve (for profiler runs)")
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
    if a.no_extra:
        P, psi = _plan(w)
        u0, uinit = _inputs(w, torch)
        dt, each, r = _timed_solves(P, u0, uinit, a.steps, a.warmup, torch)
        print(json.dumps({"workload": a.workload, "ms_per_step": round(dt * 1e3, 4),
                          "iterations": r.iters, "final_residual": r.hist[-1],
                          "kernels": P.describe()}), flush=True)
        P.close()
        return
    steps = max(a.steps, 1)
    P, u0, uinit, rec, ref, dt, each = solve_record(a.workload, w, steps, a.warmup, torch)
    line = {"metric": METRIC, "value": w["nx"] * w["nt"] / dt, "unit": "DOF/s",
            "n_gpus": 1, "steps": steps, "warmup": a.warmup,
            "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if w["precision"] == "fp64" else "f32+f64",
            "data": "synthetic",
            "config": {"workload": a.workload, "scheme": w["scheme"], "nx": w["nx"],
                       "nt": w["nt"], "cfl": w["cfl"], "m": w["m"],
                       "levels": w["levels"], "cycle": w["cycle"], "tol": TOL,
                       "precision": w["precision"], "psi_rule": w["psi_rule"],
                       "psi_nnz": rec["psi_nnz"]},
            "iterations": rec["iterations"], "final_residual": rec["final_residual"],
            "step_ms": rec["step_ms"],
            "error_vs_fp64_reference": rec["error_vs_fp64_reference"],
            "reference_residual": rec.get("reference_residual"),
            "kernels": rec["kernels"], "roofline": rec["roofline"],
            "ms_by_class": rec["ms_by_class"], "by_pass": rec["by_pass"],
            "fine_passes": {"fp64": rec["fine_passes_fp64"], "fp32": rec["fine_passes_fp32"]}}
    tseq = gpu_sequential(P, w, u0, torch)
    line["gpu_sequential"] = {"ms": round(tseq * 1e3, 3),
                              "dof_per_s": w["nx"] * w["nt"] / tseq,
                              "mgrit_speedup": round(tseq / dt, 2)}
    P.close()
    if w["precision"] == "fp32":
        # the same solve in plain FP64, the same number of timed steps
        P64, _, _, r64, _, dt64, _ = solve_record(a.workload, w, steps, a.warmup, torch,
                                                  "fp64", ref)
        P64.close()
        line["fp64"] = r64
        line["fp32_vs_fp64"] = {
            "speedup_median": round(r64["step_ms"]["median"] / rec["step_ms"]["median"], 4),
            "spread_fp32": round(rec["step_ms"]["p95"] / rec["step_ms"]["median"] - 1, 4),
            "spread_fp64": round(r64["step_ms"]["p95"] / r64["step_ms"]["median"] - 1, 4)}
        # the other FP32 form: every inner fine pass in FP32 inside FP64
        # iterative refinement (the residual of the iterate in FP64)
        Pir, _, _, rir, _, _, _ = solve_record(a.workload, w, max(5, steps // 2), a.warmup,
                                               torch, "fp32_ir", ref)
        Pir.close()
        line["fp32_ir"] = rir
        line["fp32_vs_fp64"]["speedup_median_ir"] = round(
            r64["step_ms"]["median"] / rir["step_ms"]["median"], 4)
    extra = {}
    if w["psi_rule"] == "bound":  # the same solve with the Sec. 4.4 width rule
        ww = dict(w, psi_rule="window")
        Pw, _, _, rw, _, _, _ = solve_record(a.workload, ww, 5, 1, torch, None, ref)
        Pw.close()
        extra[a.workload + "@window_rule"] = rw
    for name in inputs.WORKLOADS:
        if name == a.workload:
            continue
        try:
            wn = dict(inputs.WORKLOADS[name])
            Pn, _, _, rn, refn, _, _ = solve_record(name, wn, 5, 1, torch)
            Pn.close()
            extra[name] = rn
            if wn["precision"] == "fp32":
                Pf, _, _, rf, _, _, _ = solve_record(name, wn, 5, 1, torch, "fp64", refn)
                Pf.close()
                extra[name + "@fp64"] = rf
        except Exception as e:  # report, keep the main line
            extra[name] = {"error": str(e)}
        torch.cuda.empty_cache()
    line["workloads"] = extra
    if a.serve > 0:
        line["serving"] = serving(a.serve, torch)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
