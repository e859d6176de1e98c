#!/usr/bin/env python3
"""Benchmark: CN time steps per second of the multigrid-preconditioned GMRES solver at 2047^2.

Workload (synthetic, shaped like the paper's examples): the single large anisotropic instance
alpha = 1.2, beta = 1.9 on the unit square, n1 = n2 = 2047 (4.19 M unknowns), variable
coefficients d+ = 1+x+y^2, d- = 2-x+y, e+ = 1+xy, e- = 1.5+0.5 sin(pi x) y, tau = 1/16, 16 CN steps,
source = manufactured term + seeded N(0,1) field (seed 3), GMRES(20) to relative residual 1e-10,
one geometric V(1,1) cycle per iteration.  A step is one CN step: right-hand side plus solve.

Prints one JSON line: the mixed-precision (FP32 preconditioner, FP64 outer) throughput as `value`,
the plain FP64 throughput beside it, per-step latency percentiles, iterations per step, the error of
the mixed result against the FP64 GPU result, the live-timed roofline of the dominant kernel, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MG-GMRES CN time-steps/s at 2047² + p50/p99 latency, mixed vs FP64 plain"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs of this workload
# (scaled by a copy of known size), keyed by kernel family, with the hash of the source file the
# kernels were built from: the figure is reported only while that source is unchanged.
PMC_TRAFFIC = {
    "cgs": {"bytes_per_launch": 396.98e6, "source": "paper_1706_06844_amd/csrc/krylov.hip",
            "sha256": "30ed1c7dd8db1a5f9ae70a84a55906ba20b0655fef489e8df2eb1f4f302baef9", "summary": "profiles/cgs_pass_c3_2047_mixed.md"},
}


def measured_traffic(family):
    import hashlib

    e = PMC_TRAFFIC.get(family)
    if not e:
        return None
    try:
        with open(os.path.join(ROOT, e["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != e["sha256"]:
                return None
    except OSError:
        return None
    return e["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2047)
    ap.add_argument("--maxit", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=24)
    ap.add_argument("--only", choices=["mixed", "fp64", "bf16"], default=None)
    ap.add_argument("--bf16", action="store_true",
                    help="also time the V-cycle with BF16 MFMA operator passes on its large levels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 2047^2 FP64 field (33.5 MB) three times with torch, so that a "
                         "counter run sees a kernel of known traffic")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(prec, p, dev_fields, S, phis, u0, steps, warmup, maxit, profile_family=None):
    import torch

    from paper_1706_06844_amd import fde

    s = fde.fde_problem_default(p.alpha, p.beta, p.n1, p.n2, p.tau, precision=prec, maxit=maxit)
    h = fde.fde_setup(s, *dev_fields)
    u = torch.empty_like(u0)
    un = torch.empty_like(u0)

    def run(k, tag):
        u.copy_(u0)
        lat, its, reo = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, b = u, un
        for m in range(1, k + 1):
            ts = time.perf_counter()
            st = fde.fde_step_sources(h, a, [f((m - 0.5) * p.tau) for f in phis], S, b)
            lat.append(time.perf_counter() - ts)
            its.append(st["iters"])
            reo.append(st["reorth_steps"])
            if not st["converged"]:
                raise RuntimeError(f"{tag}: step {m} did not converge: {st}")
            a, b = b, a
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, its, reo, a

    # warmup, with every kernel family timed to find the dominant one
    fde.fde_profile_enable(h)
    run(warmup, "warmup")
    prof = fde.fde_profile_read(h)
    fam = profile_family
    cand = {k: v for k, v in prof.items() if v["launches"] > 0}
    if fam is None and cand:
        fam = max(cand, key=lambda k: cand[k]["ms"])
    fde.fde_profile_reset(h)
    # without warmup there is nothing to choose from: time every family in the timed run
    fde.fde_profile_enable(h, 1 << fde.L.KFAM.index(fam) if fam else (1 << len(fde.L.KFAM)) - 1)
    elapsed, lat, its, reo, u_final = run(steps, "timed")
    timed = fde.fde_profile_read(h)
    if fam is None:
        prof = timed
        fam = max(timed, key=lambda k: timed[k]["ms"])
    live = timed[fam]
    out = {"elapsed": elapsed, "lat": lat, "iters": its, "u": u_final.clone(), "family": fam,
           "live": live, "warm_profile": prof, "reorth": reo}
    h.close()
    return out


def cpu_baseline(p, iters_per_step, sample_iters):
    """Oracle (FP64 CPU) on a bounded sample of the same workload: the right-hand side of step 1 and
    the first `sample_iters` FGMRES iterations, scaled to a whole step with the GPU's mean iteration
    count."""
    import workloads
    from oracle import multigrid as omg
    from oracle.cn import rhs
    from oracle.krylov import fgmres
    from oracle.operator import operator_from_problem

    threads = None
    try:
        from threadpoolctl import threadpool_info

        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        pass
    t_setup = time.perf_counter()
    op = operator_from_problem(p, 0.0)
    vc = omg.VCycle(omg.geometric_hierarchy(op))
    u0 = workloads.sample_u0(p)
    v = workloads.sample_source(p, 0.5 * p.tau)
    t_setup = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    b = rhs(op, u0, v)
    t_rhs = time.perf_counter() - t0
    t1 = time.perf_counter()
    fgmres(op.apply, b, vc, rtol=1e-10, restart=20, maxit=sample_iters)
    t_it = time.perf_counter() - t1
    # the sample also includes one residual evaluation at the start and one at the end
    per_iter = t_it / sample_iters
    per_step = t_rhs + iters_per_step * per_iter
    model = ""
    try:
        model = open("/proc/cpuinfo").read().split("model name")[1].split("\n")[0].strip(": \t")
    except Exception:
        pass
    return {"value": 1.0 / per_step, "unit": "CN steps/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": (f"C3 step 1 at {p.n1}^2: right-hand side + first {sample_iters} FGMRES(20) "
                       f"iterations ({t_rhs + t_it:.1f} s, setup {t_setup:.1f} s excluded), scaled by "
                       f"{iters_per_step:.1f} iterations/step"),
            "host_cpus": os.cpu_count(), "cpu_model": model}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); independent instances "
              "would be sharded across GPUs without communication, which this build does not "
              "measure.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads
    from paper_1706_06844_amd import fde

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p = workloads.config_c3(args.n, 16)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    dev_fields = [d(f) for f in workloads.sample(p, 0.0)]
    phis, fields = workloads.source_terms(p)
    S = [d(f) for f in fields]
    u0 = d(workloads.sample_u0(p))
    if args.copy_calibration:
        dst = torch.empty_like(u0)
        for _ in range(3):
            dst.copy_(u0)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {u0.numel() * 8} bytes")
    res = {}
    order = [("mixed", fde.FDE_MIXED_FP32), ("fp64", fde.FDE_FP64), ("bf16", fde.FDE_MIXED_BF16GEMM)]
    for name, prec in order:
        if args.only and args.only != name:
            continue
        if name == "bf16" and not (args.bf16 or args.only == "bf16"):
            continue
        log(f"{name}: {args.warmup} warmup + {args.steps} timed CN steps at {args.n}^2")
        res[name] = run_precision(prec, p, dev_fields, S, phis, u0, args.steps, args.warmup, args.maxit)
        r = res[name]
        log(f"{name}: {args.steps / r['elapsed']:.3f} steps/s, mean iters {np.mean(r['iters']):.1f}, "
            f"dominant {r['family']}")
    main_name = "mixed" if "mixed" in res else ("fp64" if "fp64" in res else "bf16")
    m = res[main_name]
    lat_ms = np.array(m["lat"]) * 1e3
    live = m["live"]
    bytes_per_launch = live["bytes"] / max(live["launches"], 1)
    ms_per_launch = live["ms"] / max(live["launches"], 1)
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9 if live["launches"] else 0.0
    out = {
        "metric": METRIC,
        "value": args.steps / m["elapsed"],
        "unit": "CN steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * m["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f64+f32", "fp64": "f64", "bf16": "f64+f32+bf16"}[main_name],
        "data": "synthetic",
        "config": {"workload": f"C3 anisotropic instance {args.n}x{args.n}, alpha=1.2, beta=1.9, "
                               "C2 variable coefficients, tau=1/16, manufactured + N(0,1) source "
                               "(seed 3)",
                   "precision": {"mixed": "FP32 V-cycle in FP64 flexible GMRES", "fp64": "FP64",
                                 "bf16": "V-cycle with BF16 MFMA operator passes (FP32 accumulation) in FP64 "
                                         "flexible GMRES"}[main_name],
                   "gmres": "GMRES(20), rtol 1e-10, x0 = 0", "multigrid": "geometric V(1,1), damped Jacobi 0.7"},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "iters_per_step": float(np.mean(m["iters"])),
        "reorth_fraction": float(np.sum(m["reorth"]) / max(np.sum(m["iters"]), 1)),
        "roofline": {"bound": "hbm", "kernel_family": m["family"], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(m["family"]), "bytes_per_launch": bytes_per_launch,
                     "us_per_launch": 1e3 * ms_per_launch, "launches": live["launches"]},
    }
    if "fp64" in res and main_name == "mixed":
        f = res["fp64"]
        out["fp64_value"] = args.steps / f["elapsed"]
        out["fp64_ms_per_step"] = 1e3 * f["elapsed"] / args.steps
        out["fp64_iters_per_step"] = float(np.mean(f["iters"]))
        out["fp64_p50_ms"] = float(np.percentile(np.array(f["lat"]) * 1e3, 50))
        out["fp64_p99_ms"] = float(np.percentile(np.array(f["lat"]) * 1e3, 99))
        du = (m["u"] - f["u"]).double()
        out["err_mixed_vs_fp64"] = float(torch.linalg.norm(du) / torch.linalg.norm(f["u"]))
        out["mixed_speedup_vs_fp64"] = out["value"] / out["fp64_value"]
    if "bf16" in res and main_name != "bf16":
        g = res["bf16"]
        ref = res["fp64"]["u"] if "fp64" in res else m["u"]
        out["bf16_value"] = args.steps / g["elapsed"]
        out["bf16_ms_per_step"] = 1e3 * g["elapsed"] / args.steps
        out["bf16_iters_per_step"] = float(np.mean(g["iters"]))
        out["err_bf16_vs_fp64"] = float(torch.linalg.norm((g["u"] - ref).double()) / torch.linalg.norm(ref))
        out["bf16_warm_profile_ms"] = {k: round(v["ms"], 3) for k, v in g["warm_profile"].items()}
    out["warm_profile_ms"] = {k: round(v["ms"], 3) for k, v in m["warm_profile"].items()}
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(p, out["iters_per_step"], args.cpu_sample_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
