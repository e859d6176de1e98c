#!/usr/bin/env python3
"""Benchmark: CN time steps per second of the multigrid-preconditioned GMRES solver at 2047^2.

Workload (synthetic, shaped like the paper's examples): the single large anisotropic instance
alpha = 1.2, beta = 1.9 on the unit square, n1 = n2 = 2047 (4.19 M unknowns), variable
coefficients d+ = 1+x+y^2, d- = 2-x+y, e+ = 1+xy, e- = 1.5+0.5 sin(pi x) y, tau = 1/16, 16 CN steps,
source = manufactured term + seeded N(0,1) field (seed 3), GMRES(20) to relative residual 1e-10,
one geometric V(1,1) cycle per iteration.  A step is one CN step: right-hand side plus solve.

Prints one JSON line: the mixed-precision throughput as `value` (the FP32 V-cycle as the
preconditioner of FP64 flexible GMRES: FP64 basis, Arnoldi products, inner products, Givens
rotations and true residuals), plain FP64 (`fp64_*`) and the FP32-restart-cycle modes (`cycle_*`,
`cycle16_*`) beside it, per-step latency percentiles, iterations per step, the errors against the
FP64 GPU result, the live-timed roofline of the dominant kernel, the FP64 CPU oracle timed on a
bounded sample of the same workload, and the 511^2 C2 workload run in full by the GPU and by the
oracle (all host cores and one thread).
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
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
# live timing of the dominant kernel samples every PROFILE_STRIDE-th launch (coprime to the two or three
# Gram-Schmidt passes per step and to the restart length 20)
PROFILE_STRIDE = 17

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs of this workload
# (scaled by a copy of known size), keyed by kernel family, with the hash of the source files the
# kernel is built from: the figure is reported only while those sources are unchanged.
PMC_TRAFFIC = {
    # cgs_kernel<double, double, *> (FP64 Gram-Schmidt passes): per executed pass of one C3 step with
    # the FP32 V-cycle in FP64 GMRES (1080 executed of 1606 dispatches)
    "cgs": {"bytes_per_launch": 390.00e6,
             "sources": ['paper_1706_06844_amd/csrc/krylov.hip', 'paper_1706_06844_amd/csrc/common.h', 'paper_1706_06844_amd/csrc/fft.h'],
             "sha256": "5f4536c500e2326c4c0e254f4e5ff7ba1d5c8cb1b33bf21c2b10e2c3f14644be",
             "summary": "profiles/gram_schmidt_fp64_c3_2047.md"},
    # toep_y_kernel<float, float, 4096, false>: 1052 dispatches of the same step
    "mg0_y": {"bytes_per_launch": 70.98e6,
              "sources": ['paper_1706_06844_amd/csrc/toeplitz.hip', 'paper_1706_06844_amd/csrc/toep_dev.h', 'paper_1706_06844_amd/csrc/fft.h', 'paper_1706_06844_amd/csrc/common.h'],
              "sha256": "d83e1263bf063f26c450e3c3026638915c19d52f25c4ce8381a31ea1f9c2f556",
              "summary": "profiles/fft_column_pass_c3_2047.md"},
}


def measured_traffic(family):
    import hashlib

    e = PMC_TRAFFIC.get(family)
    if not e:
        return None
    h = hashlib.sha256()
    try:
        for src in e["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return e["bytes_per_launch"] if h.hexdigest() == e["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2047)
    ap.add_argument("--maxit", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the C2 (511^2) GPU and oracle comparison")
    ap.add_argument("--no-c4", action="store_true", help="skip the C4 (64 batched instances) keys")
    ap.add_argument("--c4-modes", type=str, default="mixed,fp64,cycle",
                    help="--workload c4: precision modes (the first of mixed/fp64/cycle present gives the value)")
    ap.add_argument("--c4-slots", type=int, default=0,
                    help="--workload c4: slots per group (0: the count of the most frequent size)")
    ap.add_argument("--c4-piece", type=int, default=0,
                    help="--workload c4: Arnoldi steps per issued piece of a restart cycle (0: whole cycles)")
    ap.add_argument("--c4-grouped-only", action="store_true",
                    help="--workload c4: grouped batching only (no ungrouped and one-at-a-time runs)")
    ap.add_argument("--cpu-sample-iters", type=int, default=24)
    ap.add_argument("--only", choices=["cycle16", "cycle", "mixed", "fp64", "bf16"], default=None)
    ap.add_argument("--workload", choices=["c3", "c4", "c5"], default="c3",
                    help="c3: the single 2047^2 instance (default, the headline line); c4: 64 batched "
                         "instances; c5: served requests with Poisson arrivals")
    ap.add_argument("--c5-count", type=int, default=200, help="measured requests")
    ap.add_argument("--c5-warmup", type=int, default=20, help="warm-up requests before the measured ones")
    ap.add_argument("--c5-kmax", type=int, default=11, help="largest grid 2^k - 1 of the served requests")
    ap.add_argument("--c5-max-running", type=int, default=2,
                    help="ungrouped requests with a cycle piece in flight at once (0: no limit)")
    ap.add_argument("--c5-piece", type=int, default=5,
                    help="Arnoldi steps per issued piece of a restart cycle (0: whole cycles)")
    ap.add_argument("--c5-lanes", type=int, default=0,
                    help="streams shared by the batch: larger requests on one, groups on the others (0: own streams)")
    ap.add_argument("--c5-busy-running", type=int, default=1,
                    help="ungrouped (larger) requests with a piece in flight while a group has work (-1: no cap)")
    ap.add_argument("--c5-loads", type=str, default="0.9",
                    help="with --c5-qps auto: arrival rates as fractions of the saturation rate")
    ap.add_argument("--c5-compare", action="store_true",
                    help="also run at the highest load: the other busy cap, the plain policy and FP64")
    ap.add_argument("--c5-qps", type=str, default="auto",
                    help="comma-separated arrival rates, or 'auto' for the --c5-loads fractions of the saturation rate")
    ap.add_argument("--bf16", action="store_true",
                    help="also time the V-cycle with BF16 MFMA operator passes on its large levels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 2047^2 FP64 field (33.5 MB) three times with torch, so that a "
                         "counter run sees a kernel of known traffic")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_groups(prec):
    """Profiling families that time a single kernel (template variants of one kernel count as one):
    the candidates for the dominant kernel.  The coarser-level and transfer families hold several
    different kernels at several sizes.  (With FP32 cycles the Arnoldi product runs the fine-level
    FP32 FFT kernels and is timed in the mg0 families.)"""
    from paper_1706_06844_amd import fde

    several = ("cgs_finalize", "mgc_y", "mgc_x", "transfer")
    return {f: [f] for f in fde.L.KFAM if f not in several}


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

    groups = kernel_groups(prec)

    def group_sum(prof, g):
        fams = groups[g]
        return {k: sum(prof[f][k] for f in fams) for k in ("launches", "ms", "bytes")}

    def dominant(prof):
        cand = {g: group_sum(prof, g) for g in groups}
        cand = {g: v for g, v in cand.items() if v["launches"] > 0}
        return max(cand, key=lambda g: cand[g]["ms"]) if cand else None

    # warmup, with every kernel family timed to find the dominant kernel
    fde.fde_profile_enable(h)
    run(warmup, "warmup")
    prof = fde.fde_profile_read(h)
    fam = profile_family or dominant(prof)
    fde.fde_profile_reset(h)
    # without warmup there is nothing to choose from: time every family in the timed run
    if fam is None:
        mask = (1 << len(fde.L.KFAM)) - 1
    else:
        mask = 0
        for f in groups[fam]:
            mask |= 1 << fde.L.KFAM.index(f)
        if fam == "cgs":  # wide passes' partials are combined by a separate one-workgroup kernel
            mask |= 1 << fde.L.KFAM.index("cgs_finalize")
    fde.fde_profile_enable(h, mask)
    # a sparse sample of the family's launches: every event pair costs the stream some microseconds
    fde.fde_profile_stride(h, PROFILE_STRIDE)
    elapsed, lat, its, reo, u_final = run(steps, "timed")
    timed = fde.fde_profile_read(h)
    if fam is None:
        prof = timed
        fam = dominant(timed)
    live = group_sum(timed, fam)
    fin = timed.get("cgs_finalize") if fam == "cgs" else None
    out = {"elapsed": elapsed, "lat": lat, "iters": its, "u": u_final.clone(), "family": fam,
           "live": live, "fin": fin, "warm_profile": prof, "reorth": reo}
    h.close()
    return out


def copy_bandwidth(nbytes=33521672, reps=20):
    """Device-to-device copy of a field (torch), timed with events: the practical HBM rate the
    streaming kernels are compared with besides the nominal peak (GB/s counting read + write)."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    return 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9


def family_rates(prof, n1, n2):
    """Per kernel family of a fully timed step: launches, mean duration and algorithmic GB/s; for the
    fine-level FFT passes also the transform arithmetic (5 L log2 L flops per complex transform, three
    transforms per pair of rows or columns) against the vector peak of their precision."""
    import math

    L1 = 1 << math.ceil(math.log2(2 * n1 - 1))
    L2 = 1 << math.ceil(math.log2(2 * n2 - 1))
    fft_flops = {"y": 3 * 5 * L2 * math.log2(L2) * math.ceil(n1 / 2),
                 "x": 3 * 5 * L1 * math.log2(L1) * math.ceil(n2 / 2)}
    out = {}
    for fam, v in prof.items():
        if not v["launches"] or v["ms"] <= 0:
            continue
        us = 1e3 * v["ms"] / v["launches"]
        r = {"launches": int(v["launches"]), "us_per_launch": round(us, 2)}
        if v["bytes"] > 0:
            gbs = v["bytes"] / v["launches"] / (us * 1e-6) / 1e9
            r["GB_s"] = round(gbs, 1)
            r["frac_hbm"] = round(gbs / HBM_PEAK_GBS, 4)
        if fam in ("outer_y", "outer_x", "mg0_y", "mg0_x"):
            fl = fft_flops[fam[-1]] / (us * 1e-6) / 1e12
            peak = FP64_VALU_PEAK_TFLOPS if fam.startswith("outer") else FP32_VALU_PEAK_TFLOPS
            r["fft_TFLOPs"] = round(fl, 2)
            r["frac_valu"] = round(fl / peak, 4)
        out[fam] = r
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

    threads = blas_threads()
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


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        return None


def c2_comparison(steps_gpu=32, steps_cpu=2):
    """The C2 workload (511^2, alpha = 1.8, beta = 1.6, variable coefficients, 32 CN steps, seed 2)
    on the GPU in full (FP32 V-cycle in FP64 GMRES, and plain FP64), and the oracle (its FGMRES(50)
    with its V-cycle to 1e-12) on the first steps with all host cores and with one thread; the GPU's
    state after those steps is compared with the oracle's."""
    import torch

    import workloads
    from oracle.cn import IterativeSolver, cn_run
    from paper_1706_06844_amd import fde

    p = workloads.config_c2(511, 32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    F = [d(f) for f in workloads.sample(p, 0.0)]
    phis, fields = workloads.source_terms(p)
    S = [d(f) for f in fields]
    u0 = d(workloads.sample_u0(p))
    gpu = {}
    for name, prec in (("mixed", fde.FDE_MIXED_FP32), ("fp64", fde.FDE_FP64)):
        h = fde.fde_setup(fde.fde_problem_default(p.alpha, p.beta, p.n1, p.n2, p.tau, precision=prec), *F)
        a, b = u0.clone(), torch.empty_like(u0)
        fde.fde_step_sources(h, a, [f(0.5 * p.tau) for f in phis], S, b)  # warm-up
        a.copy_(u0)
        its, early = [], None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for m in range(1, steps_gpu + 1):
            st = fde.fde_step_sources(h, a, [f((m - 0.5) * p.tau) for f in phis], S, b)
            its.append(st["iters"])
            a, b = b, a
            if m == steps_cpu:
                early = a.clone()
        torch.cuda.synchronize()
        gpu[name] = {"steps_per_s": steps_gpu / (time.perf_counter() - t0), "iters_per_step": float(np.mean(its)),
                     "early": early.cpu().numpy()}
        h.close()
    from threadpoolctl import threadpool_limits

    t0 = time.perf_counter()
    ref = cn_run(p, steps=steps_cpu, solver=IterativeSolver(rtol=1e-12)).u
    t_all = (time.perf_counter() - t0) / steps_cpu
    cores = blas_threads()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        cn_run(p, steps=1, solver=IterativeSolver(rtol=1e-12))
        t_one = time.perf_counter() - t0
    err = {k: float(np.linalg.norm(v["early"] - ref) / np.linalg.norm(ref)) for k, v in gpu.items()}
    return {"workload": "C2 511x511, alpha=1.8, beta=1.6, variable coefficients, tau=1/32, 32 CN steps, "
                        "manufactured + N(0,1) source (seed 2), rtol 1e-10",
            "gpu_mixed_steps_per_s": gpu["mixed"]["steps_per_s"], "gpu_fp64_steps_per_s": gpu["fp64"]["steps_per_s"],
            "gpu_mixed_iters_per_step": gpu["mixed"]["iters_per_step"],
            "gpu_fp64_iters_per_step": gpu["fp64"]["iters_per_step"],
            "oracle_steps_per_s": 1.0 / t_all, "oracle_cores": cores,
            "oracle_steps_per_s_1_thread": 1.0 / t_one,
            "oracle_sample": f"first {steps_cpu} steps with all cores, the first step with one thread",
            f"err_mixed_vs_oracle_after_{steps_cpu}_steps": err["mixed"],
            f"err_fp64_vs_oracle_after_{steps_cpu}_steps": err["fp64"]}


def exp_terms(p):
    """(coef, rate, fields) with phi_k(t) = coef_k exp(rate_k t) for the workload's source terms."""
    import math

    import workloads

    phis, fields = workloads.source_terms(p)
    coef, rate = [], []
    for f in phis:
        c0, c1 = float(f(0.0)), float(f(1.0))
        coef.append(c0)
        rate.append(math.log(c1 / c0) if c0 != 0.0 else 0.0)
    return coef, rate, fields


def host_request(p):
    import workloads

    coef, rate, fields = exp_terms(p)
    return {"p": p, "F": [np.ascontiguousarray(f) for f in workloads.sample(p, 0.0)], "S": fields,
            "u0": workloads.sample_u0(p), "coef": coef, "rate": rate}


def admit(b, hr, precision, rtol, maxit):
    import torch

    from paper_1706_06844_amd import fde

    p = hr["p"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    s = fde.fde_problem_default(p.alpha, p.beta, p.n1, p.n2, p.tau, precision=precision, rtol=rtol, maxit=maxit)
    s.a1, s.b1, s.a2, s.b2 = p.a1, p.b1, p.a2, p.b2
    F = [d(f) for f in hr["F"]]
    return fde.fde_batch_admit(b, s, *F, d(hr["u0"]), p.M, 0.0, hr["coef"], hr["rate"], [d(f) for f in hr["S"]])


def c4_results(modes=("mixed", "fp64", "cycle"), ungrouped=True, sequential=True, piece=0, slots=0):
    """C4: 64 uneven instances (n in {127,255,511}, 8 CN steps, rtol 1e-9) resident together.  Per
    precision mode: grouped batching (one group per size; every kernel of a restart cycle launched
    once over the solving members), optionally ungrouped batching (a stream and a graph per instance)
    and the instances one after another; grouped results are checked bitwise against the others."""
    import torch

    import workloads
    from paper_1706_06844_amd import fde

    precs = {"mixed": fde.FDE_MIXED_FP32, "fp64": fde.FDE_FP64, "cycle": fde.FDE_MIXED_FP32_CYCLE}
    probs = workloads.config_c4_instances(64, 4, 8)
    reqs = [host_request(p) for p in probs]
    # one group per size by default: as many slots as instances of the most frequent size
    slots = slots or max(sum(1 for p in probs if p.n1 == n) for n in {p.n1 for p in probs})

    marker = torch.empty(7, device="cuda:0")

    def batched(prec, grouped):
        # admission (resident setup, graph capture) outside the timed region; a fill of a small
        # tensor before and after it marks the region in kernel traces
        b = fde.fde_batch_create(200 << 30)
        if grouped:
            fde.fde_batch_set_grouping(b, 511, slots)
        fde.fde_batch_set_policy(b, 0, piece)
        ids = [admit(b, r, prec, 1e-9, 2000) for r in reqs]
        assert min(ids) >= 0
        marker.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while fde.fde_batch_step(b) > 0:
            pass
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        marker.fill_(2.0)
        finals, iters = [], 0
        for rid, p in zip(ids, probs):
            u = torch.empty((p.n2, p.n1), dtype=torch.float64, device="cuda:0")
            st, it = fde.fde_batch_poll(b, rid, u)
            assert st == 1, (rid, st)
            finals.append(u)
            iters += it
        b.close()
        return tb, finals, iters

    out = {"steps": sum(p.M for p in probs), "unknown_steps": sum(p.n1 * p.n2 * p.M for p in probs),
           "slots": slots}
    for name in modes:
        prec = precs[name]
        tg, finals, iters = batched(prec, True)
        r = {"grouped_s": tg, "iters": iters}
        if ungrouped:
            tb, ufinals, uiters = batched(prec, False)
            r["batched_s"] = tb
            r["grouped_equals_ungrouped"] = uiters == iters and all(bool(torch.equal(a, c))
                                                                    for a, c in zip(finals, ufinals))
        if sequential:
            # one resident instance at a time, same steps (setup outside the timed region)
            ts, maxdiff = 0.0, 0.0
            for r_, p, f in zip(reqs, probs, finals):
                b1 = fde.fde_batch_create(200 << 30)
                i1 = admit(b1, r_, prec, 1e-9, 2000)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                while fde.fde_batch_step(b1) > 0:
                    pass
                torch.cuda.synchronize()
                ts += time.perf_counter() - t1
                u = torch.empty((p.n2, p.n1), dtype=torch.float64, device="cuda:0")
                fde.fde_batch_poll(b1, i1, u)
                maxdiff = max(maxdiff, float((u - f).abs().max()))
                b1.close()
            r["sequential_s"] = ts
            r["max_diff_alone_vs_grouped"] = maxdiff
        out[name] = r
        log(f"c4 {name}: " + ", ".join(f"{k} {v:.3f}" if isinstance(v, float) else f"{k} {v}" for k, v in r.items()))
    return out


def c4_summary(c4):
    """The C4 keys of a JSON line: CN steps/s per mode and batching layout."""
    steps = c4["steps"]
    out = {"slots_per_group": c4["slots"]}
    for name in ("mixed", "fp64", "cycle"):
        if name not in c4:
            continue
        r = c4[name]
        out[f"{name}_grouped_steps_per_s"] = steps / r["grouped_s"]
        if "batched_s" in r:
            out[f"{name}_ungrouped_steps_per_s"] = steps / r["batched_s"]
            out[f"{name}_grouped_equals_ungrouped"] = r["grouped_equals_ungrouped"]
        if "sequential_s" in r:
            out[f"{name}_one_at_a_time_steps_per_s"] = steps / r["sequential_s"]
            out[f"{name}_max_diff_alone_vs_grouped"] = r["max_diff_alone_vs_grouped"]
        out[f"{name}_iters"] = r["iters"]
    if "mixed" in c4 and "fp64" in c4:
        out["mixed_speedup_vs_fp64"] = c4["fp64"]["grouped_s"] / c4["mixed"]["grouped_s"]
    return out


def run_c4(args):
    """The C4 line: the value is grouped batching with the FP32 V-cycle inside FP64 flexible GMRES."""
    c4 = c4_results(modes=tuple(args.c4_modes.split(",")), ungrouped=not args.c4_grouped_only,
                    sequential=not args.c4_grouped_only, piece=args.c4_piece, slots=args.c4_slots)
    name = "mixed" if "mixed" in c4 else args.c4_modes.split(",")[0]
    m = c4[name]
    line = {
        "metric": "C4 batched CN steps/s (64 uneven instances, FP32 V-cycle in FP64 FGMRES)"
                  if name == "mixed" else f"C4 batched CN steps/s (64 uneven instances, {name})",
        "value": c4["steps"] / m["grouped_s"], "unit": "CN steps/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "C4: 64 instances (seed 4), n in {127,255,511}, alpha,beta ~ U[1.1,1.9], "
                               "c(1+ax+by^2) coefficients, tau=1/8, 8 CN steps, rtol 1e-9",
                   "precision": "FP32 V-cycle in FP64 flexible GMRES (cycle: FP32 restart cycles refining "
                                "the FP64 iterate from FP64 true residuals)",
                   "batching": "grouped: one group per size, every restart-cycle kernel launched once over "
                               "the solving members"},
        "unknown_updates_per_s": c4["unknown_steps"] / m["grouped_s"],
    }
    line.update(c4_summary(c4))
    print(json.dumps(line), flush=True)


def serve(reqs, prec, budget, warm, max_running=0, group=(0, 0), piece=0, busy_running=-1, lanes=0):
    """Continuous batching: requests join the batch as they arrive and memory allows; returns the
    measured requests' latencies (arrival -> result copied out), their grid sides and the span.
    max_running caps the ungrouped requests with a cycle piece in flight (least work left first);
    piece > 0 issues restart cycles in pieces of that many Arnoldi steps; group = (max_n, slots)
    shares batched launches among requests of one shape up to max_n; busy_running caps the ungrouped
    requests with a piece in flight while a group has work (-1: no extra cap)."""
    import torch

    from paper_1706_06844_amd import fde

    b = fde.fde_batch_create(budget)
    if lanes:
        fde.fde_batch_set_lanes(b, lanes)
    if group[0] > 0:
        fde.fde_batch_set_grouping(b, group[0], group[1])
    fde.fde_batch_set_policy(b, max_running, piece, busy_running)
    pending = sorted(range(len(reqs)), key=lambda i: reqs[i]["arrival"])
    queue, inflight, lat, done_t = [], {}, {}, {}
    t_start = time.perf_counter()
    while pending or queue or inflight:
        now = time.perf_counter() - t_start
        while pending and reqs[pending[0]]["arrival"] <= now:
            queue.append(pending.pop(0))
        while queue:
            i = queue[0]
            rid = admit(b, reqs[i]["hr"], prec, 1e-9, 4000)
            if rid == fde.FDE_EAGAIN:
                if not inflight:
                    raise RuntimeError("a request does not fit the budget on its own")
                break
            inflight[rid] = i
            queue.pop(0)
        if not inflight:
            if pending:
                time.sleep(max(0.0, reqs[pending[0]]["arrival"] - (time.perf_counter() - t_start)))
            continue
        fde.fde_batch_step(b)
        for rid, i in list(inflight.items()):
            if fde.fde_batch_poll(b, rid)[0] == 0:  # status only: no output buffer per poll
                continue
            p = reqs[i]["hr"]["p"]
            u = torch.empty((p.n2, p.n1), dtype=torch.float64, device="cuda:0")
            st, _ = fde.fde_batch_poll(b, rid, u)
            if st:
                t = time.perf_counter() - t_start
                lat[i] = t - reqs[i]["arrival"]
                done_t[i] = t
                del inflight[rid]
                if len(done_t) % 10 == 0:
                    log(f"c5 serve: {len(done_t)} of {len(reqs)} requests done at {t:.0f} s")
    b.close()
    meas = [i for i in range(len(reqs)) if i >= warm]
    span = max(done_t[i] for i in meas) - min(reqs[i]["arrival"] for i in meas)
    return [lat[i] for i in meas], [reqs[i]["hr"]["p"].n1 for i in meas], span


def latency_stats(lat, sides, solo=None):
    """p50/p99 over all measured requests and per grid side (ms); with the requests' latencies alone
    on the device (solo), also of the slowdown latency / solo latency."""
    lat_ms = np.array(lat) * 1e3
    out = {"p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99))}
    sl = None if solo is None else np.array(lat) / np.array(solo)
    if sl is not None:
        out["slowdown_p50"] = float(np.percentile(sl, 50))
        out["slowdown_p99"] = float(np.percentile(sl, 99))
    per = {}
    for n in sorted(set(sides)):
        idx = [j for j, m in enumerate(sides) if m == n]
        v = lat_ms[idx]
        per[str(n)] = {"count": int(v.size), "p50_ms": float(np.percentile(v, 50)),
                       "p99_ms": float(np.percentile(v, 99))}
        if sl is not None:
            per[str(n)]["slowdown_p50"] = float(np.percentile(sl[idx], 50))
            per[str(n)]["slowdown_p99"] = float(np.percentile(sl[idx], 99))
    out["by_side"] = per
    return out


def run_c5(args):
    """Served requests (Poisson arrivals, seed 5): n = 2^k - 1 with k uniform in 6..kmax, 8..128
    steps each; solves/s, CN steps/s, p50/p99 latency overall and per grid side.  Requests up to
    511^2 share grouped launches; restart cycles are issued in pieces of --c5-piece Arnoldi steps and
    the larger requests are scheduled least-work-first with at most --c5-max-running pieces in
    flight.  Runs: each request alone, saturation (all requests at t = 0), then the --c5-loads
    fractions of the saturation rate with that policy (default 90 %); with --c5-compare also, at the
    highest load, the other busy cap, the plain policy (whole cycles, every due cycle issued at once)
    and FP64.
    Slowdowns divide each request's latency by its latency alone on the device (mixed precision)."""
    import workloads

    warm = args.c5_warmup
    count = warm + args.c5_count
    ks = tuple(range(6, args.c5_kmax + 1))
    base = workloads.config_c5_requests(1.0, count=count, seed=5, ks=ks)
    hrs = [host_request(r.problem) for r in base]
    gaps = np.diff([0.0] + [r.arrival for r in base])  # arrivals at qps 1; scaled per run
    budget = 200 << 30
    group = (511, 16)

    def reqs_at(qps):
        t = np.cumsum(gaps) / qps
        return [{"hr": hrs[i], "arrival": float(t[i])} for i in range(count)]

    from paper_1706_06844_amd import fde

    steps_meas = sum(hrs[i]["p"].M for i in range(warm, count))
    cap, piece, gf, lanes = args.c5_max_running, args.c5_piece, args.c5_busy_running, args.c5_lanes
    # every measured request alone on the device, one after another in one batch (so that groups,
    # once created, are reused as in the loaded runs): the reference for slowdowns
    import torch

    solo = []
    b = fde.fde_batch_create(budget)
    fde.fde_batch_set_grouping(b, group[0], group[1])
    fde.fde_batch_set_policy(b, 0, piece)
    for i in range(count):
        t0 = time.perf_counter()
        rid = admit(b, hrs[i], fde.FDE_MIXED_FP32, 1e-9, 4000)
        while fde.fde_batch_step(b) > 0:
            pass
        p = hrs[i]["p"]
        u = torch.empty((p.n2, p.n1), dtype=torch.float64, device="cuda:0")
        st, _ = fde.fde_batch_poll(b, rid, u)
        assert st >= 1, (i, st)
        if i >= warm:
            solo.append(time.perf_counter() - t0)
        if (i + 1) % 10 == 0:
            log(f"c5 solo: {i + 1} of {count} requests done")
    b.close()
    log(f"c5 solo: {sum(solo):.1f} s in all, largest {max(solo):.1f} s")
    mix = {str(2 ** k - 1): sum(1 for i in range(warm, count) if hrs[i]["p"].n1 == 2 ** k - 1) for k in ks}
    lat0, sides0, span0 = serve(reqs_at(1e9), fde.FDE_MIXED_FP32, budget, warm, cap, group, piece, gf, lanes)
    sat = args.c5_count / span0
    log(f"c5 saturation: {sat:.3f} solves/s ({span0:.1f} s)")
    loads = [float(f) for f in args.c5_loads.split(",")]
    rates = [f * sat for f in loads] if args.c5_qps == "auto" else [float(q) for q in args.c5_qps.split(",")]
    plan = [(q, "mixed", cap, piece, gf) for q in rates]
    if args.c5_qps == "auto" and args.c5_compare:
        # at 90 %: the other busy cap (0 if it is set, else 1), the plain policy and FP64
        plan += [(rates[-1], "mixed", cap, piece, 0 if gf != 0 else 1),
                 (rates[-1], "mixed", 0, 0, -1), (rates[-1], "fp64", cap, piece, gf)]
    runs = []
    for qps, name, mr, pc, g1 in plan:
        prec = fde.FDE_MIXED_FP32 if name == "mixed" else fde.FDE_FP64
        lat, sides, span = serve(reqs_at(qps), prec, budget, warm, mr, group, pc, g1, lanes if mr else 0)
        r = {"qps": qps, "precision": name, "max_running": mr, "piece_steps": pc, "busy_running": g1,
             "solves_per_s": args.c5_count / span, "cn_steps_per_s": steps_meas / span}
        r.update(latency_stats(lat, sides, solo if name == "mixed" else None))
        runs.append(r)
        log(f"c5 qps {qps:.3f} {name} max_running {mr} piece {pc} busy_running {g1}: "
            f"{args.c5_count / span:.3f} solves/s, "
            f"p50 {r['p50_ms']:.0f} ms, p99 {r['p99_ms']:.0f} ms")
    hi = [r for r in runs if r["precision"] == "mixed" and r["max_running"] == cap and r["piece_steps"] == piece
          and r["busy_running"] == gf][-1]
    line = {
        "metric": "C5 served solves/s with p50/p99 latency (continuous batching, mixed vs FP64)",
        "value": hi["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"C5: Poisson arrivals (seed 5), {args.c5_count} measured requests after "
                               f"{warm} warm-up, n = 2^k - 1 with k in 6..{args.c5_kmax}, 8..128 CN "
                               "steps each (tau = 1/M), rtol 1e-9, FP32 V-cycle in FP64 FGMRES",
                   "request_mix": mix,
                   "policy": f"sides <= 511 grouped (16 slots); restart cycles in pieces of {piece} Arnoldi "
                             f"steps; larger requests least work left first, at most {cap} with a piece in "
                             f"flight, {gf} while a group has work (the 'plain' run: whole cycles, no cap)"},
        "saturation_solves_per_s": sat, "saturation_cn_steps_per_s": steps_meas / span0,
        "saturation_latency": latency_stats(lat0, sides0, solo), "runs": runs,
        "solo_latency": latency_stats(solo, sides0),
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); independent instances "
              "would be sharded across GPUs without communication, which this benchmark does not "
              "measure.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads
    from paper_1706_06844_amd import fde

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c5":
        return run_c5(args)
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
    order = [("cycle16", fde.FDE_MIXED_CYCLE_BF16), ("cycle", fde.FDE_MIXED_FP32_CYCLE), ("mixed", fde.FDE_MIXED_FP32),
             ("fp64", fde.FDE_FP64), ("bf16", fde.FDE_MIXED_BF16GEMM)]
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
    # the value: the FP32 V-cycle inside FP64 flexible GMRES (FP64 basis, Arnoldi products, inner
    # products, Givens and true residuals); the FP32-cycle modes are reported beside it
    main_name = next(k for k in ("mixed", "cycle16", "cycle", "fp64", "bf16") if k in res)
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
        "dtype": {"cycle16": "f64+f32+bf16", "cycle": "f64+f32", "mixed": "f64+f32", "fp64": "f64",
                  "bf16": "f64+f32+bf16"}[main_name],
        "data": "synthetic",
        "config": {"workload": f"C3 anisotropic instance {args.n}x{args.n}, alpha=1.2, beta=1.9, "
                               "C2 variable coefficients, tau=1/16, manufactured + N(0,1) source "
                               "(seed 3)",
                   "precision": {"cycle16": "FP32 V-cycle and FP32 restart cycles (Arnoldi products, "
                                            "orthogonalisation; basis stored in BF16) refining the FP64 iterate "
                                            "from FP64 true residuals",
                                 "cycle": "FP32 V-cycle and FP32 restart cycles (basis, Arnoldi products) "
                                          "refining the FP64 iterate from FP64 true residuals",
                                 "mixed": "FP32 V-cycle in FP64 flexible GMRES", "fp64": "FP64",
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
    if m.get("fin") and m["fin"]["launches"]:
        f = m["fin"]
        us_fin = 1e3 * f["ms"] / f["launches"]
        stage_us = 1e3 * ms_per_launch + us_fin
        out["roofline"]["finalize_us_per_launch"] = us_fin
        # the whole Gram-Schmidt stage: pass plus the combination of its partials
        out["roofline"]["stage_achieved_with_finalize"] = bytes_per_launch / (stage_us * 1e-6) / 1e9
    ref = res["fp64"]["u"] if "fp64" in res else None

    def err_vs_fp64(r):
        return float(torch.linalg.norm((r["u"] - ref).double()) / torch.linalg.norm(ref))

    if ref is not None and main_name != "fp64":
        out["err_vs_fp64"] = err_vs_fp64(m)
    for name, r in res.items():
        if name == main_name:
            continue
        out[f"{name}_value"] = args.steps / r["elapsed"]
        out[f"{name}_ms_per_step"] = 1e3 * r["elapsed"] / args.steps
        out[f"{name}_iters_per_step"] = float(np.mean(r["iters"]))
        out[f"{name}_p50_ms"] = float(np.percentile(np.array(r["lat"]) * 1e3, 50))
        out[f"{name}_p99_ms"] = float(np.percentile(np.array(r["lat"]) * 1e3, 99))
        if ref is not None and name != "fp64":
            out[f"err_{name}_vs_fp64"] = err_vs_fp64(r)
        out[f"{name}_warm_profile_ms"] = {k: round(v["ms"], 3) for k, v in r["warm_profile"].items()}
    if "fp64" in res and main_name != "fp64":
        out["speedup_vs_fp64"] = out["value"] / out["fp64_value"]
    out["warm_profile_ms"] = {k: round(v["ms"], 3) for k, v in m["warm_profile"].items()}
    # every family of one fully timed step (events around each launch, so slightly slower than the
    # timed run): rates against HBM and, for the fine-level transforms, against the vector peak
    out["family_rates"] = family_rates(m["warm_profile"], p.n1, p.n2)
    copy_gbs = copy_bandwidth()
    out["roofline"]["copy_GB_s"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(p, out["iters_per_step"], args.cpu_sample_iters)
    if not args.no_c2:
        log("c2: 511^2 on the GPU (32 steps) and the oracle (2 steps all cores, 1 step one thread)")
        out["c2"] = c2_comparison()
    if not args.no_c4:
        log("c4: 64 batched instances, grouped (mixed, fp64) and ungrouped (mixed)")
        c4 = c4_results(modes=("mixed",), ungrouped=True, sequential=False)
        c4.update(c4_results(modes=("fp64",), ungrouped=False, sequential=False))
        out["c4"] = c4_summary(c4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
