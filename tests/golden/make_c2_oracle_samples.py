"""Writes c2_oracle_32_steps.json: the oracle's C2 run (511^2, alpha = 1.8, beta = 1.6, variable
coefficients, tau = 1/32, all 32 CN steps of eq. (system), manufactured + N(0,1) source with seed 2)
reduced to what a test can compare with a GPU run: the 2-norm of u^(16) and u^(32), their values at
2048 seeded sample points, and their inner products with four seeded N(0,1) probe fields.

Calls only the oracle (its FGMRES(50) with its geometric V-cycle to relative residual 1e-12, the
tightest it reaches at 511^2) and the seeded input generators.  Run from the repository root:
    python tests/golden/make_c2_oracle_samples.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle.cn import IterativeSolver, cn_run  # noqa: E402

SAMPLE_SEED = 20
PROBE_SEEDS = (21, 22, 23, 24)
N_SAMPLES = 2048


def sample_points(n2, n1):
    rng = np.random.default_rng(SAMPLE_SEED)
    js = np.concatenate([[0, 0, n2 - 1, n2 - 1], rng.integers(0, n2, N_SAMPLES - 4)])
    is_ = np.concatenate([[0, n1 - 1, 0, n1 - 1], rng.integers(0, n1, N_SAMPLES - 4)])
    return js, is_


def probes(n2, n1):
    return [np.random.default_rng(s).standard_normal((n2, n1)) for s in PROBE_SEEDS]


def reduce_field(u):
    js, is_ = sample_points(*u.shape)
    return {"norm2": float(np.linalg.norm(u)), "values": [float(v) for v in u[js, is_]],
            "probes": [float(np.vdot(q, u)) for q in probes(*u.shape)]}


def main():
    p = workloads.config_c2(511, 32)
    solver = IterativeSolver(rtol=1e-12)
    t0 = time.perf_counter()
    half = cn_run(p, steps=16, solver=solver)
    full = cn_run(p, steps=16, solver=solver, u0=half.u, t0=16 * p.tau)
    out = {"workload": "C2 511x511, alpha=1.8, beta=1.6, tau=1/32, noise seed 2",
           "solver": "oracle FGMRES(50) + geometric V(1,1), rtol 1e-12",
           "sample_seed": SAMPLE_SEED, "probe_seeds": list(PROBE_SEEDS), "n_samples": N_SAMPLES,
           "oracle_iters": half.iters + full.iters,
           "step16": reduce_field(half.u), "step32": reduce_field(full.u)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_32_steps.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} in {time.perf_counter() - t0:.1f} s")


if __name__ == "__main__":
    main()
