"""Parity of the benchmarked path at full size and over whole runs.

* The FP32 fine-level operator of the 2047^2 anisotropic instance (length-4096 transforms, the plan
  the benchmark runs) in its three epilogues -- y = A x, r = b - A x, and the damped-Jacobi update --
  element by element against the oracle's FP64 operator of eq. (AxAy) / (system).
* The FP32 V-cycle (Sec. 4 V-cycle with the Sec. 4.2 settings) at 1023^2 and 2047^2 against the
  oracle's V-cycle.
* The BF16 MFMA passes at 2047^2 against an FP64 evaluation of the same BF16-rounded factors.
* The 511^2 analogue of the anisotropic instance (alpha = 1.2, beta = 1.9, same coefficients and
  time step): one CN step in every precision against the oracle's solve of eq. (system).
* All 32 steps of the 511^2 C2 run against the oracle's run, at the samples stored by
  tests/golden/make_c2_oracle_samples.py.

Tolerances, from the arithmetic: an FP32 length-L transform product loses about u32 log2(L) in
relative 2-norm (u32 = 6e-8, log2 4096 = 12), so the FP32 operator must match to 2e-6; a V-cycle is a
short chain of such products, 1e-5; solves stop on the FP64 true residual 1e-10, and the solution
must match the oracle to 1e-9 (relative 2-norm), as for every other solve.
"""
import json
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import multigrid as omg
from oracle.cn import IterativeSolver, cn_run
from oracle.operator import operator_from_problem
from paper_1706_06844_amd import fde

from .gpu_util import dev, host, make_handle, note, rel

pytestmark = pytest.mark.gpu

F32 = fde.FDE_MIXED_FP32
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.fixture(scope="module")
def c3_fine():
    p = workloads.config_c3(2047, 16)
    h = make_handle(p, precision=F32, maxit=4000)
    op = operator_from_problem(p, 0.0)
    yield p, h, op
    h.close()


def _check_fp32(got, ref, what):
    e2 = rel(got, ref)
    emax = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    note(f"{what}: rel 2-norm {e2:.2e}, max {emax:.2e}")
    assert e2 <= 2e-6 and emax <= 1e-5


def test_fp32_fine_apply_2047(c3_fine):
    p, h, op = c3_fine
    U = _rand((2047, 2047), 31)
    y = dev(np.zeros_like(U))
    fde.fde_apply(h, 0, F32, dev(U), y)
    _check_fp32(host(y), op.apply(U), "FP32 2047 apply")


def test_fp32_fine_residual_2047(c3_fine):
    p, h, op = c3_fine
    U, B = _rand((2047, 2047), 32), _rand((2047, 2047), 33)
    r = dev(np.zeros_like(U))
    fde.fde_residual(h, 0, F32, dev(B), dev(U), r)
    _check_fp32(host(r), B - op.apply(U), "FP32 2047 residual")


def test_fp64_outer_residual_2047(c3_fine):
    # the FP64 operator's residual epilogue (true residuals of every restart cycle)
    p, h, op = c3_fine
    U, B = _rand((2047, 2047), 34), _rand((2047, 2047), 35)
    r = dev(np.zeros_like(U))
    fde.fde_residual(h, 0, fde.FDE_FP64, dev(B), dev(U), r)
    ref = B - op.apply(U)
    assert rel(host(r), ref) <= 1e-12


def test_fp32_fine_jacobi_2047(c3_fine):
    p, h, op = c3_fine
    X0, B = _rand((2047, 2047), 36), _rand((2047, 2047), 37)
    x = dev(X0)
    fde.fde_smooth(h, 0, F32, dev(B), x, False)
    _check_fp32(host(x), omg.jacobi(op, B, X0, 0.7), "FP32 2047 Jacobi")
    x0 = dev(X0)
    fde.fde_smooth(h, 0, F32, dev(B), x0, True)
    _check_fp32(host(x0), omg.jacobi(op, B, np.zeros_like(B), 0.7), "FP32 2047 Jacobi from zero")


@pytest.mark.parametrize("n", [1023, 2047])
def test_fp32_vcycle_full_size(n):
    note(f"FP32 V-cycle {n}^2")
    p = workloads.config_c3(n, 16)
    h = make_handle(p, precision=F32, maxit=4000)
    vc = omg.VCycle(omg.geometric_hierarchy(operator_from_problem(p, 0.0)))
    B = _rand((n, n), 41)
    x = dev(np.zeros_like(B))
    fde.fde_vcycle(h, dev(B), x)
    e = rel(host(x), vc(B))
    note(f"FP32 V-cycle {n}^2: rel 2-norm {e:.2e}")
    assert e <= 1e-5
    h.close()


def test_bf16_fine_apply_2047():
    from .test_gpu_bf16 import bf16_level_apply

    p = workloads.config_c3(2047, 16)
    h = make_handle(p, precision=fde.FDE_MIXED_BF16GEMM, maxit=4000)
    L = omg.geometric_hierarchy(operator_from_problem(p, 0.0))[0]
    U = _rand((2047, 2047), 43)
    y = dev(np.zeros_like(U))
    fde.fde_apply(h, 0, F32, dev(U), y)
    got = host(y)
    e = rel(got, bf16_level_apply(L, U))
    note(f"BF16 MFMA 2047 apply vs rounded factors: {e:.2e}")
    assert e <= 2e-6
    h.close()


# ---- the anisotropic instance at 511^2: one CN step in every precision ----
ALL_PRECS = [fde.FDE_FP64, fde.FDE_MIXED_FP32, fde.FDE_MIXED_FP32_CYCLE, fde.FDE_MIXED_CYCLE_BF16,
             fde.FDE_MIXED_BF16GEMM]


@pytest.fixture(scope="module")
def c3_511_oracle():
    p = workloads.config_c3(511, 16)
    note("oracle: one C3-analogue step at 511^2 (rtol 1e-12)")
    return p, cn_run(p, steps=1, solver=IterativeSolver(rtol=1e-12, maxit=3000)).u


@pytest.mark.parametrize("prec", ALL_PRECS)
def test_c3_analogue_511_step_matches_oracle(prec, c3_511_oracle):
    p, ref = c3_511_oracle
    h = make_handle(p, precision=prec, maxit=4000)
    phis, fields = workloads.source_terms(p)
    un = dev(np.zeros((p.n2, p.n1)))
    st = fde.fde_step_sources(h, dev(workloads.sample_u0(p)), [f(0.5 * p.tau) for f in phis],
                              [dev(f) for f in fields], un)
    e = rel(host(un), ref)
    note(f"C3 analogue 511^2 prec={prec}: {st['iters']} iterations, rel err vs oracle {e:.2e}")
    assert st["converged"] and st["relres_true"] <= 1e-10
    assert e <= 1e-9
    h.close()


# ---- all 32 steps of C2 against the oracle's run (stored samples) ----
def _golden_c2():
    with open(os.path.join(GOLDEN, "c2_oracle_32_steps.json")) as f:
        return json.load(f)


def _golden_script():
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_c2_oracle_samples",
                                                  os.path.join(GOLDEN, "make_c2_oracle_samples.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _compare_reduced(u, g, what):
    gs = _golden_script()
    probes, sample_points = gs.probes, gs.sample_points
    js, is_ = sample_points(*u.shape)
    ref = np.array(g["values"])
    rms = g["norm2"] / np.sqrt(u.size)
    e_pts = np.max(np.abs(u[js, is_] - ref)) / rms
    e_norm = abs(np.linalg.norm(u) - g["norm2"]) / g["norm2"]
    e_probe = max(abs(np.vdot(q, u) - r) / (np.linalg.norm(q) * g["norm2"])
                  for q, r in zip(probes(*u.shape), g["probes"]))
    note(f"{what}: samples {e_pts:.2e} (of rms), norm {e_norm:.2e}, probes {e_probe:.2e}")
    assert e_pts <= 1e-9 and e_norm <= 1e-9 and e_probe <= 1e-9


@pytest.mark.parametrize("prec", [fde.FDE_FP64, fde.FDE_MIXED_FP32])
def test_c2_all_32_steps_match_oracle(prec):
    g = _golden_c2()
    p = workloads.config_c2(511, 32)
    h = make_handle(p, precision=prec)
    phis, fields = workloads.source_terms(p)
    S = [dev(f) for f in fields]
    u = dev(workloads.sample_u0(p))
    un = torch.empty_like(u)
    for m in range(1, 33):
        st = fde.fde_step_sources(h, u, [f((m - 0.5) * p.tau) for f in phis], S, un)
        assert st["converged"], (m, st)
        u, un = un, u
        if m == 16:
            _compare_reduced(host(u), g["step16"], f"C2 step 16 prec={prec}")
    _compare_reduced(host(u), g["step32"], f"C2 step 32 prec={prec}")
    h.close()
