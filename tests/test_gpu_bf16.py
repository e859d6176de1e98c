"""BF16 MFMA operator passes (FP32 accumulation) of the V-cycle against the oracle.

Exactness pin: the kernels multiply BF16-rounded field values by BF16-rounded scaled weights and
accumulate in FP32, so they must agree with an FP64 evaluation of the same rounded factors to FP32
accuracy.  Against the unrounded operator they agree to BF16 accuracy; inside flexible GMRES the
solution still meets the FP64 tolerance.
"""
import numpy as np
import pytest

import workloads
from oracle import multigrid as omg
from oracle.cn import IterativeSolver, rhs, solve_step
from oracle.operator import operator_from_problem
from oracle.weights import wsgd
from paper_1706_06844_amd import fde

from .gpu_util import dev, host, make_handle, note, rel

pytestmark = pytest.mark.gpu

BF = fde.FDE_MIXED_BF16GEMM
F32 = fde.FDE_MIXED_FP32


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def bf16_round(a):
    """Round float64 values to BF16 (through FP32, ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def toeplitz_from(wv, n):
    i = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    m = i - k + 1
    return np.where((m >= 0) & (m <= n), wv[np.clip(m, 0, n)], 0.0)


def bf16_level_apply(L, U):
    """A x with the BF16-rounded factors the MFMA kernels use (FP64 arithmetic otherwise)."""
    sx = 0.5 * L.tau / L.hx ** L.alpha
    sy = 0.5 * L.tau / L.hy ** L.beta
    Tx = toeplitz_from(bf16_round(sx * wsgd(L.alpha, L.n1)), L.n1)
    Ty = toeplitz_from(bf16_round(sy * wsgd(L.beta, L.n2)), L.n2)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Ub = bf16_round(U)
    lx = f32(L.dp) * (Ub @ Tx.T) + f32(L.dm) * (Ub @ Tx)
    ly = f32(L.ep) * (Ty @ Ub) + f32(L.em) * (Ty.T @ Ub)
    return f32(U) - (lx + ly)


@pytest.mark.parametrize("n1,n2", [(511, 511), (1023, 1023), (511, 1023)])
def test_bf16_level_apply_matches_rounded_factors(n1, n2):
    note(f"bf16 apply {n1}x{n2}")
    p = workloads.config_c3(n1, 16)
    p.n2 = n2
    h = make_handle(p, precision=BF)
    L = omg.geometric_hierarchy(operator_from_problem(p, 0.0))[0]
    U = _rand((n2, n1), 5)
    y = dev(np.zeros_like(U))
    fde.fde_apply(h, 0, F32, dev(U), y)
    got = host(y)
    assert rel(got, bf16_level_apply(L, U)) <= 2e-6
    assert rel(got, L.apply(U)) <= 2e-2  # BF16 against the exact operator


def test_bf16_smoother_and_residual():
    n = 511
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=BF)
    L = omg.geometric_hierarchy(operator_from_problem(p, 0.0))[0]
    B, X0 = _rand((n, n), 1), _rand((n, n), 2)
    x = dev(X0)
    fde.fde_smooth(h, 0, F32, dev(B), x, False)
    d = dev(np.zeros_like(B))
    fde.fde_level_diag(h, 0, d)
    dinv = 0.7 / host(d)
    ref = X0 + dinv * (B - bf16_level_apply(L, X0))
    assert rel(host(x), ref) <= 2e-6


@pytest.mark.parametrize("n", [511, 1023])
def test_bf16_vcycle_close_to_fp32(n):
    p = workloads.config_c2(n, 32)
    B = _rand((n, n), 9)
    out = {}
    for prec in (F32, BF):
        h = make_handle(p, precision=prec)
        x = dev(np.zeros_like(B))
        fde.fde_vcycle(h, dev(B), x)
        out[prec] = host(x)
    note(f"bf16 vs fp32 vcycle n={n}: {rel(out[BF], out[F32]):.2e}")
    assert rel(out[BF], out[F32]) <= 2e-2


def test_bf16_c2_step_matches_oracle():
    n = 511
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=BF)
    op = operator_from_problem(p, 0.0)
    u0 = workloads.sample_u0(p)
    v = workloads.sample_source(p, 0.5 * p.tau)
    un = dev(np.zeros_like(u0))
    st = fde.fde_step(h, dev(u0), dev(v), un)
    assert st["converged"]
    note(f"bf16 C2 step: {st['iters']} iterations")
    ref = solve_step(op, rhs(op, u0, v), IterativeSolver(rtol=1e-12))
    assert rel(host(un), ref) <= 1e-9


def test_bf16_c3_step_matches_fp64_gpu():
    n = 2047
    p = workloads.config_c3(n, 16)
    u0 = workloads.sample_u0(p)
    v = workloads.sample_source(p, 0.5 * p.tau)
    res, its = {}, {}
    for prec in (fde.FDE_FP64, BF):
        h = make_handle(p, precision=prec, maxit=4000)
        un = dev(np.zeros_like(u0))
        st = fde.fde_step(h, dev(u0), dev(v), un)
        assert st["converged"]
        res[prec], its[prec] = host(un), st["iters"]
        h.close()
    note(f"C3 step iterations fp64 {its[fde.FDE_FP64]} bf16 {its[BF]}")
    assert rel(res[BF], res[fde.FDE_FP64]) <= 1e-9
