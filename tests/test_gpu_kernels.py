"""Kernel-level parity of the HIP path against the FP64 oracle.

Each call goes through the C ABI (libfde) via the Python binding; the expected values come from the
oracle only.  FP64 results must agree to rounding (1e-12 relative 2-norm for the FFT operator, as
required for the FFT-versus-direct matvec); FP32 results to what single precision allows (1e-5).
"""
import numpy as np
import pytest

import workloads
from oracle import multigrid as omg
from oracle.operator import operator_from_problem
from paper_1706_06844_amd import fde

from .gpu_util import dev, host, make_handle, note, rel

pytestmark = pytest.mark.gpu


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("n", [7, 15, 31, 63, 127, 255, 511])
def test_outer_apply_fp64_matches_oracle(n):
    note(f"outer apply fp64 n={n}")
    p = workloads.config_c2(n, 32)
    h = make_handle(p)
    op = operator_from_problem(p, 0.0)
    U = _rand((n, n), n)
    y = dev(np.zeros((n, n)))
    fde.fde_apply(h, 0, fde.FDE_FP64, dev(U), y)
    assert rel(host(y), op.apply(U)) <= 1e-12


@pytest.mark.parametrize("n1,n2", [(63, 127), (127, 63), (31, 63)])
def test_outer_apply_rectangular(n1, n2):
    note(f"outer apply rect {n1}x{n2}")
    p = workloads.config_c2(n1, 32)
    p.n2 = n2
    h = make_handle(p)
    op = operator_from_problem(p, 0.0)
    U = _rand((n2, n1), 7)
    y = dev(np.zeros((n2, n1)))
    fde.fde_apply(h, 0, fde.FDE_FP64, dev(U), y)
    assert rel(host(y), op.apply(U)) <= 1e-12


def test_outer_apply_smooth_input_relative_to_abs_operator():
    # On smooth inputs the weights' zero sum cancels; compare against |A||x| as well.
    n = 255
    p = workloads.config_c3(n, 16)
    h = make_handle(p)
    op = operator_from_problem(p, 0.0)
    X, Y = workloads.grid(p)
    U = np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    y = dev(np.zeros((n, n)))
    fde.fde_apply(h, 0, fde.FDE_FP64, dev(U), y)
    ref = op.apply(U)
    absop = np.abs(U) + 0.5 * p.tau * (
        op.dp * (np.abs(U) @ np.abs(op.Tx.T)) + op.dm * (np.abs(U) @ np.abs(op.Tx))
        + op.ep * (np.abs(op.Ty) @ np.abs(U)) + op.em * (np.abs(op.Ty.T) @ np.abs(U)))
    assert np.max(np.abs(host(y) - ref) / absop) <= 1e-13


def test_outer_apply_2047_sampled():
    note("outer apply 2047 sampled")
    n = 2047
    p = workloads.config_c3(n, 16)
    h = make_handle(p)
    op = operator_from_problem(p, 0.0)
    U = _rand((n, n), 3)
    y = dev(np.zeros((n, n)))
    fde.fde_apply(h, 0, fde.FDE_FP64, dev(U), y)
    rng = np.random.default_rng(11)
    js = np.concatenate([[0, 0, n - 1, n - 1, 1023], rng.integers(0, n, 60)])
    is_ = np.concatenate([[0, n - 1, 0, n - 1, 1024], rng.integers(0, n, 60)])
    ref = op.apply_points(U, js, is_)
    got = host(y)[js, is_]
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("prec", [fde.FDE_FP64, fde.FDE_MIXED_FP32])
def test_level_operators_match_geometric_hierarchy(prec):
    n = 255
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec)
    lv = omg.geometric_hierarchy(operator_from_problem(p, 0.0))
    assert fde.fde_num_levels(h) == len(lv)
    tol = 1e-12 if prec == fde.FDE_FP64 else 2e-6
    for l, L in enumerate(lv):
        note(f"level {l} apply prec={prec}")
        assert fde.fde_level_size(h, l) == (L.n1, L.n2)
        U = _rand((L.n2, L.n1), 100 + l)
        y = dev(np.zeros_like(U))
        fde.fde_apply(h, l, prec, dev(U), y)
        assert rel(host(y), L.apply(U)) <= tol, l
        d = dev(np.zeros_like(U))
        fde.fde_level_diag(h, l, d)
        np.testing.assert_allclose(host(d), L.diag(), rtol=1e-14 if prec == fde.FDE_FP64 else 1e-6)


def test_fp32_fft_levels_match_geometric_hierarchy():
    # the FFT passes of the FP32 levels 1023^2 (length 2048) and 511^2 (length 1024): each length
    # has its own elements-per-thread plan
    n = 1023
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=fde.FDE_MIXED_FP32)
    lv = omg.geometric_hierarchy(operator_from_problem(p, 0.0))
    for l in (0, 1):
        L = lv[l]
        note(f"FP32 FFT level {l} ({L.n1}^2)")
        U = _rand((L.n2, L.n1), 200 + l)
        y = dev(np.zeros_like(U))
        fde.fde_apply(h, l, fde.FDE_MIXED_FP32, dev(U), y)
        assert rel(host(y), L.apply(U)) <= 2e-6, l


@pytest.mark.parametrize("prec", [fde.FDE_FP64, fde.FDE_MIXED_FP32])
def test_smoother_and_transfers_match_oracle(prec):
    n = 127
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec)
    lv = omg.geometric_hierarchy(operator_from_problem(p, 0.0))
    tol = 1e-12 if prec == fde.FDE_FP64 else 2e-6
    for l in range(len(lv) - 1):
        note(f"smooth/restrict/prolong level {l} prec={prec}")
        L = lv[l]
        B, X0 = _rand((L.n2, L.n1), l), _rand((L.n2, L.n1), 50 + l)
        x = dev(X0)
        fde.fde_smooth(h, l, prec, dev(B), x, False)
        assert rel(host(x), omg.jacobi(L, B, X0, 0.7)) <= tol
        x0 = dev(X0)
        fde.fde_smooth(h, l, prec, dev(B), x0, True)
        assert rel(host(x0), omg.jacobi(L, B, np.zeros_like(B), 0.7)) <= tol
        rc = dev(np.zeros((lv[l + 1].n2, lv[l + 1].n1)))
        fde.fde_restrict(h, l, prec, dev(B), rc)
        assert rel(host(rc), omg.restrict(B, L.n1, L.n2)) <= (1e-15 if prec == fde.FDE_FP64 else 1e-6)
        E = _rand((lv[l + 1].n2, lv[l + 1].n1), 70 + l)
        xf = dev(X0)
        fde.fde_prolong(h, l, prec, dev(E), xf)
        assert rel(host(xf), X0 + omg.prolong(E, L.n1, L.n2)) <= (1e-15 if prec == fde.FDE_FP64 else 1e-6)


def test_coarse_solve_matches_dense_solve():
    p = workloads.config_c2(63, 32)
    h = make_handle(p)
    lv = omg.geometric_hierarchy(operator_from_problem(p, 0.0))
    C = lv[-1]
    B = _rand((C.n2, C.n1), 5)
    x = dev(np.zeros_like(B))
    fde.fde_coarse_solve(h, dev(B), x)
    ref = np.linalg.solve(C.dense(), B.ravel()).reshape(B.shape)
    assert rel(host(x), ref) <= 1e-13


@pytest.mark.parametrize("n,prec", [(15, fde.FDE_FP64), (63, fde.FDE_FP64), (255, fde.FDE_FP64),
                                    (511, fde.FDE_FP64), (63, fde.FDE_MIXED_FP32),
                                    (255, fde.FDE_MIXED_FP32)])
def test_vcycle_matches_oracle(n, prec):
    note(f"vcycle n={n} prec={prec}")
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec)
    vc = omg.VCycle(omg.geometric_hierarchy(operator_from_problem(p, 0.0)))
    B = _rand((n, n), 9)
    x = dev(np.zeros_like(B))
    fde.fde_vcycle(h, dev(B), x)
    assert rel(host(x), vc(B)) <= (1e-12 if prec == fde.FDE_FP64 else 1e-5)


def test_vcycle_with_more_smoothing_steps():
    n = 127
    p = workloads.config_c2(n, 32)
    h = make_handle(p, nu_pre=2, nu_post=3)
    vc = omg.VCycle(omg.geometric_hierarchy(operator_from_problem(p, 0.0)), nu_pre=2, nu_post=3)
    B = _rand((n, n), 19)
    x = dev(np.zeros_like(B))
    fde.fde_vcycle(h, dev(B), x)
    assert rel(host(x), vc(B)) <= 1e-12
