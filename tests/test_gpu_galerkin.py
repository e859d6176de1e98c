"""Galerkin coarse operators on the GPU (factored form) against the oracle.

The oracle's Galerkin levels are R ... R A_0 P ... P applied by composition (and, on small grids, the
dense triple products); the GPU never forms them.  FP64 results agree to rounding, FP32 to single
precision.
"""
import numpy as np
import pytest

import workloads
from oracle import multigrid as omg
from oracle.cn import rhs, solve_step
from oracle.operator import operator_from_problem
from paper_1706_06844_amd import fde

from .gpu_util import dev, host, make_handle, note, rel

pytestmark = pytest.mark.gpu

GAL = fde.FDE_MG_GALERKIN


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("n1,n2,prec", [(31, 31, fde.FDE_FP64), (63, 63, fde.FDE_FP64), (127, 127, fde.FDE_FP64),
                                        (255, 255, fde.FDE_FP64), (63, 127, fde.FDE_FP64),
                                        (127, 127, fde.FDE_MIXED_FP32)])
def test_galerkin_level_apply_and_diag(n1, n2, prec):
    p = workloads.config_c2(n1, 32)
    p.n2 = n2
    h = make_handle(p, precision=prec, mg_variant=GAL)
    op = operator_from_problem(p, 0.0)
    lv = omg.galerkin_hierarchy_composed(op)
    assert fde.fde_num_levels(h) == len(lv)
    tol = 1e-12 if prec == fde.FDE_FP64 else 3e-6
    for l in range(1, len(lv)):
        L = lv[l]
        note(f"galerkin level {l} ({L.n1}x{L.n2}) of {n1}x{n2} prec={prec}")
        assert fde.fde_level_size(h, l) == (L.n1, L.n2)
        U = _rand((L.n2, L.n1), 300 + l)
        y = dev(np.zeros_like(U))
        fde.fde_apply(h, l, prec, dev(U), y)
        assert rel(host(y), L.apply(U)) <= tol, l
        d = dev(np.zeros_like(U))
        fde.fde_level_diag(h, l, d)
        np.testing.assert_allclose(host(d), L.diag(), rtol=1e-12 if prec == fde.FDE_FP64 else 2e-6)


def test_galerkin_level_matches_dense_triple_product():
    n = 31
    p = workloads.config_c2(n, 32)
    h = make_handle(p, mg_variant=GAL)
    dense = omg.galerkin_hierarchy_dense(operator_from_problem(p, 0.0))
    for l in range(1, len(dense)):
        A = dense[l].dense()
        U = _rand((dense[l].n2, dense[l].n1), 40 + l)
        y = dev(np.zeros_like(U))
        fde.fde_apply(h, l, fde.FDE_FP64, dev(U), y)
        assert rel(host(y).ravel(), A @ U.ravel()) <= 1e-12


@pytest.mark.parametrize("n", [63, 255])
def test_galerkin_coarsest_solve(n):
    p = workloads.config_c2(n, 32)
    h = make_handle(p, mg_variant=GAL)
    lv = omg.galerkin_hierarchy_composed(operator_from_problem(p, 0.0))
    C = lv[-1]
    B = _rand((C.n2, C.n1), 8)
    x = dev(np.zeros_like(B))
    fde.fde_coarse_solve(h, dev(B), x)
    ref = np.linalg.solve(C.dense(), B.ravel()).reshape(B.shape)
    assert rel(host(x), ref) <= 1e-12


@pytest.mark.parametrize("n,prec", [(63, fde.FDE_FP64), (127, fde.FDE_FP64), (255, fde.FDE_FP64),
                                    (127, fde.FDE_MIXED_FP32)])
def test_galerkin_vcycle_matches_oracle(n, prec):
    note(f"galerkin vcycle n={n} prec={prec}")
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec, mg_variant=GAL)
    vc = omg.VCycle(omg.galerkin_hierarchy_composed(operator_from_problem(p, 0.0)))
    B = _rand((n, n), 12)
    x = dev(np.zeros_like(B))
    fde.fde_vcycle(h, dev(B), x)
    assert rel(host(x), vc(B)) <= (1e-11 if prec == fde.FDE_FP64 else 2e-5)


@pytest.mark.parametrize("prec", [fde.FDE_FP64, fde.FDE_MIXED_FP32])
def test_galerkin_solve_matches_dense_lu(prec):
    n = 63
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec, mg_variant=GAL)
    op = operator_from_problem(p, 0.0)
    B = _rand((n, n), 21)
    x = dev(np.zeros_like(B))
    st = fde.fde_solve(h, dev(B), x)
    assert st["converged"]
    ref = solve_step(op, B)
    assert rel(host(x), ref) <= 1e-9


def test_galerkin_and_geometric_iteration_counts_c1():
    # the paper's tables give (almost) the same counts for both coarse operators
    p = workloads.config_c1(63)
    op = operator_from_problem(p, 0.0)
    u0 = workloads.sample_u0(p)
    b = rhs(op, u0, workloads.sample_source(p, 0.5 * p.tau))
    its = {}
    for v in (fde.FDE_MG_GEOMETRIC, GAL):
        h = make_handle(p, mg_variant=v)
        x = dev(np.zeros_like(b))
        st = fde.fde_solve(h, dev(b), x)
        assert st["converged"]
        its[v] = st["iters"]
        assert rel(host(x), solve_step(op, b)) <= 1e-9
    note(f"C1 iterations geometric {its[fde.FDE_MG_GEOMETRIC]} galerkin {its[GAL]}")
    assert abs(its[fde.FDE_MG_GEOMETRIC] - its[GAL]) <= 2


def test_galerkin_c2_step_matches_oracle():
    n = 255
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=fde.FDE_MIXED_FP32, mg_variant=GAL)
    op = operator_from_problem(p, 0.0)
    u0 = workloads.sample_u0(p)
    v = workloads.sample_source(p, 0.5 * p.tau)
    un = dev(np.zeros_like(u0))
    st = fde.fde_step(h, dev(u0), dev(v), un)
    assert st["converged"]
    from oracle.cn import IterativeSolver

    ref = solve_step(op, rhs(op, u0, v), IterativeSolver(rtol=1e-12))
    assert rel(host(un), ref) <= 1e-9


# ---- the band preconditioner P_2 (Sec. 4.3): the Laplacian in place of the fractional factors ----
def _band_operator(p):
    # r P_2 of Sec. 4.3: the Laplacian matrix in place of the fractional factors, with the system's
    # scalings tau/(2 hx^alpha), tau/(2 hy^beta)
    from oracle.operator import band_operator

    return band_operator(operator_from_problem(p, 0.0))


@pytest.mark.parametrize("prec", [fde.FDE_FP64, fde.FDE_MIXED_FP32])
def test_band_hierarchy_and_vcycle(prec):
    n = 63
    p = workloads.config_c2(n, 32)
    h = make_handle(p, precision=prec, mg_variant=fde.FDE_MG_BAND)
    opb = _band_operator(p)
    lv = omg.galerkin_hierarchy_composed(opb)
    assert fde.fde_num_levels(h) == len(lv)
    tol = 1e-12 if prec == fde.FDE_FP64 else 3e-6
    for l in range(len(lv)):
        U = _rand((lv[l].n2, lv[l].n1), 500 + l)
        y = dev(np.zeros_like(U))
        fde.fde_apply(h, l, prec, dev(U), y)
        assert rel(host(y), lv[l].apply(U)) <= tol, l
    B = _rand((n, n), 17)
    x = dev(np.zeros_like(B))
    fde.fde_vcycle(h, dev(B), x)
    assert rel(host(x), omg.VCycle(lv)(B)) <= (1e-11 if prec == fde.FDE_FP64 else 2e-5)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_band_preconditioned_solve(cfg):
    from oracle.krylov import fgmres

    n = 63 if cfg == "c1" else 127
    p = workloads.config_c1(n) if cfg == "c1" else workloads.config_c2(n, 32)
    op = operator_from_problem(p, 0.0)
    b = rhs(op, workloads.sample_u0(p), workloads.sample_source(p, 0.5 * p.tau))
    its = {}
    for v in (fde.FDE_MG_GEOMETRIC, fde.FDE_MG_BAND):
        h = make_handle(p, mg_variant=v, maxit=1000)
        x = dev(np.zeros_like(b))
        st = fde.fde_solve(h, dev(b), x)
        assert st["converged"]
        its[v] = st["iters"]
        assert rel(host(x), solve_step(op, b)) <= 1e-9
    ref = fgmres(op.apply, b, omg.VCycle(omg.galerkin_hierarchy_composed(_band_operator(p))), rtol=1e-10,
                 restart=20, maxit=1000)
    note(f"{cfg} n={n}: GMRES iterations with the multigrid preconditioner {its[fde.FDE_MG_GEOMETRIC]}, "
         f"with the band preconditioner {its[fde.FDE_MG_BAND]} (oracle {ref.iters})")
    assert abs(its[fde.FDE_MG_BAND] - ref.iters) <= 2
