"""The entry point that allocates nothing (fde_apply_noalloc) against the handle's FP64 system
operator (fde_apply at level 0, FDE_FP64) and the oracle's operator of eq. (system): two calls in a
row, the second on a smaller grid, then a rectangular one, and even sides; the FP64 bar of the
operator (1e-12 relative 2-norm).  Sizes beyond the static buffer are rejected with FDE_EINVAL."""
import numpy as np
import pytest
import torch

import workloads
from oracle.operator import operator_from_problem
from paper_1706_06844_amd import fde

from .gpu_util import dev, host, make_handle, note, problem_struct, rel

pytestmark = pytest.mark.gpu


def _case(p, seed):
    F = [dev(f) for f in workloads.sample(p, 0.0)]
    U = np.random.default_rng(seed).standard_normal((p.n2, p.n1))
    y = dev(np.full_like(U, np.nan))
    fde.fde_apply_noalloc(problem_struct(p), *F, dev(U), y)
    torch.cuda.synchronize()
    h = make_handle(p)
    yh = dev(np.zeros_like(U))
    fde.fde_apply(h, 0, fde.FDE_FP64, dev(U), yh)
    h.close()
    got, ref_h, ref_o = host(y), host(yh), operator_from_problem(p, 0.0).apply(U)
    note(f"no-alloc apply {p.n1}x{p.n2}: vs fde_apply {rel(got, ref_h):.2e}, vs oracle {rel(got, ref_o):.2e}")
    assert np.all(np.isfinite(got))
    assert rel(got, ref_h) <= 1e-12 and rel(got, ref_o) <= 1e-12


def test_noalloc_apply_matches_handle_twice_then_smaller():
    _case(workloads.config_c2(511, 32), 1)          # alpha 1.8, beta 1.6, variable coefficients
    _case(workloads.config_c3(127, 16), 2)          # smaller grid, other orders: every table rebuilt
    p = workloads.config_c2(63, 32)
    p.n2 = 127
    _case(p, 3)                                      # rectangular


def test_noalloc_apply_on_even_sides():
    # the paper's even grids: embedding length 2n
    _case(workloads.example1(64), 4)
    p = workloads.config_c2(128, 32)
    p.n2 = 63
    _case(p, 5)


def test_noalloc_rejects_grids_beyond_its_buffer():
    p = workloads.config_c3(2047, 16)
    z = dev(np.zeros((7, 7)))
    with pytest.raises(fde.FdeError) as e:
        fde.fde_apply_noalloc(problem_struct(p), z, z, z, z, z, dev(np.zeros((7, 7))))
    assert e.value.code == fde.FDE_EINVAL and "FDE_NOALLOC_MAX_N" in str(e.value)
