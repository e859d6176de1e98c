"""Grouped batching: requests of one shape share a group whose restart cycle is replayed from captured
graphs whose every kernel is launched once over the members that solve (grid z indexes a table of
their slot offsets).

Each member must give what the same problem gives alone (fde_step_sources on its own handle: the same
kernels over the same data, so the same result to rounding-free equality in practice, asserted to
1e-14), whatever the other slots hold -- empty slots, members at other steps, members that joined
late or left early.  A few members are also checked against the oracle's CN run (1e-9, as for every
solve).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle.cn import IterativeSolver, cn_run
from paper_1706_06844_amd import fde

from .gpu_util import dev, exp_source_terms, host, note, problem_struct, rel, solo_run

pytestmark = pytest.mark.gpu


def _instances(count, sizes, seed, M):
    rng = np.random.default_rng(seed)
    return [workloads.random_instance(rng, sizes, f"g{i}", M, seed + 1000 * i) for i in range(count)]


def _admit(b, p, precision, keep, **kw):
    coef, rate, fields = exp_source_terms(p)
    F = [dev(f) for f in workloads.sample(p, 0.0)]
    S = [dev(f) for f in fields]
    u0 = dev(workloads.sample_u0(p))
    keep.append((F, S, u0))
    rid = fde.fde_batch_admit(b, problem_struct(p, precision, **kw), *F, u0, p.M, 0.0, coef, rate, S)
    assert rid >= 0
    return rid


def _drain(b, ids, shapes, on_step=None):
    out = {}
    pending = set(ids)
    calls = 0
    while pending:
        fde.fde_batch_step(b)
        calls += 1
        if on_step is not None:
            on_step(calls, pending)
        for rid in list(pending):
            n2, n1 = shapes[rid]
            u = torch.empty((n2, n1), dtype=torch.float64, device="cuda:0")
            st, it = fde.fde_batch_poll(b, rid, u)
            if st:
                assert st == 1, f"request {rid} hit the iteration limit"
                out[rid] = (host(u), it)
                pending.discard(rid)
    return out


def _check_solo(res, ids, probs, precision, **kw):
    for rid, p in zip(ids, probs):
        ref, its = solo_run(p, p.M, precision, **kw)
        got, bits = res[rid]
        note(f"member {rid} n={p.n1} alpha={p.alpha:.3f}: max diff {np.max(np.abs(got - ref)):.2e}, "
             f"iters {bits} vs {its}")
        assert bits == its
        assert rel(got, ref) <= 1e-14


@pytest.mark.parametrize("precision,piece", [(fde.FDE_FP64, 0), (fde.FDE_MIXED_FP32, 0),
                                             (fde.FDE_MIXED_FP32_CYCLE, 0), (fde.FDE_MIXED_CYCLE_BF16, 0),
                                             (fde.FDE_MIXED_FP32, 5), (fde.FDE_FP64, 3)])
def test_group_members_equal_solo(precision, piece):
    # 5 members in a group of 8 slots (3 stay empty); different orders, coefficients and sources;
    # cycles whole or in pieces of `piece` Arnoldi steps
    probs = _instances(5, (63,), 21, 3)
    b = fde.fde_batch_create(8 << 30)
    fde.fde_batch_set_grouping(b, 127, 8)
    fde.fde_batch_set_policy(b, 0, piece)
    keep, ids, shapes = [], [], {}
    for p in probs:
        ids.append(_admit(b, p, precision, keep))
        shapes[ids[-1]] = (p.n2, p.n1)
    res = _drain(b, ids, shapes)
    _check_solo(res, ids, probs, precision)
    assert fde.fde_batch_info(b)[0] == 0
    b.close()


@pytest.mark.parametrize("lanes", [0, 4])
def test_group_join_leave_and_mixed_shapes(lanes):
    # members join while the group is stepping, one is cancelled mid-run and its slot reused; a
    # larger request beyond the size limit runs ungrouped beside the group; with lanes the batch's
    # shared streams carry them
    precision = fde.FDE_MIXED_FP32
    probs = _instances(6, (127,), 33, 4)
    big = _instances(1, (255,), 34, 3)[0]
    b = fde.fde_batch_create(8 << 30)
    if lanes:
        fde.fde_batch_set_lanes(b, lanes)
    fde.fde_batch_set_grouping(b, 127, 4)
    keep, ids, shapes = [], [], {}
    for p in probs[:3]:
        ids.append(_admit(b, p, precision, keep))
        shapes[ids[-1]] = (p.n2, p.n1)
    rbig = _admit(b, big, precision, keep)
    shapes[rbig] = (big.n2, big.n1)
    fde.fde_batch_step(b)
    fde.fde_batch_step(b)
    fde.fde_batch_cancel(b, ids[1])  # frees a slot mid-solve
    kept = [ids[0], ids[2]]
    kept_probs = [probs[0], probs[2]]
    for p in probs[3:]:  # one takes the freed slot, one the empty one, one opens a second group
        kept.append(_admit(b, p, precision, keep))
        kept_probs.append(p)
        shapes[kept[-1]] = (p.n2, p.n1)
    res = _drain(b, kept + [rbig], shapes)
    _check_solo(res, kept + [rbig], kept_probs + [big], precision)
    b.close()


def test_group_members_match_oracle():
    probs = _instances(3, (63,), 55, 2)
    b = fde.fde_batch_create(8 << 30)
    fde.fde_batch_set_grouping(b, 63, 4)
    keep, ids, shapes = [], [], {}
    for p in probs:
        ids.append(_admit(b, p, fde.FDE_MIXED_FP32, keep))
        shapes[ids[-1]] = (p.n2, p.n1)
    res = _drain(b, ids, shapes)
    for rid, p in zip(ids, probs):
        ref = cn_run(p, steps=p.M, solver=IterativeSolver(rtol=1e-12, maxit=3000)).u
        e = rel(res[rid][0], ref)
        note(f"member {rid} vs oracle CN run ({p.M} steps): {e:.2e}")
        assert e <= 1e-9
    b.close()


def test_grouping_arguments():
    b = fde.fde_batch_create(1 << 30)
    with pytest.raises(fde.FdeError):
        fde.fde_batch_set_grouping(b, 127, 0)
    with pytest.raises(fde.FdeError):
        fde.fde_batch_set_grouping(b, 127, 2000)
    fde.fde_batch_set_grouping(b, 0, 0)  # off
    p = _instances(1, (31,), 3, 1)[0]
    keep = []
    rid = _admit(b, p, fde.FDE_FP64, keep)
    with pytest.raises(fde.FdeError):  # only on an empty batch
        fde.fde_batch_set_grouping(b, 127, 4)
    _drain(b, [rid], {rid: (p.n2, p.n1)})
    b.close()


@pytest.mark.parametrize("precision", [fde.FDE_MIXED_FP32, fde.FDE_FP64])
def test_group_with_fft_levels_equals_solo(precision):
    # 511^2 members: the outer operator and the fine levels run the FFT passes in their batched
    # instantiation (slot table), the coarser ones the tiled and one-workgroup kernels
    probs = _instances(3, (511,), 71, 2)
    b = fde.fde_batch_create(16 << 30)
    fde.fde_batch_set_grouping(b, 511, 4)
    keep, ids, shapes = [], [], {}
    for p in probs:
        ids.append(_admit(b, p, precision, keep))
        shapes[ids[-1]] = (p.n2, p.n1)
    res = _drain(b, ids, shapes)
    _check_solo(res, ids, probs, precision)
    b.close()


def test_group_on_even_sides_equals_solo():
    # the paper's even grids in a group: 64^2 -> 32 -> 16 -> 8
    probs = _instances(3, (64,), 73, 3)
    b = fde.fde_batch_create(8 << 30)
    fde.fde_batch_set_grouping(b, 64, 4)
    fde.fde_batch_set_policy(b, 0, 5)
    keep, ids, shapes = [], [], {}
    for p in probs:
        ids.append(_admit(b, p, fde.FDE_MIXED_FP32, keep))
        shapes[ids[-1]] = (p.n2, p.n1)
    res = _drain(b, ids, shapes)
    _check_solo(res, ids, probs, fde.FDE_MIXED_FP32)
    b.close()
