"""Python binding of libfde with the C ABI's names (include/fde.h).

Arguments are torch tensors in device memory (float64, contiguous, on the current HIP device); the
functions only marshal pointers and sizes.  PyTorch supplies device memory and streams; every step
of the solver runs in libfde's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L
from ._lib import (FDE_EAGAIN, FDE_EDEVICE, FDE_EINVAL, FDE_ENEGCOEF, FDE_ENOCONV, FDE_ENOMEM,  # noqa
                   FDE_ENONFINITE, FDE_FP64, FDE_MG_BAND, FDE_MG_GALERKIN, FDE_MG_GEOMETRIC,
                   FDE_MIXED_BF16GEMM, FDE_MIXED_CYCLE_BF16, FDE_MIXED_FP32_CYCLE,
                   FDE_MIXED_FP32, FDE_OK, fde_problem, fde_stats)


class FdeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfde error {code}: {msg}")
        self.code = code


def _lib():
    return L.load()


def _ptr(t: Optional[torch.Tensor], name: str = "tensor", dtype=torch.float64) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(rc: int, h=None) -> int:
    if rc < 0:
        msg = _lib().fde_last_error(h.ptr if h is not None else None)
        raise FdeError(rc, msg.decode() if msg else "")
    return rc


def fde_problem_default(alpha: float, beta: float, n1: int, n2: int, tau: float, **kw) -> fde_problem:
    p = fde_problem()
    _lib().fde_problem_default(ctypes.byref(p), alpha, beta, n1, n2, tau)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class Handle:
    """Owns an fde_handle; destroyed with fde_destroy."""

    def __init__(self, ptr: int, problem: fde_problem):
        self.ptr = ptr
        self.problem = problem

    def close(self):
        if self.ptr:
            _lib().fde_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n1(self):
        return self.problem.n1

    @property
    def n2(self):
        return self.problem.n2


def fde_setup(problem: fde_problem, dp, dm, ep, em, stream=None) -> Handle:
    out = ctypes.c_void_p()
    rc = _lib().fde_setup(ctypes.byref(problem), _ptr(dp, "dp"), _ptr(dm, "dm"), _ptr(ep, "ep"),
                          _ptr(em, "em"), _stream_ptr(stream), ctypes.byref(out))
    _check(rc)
    return Handle(out.value, problem)


def fde_update_coeffs(h: Handle, dp, dm, ep, em) -> None:
    _check(_lib().fde_update_coeffs(h.ptr, _ptr(dp), _ptr(dm), _ptr(ep), _ptr(em)), h)


def _stats_result(rc: int, st: fde_stats, h: Handle) -> Dict:
    _check(rc, h)
    d = st.as_dict()
    d["rc"] = rc
    return d


def fde_step(h: Handle, u_prev, v_half, u_next) -> Dict:
    st = fde_stats()
    rc = _lib().fde_step(h.ptr, _ptr(u_prev, "u_prev"), _ptr(v_half, "v_half"), _ptr(u_next, "u_next"),
                         ctypes.byref(st))
    return _stats_result(rc, st, h)


def fde_step_sources(h: Handle, u_prev, phis: Sequence[float], fields: Sequence[torch.Tensor], u_next,
                     want_stats: bool = True) -> Optional[Dict]:
    n = len(phis)
    phi = (ctypes.c_double * max(n, 1))(*phis)
    S = (ctypes.c_void_p * max(n, 1))(*[_ptr(f, "source") for f in fields])
    st = fde_stats()
    rc = _lib().fde_step_sources(h.ptr, _ptr(u_prev, "u_prev"), n, phi, S, _ptr(u_next, "u_next"),
                                 ctypes.byref(st) if want_stats else None)
    return _stats_result(rc, st, h) if want_stats else (_check(rc, h) and None)


def fde_solve(h: Handle, b, x) -> Dict:
    st = fde_stats()
    rc = _lib().fde_solve(h.ptr, _ptr(b, "b"), _ptr(x, "x"), ctypes.byref(st))
    return _stats_result(rc, st, h)


def fde_solve_mg(h: Handle, b, x, max_cycles: int = 200) -> Dict:
    st = fde_stats()
    rc = _lib().fde_solve_mg(h.ptr, _ptr(b, "b"), _ptr(x, "x"), int(max_cycles), ctypes.byref(st))
    return _stats_result(rc, st, h)


def fde_num_levels(h: Handle) -> int:
    return _check(_lib().fde_num_levels(h.ptr), h)


def fde_level_size(h: Handle, level: int):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().fde_level_size(h.ptr, level, ctypes.byref(a), ctypes.byref(b)), h)
    return a.value, b.value


def fde_apply(h: Handle, level: int, prec: int, x, y) -> None:
    _check(_lib().fde_apply(h.ptr, level, prec, _ptr(x, "x"), _ptr(y, "y")), h)


def fde_residual(h: Handle, level: int, prec: int, b, x, r) -> None:
    _check(_lib().fde_residual(h.ptr, level, prec, _ptr(b, "b"), _ptr(x, "x"), _ptr(r, "r")), h)


def fde_smooth(h: Handle, level: int, prec: int, b, x, zero_guess: bool) -> None:
    _check(_lib().fde_smooth(h.ptr, level, prec, _ptr(b, "b"), _ptr(x, "x"), int(zero_guess)), h)


def fde_restrict(h: Handle, level: int, prec: int, r, rc) -> None:
    _check(_lib().fde_restrict(h.ptr, level, prec, _ptr(r, "r"), _ptr(rc, "rc")), h)


def fde_prolong(h: Handle, level: int, prec: int, e, x) -> None:
    _check(_lib().fde_prolong(h.ptr, level, prec, _ptr(e, "e"), _ptr(x, "x")), h)


def fde_coarse_solve(h: Handle, b, x) -> None:
    _check(_lib().fde_coarse_solve(h.ptr, _ptr(b, "b"), _ptr(x, "x")), h)


def fde_vcycle(h: Handle, b, x) -> None:
    _check(_lib().fde_vcycle(h.ptr, _ptr(b, "b"), _ptr(x, "x")), h)


def fde_level_diag(h: Handle, level: int, diag) -> None:
    _check(_lib().fde_level_diag(h.ptr, level, _ptr(diag, "diag")), h)


def fde_sync(h: Handle) -> None:
    _check(_lib().fde_sync(h.ptr), h)


def fde_profile_enable(h: Handle, mask: int = (1 << len(L.KFAM)) - 1) -> None:
    _check(_lib().fde_profile_enable(h.ptr, mask), h)


def fde_profile_stride(h: Handle, every: int) -> None:
    _check(_lib().fde_profile_stride(h.ptr, every), h)


def fde_profile_reset(h: Handle) -> None:
    _check(_lib().fde_profile_reset(h.ptr), h)


def fde_profile_read(h: Handle) -> Dict[str, Dict]:
    out = {}
    for k, name in enumerate(L.KFAM):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(_lib().fde_profile_read(h.ptr, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), h)
        out[name] = {"launches": n.value, "ms": ms.value, "bytes": by.value}
    return out


# ---- batching and serving --------------------------------------------------------------------------
def fde_footprint(problem: fde_problem) -> int:
    return int(_lib().fde_footprint(ctypes.byref(problem)))


class Batch:
    """Owns an fde_batch; destroyed with fde_batch_destroy."""

    def __init__(self, ptr: int, budget: int):
        self.ptr = ptr
        self.budget = budget
        self._keep = {}

    def close(self):
        if self.ptr:
            _lib().fde_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fde_batch_create(budget_bytes: int, stream=None) -> Batch:
    out = ctypes.c_void_p()
    rc = _lib().fde_batch_create(ctypes.c_size_t(budget_bytes), _stream_ptr(stream), ctypes.byref(out))
    _check(rc)
    return Batch(out.value, budget_bytes)


def fde_batch_destroy(b: Batch) -> None:
    b.close()


def fde_batch_set_grouping(b: Batch, max_n: int, slots: int) -> None:
    """Requests of one shape with max(n1, n2) <= max_n share a group of `slots` slots (0 turns it off)."""
    _check(_lib().fde_batch_set_grouping(b.ptr, int(max_n), int(slots)))


def fde_batch_set_lanes(b: Batch, lanes: int) -> None:
    """Ungrouped requests on one stream and the groups on lanes - 1 others, created together (0: a
    stream per request and group)."""
    _check(_lib().fde_batch_set_lanes(b.ptr, int(lanes)))


def fde_batch_set_policy(b: Batch, max_running: int, piece_steps: int = 0, busy_running: int = -1) -> None:
    """Restart cycles issued in pieces of piece_steps Arnoldi steps (0: whole cycles); at most
    max_running ungrouped requests with a piece in flight, least work left first (0: no limit), and
    at most busy_running of them while a group has work (-1: no extra limit)."""
    _check(_lib().fde_batch_set_policy(b.ptr, int(max_running), int(piece_steps), int(busy_running)))


def fde_batch_admit(b: Batch, problem: fde_problem, dp, dm, ep, em, u0, nsteps: int, t0: float = 0.0,
                    coef: Sequence[float] = (), rate: Sequence[float] = (),
                    fields: Sequence[torch.Tensor] = ()) -> int:
    """Returns the request id (>= 0) or FDE_EAGAIN (the request does not fit the budget now)."""
    n = len(fields)
    if len(coef) != n or len(rate) != n:
        raise ValueError("coef, rate and fields must have the same length")
    c = (ctypes.c_double * max(n, 1))(*coef)
    r = (ctypes.c_double * max(n, 1))(*rate)
    S = (ctypes.c_void_p * max(n, 1))(*[_ptr(f, "source") for f in fields])
    rc = _lib().fde_batch_admit(b.ptr, ctypes.byref(problem), _ptr(dp, "dp"), _ptr(dm, "dm"), _ptr(ep, "ep"),
                                _ptr(em, "em"), _ptr(u0, "u0"), int(nsteps), float(t0), n, c, r, S)
    if rc == FDE_EAGAIN:
        return rc
    if rc < 0:
        raise FdeError(rc, "fde_batch_admit failed")
    return rc


def fde_batch_step(b: Batch) -> int:
    rc = _lib().fde_batch_step(b.ptr)
    if rc < 0:
        raise FdeError(rc, "fde_batch_step failed")
    return rc


def fde_batch_poll(b: Batch, rid: int, u_out=None):
    """(status, iterations): status 1 finished, 2 finished with steps at the iteration limit,
    0 still stepping; raises on errors."""
    it = ctypes.c_int64()
    rc = _lib().fde_batch_poll(b.ptr, rid, _ptr(u_out, "u_out"), ctypes.byref(it))
    if rc < 0:
        raise FdeError(rc, f"request {rid} failed")
    return rc, it.value


def fde_batch_cancel(b: Batch, rid: int) -> None:
    _check(_lib().fde_batch_cancel(b.ptr, rid))


def fde_batch_info(b: Batch):
    a, by = ctypes.c_int32(), ctypes.c_size_t()
    _check(_lib().fde_batch_info(b.ptr, ctypes.byref(a), ctypes.byref(by)))
    return a.value, by.value


def fde_apply_noalloc(problem: fde_problem, dp, dm, ep, em, x, y, stream=None) -> None:
    """y = (I - tau/2 L) x without a handle and without device allocation (asynchronous on stream)."""
    _check(_lib().fde_apply_noalloc(ctypes.byref(problem), _ptr(dp, "dp"), _ptr(dm, "dm"), _ptr(ep, "ep"),
                                    _ptr(em, "em"), _ptr(x, "x"), _ptr(y, "y"), _stream_ptr(stream)))
