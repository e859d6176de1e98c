"""Helpers shared by the GPU tests: build a solver handle for a workload problem and move fields."""
import sys

import numpy as np
import torch

import workloads
from paper_1706_06844_amd import fde


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def problem_struct(p, precision=fde.FDE_FP64, **kw):
    s = fde.fde_problem_default(p.alpha, p.beta, p.n1, p.n2, p.tau)
    s.a1, s.b1, s.a2, s.b2 = p.a1, p.b1, p.a2, p.b2
    s.precision = precision
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def make_handle(p, precision=fde.FDE_FP64, t=0.0, **kw):
    fields = [dev(f) for f in workloads.sample(p, t)]
    h = fde.fde_setup(problem_struct(p, precision, **kw), *fields)
    h._keep = fields
    return h


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def exp_source_terms(p):
    """Source terms of p as (coef, rate, fields) with phi_k(t) = coef_k exp(rate_k t); the problems'
    time factors are exponentials (or constants), recovered from their values at t = 0 and 1."""
    import math

    phis, fields = workloads.source_terms(p)
    coef, rate = [], []
    for f in phis:
        c0, c1 = float(f(0.0)), float(f(1.0))
        coef.append(c0)
        rate.append(math.log(c1 / c0) if c0 != 0.0 else 0.0)
    return coef, rate, fields


def solo_run(p, steps, precision=fde.FDE_FP64, **kw):
    """The reference for batched runs: fde_step_sources step by step on one handle."""
    import math

    h = make_handle(p, precision, **kw)
    coef, rate, fields = exp_source_terms(p)
    S = [dev(f) for f in fields]
    u = dev(workloads.sample_u0(p))
    un = torch.empty_like(u)
    iters = 0
    for m in range(1, steps + 1):
        t = (m - 0.5) * p.tau
        phi = [c * math.exp(r * t) for c, r in zip(coef, rate)]
        st = fde.fde_step_sources(h, u, phi, S, un)
        iters += st["iters"]
        u, un = un, u
    out = host(u)
    h.close()
    return out, iters
