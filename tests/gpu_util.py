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
