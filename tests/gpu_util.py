"""Helpers of the GPU parity tests: device placement of seeded inputs and
comparison norms.  Everything here is marshalling; no solver arithmetic."""
import sys

import numpy as np

import wdgen


def torch_mod():
    import torch
    return torch


def dev(a: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def field_set(dims, eps, gseed, nrhs, sseed):
    U = wdgen.gauge_field(dims, eps, gseed)
    psi = wdgen.gaussian_source(dims, nrhs, sseed)
    return U, psi
