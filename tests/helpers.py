"""Shared helpers of the GPU parity tests (input marshalling and tolerance checks)."""
import functools
import sys

import numpy as np
import torch

from paper_2404_16039_amd import gen

# tolerances of the two paths: relative to the natural error scale of each result
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
F64, F32 = 1, 0


def prec_of(dtype):
    return F64 if dtype == torch.float64 else F32


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy()


def counters():
    return torch.zeros(4, dtype=torch.int64, device="cuda")


def say(*a):
    """Name the case before each GPU step (so a failing run says what it was doing)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def within(got, ref, scale, tol, what):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    err = np.abs(got - ref)
    bound = tol * scale
    bad = ~(err <= bound)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tol {tol}: got {got.ravel()[i]} "
                             f"ref {ref.ravel()[i]} scale {scale.ravel()[i]} max rel "
                             f"{np.max(err / np.maximum(scale, 1e-300)):.3e}")
    return float(np.max(err / np.maximum(scale, 1e-300))) if err.size else 0.0


@functools.lru_cache(maxsize=4)
def cube(n, jitter=0.15):
    return gen.cube_mesh(n, jitter=jitter)


@functools.lru_cache(maxsize=4)
def square(n, jitter=0.2):
    return gen.square_mesh(n, jitter=jitter)
