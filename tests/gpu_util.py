"""Helpers shared by the GPU tests (inputs and comparisons only)."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    return t.detach().to("cpu", torch.complex128).numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_eps(rng, ny, nx):
    """Inhomogeneous permittivity with both signs of Re and some loss (never 0)."""
    e = 1.0 + 6.0 * rng.random((ny, nx)) - 3.0 * (rng.random((ny, nx)) < 0.2) * 3.0
    return (e + 0.7j * rng.random((ny, nx))).astype(np.complex128)
