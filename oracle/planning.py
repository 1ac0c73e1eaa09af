"""Deflation size and memory planning of Section 5 (the systematic application of the
regularized and deflated solver).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``segment_image_radius`` / ``deflation_radius``: the deflation bound.  Every dense line
  segment [1, eps(x)/eps_b] of the spectrum of A is mapped through eq. EigenvaluesArA, the
  eigenvalue map of the regularized matrix A_R A, and the point of largest magnitude over
  all segments is the radius R beyond which eigenvalues are deflated.  The segment is
  sampled densely (the paper: "a small numerical routine, which produces a discretized
  image").
* ``plan_memory``: the five planning steps of Section 5 for a memory budget M (bytes), the
  ratio beta = r / (3N) of deflated eigenvalues, k points per smallest medium wavelength and
  restart = x r: the largest affordable grid N_max from M_A + M_prec = M with M_A = 720 N
  and M_prec = 16 r^2 + 48 N r + 48 N restart (16-byte complex values, 3N unknowns), then
  the largest object size (sqrt(N_max) - 1) / alpha.
* ``fair_restart``: the fair-memory comparison of Section 4's and Section 5's tables: the
  unpreconditioned system gets restart + r, the deflated one restart.
"""

from __future__ import annotations

import math

import numpy as np

from .spectral import homogeneous_map


def segment_image_radius(eps: complex, samples: int = 4001) -> float:
    """max |lam'| over lam on [1, eps], lam' = [1 + (1 - lam)/eps] lam (eq. EigenvaluesArA,
    eps_b = 1), with the segment sampled at `samples` equispaced points."""
    t = np.linspace(0.0, 1.0, samples)
    lam = 1.0 + t * (complex(eps) - 1.0)
    return float(np.abs(homogeneous_map(lam, complex(eps))).max())


def deflation_radius(eps_cells, samples: int = 4001) -> float:
    """Section 5's deflation bound for an inhomogeneous object: the segment mapping applied
    to [1, eps(x)] for every cell x, the largest magnitude over all of them."""
    vals = np.unique(np.asarray(eps_cells, dtype=np.complex128).ravel())
    return max(segment_image_radius(e, samples) for e in vals)


def plan_memory(M_bytes: float, beta: float, ppw: float, x: float, eps_real_max: float) -> dict:
    """The planning steps of Section 5, in the paper's order and units."""
    alpha = ppw * math.sqrt(eps_real_max)
    s = beta * beta + beta + x * beta
    n_max = (math.sqrt(900.0 + M_bytes * s) - 30.0) / (12.0 * s)
    a_max = (math.sqrt(n_max) - 1.0) / alpha
    # grid of the largest affordable object: nodes = alpha a/lambda + 1 per side, rounded down
    nodes = int(math.floor(alpha * a_max + 1.0 + 1e-9))
    N = nodes * nodes
    r = int(math.ceil(3.0 * N * beta - 1e-9))
    restart = int(math.floor(x * r + 0.5))  # restart = x r, rounded half up
    return {"alpha": alpha, "n_max": n_max, "a_over_lambda_max": a_max, "nodes": nodes, "N": N,
            "unknowns": 3 * N, "r": r, "restart": restart, "restart_unpreconditioned": fair_restart(restart, r),
            "M_A": 720.0 * N, "M_prec": 16.0 * r * r + 48.0 * N * r + 48.0 * N * restart}


def fair_restart(restart: int, r: int) -> int:
    """Restart of the unpreconditioned system given the same memory: restart + r."""
    return restart + r
