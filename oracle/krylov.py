"""Short-memory Krylov solvers for the preconditioned system, for comparison with restarted GMRES.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Conclusions of Zouros & Budko note that any memory-efficient Krylov solver that works on the
original system A u = b also applies to the regularized and deflated system A_R A P^-1 v = A_R b,
and name Bi-CGSTAB, restarted GCR and IDR.  The paper gives no listing for them; the two here
follow their published definitions, written as plain dense-matrix numpy code:

* ``bicgstab`` -- H. A. van der Vorst, "Bi-CGSTAB: a fast and smoothly converging variant of Bi-CG
  for the solution of nonsymmetric linear systems", SIAM J. Sci. Stat. Comput. 13 (1992):
  the shadow residual is the initial residual, one BiCG step followed by one minimal-residual
  (GMRES(1)) step per iteration.
* ``gcr`` -- S. C. Eisenstat, H. C. Elman, M. H. Schultz, "Variational iterative methods for
  nonsymmetric systems of linear equations", SIAM J. Numer. Anal. 20 (1983): each new direction
  is made A-orthogonal (its image orthonormal) to the kept ones, the residual is reduced along
  its image; with restart m the kept directions are dropped every m steps.

Both take the operator as a dense matrix (or a callable), a right preconditioner as a callable,
and return the iterate, the residual norms of the recurrence and the number of operator
applications.  Complex arithmetic in FP64; inner products conjugate their first argument.
"""
from __future__ import annotations

import numpy as np


def _op(M):
    return M if callable(M) else (lambda x: M @ x)


def bicgstab(M, b, x0=None, tol=1e-10, maxiter=1000, prec=None):
    """Right-preconditioned Bi-CGSTAB on M (P^-1 v) = b, x = P^-1 v (prec = P^-1, identity if None).

    Returns (x, residual norms after every iteration, applications of M).  Stops when the
    recurrence residual is below tol ||b|| or on a breakdown (rho = 0 or (r^, v) = 0)."""
    A = _op(M)
    P = prec if prec is not None else (lambda x: x)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A(x)
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    hist = [np.linalg.norm(r)]
    nb = np.linalg.norm(b)
    apps = 0
    for _ in range(maxiter):
        rho1 = np.vdot(rh, r)
        if rho1 == 0:
            break
        beta = (rho1 / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = P(p)
        v = A(ph)
        apps += 1
        rv = np.vdot(rh, v)
        if rv == 0:
            break
        alpha = rho1 / rv
        s = r - alpha * v
        sh = P(s)
        t = A(sh)
        apps += 1
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho = rho1
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * nb or omega == 0:
            break
    return x, np.array(hist), apps


def gcr(M, b, x0=None, tol=1e-10, maxiter=1000, restart=None, prec=None):
    """Right-preconditioned restarted GCR(m) on M (P^-1 v) = b, x = P^-1 v (m = restart, None:
    keep every direction).  Each step: z = P^-1 r, q = M z; q and z are orthogonalised against
    the kept pairs (classical Gram-Schmidt twice, on q's inner products) and scaled to ||q|| = 1;
    x += (q, r) z, r -= (q, r) q.  Returns (x, residual norms after every step, applications of M)."""
    A = _op(M)
    P = prec if prec is not None else (lambda x: x)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A(x)
    Ps, Qs = [], []
    hist = [np.linalg.norm(r)]
    nb = np.linalg.norm(b)
    apps = 0
    for _ in range(maxiter):
        z = P(r)
        q = A(z)
        apps += 1
        for _pass in range(2):
            for pj, qj in zip(Ps, Qs):
                h = np.vdot(qj, q)
                q = q - h * qj
                z = z - h * pj
        nq = np.linalg.norm(q)
        if nq == 0:
            break
        q = q / nq
        z = z / nq
        a = np.vdot(q, r)
        x = x + a * z
        r = r - a * q
        Ps.append(z)
        Qs.append(q)
        if restart is not None and len(Qs) >= restart:
            Ps, Qs = [], []
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * nb:
            break
    return x, np.array(hist), apps


def gmres_residuals(M, b, steps: int) -> np.ndarray:
    """Residual norms of full (unrestarted) GMRES from x0 = 0 after 0 .. steps steps: the minimum
    of ||b - M y|| over the Krylov space, from the Arnoldi relation and a least-squares solve
    per step (used as the reference for GCR's minimal-residual property)."""
    A = _op(M)
    n = b.shape[0]
    beta = np.linalg.norm(b)
    Q = np.zeros((n, steps + 1), dtype=np.complex128)
    H = np.zeros((steps + 1, steps), dtype=np.complex128)
    Q[:, 0] = b / beta
    out = [beta]
    for j in range(steps):
        w = A(Q[:, j])
        for _pass in range(2):
            h = Q[:, : j + 1].conj().T @ w
            w = w - Q[:, : j + 1] @ h
            H[: j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            Q[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2, dtype=np.complex128)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
        out.append(np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y))
    return np.array(out)


def idrs(M, b, s=4, x0=None, tol=1e-10, maxiter=1000, prec=None, shadow=None, seed=0):
    """Right-preconditioned IDR(s) (induced dimension reduction: P. Sonneveld, M. B. van Gijzen,
    "IDR(s): a family of simple and fast algorithms for solving large nonsymmetric systems of
    linear equations", SIAM J. Sci. Comput. 31 (2008), their prototype algorithm) on
    M (P^-1 v) = b, x = P^-1 v.

    s minimal-residual steps fill the difference matrices dR = -M dU (s columns each); then every
    group of s + 1 steps builds the next residual in the intersection of the previous space with
    the orthogonal complement of the shadow space span(shadow) (n x s; random orthonormal columns
    from ``seed`` when None): c solves (shadow^H dR) c = shadow^H r, v = r - dR c, and the first
    step of the group takes a new minimal-residual parameter omega on v.  The oldest difference
    column is replaced by the new one at every step.  Returns (x, residual norms after every
    step, applications of M)."""
    A = _op(M)
    P = prec if prec is not None else (lambda x: x)
    n = b.shape[0]
    if shadow is None:
        rng = np.random.default_rng(seed)
        shadow, _ = np.linalg.qr(rng.standard_normal((n, s)) + 1j * rng.standard_normal((n, s)))
    S = np.asarray(shadow, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A(x)
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    apps = 0
    dR = np.zeros((n, s), dtype=np.complex128)
    dU = np.zeros((n, s), dtype=np.complex128)
    for k in range(s):  # the first s steps: minimal residual along the preconditioned residual
        z = P(r)
        v = A(z)
        apps += 1
        om = np.vdot(v, r) / np.vdot(v, v)
        dU[:, k] = om * z
        dR[:, k] = -om * v
        x = x + dU[:, k]
        r = r + dR[:, k]
        hist.append(np.linalg.norm(r))
    Mm = S.conj().T @ dR
    m = S.conj().T @ r
    oldest = 0
    om = 1.0
    while apps < maxiter and hist[-1] > tol * nb:
        for k in range(s + 1):
            c = np.linalg.solve(Mm, m)
            q = -dR @ c
            v = r + q
            z = P(v)
            if k == 0:
                t = A(z)
                apps += 1
                om = np.vdot(t, v) / np.vdot(t, t)
                dR[:, oldest] = q - om * t
                dU[:, oldest] = -dU @ c + om * z
            else:
                dU[:, oldest] = -dU @ c + om * z
                dR[:, oldest] = -A(dU[:, oldest])
                apps += 1
            r = r + dR[:, oldest]
            x = x + dU[:, oldest]
            dm = S.conj().T @ dR[:, oldest]
            Mm[:, oldest] = dm
            m = m + dm
            oldest = (oldest + 1) % s
            hist.append(np.linalg.norm(r))
            if hist[-1] <= tol * nb or apps >= maxiter:
                break
    return x, np.array(hist), apps
