"""Outer iterations around the hierarchical preconditioner (oracle; test infrastructure only).

* ``stationary``: x_{k+1} = x_k + A_H^{-1}(b - A x_k), stopped when ||e_k|| / ||e_0|| < tol
  with a known solution x* (§7.1, 2D cases).
* ``gmres``: GMRES preconditioned by the h-solver, relative residual < tol (§7, Tables
  2-5). Right preconditioning, so the monitored residual is the true one; restarted,
  modified Gram-Schmidt Arnoldi, Givens rotations.
* ``pcg``: preconditioned conjugate gradients (Hestenes-Stiefel) for SPD A with the SPD
  preconditioner A_H^{-1}; x_0 = 0; stop when ||b - A x_k||_2 / ||b||_2 <= tol on the
  recursive residual, then report the true residual.
* ``fpcg``: the same with the flexible beta_k = r_{k+1}^T (z_{k+1} - z_k) / r_k^T z_k of
  inexact-preconditioner CG (Golub and Ye, 1999). It is not in the paper; it is the outer loop
  read for a preconditioner applied in single precision, where z = M(r) is not exactly linear.
  With a fixed symmetric M it equals ``pcg`` in exact arithmetic (r_{k+1}^T z_k = 0).

``A`` is anything with ``@`` (a SciPy sparse matrix), ``M`` a callable r -> z.
"""
from __future__ import annotations

import numpy as np


def pcg(A, b, M, tol=1e-10, maxiter=1000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = M(r)
    p = z.copy()
    rz = r @ z
    it = 0
    hist = []
    while it < maxiter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            break
        z = M(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true_rel = np.linalg.norm(b - A @ x) / nb
    return x, it, true_rel


def fpcg(A, b, M, tol=1e-10, maxiter=1000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = M(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxiter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) / nb <= tol:
            break
        z_old = z
        z = M(r)
        rz_new = r @ z
        beta = (rz_new - r @ z_old) / rz
        rz = rz_new
        p = z + beta * p
    true_rel = np.linalg.norm(b - A @ x) / nb
    return x, it, true_rel


def gmres(A, b, M, tol=1e-10, restart=200, maxiter=1000):
    """Right-preconditioned restarted GMRES: A M y = b, x = M y. Returns (x, its, true_rel)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    total = 0
    while total < maxiter:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta / nb <= tol:
            break
        m = min(restart, maxiter - total)
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            Z[:, j] = M(V[:, j])
            w = A @ Z[:, j]
            for i in range(j + 1):
                H[i, j] = w @ V[:, i]
                w -= H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            if abs(g[j + 1]) / nb <= tol:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x += Z[:, :j_done] @ y
        if abs(g[j_done]) / nb <= tol:
            break
    true_rel = np.linalg.norm(b - A @ x) / nb
    return x, total, true_rel


def stationary(A, b, M, x_star, tol=1e-6, maxiter=1000):
    """x_{k+1} = x_k + M(b - A x_k) from x_0 = 0 until ||x_k - x*|| / ||x_0 - x*|| < tol."""
    x = np.zeros_like(b)
    e0 = np.linalg.norm(x - x_star)
    for it in range(1, maxiter + 1):
        x = x + M(b - A @ x)
        if np.linalg.norm(x - x_star) / e0 < tol:
            return x, it
    return x, maxiter
