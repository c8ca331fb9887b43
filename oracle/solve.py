"""Reference solvers for A x = b.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``dense_solve``: builds A column by column and solves with LU (tiny grids):
  the exact discrete solution.
* ``gmres``: restarted GMRES (the paper names GMRES beside Bi-CGStab as a
  suitable unpreconditioned iteration, Introduction and Discussion).  Arnoldi
  with classical Gram-Schmidt applied twice (as stable as the modified
  variant; the basis is a matrix, so each pass is two matrix-vector
  products); the small least-squares problem is solved with
  ``numpy.linalg.lstsq`` at every step; stops on the true relative residual
  ||b - A x|| / ||b|| <= tol, x0 = 0.
* ``bicgstab``: unpreconditioned Bi-CGStab as used in the numerical section.
* ``neumann``: the fixed-point iteration x <- b + (I - A) x, i.e. the Neumann
  series sum_n B^n b of the Laplace existence proof (eq. intLap), which
  converges because ||B|| < 1 there.
"""

from __future__ import annotations

import numpy as np


def _norm(v) -> float:
    return float(np.sqrt(np.vdot(v, v).real))


def dense_matrix(apply, shape) -> np.ndarray:
    size = int(np.prod(shape))
    A = np.empty((size, size), dtype=np.complex128)
    e = np.zeros(size, dtype=np.complex128)
    for k in range(size):
        e[k] = 1.0
        A[:, k] = apply(e.reshape(shape)).reshape(-1)
        e[k] = 0.0
    return A


def dense_solve(apply, b: np.ndarray) -> np.ndarray:
    A = dense_matrix(apply, b.shape)
    return np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)


def gmres(apply, b: np.ndarray, tol: float = 1e-13, restart: int = 100, maxiter: int = 2000,
          x0: np.ndarray = None):
    """Returns (x, info) with info = {'matvecs', 'rel_residual', 'converged', 'history'}."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    bnorm = _norm(b)
    info = {"matvecs": 0, "history": [], "converged": False}
    if bnorm == 0.0:
        info.update(rel_residual=0.0, converged=True)
        return np.zeros_like(b), info
    while True:
        r = b - apply(x)
        beta = _norm(r)
        rel = beta / bnorm
        info["history"].append(rel)
        if rel <= tol or info["matvecs"] >= maxiter:
            break
        m = min(restart, max(1, maxiter - info["matvecs"]))
        V = np.empty((m + 1, b.size), dtype=np.complex128)
        V[0] = (r / beta).ravel()
        Hh = np.zeros((m + 1, m), dtype=np.complex128)
        k = 0
        y = np.zeros(0)
        for j in range(m):
            w = apply(V[j].reshape(b.shape)).ravel()
            info["matvecs"] += 1
            for _ in range(2):                  # classical Gram-Schmidt, twice
                h = np.conj(V[:j + 1] @ np.conj(w))  # h_i = (V_i, w)
                w = w - V[:j + 1].T @ h
                Hh[:j + 1, j] += h
            Hh[j + 1, j] = _norm(w)
            rhs = np.zeros(j + 2, dtype=np.complex128)
            rhs[0] = beta
            y = np.linalg.lstsq(Hh[:j + 2, :j + 1], rhs, rcond=None)[0]
            est = _norm(rhs - Hh[:j + 2, :j + 1] @ y)
            k = j + 1
            if est <= 0.5 * tol * bnorm or Hh[j + 1, j] == 0 or info["matvecs"] >= maxiter:
                break
            V[j + 1] = w / Hh[j + 1, j]
        x = x + (V[:k].T @ y[:k]).reshape(b.shape)
    info["rel_residual"] = rel
    info["converged"] = rel <= tol
    return x, info


def bicgstab(apply, b: np.ndarray, tol: float = 1e-13, maxiter: int = 2000, x0=None):
    """Unpreconditioned Bi-CGStab; stops on the recomputed true residual."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    bnorm = _norm(b)
    info = {"matvecs": 0, "converged": False, "history": []}
    r = b - apply(x)
    rhat = r.copy()
    rho = alpha = om = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    while info["matvecs"] < maxiter:
        rho_new = np.vdot(rhat, r)
        beta = (rho_new / rho) * (alpha / om)
        p = r + beta * (p - om * v)
        v = apply(p)
        info["matvecs"] += 1
        alpha = rho_new / np.vdot(rhat, v)
        s = r - alpha * v
        if _norm(s) <= tol * bnorm:
            x = x + alpha * p
            r = s
            break
        t = apply(s)
        info["matvecs"] += 1
        om = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + om * s
        r = s - om * t
        rho = rho_new
        info["history"].append(_norm(r) / bnorm)
        if _norm(r) <= tol * bnorm:
            break
    rel = _norm(b - apply(x)) / bnorm
    info["rel_residual"] = rel
    info["converged"] = rel <= tol * 10
    return x, info


def neumann(apply, b: np.ndarray, tol: float = 1e-12, maxiter: int = 500):
    """x_{k+1} = b + x_k - A x_k (Neumann series of the contraction)."""
    x = b.copy()
    bnorm = _norm(b)
    for k in range(maxiter):
        r = b - apply(x)
        if _norm(r) <= tol * bnorm:
            return x, {"iterations": k, "rel_residual": _norm(r) / bnorm}
        x = x + r
    return x, {"iterations": maxiter, "rel_residual": _norm(b - apply(x)) / bnorm}
