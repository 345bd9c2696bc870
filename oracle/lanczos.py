"""Lanczos ground-state solver on the host, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's DMRG needs the lowest eigenpair of the two-site effective Hamiltonian at
every step but does not say how it is found.  This is the textbook Lanczos method:

  v_0 = theta_0 / |theta_0|
  w = H v_j;  alpha_j = Re <v_j, w>;  w -= alpha_j v_j + beta_{j-1} v_{j-1}
  w -= V (V^H w) twice (classical Gram-Schmidt, repeated once, against all v_0..v_j)
  beta_j = |w|;  v_{j+1} = w / beta_j

It stops after ``max_iter`` products with H, at breakdown (beta_j <= tol * |T|, with
|T| = max_i |alpha_i| + |beta_i| + |beta_{i-1}|), or, if ``tol_res`` is given, when
the residual norm beta_j |y_j| of the lowest Ritz pair is below ``tol_res``.  The
lowest eigenpair (E, y) of the tridiagonal T comes from LAPACK (scipy
``eigh_tridiagonal``), and the Ritz vector is V y.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos(matvec, v0: np.ndarray, max_iter: int = 30, tol: float = 1e-14,
            tol_res: float | None = None):
    """Returns (E, ritz_vector, iterations, alphas, betas)."""
    v = v0 / np.linalg.norm(v0)
    V = [v]
    alphas: list[float] = []
    betas: list[float] = []
    for j in range(max_iter):
        w = matvec(V[j])
        a = float(np.vdot(V[j], w).real)
        w = w - a * V[j]
        if j > 0:
            w = w - betas[j - 1] * V[j - 1]
        Vm = np.array(V)
        for _ in range(2):
            w = w - Vm.T @ (Vm.conj() @ w)
        b = float(np.linalg.norm(w))
        alphas.append(a)
        tnorm = max(abs(alphas[i]) + (betas[i] if i < len(betas) else b) +
                    (betas[i - 1] if i > 0 else 0.0) for i in range(len(alphas)))
        if b <= tol * tnorm:
            break
        if tol_res is not None:
            e, y = _lowest(alphas, betas)
            if b * abs(y[-1]) < tol_res:
                break
        if j == max_iter - 1:
            break
        betas.append(b)
        V.append(w / b)
    k = len(alphas)
    e, y = _lowest(alphas, betas[:k - 1])
    ritz = np.array(V[:k]).T @ y
    return e, ritz / np.linalg.norm(ritz), k, np.array(alphas), np.array(betas[:k - 1])


def _lowest(alphas, betas):
    if len(alphas) == 1:
        return alphas[0], np.ones(1)
    e, y = eigh_tridiagonal(np.array(alphas), np.array(betas[:len(alphas) - 1]),
                            select="i", select_range=(0, 0))
    return float(e[0]), y[:, 0]


def ground_state(matvec, v0: np.ndarray, tol_res: float = 1e-10, krylov: int = 30,
                 max_restarts: int = 200):
    """Lowest eigenpair to a residual |H v - E v| <= tol_res * |H| by explicitly restarted
    Lanczos: each cycle runs ``lanczos`` for ``krylov`` steps from the previous cycle's
    Ritz vector.  |H| is estimated by the largest |alpha_i| + beta_i + beta_{i-1} seen.
    Returns (E, v, residual norm, matvecs)."""
    v = v0 / np.linalg.norm(v0)
    hnorm = 0.0
    n_mv = 0
    e = float("nan")
    res = float("inf")
    for _ in range(max_restarts):
        e, v, k, al, be = lanczos(matvec, v, max_iter=krylov)
        n_mv += k
        b = np.concatenate([be, [0.0]])
        hnorm = max(hnorm, float(np.max(np.abs(al) + b + np.concatenate([[0.0], be]))))
        r = matvec(v) - e * v
        n_mv += 1
        res = float(np.linalg.norm(r))
        if res <= tol_res * hnorm:
            break
    return e, v, res, n_mv
