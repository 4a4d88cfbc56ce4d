"""Lowest eigenpair by the Lanczos method (oracle; test infrastructure).

The paper's Lanczos solver (Sec. 3.3) needs only the product x += H y.  It
gives no tolerance, iteration cap or reorthogonalisation scheme; the reading
used here: the initial vector is normalised, every new Lanczos vector is
orthogonalised twice against all previous ones (full reorthogonalisation),
the tridiagonal matrix is diagonalised after each step, and the run stops
when the residual estimate beta_j |u_j| of the lowest Ritz pair is at most
``tol`` or after ``max_iter`` steps.  The returned residual is recomputed
explicitly as || H psi - E psi ||.
"""
from __future__ import annotations

import numpy as np


def tridiagonal(alphas, betas):
    """Dense symmetric tridiagonal matrix from its diagonal and off-diagonal."""
    n = len(alphas)
    T = np.diag(np.asarray(alphas, dtype=float))
    for i in range(n - 1):
        T[i, i + 1] = T[i + 1, i] = betas[i]
    return T


def lanczos_ground(matvec, v0, max_iter=300, tol=1e-10):
    """(E0, psi, iterations, residual) for the lowest eigenpair of H."""
    v = np.array(v0, dtype=float)
    v /= np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    theta, u = None, None
    it = 0
    for it in range(1, max_iter + 1):
        w = matvec(V[-1])
        a = float(np.dot(V[-1], w))
        w = w - a * V[-1]
        if len(V) > 1:
            w = w - betas[-1] * V[-2]
        Vm = np.array(V).T
        for _ in range(2):
            w = w - Vm @ (Vm.T @ w)
        b = float(np.linalg.norm(w))
        alphas.append(a)
        evals, evecs = np.linalg.eigh(tridiagonal(alphas, betas))
        theta, u = float(evals[0]), evecs[:, 0]
        if b * abs(u[-1]) <= tol or b <= 1e-300:
            break
        betas.append(b)
        V.append(w / b)
    Vm = np.array(V[:len(alphas)]).T
    psi = Vm @ u
    psi /= np.linalg.norm(psi)
    r = matvec(psi) - theta * psi
    return theta, psi, it, float(np.linalg.norm(r))
