"""Multistart brute-force minimiser of problem (5) for tiny inputs.

TEST INFRASTRUCTURE (see oracle/swlr.py).  Independent of Algorithm 1: it
parametrises a rank-r matrix as X = L R^T and minimises
F(X) = ||(A - X) o [W1 1]||_F^2 by L-BFGS from many random starts, keeping the
best value.  Problem (5) is non-convex (Section 1 notes there is no closed form
for general weights), so many starts are taken.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def brute_force(A, W1, k, r, starts=200, seed=0, gtol=1e-14, maxiter=20000, w2=None):
    """w2: optional weights of the columns of the second block (eq. (6) with
    W2(i, j) = w2_j); default 1."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    W = np.ones((m, n))
    W[:, :k] = W1
    if w2 is not None:
        W[:, k:] = np.asarray(w2, dtype=np.float64)[None, :]
    W2 = W * W
    rng = np.random.Generator(np.random.PCG64(seed))

    def f_and_g(z):
        L = z[:m * r].reshape(m, r)
        R = z[m * r:].reshape(n, r)
        Res = A - L @ R.T
        f = np.sum(W2 * Res * Res)
        G = -2.0 * W2 * Res
        return f, np.concatenate([(G @ R).ravel(), (G.T @ L).ravel()])

    best_f, best_X = np.inf, None
    scale = np.sqrt(np.linalg.norm(A) / np.sqrt(r * max(m, n)))
    for _ in range(starts):
        z0 = scale * rng.standard_normal(m * r + n * r)
        out = minimize(f_and_g, z0, jac=True, method="L-BFGS-B",
                       options=dict(gtol=gtol, ftol=1e-16, maxiter=maxiter, maxcor=30))
        if out.fun < best_f:
            best_f = float(out.fun)
            L = out.x[:m * r].reshape(m, r)
            R = out.x[m * r:].reshape(n, r)
            best_X = L @ R.T
    return best_f, best_X
