"""FP64 CPU oracle for the special weighted low-rank approximation (sWLR).

TEST INFRASTRUCTURE.  This is a plain, slow, obviously correct reference of
the method in Dutta & Li, "A Fast Algorithm for a Weighted Low Rank
Approximation" (arXiv 1703.06303).  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import or run it.  It shares no code with
the GPU library: NumPy/LAPACK primitives (Householder QR, SVD, LU solves) are
used as single steps, in the order the paper states them, in float64.

Problem (5):   min over X1, X2 with rank([X1 X2]) <= r of
                   ||(A1 - X1) o W1||_F^2 + ||A2 - X2||_F^2
where A = [A1 A2] is m x n, A1 the first k columns, W1 (m x k) > 0 and o the
entrywise product.

Functions and the passage each follows:
  objective                 problem (5) / the objective F of problem (8)
  hard_threshold            eq. (2): H_r(M) = U Sigma_r V^T (Eckart-Young-Mirsky)
  ghs                       Theorem 1 (Golub-Hoffman-Stewart), eq. (4)
  closed_form_column_weights  a derived special case of (5): W1(i, j) = w_j
  swlr                      Algorithm 1 (Section 3), with the X1 row update
                            below eq. (9) and the stopping rule of Section 4.1
  round_bf16                BF16 rounding (IEEE binary32 truncated to 8 exponent
                            and 7 fraction bits, round to nearest even)
  swlr_mixed                the reduced-precision schedule: Algorithm 1 with
                            step 7's A2 product on bf16(A2) to a looser
                            threshold, then one exact sweep of Algorithm 1
  objective_colweights,     eq. (6) with W2(i, j) = w2_j (one weight per
  swlr_colweights           column of the unweighted block), reduced to
                            problem (5) by scaling the columns of A2

Readings taken where the paper is loose (all listed in the design notes):
  * X_p = [X1_p, X1_p C_p + D_p] uses the C_p, D_p computed from X1_p; on
    convergence X_p is returned, with no trailing X1 update.
  * Error_p = ||X_p - X_{p-1}||_F; stop when Error_p < tol or
    Error_p / ||X_{p-1}||_F < tol (tol = 1e-7 in the paper), or at max_sweeps.
    "sweeps" is the number of X1 updates done.
  * The rows of the X1 update are independent (E_p is fixed before the loop).
  * 0 <= k <= r <= min(m, n); k = 0 reduces to H_r(A); r = k gives D = 0.
  * W1 entries must be > 0 and finite; a numerically rank-deficient X1 is an
    error (the paper assumes rank(X1) = k).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

# Status codes (same meaning as the library's, defined independently here).
OK, MAX_SWEEPS = 0, 1
E_ARG, E_WEIGHT, E_NONFINITE, E_RANK = -1, -2, -3, -4


class OracleError(ValueError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


@dataclass
class OracleResult:
    X1: np.ndarray
    X2: np.ndarray
    status: int
    sweeps: int
    F: list = field(default_factory=list)          # F(X_p) for p = 0..sweeps
    err: list = field(default_factory=list)        # Error_p for p = 1..sweeps
    rel: list = field(default_factory=list)        # Error_p / ||X_{p-1}||_F
    half: list = field(default_factory=list)       # F(X1_{p+1}, C_p, D_p)
    C: np.ndarray | None = None
    V: np.ndarray | None = None                     # top r-k right singular vectors
    sigma: np.ndarray | None = None                 # all singular values of P^perp A2
    gap: float = float("inf")                       # sigma_l - sigma_{l+1}

    @property
    def X(self):
        return np.hstack([self.X1, self.X2])


def objective(A, W1, X, k):
    """F of problem (5): weighted misfit on the first k columns plus the plain
    misfit on the rest."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    f1 = np.sum(((A[:, :k] - X[:, :k]) * W1) ** 2)
    f2 = np.sum((A[:, k:] - X[:, k:]) ** 2)
    return float(f1 + f2)


def hard_threshold(M, r):
    """Eq. (2): keep the r largest singular values of M, zero the rest."""
    M = np.asarray(M, dtype=np.float64)
    if r <= 0 or M.size == 0:
        return np.zeros_like(M)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    r = min(r, s.size)
    return (U[:, :r] * s[:r]) @ Vt[:r]


def ghs(A1, A2, r, rank_tol=None):
    """Theorem 1 (eq. (4)): the minimiser of ||A2 - X2|| subject to
    rank([A1 X2]) <= r is P_{A1} A2 + H_{r-k}(P^perp_{A1} A2) with
    k = rank(A1).  The projector is built from an SVD basis of A1."""
    A1 = np.asarray(A1, dtype=np.float64)
    A2 = np.asarray(A2, dtype=np.float64)
    if A1.shape[1] == 0:
        return hard_threshold(A2, r)
    U, s, _ = np.linalg.svd(A1, full_matrices=False)
    tol = rank_tol if rank_tol is not None else max(A1.shape) * np.finfo(float).eps * s[0]
    kk = int(np.sum(s > tol))
    if r < kk:
        raise OracleError(E_ARG, "Theorem 1 needs r >= rank(A1)")
    Uk = U[:, :kk]
    proj = Uk @ (Uk.T @ A2)
    return proj + hard_threshold(A2 - proj, r - kk)


def closed_form_column_weights(A, w, k, r):
    """Derived special case of problem (5).  If W1(i, j) = w_j for every row
    (the same weight down each column), put S = diag(w_1..w_k, 1..1).  Then
    F = ||(A - X) S||_F^2 and rank(X S) = rank(X), so by eq. (2) the minimiser
    is X* = H_r(A S) S^{-1} and F* = sum_{i > r} sigma_i(A S)^2."""
    A = np.asarray(A, dtype=np.float64)
    s = np.ones(A.shape[1])
    s[:k] = np.asarray(w, dtype=np.float64)
    X = hard_threshold(A * s, r) / s
    sv = np.linalg.svd(A * s, compute_uv=False)
    return X, float(np.sum(sv[r:] ** 2))


def _validate(A, W1, k, r):
    if A.ndim != 2:
        raise OracleError(E_ARG, "A must be a matrix")
    m, n = A.shape
    if not (0 <= k <= r <= min(m, n)):
        raise OracleError(E_ARG, f"need 0 <= k <= r <= min(m, n); got k={k} r={r} m={m} n={n}")
    if not np.all(np.isfinite(A)):
        raise OracleError(E_NONFINITE, "A has a non-finite entry")
    if k > 0:
        if W1.shape != (m, k):
            raise OracleError(E_ARG, "W1 must be m x k")
        if not np.all(np.isfinite(W1)) or not np.all(W1 > 0):
            raise OracleError(E_WEIGHT, "W1 entries must be finite and > 0")


def swlr(A, W1, k, r, tol=1e-7, max_sweeps=200, X1_0=None, row_chunk=4096, A2_update=None):
    """Algorithm 1 (sWLR), literally, in float64.

    A: m x n; W1: m x k array or a scalar; X1_0: m x k start (the paper
    draws it at random; callers pass it so every implementation starts from
    the same point).  tol <= 0 runs exactly max_sweeps X1 updates.

    A2_update (m x (n - k), optional; not in the paper): a stand-in for A2 in
    step 7's product only.  Writing E_p = A1 o W1 o W1 + A2 Z + X1_p T with
    Z = (I - V V^T) C_p^T and T = C_p V V^T C_p^T (D_p = P_perp A2 V V^T),
    the term A2 Z takes A2_update instead: E_p gains (A2_update - A2) Z.
    Every other step (QR, C_p, D_p, the objective and Error_p) uses A2.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if np.isscalar(W1):
        W1 = np.full((m, k), float(W1))
    W1 = np.asarray(W1, dtype=np.float64)
    _validate(A, W1, k, r)
    if max_sweeps < 0:
        raise OracleError(E_ARG, "max_sweeps must be >= 0")
    A1, A2 = A[:, :k], A[:, k:]
    ell = r - k

    if k == 0:
        # No weighted block: problem (5) is problem (1), solved by eq. (2).
        X2 = hard_threshold(A, r)
        res = OracleResult(X1=np.zeros((m, 0)), X2=X2, status=OK, sweeps=0)
        res.F = [objective(A, W1, X2, 0)]
        return res

    if X1_0 is None:
        raise OracleError(E_ARG, "X1_0 is required (pass the same start to every implementation)")
    X1 = np.array(X1_0, dtype=np.float64).reshape(m, k)
    W1sq = W1 * W1
    eps = np.finfo(np.float64).eps

    res = OracleResult(X1=X1, X2=np.zeros((m, n - k)), status=MAX_SWEEPS, sweeps=0)
    X_prev = None
    p = 0
    while True:
        # Algorithm 1, step 4: QR of X1_p.
        Q, R = np.linalg.qr(X1, mode="reduced")
        d = np.abs(np.diag(R))
        if d.min() <= k * eps * d.max():
            raise OracleError(E_RANK, f"X1 is numerically rank deficient at sweep {p}")
        # Step 5: C_p = R^{-1} Q^T A2.
        B = Q.T @ A2
        C = solve_triangular(R, B, lower=False)
        # Steps 4 and 6: SVD of (I - Q Q^T) A2 and D_p = U (Sigma)_{r-k} V^T.
        N = A2 - Q @ B
        U, s, Vt = np.linalg.svd(N, full_matrices=False)
        if ell > 0:
            D = (U[:, :ell] * s[:ell]) @ Vt[:ell]
        else:
            D = np.zeros_like(A2)
        X2 = X1 @ C + D
        X = np.hstack([X1, X2])
        res.F.append(objective(A, W1, X, k))
        res.C, res.V, res.sigma = C, Vt[:ell].T.copy(), s
        res.gap = float(s[ell - 1] - s[ell]) if 0 < ell < s.size else float("inf")
        res.X1, res.X2, res.sweeps = X1, X2, p
        # Stopping rule (Section 4.1), tested on X_p against X_{p-1}.
        if X_prev is not None:
            e = float(np.linalg.norm(X - X_prev))
            nrm = float(np.linalg.norm(X_prev))
            res.err.append(e)
            res.rel.append(e / nrm if nrm > 0 else float("inf"))
            if tol > 0 and (e < tol or (nrm > 0 and e / nrm < tol)):
                res.status = OK
                return res
        if p >= max_sweeps:
            res.status = MAX_SWEEPS
            return res
        # Step 7: E_p = A1 o W1 o W1 + (A2 - D_p) C_p^T.
        E = A1 * W1sq + (A2 - D) @ C.T
        if A2_update is not None and ell > 0:
            V = Vt[:ell].T
            E = E + (A2_update - A2) @ (C.T - V @ (V.T @ C.T))
        elif A2_update is not None:
            E = E + (A2_update - A2) @ C.T
        S = C @ C.T
        # Steps 8-9: row i of X1_{p+1} = E(i,:) (diag(W1(i,:)^2) + C C^T)^{-1}.
        X1_new = np.empty_like(X1)
        for i0 in range(0, m, row_chunk):
            i1 = min(m, i0 + row_chunk)
            K = np.broadcast_to(S, (i1 - i0, k, k)).copy()
            K[:, np.arange(k), np.arange(k)] += W1sq[i0:i1]
            X1_new[i0:i1] = np.linalg.solve(K, E[i0:i1, :, None])[:, :, 0]
        res.half.append(float(np.sum(((A1 - X1_new) * W1) ** 2)
                              + np.sum((A2 - X1_new @ C - D) ** 2)))
        X_prev = X
        X1 = X1_new
        p += 1


def round_bf16(x):
    """Nearest BF16 value of each float32 entry (ties to the even BF16
    neighbour), returned as float64.  A BF16 number is the upper 16 bits of
    an IEEE binary32 number: sign, 8 exponent bits, 7 fraction bits."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep = u >> 16
    rest = u & 0xFFFF
    up = (rest > 0x8000) | ((rest == 0x8000) & (keep & 1 == 1))
    keep = keep + up.astype(np.uint64)
    return (keep << 16).astype(np.uint32).view(np.float32).astype(np.float64)


# Threshold of the reduced-precision phase (a reading of this project: the
# paper has no mixed-precision schedule).
MIXED_TOL = 1e-5


def swlr_mixed(A, W1, k, r, tol=1e-7, max_sweeps=200, X1_0=None, mixed_tol=MIXED_TOL):
    """Reduced-precision schedule, in float64 arithmetic.

    Phase 1: Algorithm 1 on A with step 7's product A2 Z taken with bf16(A2)
    (A2 rounded to BF16 from float32; `swlr`'s A2_update), every other step
    exact, stopping at max(tol, mixed_tol) (tol > 0) or after max_sweeps - 1
    X1 updates.  Phase 2: Algorithm 1 on A from the X1 reached, for one more
    X1 update when max_sweeps allows it.  The result is phase 2's X_p with
    sweeps = all X1 updates and the status of phase 1."""
    A = np.asarray(A, dtype=np.float64)
    if k == 0:
        return swlr(A, W1, k, r, tol=tol, max_sweeps=max_sweeps, X1_0=X1_0)
    A2b = round_bf16(A[:, k:])
    tol1 = max(tol, mixed_tol) if tol > 0 else tol
    first = swlr(A, W1, k, r, tol=tol1, max_sweeps=max(max_sweeps - 1, 0), X1_0=X1_0,
                 A2_update=A2b)
    extra = min(first.sweeps + 1, max_sweeps) - first.sweeps
    second = swlr(A, W1, k, r, tol=0.0, max_sweeps=extra, X1_0=first.X1)
    second.sweeps = first.sweeps + extra
    second.status = first.status
    second.F = first.F + second.F[1:]  # phase 2 re-evaluates X_p: F_p once
    return second


def objective_colweights(A, W1, w2, X, k):
    """Eq. (6) with W = [W1, 1 w2^T]: ||(A1 - X1) o W1||_F^2 +
    ||(A2 - X2) diag(w2)||_F^2."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    w2 = np.asarray(w2, dtype=np.float64)
    f1 = np.sum(((A[:, :k] - X[:, :k]) * W1) ** 2)
    f2 = np.sum(((A[:, k:] - X[:, k:]) * w2) ** 2)
    return float(f1 + f2)


def swlr_colweights(A, W1, w2, k, r, tol=1e-7, max_sweeps=200, X1_0=None):
    """Eq. (6) restricted to weights that are constant down each column of
    the second block, W2(i, j) = w2_j > 0.  With D2 = diag(w2),
    ||(A2 - X2) D2|| = ||A2 D2 - X2 D2|| and rank([X1, X2 D2]) = rank([X1, X2])
    (D2 is invertible), so (X1, X2) solves it exactly when (X1, X2 D2) solves
    problem (5) for [A1, A2 D2].  Algorithm 1 runs on that problem; its
    iterates, Error_p and the stopping rule are those of the reduced problem,
    and X2 is returned unscaled (X2 D2 D2^-1).  F is the eq. (6) objective,
    which equals the reduced problem's."""
    A = np.asarray(A, dtype=np.float64)
    w2 = np.asarray(w2, dtype=np.float64).reshape(-1)
    if w2.shape != (A.shape[1] - k,):
        raise OracleError(E_ARG, "w2 must have n - k entries")
    if not np.all(np.isfinite(w2)) or not np.all(w2 > 0):
        raise OracleError(E_WEIGHT, "w2 entries must be finite and > 0")
    As = A.copy()
    As[:, k:] = A[:, k:] * w2
    res = swlr(As, W1, k, r, tol=tol, max_sweeps=max_sweeps, X1_0=X1_0)
    res.X2 = res.X2 / w2
    return res


def stationarity_residual(A, W1, k, X1, C, D):
    """Norm of the X1-gradient of F(X1, C, D) (the equation below eq. (9)),
    relative to the norm of its first term's scale.  Zero at a fixed point of
    the X1 update."""
    A1, A2 = A[:, :k], A[:, k:]
    G = (A1 - X1) * W1 * W1 + (A2 - X1 @ C - D) @ C.T
    scale = np.linalg.norm(A1 * W1 * W1) + np.linalg.norm(A2 @ C.T)
    return float(np.linalg.norm(G) / scale)
