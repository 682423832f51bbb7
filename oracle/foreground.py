"""Foreground extraction from an sWLR background estimate, scored against a
known mask (the background-subtraction use of the method, Section 4).

TEST INFRASTRUCTURE (see oracle/swlr.py).  Plain float64 NumPy.

The paper estimates the background X of a video matrix A (one frame per
column) and treats what X does not explain as foreground; it scores the
estimate with SSIM against ground truth and does not state how a foreground
mask is read off.  Reading taken here: pixel (i, j) is foreground when
|A(i, j) - X(i, j)| > tau for a threshold tau > 0 given by the caller.

  foreground_mask   |A - X| > tau, entrywise (uint8 0/1, m x n)
  mask_counts       true positives, false positives, false negatives and
                    true negatives of a mask against a reference mask
  residual_from_factors
                    |A - X| for X = [X1, X1 C + (A2 - X1 C) V V^T] (the
                    returned X_p of Algorithm 1: X2_p = X1_p C_p + D_p with
                    D_p = (P^perp A2) V V^T, eq. (2))
"""
from __future__ import annotations

import numpy as np


def foreground_mask(A, X, tau):
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    return (np.abs(A - X) > tau).astype(np.uint8)


def mask_counts(mask, truth):
    """(TP, FP, FN, TN) of a 0/1 mask against a 0/1 reference."""
    m = np.asarray(mask).astype(bool)
    t = np.asarray(truth).astype(bool)
    return (int(np.sum(m & t)), int(np.sum(m & ~t)), int(np.sum(~m & t)),
            int(np.sum(~m & ~t)))


def residual_from_factors(A, X1, C, V, k):
    """|A - X| with X2 = X1 C + (A2 - X1 C) V V^T."""
    A = np.asarray(A, dtype=np.float64)
    X1 = np.asarray(X1, dtype=np.float64)
    A2 = A[:, k:]
    U = A2 - X1 @ C
    R2 = U - (U @ V) @ V.T
    return np.hstack([np.abs(A[:, :k] - X1), np.abs(R2)])
