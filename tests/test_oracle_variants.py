"""Pins of the oracle's variants: eq. (6) with one weight per column of the
unweighted block (reduced to problem (5) by column scaling), and foreground
masks read off a background estimate (Section 4's use of the method)."""
import numpy as np
import pytest

from gen import video
from oracle import foreground as FG
from oracle import swlr as O
from oracle.bruteforce import brute_force


def test_colweights_constant_w1_closed_form():
    """Constant W1 = c and column weights w2: with S = diag(c, .., c, w2),
    the objective is ||(A - X) S||^2 and rank(X S) = rank(X), so the
    minimiser is H_r(A S) S^-1 (eq. (2), Eckart-Young-Mirsky)."""
    inst = video.make_instance(9, 10, 30, 4, 7, 2, fg="bernoulli", w1=("const", 50.0), seed=3)
    w2 = video.column_weights(inst.n - inst.k, seed=4)
    s = np.concatenate([np.full(inst.k, 50.0), w2])
    Xs = O.hard_threshold(inst.A * s, inst.r) / s
    Fs = float(np.sum(np.linalg.svd(inst.A * s, compute_uv=False)[inst.r:] ** 2))
    res = O.swlr_colweights(inst.A, 50.0, w2, inst.k, inst.r, tol=1e-14, max_sweeps=3000,
                            X1_0=inst.X1_0)
    assert np.linalg.norm(res.X - Xs) <= 1e-9 * np.linalg.norm(Xs)
    assert res.F[-1] == pytest.approx(Fs, rel=1e-10)
    W1 = np.full((inst.m, inst.k), 50.0)
    assert O.objective_colweights(inst.A, W1, w2, res.X, inst.k) == pytest.approx(Fs, rel=1e-10)


def test_colweights_unit_weights_is_plain_method():
    inst = video.small(seed=8)
    a = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=5, X1_0=inst.X1_0)
    b = O.swlr_colweights(inst.A, inst.W1, np.ones(inst.n - inst.k), inst.k, inst.r, tol=0.0,
                          max_sweeps=5, X1_0=inst.X1_0)
    assert np.array_equal(a.X, b.X) and a.F == b.F


@pytest.mark.parametrize("seed", [1, 2])
def test_colweights_bruteforce_tiny(seed):
    """Log-uniform W1 and random column weights on a tiny instance: the
    converged objective equals a multistart L-BFGS minimiser of the eq. (6)
    objective (independent of Algorithm 1)."""
    inst = video.make_instance(2, 4, 6, 2, 3, 1, fg="bernoulli", w1=("loguniform", 0.0, 1.5),
                               seed=40 + seed)
    w2 = video.column_weights(inst.n - inst.k, seed=50 + seed, lo=0.3, hi=3.0)
    res = O.swlr_colweights(inst.A, inst.W1, w2, inst.k, inst.r, tol=1e-15, max_sweeps=20000,
                            X1_0=inst.X1_0)
    fb, _ = brute_force(inst.A, inst.W1, inst.k, inst.r, starts=60, seed=seed, w2=w2)
    F = O.objective_colweights(inst.A, inst.W1, w2, res.X, inst.k)
    assert F == pytest.approx(res.F[-1], rel=1e-12)
    assert F <= fb * (1 + 1e-9) + 1e-14
    assert fb <= F * (1 + 1e-7) + 1e-14


def test_colweights_rejects_bad_weights():
    inst = video.small(seed=2)
    w2 = np.ones(inst.n - inst.k)
    w2[1] = 0.0
    with pytest.raises(O.OracleError) as e:
        O.swlr_colweights(inst.A, inst.W1, w2, inst.k, inst.r, X1_0=inst.X1_0)
    assert e.value.code == O.E_WEIGHT
    with pytest.raises(O.OracleError):
        O.swlr_colweights(inst.A, inst.W1, w2[:-1], inst.k, inst.r, X1_0=inst.X1_0)


def test_mask_counts_hand_example():
    mask = np.array([[1, 0, 1], [0, 0, 1]], dtype=np.uint8)
    truth = np.array([[1, 1, 0], [0, 0, 1]], dtype=np.uint8)
    assert FG.mask_counts(mask, truth) == (2, 1, 1, 2)
    assert FG.foreground_mask(np.array([[0.0, 1.0]]), np.array([[0.5, 0.9]]), 0.3).tolist() == [[1, 0]]


def test_residual_from_factors_is_the_assembled_iterate():
    """The factor form X2 = X1 C + (A2 - X1 C) V V^T reproduces the iterate
    the oracle assembles from the SVD (X2 = X1 C + D with D = U_l S_l V_l^T)."""
    inst = video.small(m_hw=(10, 12), n=20, k=4, r=8, seed=6)
    res = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=3, X1_0=inst.X1_0)
    R = FG.residual_from_factors(inst.A, res.X1, res.C, res.V, inst.k)
    assert np.allclose(R, np.abs(inst.A - res.X), rtol=0, atol=1e-12)


def test_mask_recovers_generator_foreground():
    """With a large weight on background-only frames the background estimate
    leaves the foreground in A - X: a threshold between the noise (sigma
    0.01) and the foreground magnitudes (>= 0.5) recovers the generator's
    support almost exactly."""
    inst = video.make_instance(20, 24, 60, 10, 12, 2, fg="bernoulli", fg_p=0.05, fg_lo=0.5,
                               fg_hi=1.0, noise=0.01, w1=("const", 1e3), seed=11)
    res = O.swlr(inst.A, inst.w1_const, inst.k, inst.r, tol=1e-10, max_sweeps=500,
                 X1_0=inst.X1_0)
    tp, fp, fn, tn = FG.mask_counts(FG.foreground_mask(inst.A, res.X, 0.25), inst.fg)
    assert tp + fp + fn + tn == inst.A.size
    assert tp / (tp + fn) >= 0.95 and tp / (tp + fp) >= 0.95
