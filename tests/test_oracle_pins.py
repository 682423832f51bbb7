"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a limit, a hand-derived example, a brute-force minimiser, or an
invariant of problem (5).  Together they catch a dropped term, a wrong sign or
index, or a transposed operand anywhere in the oracle's sweep.
"""
import json
import os

import numpy as np
import pytest

from gen import video
from oracle import swlr as O
from oracle.bruteforce import brute_force

HERE = os.path.dirname(os.path.abspath(__file__))


def _orth(rng, m, n):
    q, r = np.linalg.qr(rng.standard_normal((m, n)))
    return q * np.sign(np.diag(r))


def _relerr(X, Y):
    return np.linalg.norm(X - Y) / np.linalg.norm(Y)


# -- closed forms ---------------------------------------------------------------

def test_golden_hand_example():
    """Hand-derived fixture (tests/golden/diag3.json)."""
    g = json.load(open(os.path.join(HERE, "golden", "diag3.json")))
    A = np.array(g["A"])
    for case in g["cases"]:
        X0 = np.array([[0.3], [-1.0], [0.7]])
        res = O.swlr(A, g["w"], g["k"], case["r"], tol=1e-15, max_sweeps=500, X1_0=X0)
        assert np.allclose(res.X, np.array(case["X"]), atol=1e-12)
        assert res.F[-1] == pytest.approx(case["F"], rel=1e-12)


def test_constant_weight_closed_form_config1():
    """Config 1 has W1 = 1e3 everywhere: X* = H_r(A S) S^-1 (derived from (5) and (2))."""
    inst = video.config1()
    res = O.swlr(inst.A, inst.w1_const, inst.k, inst.r, tol=1e-13, max_sweeps=500,
                 X1_0=inst.X1_0)
    Xc, Fc = O.closed_form_column_weights(inst.A, np.full(inst.k, inst.w1_const), inst.k, inst.r)
    assert res.status == O.OK
    assert _relerr(res.X, Xc) < 1e-10
    assert abs(res.F[-1] - Fc) / Fc < 1e-12


def test_column_weights_closed_form():
    """Distinct weights per column (W1(i, j) = w_j): catches a transposed W1."""
    inst = video.small(m_hw=(8, 10), n=14, k=4, r=6, seed=3)
    w = np.array([3.0, 40.0, 7.0, 900.0])
    W1 = np.tile(w, (inst.m, 1))
    res = O.swlr(inst.A, W1, inst.k, inst.r, tol=1e-14, max_sweeps=3000, X1_0=inst.X1_0)
    Xc, Fc = O.closed_form_column_weights(inst.A, w, inst.k, inst.r)
    assert _relerr(res.X, Xc) < 1e-8
    assert abs(res.F[-1] - Fc) / Fc < 1e-11


def test_k0_is_eckart_young():
    """k = 0: problem (5) is problem (1); eq. (2) with a matrix built from a known SVD."""
    rng = np.random.default_rng(5)
    m, n, r = 40, 12, 4
    U, V = _orth(rng, m, n), _orth(rng, n, n)
    s = np.array([9.0, 7.0, 6.5, 5.0, 2.0, 1.5, 1.0, 0.7, 0.5, 0.3, 0.2, 0.1])
    A = (U * s) @ V.T
    res = O.swlr(A, np.zeros((m, 0)), 0, r)
    X = (U[:, :r] * s[:r]) @ V[:, :r].T
    assert _relerr(res.X, X) < 1e-13
    assert res.F[-1] == pytest.approx(np.sum(s[r:] ** 2), rel=1e-12)


def test_uniform_weight_is_eckart_young():
    """W1 = 1: problem (5) is again problem (1), solved by H_r(A) (gapped, known SVD)."""
    rng = np.random.default_rng(6)
    m, n, k, r = 30, 8, 2, 3
    U, V = _orth(rng, m, n), _orth(rng, n, n)
    s = np.array([10.0, 8.0, 6.0, 1.0, 0.8, 0.5, 0.3, 0.1])
    A = (U * s) @ V.T
    X1_0 = rng.standard_normal((m, k))
    res = O.swlr(A, np.ones((m, k)), k, r, tol=1e-15, max_sweeps=20000, X1_0=X1_0)
    X = (U[:, :r] * s[:r]) @ V[:, :r].T
    assert _relerr(res.X, X) < 1e-9
    assert res.F[-1] == pytest.approx(np.sum(s[r:] ** 2), rel=1e-11)


def test_exact_low_rank_is_recovered():
    """rank(A) <= r: X = A and F = 0 for any positive W1."""
    rng = np.random.default_rng(7)
    m, n, k, r = 25, 9, 3, 4
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    W1 = 10 ** rng.uniform(0, 3, size=(m, k))
    res = O.swlr(A, W1, k, r, tol=1e-15, max_sweeps=500, X1_0=rng.standard_normal((m, k)))
    assert _relerr(res.X, A) < 1e-10
    assert res.F[-1] < 1e-18 * np.sum(A ** 2) * 1e3


# -- the GHS limit (Theorem 1) ----------------------------------------------------

def test_large_weight_limit_is_ghs_with_slope_minus_two():
    """W1 = c -> inf forces X1 -> A1, and X2 -> GHS(A1, A2) (Theorem 1).
    The leading correction is O(c^-2)."""
    inst = video.small(m_hw=(8, 10), n=16, k=3, r=6, seed=11)
    A1, A2 = inst.A[:, :3], inst.A[:, 3:]
    X2_ghs = O.ghs(A1, A2, inst.r)
    errs = []
    for c in (1e2, 1e3, 1e4):
        res = O.swlr(inst.A, c, 3, inst.r, tol=1e-15, max_sweeps=2000, X1_0=inst.X1_0)
        errs.append(np.linalg.norm(res.X2 - X2_ghs) / np.linalg.norm(X2_ghs))
        assert np.linalg.norm(res.X1 - A1) / np.linalg.norm(A1) < 10.0 / c ** 2
    slopes = np.diff(np.log10(errs))
    assert np.all(np.abs(slopes + 2.0) < 0.15), (errs, slopes)


# -- brute force ---------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_bruteforce_tiny(seed):
    """On a 7 x 5 problem with row- and column-varying weights, the converged
    objective equals the best of a 150-start L-BFGS minimiser over X = L R^T."""
    rng = np.random.default_rng(100 + seed)
    m, n, k, r = 7, 5, 2, 3
    A = rng.standard_normal((m, n))
    W1 = 10 ** rng.uniform(0, 2, size=(m, k))
    fb, Xb = brute_force(A, W1, k, r, starts=150, seed=seed)
    best = np.inf
    for s in range(5):
        res = O.swlr(A, W1, k, r, tol=1e-15, max_sweeps=20000,
                     X1_0=rng.standard_normal((m, k)))
        best = min(best, res.F[-1])
    assert best <= fb * (1 + 1e-9)
    assert best >= fb * (1 - 1e-9)


# -- invariants of the sweep -------------------------------------------------------

@pytest.fixture(scope="module")
def small_run():
    inst = video.small(m_hw=(10, 12), n=20, k=4, r=7, seed=21,
                       w1=("loguniform", 0.5, 3.0))
    res = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-14, max_sweeps=3000,
                 X1_0=inst.X1_0)
    return inst, res


def test_objective_monotone(small_run):
    """Both half-steps are exact block minimisers (the GHS step over C, D and
    the row update over X1), so F never increases."""
    _, res = small_run
    F, H = np.array(res.F), np.array(res.half)
    scale = F[0]
    # F(X_p) >= F(X1_{p+1}, C_p, D_p) >= F(X_{p+1})
    assert np.all(H - F[:-1] <= 1e-13 * scale)
    assert np.all(F[1:] - H <= 1e-13 * scale)


def test_theorem2_invariant(small_run):
    """Theorem 2: at a solution X2 = P_{X1} A2 + H_{r-k}(P^perp_{X1} A2)."""
    inst, res = small_run
    X2 = O.ghs(res.X1, inst.A[:, inst.k:], inst.r)
    assert _relerr(res.X2, X2) < 1e-12


def test_x1_stationarity(small_run):
    """The X1 gradient of F(X1, C, D) vanishes at the fixed point."""
    inst, res = small_run
    A2 = inst.A[:, inst.k:]
    D = res.X2 - res.X1 @ res.C
    assert O.stationarity_residual(inst.A, inst.W1, inst.k, res.X1, res.C, D) < 1e-12


def test_rank_bound(small_run):
    inst, res = small_run
    s = np.linalg.svd(res.X, compute_uv=False)
    assert s[inst.r] < 1e-10 * s[0]
    assert np.linalg.matrix_rank(res.X1) == inst.k


def test_scale_and_permutation_invariance(small_run):
    inst, res = small_run
    k, r = inst.k, inst.r
    # A -> alpha A gives X -> alpha X, F -> alpha^2 F
    a = 3.5
    res_s = O.swlr(a * inst.A, inst.W1, k, r, tol=1e-14, max_sweeps=3000, X1_0=inst.X1_0)
    assert _relerr(res_s.X, a * res.X) < 1e-9
    assert res_s.F[-1] == pytest.approx(a * a * res.F[-1], rel=1e-11)
    # permuting rows of A and W1 permutes rows of X
    perm = np.random.default_rng(1).permutation(inst.m)
    res_p = O.swlr(inst.A[perm], inst.W1[perm], k, r, tol=1e-14, max_sweeps=3000,
                   X1_0=inst.X1_0[perm])
    assert _relerr(res_p.X, res.X[perm]) < 1e-9
    # permuting the columns of A2 permutes the columns of X2
    cp = np.random.default_rng(2).permutation(inst.n - k)
    A_c = np.hstack([inst.A[:, :k], inst.A[:, k:][:, cp]])
    res_c = O.swlr(A_c, inst.W1, k, r, tol=1e-14, max_sweeps=3000, X1_0=inst.X1_0)
    assert _relerr(res_c.X2, res.X2[:, cp]) < 1e-9


def test_stopping_rule_and_trace():
    """Section 4.1: stop when ||X_p - X_{p-1}|| (absolute or relative to
    ||X_{p-1}||) falls below tol; the trace records each Error_p."""
    inst = video.config1()
    res = O.swlr(inst.A, inst.w1_const, inst.k, inst.r, tol=1e-7, max_sweeps=100,
                 X1_0=inst.X1_0)
    assert res.status == O.OK
    assert len(res.err) == res.sweeps and len(res.F) == res.sweeps + 1
    assert res.rel[-1] < 1e-7 and all(x >= 1e-7 for x in res.rel[:-1])
    res0 = O.swlr(inst.A, inst.w1_const, inst.k, inst.r, tol=1e-7, max_sweeps=0,
                  X1_0=inst.X1_0)
    assert res0.status == O.MAX_SWEEPS and res0.sweeps == 0
    res2 = O.swlr(inst.A, inst.w1_const, inst.k, inst.r, tol=0, max_sweeps=2,
                  X1_0=inst.X1_0)
    assert res2.status == O.MAX_SWEEPS and res2.sweeps == 2


def test_r_equals_k_has_no_d_term():
    inst = video.small(seed=4, k=3, r=3)
    res = O.swlr(inst.A, inst.W1, 3, 3, tol=1e-14, max_sweeps=2000, X1_0=inst.X1_0)
    assert np.linalg.matrix_rank(res.X, tol=1e-9 * np.linalg.norm(res.X)) == 3
    assert _relerr(res.X2, res.X1 @ res.C) < 1e-13


# -- errors --------------------------------------------------------------------------

def test_error_codes():
    inst = video.small(seed=2)
    A, W1, k, r, X0 = inst.A, inst.W1, inst.k, inst.r, inst.X1_0
    with pytest.raises(O.OracleError) as e:
        O.swlr(A, W1, r + 1, r, X1_0=X0)
    assert e.value.code == O.E_ARG
    bad = W1.copy(); bad[3, 1] = 0.0
    with pytest.raises(O.OracleError) as e:
        O.swlr(A, bad, k, r, X1_0=X0)
    assert e.value.code == O.E_WEIGHT
    badA = A.copy(); badA[5, 7] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.swlr(badA, W1, k, r, X1_0=X0)
    assert e.value.code == O.E_NONFINITE
    X0d = X0.copy(); X0d[:, 2] = X0d[:, 0]
    with pytest.raises(O.OracleError) as e:
        O.swlr(A, W1, k, r, X1_0=X0d)
    assert e.value.code == O.E_RANK


# -- reduced-precision schedule --------------------------------------------------

def test_round_bf16_matches_library_and_ties():
    """BF16 rounding equals torch's float32 -> bfloat16 conversion (round to
    nearest even), including exact ties."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(50000) * 10.0 ** rng.uniform(-6, 6, 50000)).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_bf16(x), ref)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: the even neighbour is 1.
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even).
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 1 + 2.0 ** -7],
                    dtype=np.float32)
    assert np.array_equal(O.round_bf16(ties), [1.0, 1 + 2.0 ** -6, -1.0, 1 + 2.0 ** -7])


def test_mixed_schedule_special_cases():
    """With one sweep allowed, phase 1 does no update and the schedule is one
    plain sweep; on data whose A2 is already BF16-exact it is the plain
    iteration split at the phase boundary."""
    inst = video.small(m_hw=(8, 9), n=14, k=3, r=5, seed=8)
    one = O.swlr_mixed(inst.A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=1, X1_0=inst.X1_0)
    ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=1, X1_0=inst.X1_0)
    assert one.sweeps == 1 and _relerr(one.X, ref.X) < 1e-13
    A = np.round(inst.A * 16) / 16            # multiples of 1/16 below 8: BF16-exact
    mix = O.swlr_mixed(A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=4, X1_0=inst.X1_0)
    ref = O.swlr(A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=4, X1_0=inst.X1_0)
    assert mix.sweeps == 4 and _relerr(mix.X, ref.X) < 1e-12


def test_update_stand_in_enters_step7_through_z_only():
    """`swlr`'s A2_update replaces A2 in step 7's product A2 Z alone
    (Z = (I - V V^T) C^T).  Equal to A2 it is the plain sweep.  A perturbation
    G V^T along the sweep's right singular vectors leaves the update as it is
    ((I - V V^T) annihilates it).  The update is affine in the stand-in.  And a
    small perturbation that is orthogonal to col(X1), to the top left singular
    vectors of P_perp A2 and to V leaves Q, C and D unchanged, so the update
    equals the plain sweep of Algorithm 1 on [A1, A2 + perturbation] (this
    fixes the sign of the correction)."""
    inst = video.small(m_hw=(10, 12), n=30, k=4, r=7, rho=2, fg="blobs", seed=17,
                       w1=("loguniform", 1.0, 3.0))
    A, W1, k, r, X0 = inst.A, inst.W1, inst.k, inst.r, inst.X1_0
    A2 = A[:, k:]
    rng = np.random.default_rng(5)
    one = dict(tol=0.0, max_sweeps=1, X1_0=X0)
    base = O.swlr(A, W1, k, r, **one)
    same = O.swlr(A, W1, k, r, A2_update=A2.copy(), **one)
    assert np.array_equal(same.X1, base.X1)
    V = O.swlr(A, W1, k, r, tol=0.0, max_sweeps=0, X1_0=X0).V
    along = O.swlr(A, W1, k, r, A2_update=A2 + rng.standard_normal((A.shape[0], r - k)) @ V.T,
                   **one)
    assert _relerr(along.X1, base.X1) < 1e-12
    dl = 1e-3 * rng.standard_normal(A2.shape)
    x1 = O.swlr(A, W1, k, r, A2_update=A2 + dl, **one).X1
    x2 = O.swlr(A, W1, k, r, A2_update=A2 + 2 * dl, **one).X1
    assert _relerr(x2 - base.X1, 2 * (x1 - base.X1)) < 1e-9
    Q, _ = np.linalg.qr(X0)
    N = A2 - Q @ (Q.T @ A2)
    U, sv, _ = np.linalg.svd(N, full_matrices=False)
    Ul = U[:, :r - k]
    Pl = np.eye(A.shape[0]) - Q @ Q.T - Ul @ Ul.T
    Pr = np.eye(A2.shape[1]) - V @ V.T
    dp = Pl @ rng.standard_normal(A2.shape) @ Pr
    dp *= 1e-3 * sv[r - k - 1] / np.linalg.norm(dp, 2)
    stand_in = O.swlr(A, W1, k, r, A2_update=A2 + dp, **one).X1
    Ap = A.copy()
    Ap[:, k:] = A2 + dp
    plain = O.swlr(Ap, W1, k, r, **one).X1
    assert _relerr(stand_in, plain) < 1e-10


def test_mixed_schedule_meets_objective():
    """Sweeps with the BF16 update product to 1e-5 and one exact sweep land
    within 1e-6 of the converged objective (the accuracy the schedule is
    meant for)."""
    inst = video.small(m_hw=(24, 32), n=60, k=8, r=11, rho=3, fg="blobs", seed=12,
                       w1=("loguniform", 1.0, 4.0))
    ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0)
    mix = O.swlr_mixed(inst.A, inst.W1, inst.k, inst.r, tol=1e-7, max_sweeps=200,
                       X1_0=inst.X1_0)
    assert mix.status == O.OK
    assert abs(mix.F[-1] - ref.F[-1]) / ref.F[-1] < 1e-6
