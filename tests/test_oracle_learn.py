"""Pins of the learned-warm-start oracle (oracle/learn.py, oracle/philox.py)
against facts that do not come from the oracle itself: published test
vectors, finite differences, closed forms and invariances."""
import numpy as np
import pytest

from gen import video
from oracle import learn as L
from oracle import philox as P
from oracle import swlr as O


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator
    (Random123): counter, key -> output."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in kat:
        got = P.philox4x32_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(x) for x in got] == list(want)


def test_normals_box_muller():
    z = P.normals(12345, 200001)
    assert z.shape == (200001,)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    # a pair's squared radius is -2 ln u0 with u0 from the first two words
    x = P.philox4x32_10(np.array([7, 0, 0, 0], dtype=np.uint64),
                        np.array([12345, 0], dtype=np.uint64)).astype(float)
    u0 = (x[0] + 0.5) / 2 ** 32 + x[1] / 2 ** 64
    assert z[14] ** 2 + z[15] ** 2 == pytest.approx(-2 * np.log(u0), rel=1e-12)


def _tiny(n=6, r=2, B=3, seed=3):
    rng = np.random.default_rng(seed)
    p = L.init_params(n, r, seed=11)
    X = rng.standard_normal((B, L.D_IN))
    T = rng.standard_normal((B, n, r))
    return p, X, T


def test_backward_matches_finite_differences():
    n, r = 6, 2
    p, X, T = _tiny(n, r)

    def f(q):
        y, _ = L.forward(q, X, n, r)
        return L.loss_and_grad_y(y, T, n, r)[0]

    y, cache = L.forward(p, X, n, r)
    _, gy = L.loss_and_grad_y(y, T, n, r)
    g = L.backward(p, cache, gy, n, r)
    rng = np.random.default_rng(0)
    sizes = np.cumsum([0, 256 * 512, 256, 256 * 256, 256, n * r * 256, n * r])
    idx = np.concatenate([rng.integers(sizes[i], sizes[i + 1], 6) for i in range(6)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (f(p + e) - f(p - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-8), i


def test_loss_zero_on_any_orthonormal_basis_of_the_target():
    rng = np.random.default_rng(4)
    n, r = 9, 3
    T = rng.standard_normal((1, n, r))
    Q, _ = np.linalg.qr(T[0])
    Om, _ = np.linalg.qr(rng.standard_normal((r, r)))
    for Y in (Q, Q @ Om):
        loss, g = L.loss_and_grad_y(Y.reshape(1, -1, order="F"), T, n, r)
        assert loss < 1e-24 and np.abs(g).max() < 1e-12
    # a component orthogonal to the target costs its squared norm (plus the
    # orthonormality term)
    u = rng.standard_normal(n)
    u -= Q @ (Q.T @ u)
    u /= np.linalg.norm(u)
    Y = Q.copy()
    Y[:, 0] = 0.6 * Q[:, 0] + 0.8 * u
    loss, _ = L.loss_and_grad_y(Y.reshape(1, -1, order="F"), T, n, r, lam=0.0)
    assert loss == pytest.approx(0.64, rel=1e-12)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -2e-3, 0.5])
    p1, m, v = L.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    # m_hat = g and v_hat = g^2 at t = 1
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + L.ADAM_EPS), rtol=1e-12)


def test_adam_constant_gradient_steps_by_learning_rate():
    """With the same gradient g at every step, the bias-corrected moments are
    m_hat = g and v_hat = g^2 at every t (m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2), so each step moves p by -lr g / (|g| + eps).  A
    dropped b1 m or b2 v term, or a wrong power in a bias correction, breaks
    this from t = 2 on."""
    g = np.array([3.0, -2e-3, 0.5, -7.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    step = -0.01 * g / (np.abs(g) + L.ADAM_EPS)
    for t in range(1, 8):
        p, m, v = L.adam_step(p, g, m, v, t, 0.01)
        assert np.allclose(p, t * step, rtol=1e-12, atol=0)
        assert np.allclose(m, (1 - L.BETA1 ** t) * g, rtol=1e-12)
        assert np.allclose(v, (1 - L.BETA2 ** t) * g * g, rtol=1e-12)


def test_adam_alternating_gradient_second_step():
    """Gradients g then -g.  By hand: m_2 = b1 (1 - b1) g - (1 - b1) g
    = -(1 - b1)^2 g, so m_hat_2 = -(1 - b1) g / (1 + b1); v_2 = (1 - b2)(b2 + 1) g^2
    = (1 - b2^2) g^2, so v_hat_2 = g^2.  The second step is therefore
    +lr (1 - b1) / (1 + b1) g / (|g| + eps): with b1 = 0.9 it is 1/19 of the
    first step's size and points the other way."""
    g = np.array([2.0, -0.25])
    p1, m, v = L.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 0.1)
    p2, m, v = L.adam_step(p1, -g, m, v, 2, 0.1)
    unit = g / (np.abs(g) + L.ADAM_EPS)
    assert np.allclose(p1, -0.1 * unit, rtol=1e-12)
    assert np.allclose(p2 - p1, 0.1 * (0.1 / 1.9) * unit, rtol=1e-12)


def test_target_basis_contains_the_solution_rows():
    inst = video.small(m_hw=(10, 12), n=20, k=4, r=7, seed=21, w1=("loguniform", 0.5, 3.0))
    res = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=0.0, max_sweeps=3, X1_0=inst.X1_0)
    T = L.target_basis(res.C, res.V, inst.k, inst.r)
    Q = L.orthonormal(T)
    X = res.X
    assert np.linalg.norm(X - (X @ Q) @ Q.T) <= 1e-12 * np.linalg.norm(X)
    assert np.allclose(Q.T @ Q, np.eye(inst.r), atol=1e-12)


def test_decode_returns_the_fixed_point_for_its_row_space():
    """Once the row space is fixed, problem (5) separates over rows, and a
    fixed point of Algorithm 1 is optimal among matrices with its own row
    space (both stationarity conditions of the per-row problem are the X1
    update and D = (P_perp A2) V V^T).  The decode of that row space must
    therefore give the fixed point's X1 back, with log-uniform weights."""
    inst = video.small(m_hw=(8, 10), n=14, k=4, r=6, rho=2, seed=17)
    res = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-14, max_sweeps=2000, X1_0=inst.X1_0)
    assert res.status == O.OK
    T = L.target_basis(res.C, res.V, inst.k, inst.r)
    X1 = L.decode(inst.A, inst.W1, inst.k, T)
    assert np.linalg.norm(X1 - res.X1) <= 1e-8 * np.linalg.norm(res.X1)
    # a start off the fixed point is not returned unchanged
    T2 = T + 0.1 * np.random.default_rng(3).standard_normal(T.shape)
    assert np.linalg.norm(L.decode(inst.A, inst.W1, inst.k, T2) - res.X1) > 1e-4 * np.linalg.norm(res.X1)


def test_decode_special_cases():
    rng = np.random.default_rng(9)
    m, n, k, r = 40, 12, 3, 5
    A = rng.standard_normal((m, n))
    W1 = 10.0 ** rng.uniform(0, 3, size=(m, k))
    # the whole of R^n as row space: the start is A1 itself, for any weights
    Yf = rng.standard_normal((n, n))
    assert np.allclose(L.decode(A, W1, k, Yf), A[:, :k], atol=1e-9)
    # unit weights: orthogonal projection of the rows of A on span(Y)
    Y = rng.standard_normal((n, r))
    Pr = Y @ np.linalg.solve(Y.T @ Y, Y.T)
    assert np.allclose(L.decode(A, 1.0, k, Y), (A @ Pr)[:, :k], atol=1e-10)
    # only the row space matters
    M = rng.standard_normal((r, r)) + 3 * np.eye(r)
    assert np.allclose(L.decode(A, W1, k, Y), L.decode(A, W1, k, Y @ M), atol=1e-9)
    # optimality in the row space: perturbing a row's coefficients raises
    # that row's weighted residual, and the decode's x1 is the optimum's
    X1 = L.decode(A, W1, k, Y)
    def row_cost(i, z):
        x = Y @ z
        return np.sum((W1[i] * (A[i, :k] - x[:k])) ** 2) + np.sum((A[i, k:] - x[k:]) ** 2)
    for i in (0, 7, 31):
        z = np.linalg.lstsq(np.vstack([W1[i][:, None] * Y[:k], Y[k:]]),
                            np.concatenate([W1[i] * A[i, :k], A[i, k:]]), rcond=None)[0]
        c0 = row_cost(i, z)
        for _ in range(5):
            assert row_cost(i, z + 1e-3 * rng.standard_normal(r)) > c0
        assert np.allclose(Y[:k] @ z, X1[i], atol=1e-9)


def test_sketch_of_a_single_entry_is_an_outer_product():
    m, n = 50, 7
    A = np.zeros((m, n))
    A[13, 4] = 2.5
    s = L.sketch(A).reshape(L.SK_ROWS, L.SK_COLS, order="F")
    om = P.normals(L.SEED_OMEGA, m * L.SK_ROWS).reshape(L.SK_ROWS, m)[:, 13]
    ps = P.normals(L.SEED_PSI, n * L.SK_COLS).reshape(L.SK_COLS, n)[:, 4]
    want = np.outer(om, ps)
    assert np.allclose(s, want / np.linalg.norm(want), atol=1e-14)
    assert np.allclose(L.sketch(3.0 * A), L.sketch(A), atol=1e-15)
