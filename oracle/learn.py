"""FP64 reference of the learned warm start (a systems extension around
Algorithm 1, not part of the paper: the paper starts from a random X1_0).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it; it shares no code with the GPU library.

What is computed (all float64 here):

Sketch.  s = vec(Om^T A Ps) / ||Om^T A Ps||_F with Om (m x 16) and Ps
(n x 32) iid N(0, 1) Philox draws (oracle/philox.py) keyed by SEED_OMEGA and
SEED_PSI, element (i, c) of Om being draw i + c m and element (j, c) of Ps
draw j + c n; vec is column-major, so s[a + 16 b] = (Om^T A Ps)[a, b].

Network.  h1 = relu(W1 s + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 with
512 -> 256 -> 256 -> n r, and Y = reshape(y, n x r) column-major
(Y[j, q] = y[j + n q]).  Parameter vector: W1 (256 x 512, row-major), b1,
W2 (256 x 256), b2, W3 (n r x 256), b3.  Start: W_l = N(0, 2 / fan_in)
draws (He scaling) keyed by seed + l, biases 0.

Target.  A solve returns X* = [X1, X1 C + D] with D = (P_perp A2) V V^T, so
X* = [X1, (P_perp A2) V] R with R = [[I_k, C], [0, V^T]] (r x n): the rows of
X* lie in the row space of R.  The target basis T = R^T (n x r).

Loss per sample, Q an orthonormal basis of the target (Cholesky QR of T):
    L = ||Y - Q Q^T Y||_F^2 + lam ||Y^T Y - I_r||_F^2
(Y's columns inside the target space, and orthonormal so that they span it),
averaged over the batch; lam = 1.

Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Decode.  The network predicts a basis Y of the row space of X*.  The start
is the best matrix with that row space under the objective of problem (5):
row i of X_0 is z_i Y^T with
    z_i = argmin_z  sum_{c<k} W1[i,c]^2 (A[i,c] - (Y z)_c)^2
                  + sum_{c>=k} (A[i,c] - (Y z)_c)^2,
a weighted least-squares problem per row (the objective separates over rows
once the row space is fixed), and X1_0 = its first k columns.  With the exact
row space of a fixed point of Algorithm 1 this returns that fixed point's X1.
"""
import numpy as np

from . import philox

D_IN, HID = 512, 256
SK_ROWS, SK_COLS = 16, 32
SEED_OMEGA, SEED_PSI = 0x5EEDA001, 0x5EEDA002
LAM = 1.0
BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def param_count(n, r):
    o = n * r
    return HID * D_IN + HID + HID * HID + HID + o * HID + o


def unpack(p, n, r):
    o = n * r
    sizes = [(HID, D_IN), (HID,), (HID, HID), (HID,), (o, HID), (o,)]
    out, off = [], 0
    for sh in sizes:
        cnt = int(np.prod(sh))
        out.append(p[off:off + cnt].reshape(sh))
        off += cnt
    return out


def init_params(n, r, seed):
    """He-scaled Gaussian weights (Philox keyed by seed + layer), zero biases."""
    o = n * r
    p = np.zeros(param_count(n, r))
    W1, b1, W2, b2, W3, b3 = unpack(p, n, r)
    W1[:] = philox.normals(seed + 1, W1.size).reshape(W1.shape) * np.sqrt(2.0 / D_IN)
    W2[:] = philox.normals(seed + 2, W2.size).reshape(W2.shape) * np.sqrt(2.0 / HID)
    W3[:] = philox.normals(seed + 3, W3.size).reshape(W3.shape) * np.sqrt(2.0 / HID)
    assert o == W3.shape[0]
    return p


def sketch(A):
    """512-value Gaussian sketch of A (m x n), normalised to unit norm."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Om = philox.normals(SEED_OMEGA, m * SK_ROWS).reshape(SK_ROWS, m).T
    Ps = philox.normals(SEED_PSI, n * SK_COLS).reshape(SK_COLS, n).T
    S = Om.T @ A @ Ps
    s = S.reshape(-1, order="F")
    return s / np.linalg.norm(s)


def forward(p, X, n, r):
    """X: B x 512.  Returns (Y: B x n r, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n, r)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def target_basis(C, V, k, r):
    """T = [[I_k, C], [0, V^T]]^T (n x r) from the solve's C (k x n2) and
    V (n2 x (r - k))."""
    n2 = C.shape[1] if k > 0 else V.shape[0]
    T = np.zeros((k + n2, r))
    T[:k, :k] = np.eye(k)
    if k > 0:
        T[k:, :k] = C.T
    T[k:, k:] = V
    return T


def orthonormal(T):
    """Cholesky QR: Q = T R^-1 with R^T R = T^T T."""
    R = np.linalg.cholesky(T.T @ T).T
    return np.linalg.solve(R.T, T.T).T


def loss_and_grad_y(y, T, n, r, lam=LAM):
    """Batch-mean loss and its gradient with respect to y (B x n r); T is
    B x n x r (targets)."""
    B = y.shape[0]
    total = 0.0
    g = np.zeros_like(y)
    I = np.eye(r)
    for b in range(B):
        Y = y[b].reshape(n, r, order="F")
        Q = orthonormal(T[b])
        Rm = Y - Q @ (Q.T @ Y)
        E = Y.T @ Y - I
        total += np.sum(Rm * Rm) + lam * np.sum(E * E)
        G = 2.0 * Rm + 4.0 * lam * (Y @ E)
        g[b] = G.reshape(-1, order="F") / B
    return total / B, g


def backward(p, cache, gy, n, r):
    """Gradient of the loss with respect to the parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n, r)
    X, z1, h1, z2, h2 = cache
    gW3 = gy.T @ h2
    gb3 = gy.sum(axis=0)
    gh2 = gy @ W3
    gz2 = gh2 * (z2 > 0)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(axis=0)
    gh1 = gz2 @ W2
    gz1 = gh1 * (z1 > 0)
    gW1 = gz1.T @ X
    gb1 = gz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(p, g, m, v, t, lr):
    """One Adam update (t = 1, 2, ...); returns new (p, m, v)."""
    m = BETA1 * m + (1 - BETA1) * g
    v = BETA2 * v + (1 - BETA2) * g * g
    mh = m / (1 - BETA1 ** t)
    vh = v / (1 - BETA2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def decode(A, W1, k, Y, row_chunk=512):
    """X1_0 from the row-space basis Y (n x r): per row, the weighted least
    squares fit z_i (QR of the stacked system [w_i * Y1; Y2] z = [w_i * a1_i;
    a2_i], Y1 = Y[:k], Y2 = Y[k:]) and X1_0[i] = Y1 z_i.  W1: m x k or a
    scalar."""
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    m, n = A.shape
    if np.isscalar(W1):
        W1 = np.full((m, k), float(W1))
    W1 = np.asarray(W1, dtype=np.float64)
    Y1, Y2 = Y[:k], Y[k:]
    X1 = np.empty((m, k))
    for i0 in range(0, m, row_chunk):
        i1 = min(m, i0 + row_chunk)
        w = W1[i0:i1]                                   # rows x k
        M = np.concatenate([w[:, :, None] * Y1[None], np.broadcast_to(Y2, (i1 - i0,) + Y2.shape)],
                           axis=1)                      # rows x n x r
        b = np.concatenate([w * A[i0:i1, :k], A[i0:i1, k:]], axis=1)
        Q, R = np.linalg.qr(M)
        z = np.linalg.solve(R, np.einsum('inr,in->ir', Q, b)[:, :, None])[:, :, 0]
        X1[i0:i1] = z @ Y1.T
    return X1
