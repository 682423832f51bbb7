"""Seeded synthetic "video" matrices for the special weighted low-rank problem.

The paper evaluates on a rendered surveillance video (its Section 4.2).  That
video is not available here, so these generators stand in for it with the same
structure: each column is one frame of h x w pixels (pixel index y*w + x), the
background is low rank, the foreground is sparse, sensor noise is additive, and
the first k frames are background only (the frames the weight W1 marks as
"almost pure background", Section 1, problem (5)).

This module only draws inputs.  It holds none of the method's arithmetic, so
both the FP64 oracle and the GPU library may be fed from it.

Model (all draws from NumPy's PCG64 stream for the given seed):
  background  U V^T with U (m x rho), V (n x rho) iid N(0, 1)
  foreground  only in columns j >= k, one of
              "bernoulli": iid Bernoulli(p) mask, magnitude U[lo, hi] with a
                           random sign
              "blobs":     8x8 pixel patches at uniform positions, painted one
                           after another (later patches overwrite) until at
                           least a fraction p of the frame is covered; values
                           U[lo, hi] per pixel
  noise       iid N(0, sigma^2) on every entry, A1 included
  fg          the foreground's support (1 where a foreground value was added;
              derived after the draws, so it changes no other value)
  W1          a constant, or iid 10**U(a, b) per entry
  X1_0        iid N(0, 1), m x k, from the stream at seed + 1
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 170306303


@dataclass
class Instance:
    """One synthetic problem: A (m x n, float64, column = frame), W1 (m x k)
    or a constant, the block split k, the rank bound r, and a start X1_0."""
    A: np.ndarray
    k: int
    r: int
    W1: np.ndarray | None
    w1_const: float
    X1_0: np.ndarray
    frame_hw: tuple
    seed: int
    meta: dict = field(default_factory=dict)
    fg: np.ndarray | None = None   # uint8 m x n: 1 where foreground was added

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    def W1_dense(self) -> np.ndarray:
        if self.W1 is not None:
            return self.W1
        return np.full((self.m, self.k), self.w1_const)


def _bernoulli_foreground(rng, m, ncols, p, lo, hi):
    mask = rng.random((m, ncols)) < p
    mag = rng.uniform(lo, hi, size=(m, ncols))
    sign = np.where(rng.random((m, ncols)) < 0.5, -1.0, 1.0)
    return np.where(mask, mag * sign, 0.0)


def _blob_foreground(rng, h, w, ncols, p, lo, hi, patch=8):
    m = h * w
    out = np.zeros((m, ncols))
    need = int(np.ceil(p * m))
    for j in range(ncols):
        frame = np.zeros((h, w))
        covered = np.zeros((h, w), dtype=bool)
        ncov = 0
        while ncov < need:
            y = int(rng.integers(0, h - patch + 1))
            x = int(rng.integers(0, w - patch + 1))
            frame[y:y + patch, x:x + patch] = rng.uniform(lo, hi, size=(patch, patch))
            before = covered[y:y + patch, x:x + patch].sum()
            covered[y:y + patch, x:x + patch] = True
            ncov += patch * patch - int(before)
        out[:, j] = frame.reshape(-1)
    return out


def make_instance(h, w, n, k, r, rho, fg="blobs", fg_p=0.10, fg_lo=0.3, fg_hi=1.0,
                  noise=0.02, w1=("loguniform", 1.0, 4.0), seed=BASE_SEED,
                  dtype=np.float64) -> Instance:
    """Draw one instance.  `w1` is ("const", c) or ("loguniform", a, b) for
    entries 10**U(a, b).  The returned A is rounded to `dtype` and held as
    float64 so that a float32 device copy and the oracle see identical values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = h * w
    U = rng.standard_normal((m, rho))
    V = rng.standard_normal((n, rho))
    A = U @ V.T
    if fg == "bernoulli":
        F = _bernoulli_foreground(rng, m, n - k, fg_p, fg_lo, fg_hi)
    elif fg == "blobs":
        F = _blob_foreground(rng, h, w, n - k, fg_p, fg_lo, fg_hi)
    elif fg == "none":
        F = np.zeros((m, n - k))
    else:
        raise ValueError(fg)
    A[:, k:] += F
    fgmask = np.zeros((m, n), dtype=np.uint8, order="F")
    fgmask[:, k:] = F != 0
    A += noise * rng.standard_normal((m, n))
    if w1[0] == "const":
        W1, wc = None, float(w1[1])
    elif w1[0] == "loguniform":
        W1, wc = 10.0 ** rng.uniform(w1[1], w1[2], size=(m, k)), 0.0
    else:
        raise ValueError(w1)
    rng0 = np.random.Generator(np.random.PCG64(seed + 1))
    X1_0 = rng0.standard_normal((m, k))
    A = np.asfortranarray(A.astype(dtype).astype(np.float64))
    if W1 is not None:
        W1 = np.asfortranarray(W1.astype(dtype).astype(np.float64))
    X1_0 = np.asfortranarray(X1_0.astype(dtype).astype(np.float64))
    return Instance(A=A, k=k, r=r, W1=W1, w1_const=wc, X1_0=X1_0, frame_hw=(h, w),
                    seed=seed, meta=dict(rho=rho, fg=fg, fg_p=fg_p, noise=noise, w1=w1),
                    fg=fgmask)


# -- the five workloads -------------------------------------------------------

def config1(seed=BASE_SEED + 10, dtype=np.float64) -> Instance:
    """30x40 frames, n=60, rank-2 background, 5% Bernoulli foreground with
    magnitude U[0.5,1] and random sign, noise 0.01, k=10, W1 = 1e3, r=12."""
    return make_instance(30, 40, 60, 10, 12, 2, fg="bernoulli", fg_p=0.05, fg_lo=0.5,
                         fg_hi=1.0, noise=0.01, w1=("const", 1e3), seed=seed, dtype=dtype)


def config2(seed=BASE_SEED + 20, dtype=np.float32) -> Instance:
    """120x160 frames, n=200, rank-3 background, 10% 8x8 blob foreground with
    values U[0.3,1], noise 0.02, k=20, W1 = 10**U(1,4), r=25."""
    return make_instance(120, 160, 200, 20, 25, 3, fg="blobs", fg_p=0.10, fg_lo=0.3,
                         fg_hi=1.0, noise=0.02, w1=("loguniform", 1.0, 4.0), seed=seed,
                         dtype=dtype)


def config3(seed=BASE_SEED + 30, dtype=np.float32) -> Instance:
    """240x320 frames, n=600, rank-5 background, 10% Bernoulli foreground with
    magnitude U[0.5,1] and random sign, noise 0.02, k=50, W1 = 1e3, r=60."""
    return make_instance(240, 320, 600, 50, 60, 5, fg="bernoulli", fg_p=0.10, fg_lo=0.5,
                         fg_hi=1.0, noise=0.02, w1=("const", 1e3), seed=seed, dtype=dtype)


C4_FRAMES = ((60, 80), (120, 160), (240, 320))


def config4_shapes(count=64, seed=BASE_SEED + 4000):
    """Shapes of the batched workload: frame size uniform over C4_FRAMES,
    n ~ U[100,400], k ~ U[5,40], r = k + U[2,8]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        h, w = C4_FRAMES[int(rng.integers(0, 3))]
        n = int(rng.integers(100, 401))
        k = int(rng.integers(5, 41))
        r = k + int(rng.integers(2, 9))
        out.append((h, w, n, k, r))
    return out


def config4_instance(i, shape, dtype=np.float32) -> Instance:
    h, w, n, k, r = shape
    return make_instance(h, w, n, k, r, 3, fg="blobs", fg_p=0.10, fg_lo=0.3, fg_hi=1.0,
                         noise=0.02, w1=("loguniform", 1.0, 4.0),
                         seed=BASE_SEED + 4000 + 1 + 2 * i, dtype=dtype)


def config5_seed(i, heldout=False) -> int:
    """Disjoint seed ranges for warm-start training and held-out evaluation."""
    return BASE_SEED + (6_000_000 if heldout else 5_000_000) + 2 * i


def column_weights(n2, seed, lo=0.5, hi=2.0):
    """Weights w2 (n2 entries, 10**U(log10 lo, log10 hi)) for the variant of
    the problem with one weight per column of the unweighted block."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=n2)


def small(m_hw=(6, 8), n=12, k=3, r=5, rho=2, w1=("loguniform", 0.0, 2.0), fg="bernoulli",
          seed=1, dtype=np.float64, noise=0.05) -> Instance:
    """A small instance for tests (defaults: 48 x 12)."""
    return make_instance(m_hw[0], m_hw[1], n, k, r, rho, fg=fg, fg_p=0.1, fg_lo=0.5,
                         fg_hi=1.0, noise=noise, w1=w1, seed=seed, dtype=dtype)
