"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), in NumPy.

TEST INFRASTRUCTURE (part of the oracle).  Random numbers that the method
draws on the device (the random start, the Gaussian sketches of the learned
warm start) are reproduced here from the generator's published definition so
that both sides see the same draws without sharing code.

Round function on a counter (c0, c1, c2, c3) with key (k0, k1):
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2   (64-bit products)
    counter <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
    key     <- (k0 + W0, k1 + W1)                  (mod 2^32)
ten times, with M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9,
W1 = 0xBB67AE85.

Normal draws: element pair e uses counter (e mod 2^32, e >> 32, 0, 0) and key
(seed mod 2^32, seed >> 32).  The four output words give two uniforms in
(0, 1), u0 = (x0 + 1/2) 2^-32 + x1 2^-64 and u1 = (x2 + 1/2) 2^-32 + x3 2^-64,
and the Box-Muller pair z0 = sqrt(-2 ln u0) cos(2 pi u1),
z1 = sqrt(-2 ln u0) sin(2 pi u1) is elements 2e and 2e + 1.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint64 array of 32-bit words, key: (..., 2).  Returns the
    (..., 4) output words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK
    for _ in range(10):
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack(c, axis=-1)


def normals(seed, count):
    """`count` N(0, 1) draws (float64) keyed by `seed`, in element order."""
    pairs = (count + 1) // 2
    e = np.arange(pairs, dtype=np.uint64)
    ctr = np.zeros((pairs, 4), dtype=np.uint64)
    ctr[:, 0] = e & np.uint64(MASK)
    ctr[:, 1] = e >> np.uint64(32)
    key = np.zeros((pairs, 2), dtype=np.uint64)
    key[:, 0] = np.uint64(seed & MASK)
    key[:, 1] = np.uint64((seed >> 32) & MASK)
    x = philox4x32_10(ctr, key).astype(np.float64)
    inv = 1.0 / 4294967296.0
    u0 = (x[:, 0] + 0.5) * inv + x[:, 1] * inv * inv
    u1 = (x[:, 2] + 0.5) * inv + x[:, 3] * inv * inv
    rad = np.sqrt(-2.0 * np.log(u0))
    z = np.empty(2 * pairs)
    z[0::2] = rad * np.cos(2.0 * np.pi * u1)
    z[1::2] = rad * np.sin(2.0 * np.pi * u1)
    return z[:count]
