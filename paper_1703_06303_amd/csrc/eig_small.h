// Small dense steps shared by the eigen kernels: an upper Cholesky and a
// parallel cyclic Jacobi eigensolver of an nb x nb matrix (nb <= 32, leading
// dimension WLRA_BMAX) in LDS, both run by wavefront 0 of the workgroup and
// followed by a workgroup barrier.
#pragma once

#include "common.h"

// Upper Cholesky in place of G (nb x nb, ld WLRA_BMAX) by wavefront 0, with an
// optional diagonal shift.  Returns nonzero on a non-positive pivot.
__device__ __forceinline__ int small_chol_wave(double *G, int nb, double shift, int *ints) {
  const int t = threadIdx.x;
  if (t < 64) {
    if (t == 0) ints[0] = 0;
    if (shift != 0.0)
      for (int a = t; a < nb; a += 64) G[a + a * WLRA_BMAX] += shift;
    wave_sync();
    for (int j = 0; j < nb; ++j) {
      if (t == 0) {
        double p = G[j + j * WLRA_BMAX];
        if (!(p > 0.0)) {
          ints[0] = 1;
          p = 1.0;
        }
        G[j + j * WLRA_BMAX] = sqrt(p);
      }
      wave_sync();
      const double rjj = G[j + j * WLRA_BMAX];
      for (int c = j + 1 + t; c < nb; c += 64) G[j + c * WLRA_BMAX] /= rjj;
      wave_sync();
      const int rem = nb - j - 1;
      for (int e = t; e < rem * rem; e += 64) {
        const int aa = j + 1 + e % rem, cc = j + 1 + e / rem;
        if (aa <= cc) G[aa + cc * WLRA_BMAX] -= G[j + aa * WLRA_BMAX] * G[j + cc * WLRA_BMAX];
      }
      wave_sync();
    }
  }
  __syncthreads();
  return ints[0];
}


// Symmetric eigendecomposition of H (nb x nb) by parallel cyclic Jacobi on
// wavefront 0 (round-robin pairing, nb/2 disjoint rotations per round).
// On return th[0..nb) is descending and S holds the eigenvectors.
__device__ __forceinline__ void small_jacobi_wave(double *H, double *S, double *th, double *rc,
                                                  double *rs, int *rp, int *rq, int *ints, int nb) {
  const int t = threadIdx.x;
  if (t < 64) {
    for (int e = t; e < WLRA_BMAX * WLRA_BMAX; e += 64) S[e] = ((e % WLRA_BMAX) == (e / WLRA_BMAX)) ? 1.0 : 0.0;
    // H = Y^T (M Y) is symmetric only to rounding: average the two triangles
    // so that the rotations can drive the off-diagonal mass to zero
    for (int e = t; e < nb * nb; e += 64) {
      const int a = e % nb, c = e / nb;
      if (a < c) {
        const double v = 0.5 * (H[a + c * WLRA_BMAX] + H[c + a * WLRA_BMAX]);
        H[a + c * WLRA_BMAX] = v;
        H[c + a * WLRA_BMAX] = v;
      }
    }
    const int nbp = nb + (nb & 1);
    const int half = nbp / 2;
    wave_sync();
    for (int sweep = 0; sweep < 40; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int e = t; e < nb * nb; e += 64) {
        const int a = e % nb, c = e / nb;
        const double v = H[a + c * WLRA_BMAX];
        tot += v * v;
        if (a != c) off += v * v;
      }
      off = wave_sum(off);
      tot = wave_sum(tot);
      // converged once the off-diagonal mass is at the rounding level of H
      if (!(off > 1e-28 * tot)) break;
      for (int round = 0; round < nbp - 1; ++round) {
        if (t < half) {
          const int x0 = t, x1 = nbp - 1 - t;
          int p = (x0 == 0) ? 0 : 1 + (x0 - 1 + round) % (nbp - 1);
          int q = (x1 == 0) ? 0 : 1 + (x1 - 1 + round) % (nbp - 1);
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          double c = 1.0, sn = 0.0;
          if (q < nb) {
            const double apq = H[p + q * WLRA_BMAX];
            if (fabs(apq) > 1e-300) {
              const double tau = (H[q + q * WLRA_BMAX] - H[p + p * WLRA_BMAX]) / (2.0 * apq);
              const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + tt * tt);
              sn = tt * c;
            }
          } else {
            q = p;  // dummy partner: identity
          }
          rp[t] = p;
          rq[t] = q;
          rc[t] = c;
          rs[t] = sn;
        }
        wave_sync();
        // rows p, q
        for (int e = t; e < half * nb; e += 64) {
          const int pr = e % half, x = e / half;
          const int p = rp[pr], q = rq[pr];
          if (p == q) continue;
          const double c = rc[pr], sn = rs[pr];
          const double hp = H[p + x * WLRA_BMAX], hq = H[q + x * WLRA_BMAX];
          H[p + x * WLRA_BMAX] = c * hp - sn * hq;
          H[q + x * WLRA_BMAX] = sn * hp + c * hq;
        }
        wave_sync();
        // columns p, q of H and of S
        for (int e = t; e < half * nb; e += 64) {
          const int pr = e % half, x = e / half;
          const int p = rp[pr], q = rq[pr];
          if (p == q) continue;
          const double c = rc[pr], sn = rs[pr];
          const double hp = H[x + p * WLRA_BMAX], hq = H[x + q * WLRA_BMAX];
          H[x + p * WLRA_BMAX] = c * hp - sn * hq;
          H[x + q * WLRA_BMAX] = sn * hp + c * hq;
          const double vp = S[x + p * WLRA_BMAX], vq = S[x + q * WLRA_BMAX];
          S[x + p * WLRA_BMAX] = c * vp - sn * vq;
          S[x + q * WLRA_BMAX] = sn * vp + c * vq;
        }
        wave_sync();
      }
    }
    // eigenvalues, sorted descending (selection sort with column swaps)
    for (int a = t; a < nb; a += 64) th[a] = H[a + a * WLRA_BMAX];
    wave_sync();
    for (int a = 0; a < nb; ++a) {
      if (t == 0) {
        int best = a;
        for (int c = a + 1; c < nb; ++c)
          if (th[c] > th[best]) best = c;
        ints[1] = best;
      }
      wave_sync();
      const int best = ints[1];
      if (best != a) {
        for (int x = t; x < nb; x += 64) {
          const double v = S[x + a * WLRA_BMAX];
          S[x + a * WLRA_BMAX] = S[x + best * WLRA_BMAX];
          S[x + best * WLRA_BMAX] = v;
        }
        if (t == 0) {
          const double v = th[a];
          th[a] = th[best];
          th[best] = v;
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
}

