// Small dense steps shared by the eigen kernels: an upper Cholesky and a
// parallel cyclic Jacobi eigensolver of an nb x nb matrix (nb <= 32, leading
// dimension WLRA_BMAX) in LDS, both run by wavefront 0 of the workgroup and
// followed by a workgroup barrier.
#pragma once

#include "common.h"

// Rotation (c, s) of the symmetric 2 x 2 Schur decomposition that zeroes hpq
// in [hpp hpq; hpq hqq]: tau = (hqq - hpp) / (2 hpq), t the root of
// t^2 + 2 tau t - 1 = 0 of smaller magnitude, sign(tau) / (|tau| +
// sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c.  Reciprocals and square
// roots go through rcp_nr / rsq_nr; for |tau| > 1e150 (tau^2 would
// overflow) t = sign(tau) / (2 |tau|), and t = 0 past 1e300.
__device__ __forceinline__ void jacobi_cs(double hpp, double hqq, double hpq, double &c,
                                          double &sn) {
  const double tau = (hqq - hpp) * rcp_nr(2.0 * hpq);
  const double at = fabs(tau);
  const double a = fma(tau, tau, 1.0);
  const double den = at > 1e150 ? 2.0 * at : at + a * rsq_nr(a);
  const double r = at < 1e300 ? rcp_nr(den) : 0.0;
  const double tt = tau >= 0 ? r : -r;
  c = rsq_nr(fma(tt, tt, 1.0));
  sn = tt * c;
}

// Upper Cholesky in place of G (nb x nb, ld WLRA_BMAX) by wavefront 0, with an
// optional diagonal shift.  Returns nonzero on a non-positive pivot.
__device__ __forceinline__ int small_chol_reg(double *G, int nb, double shift, int *ints);
__device__ __forceinline__ int small_chol_wave(double *G, int nb, double shift, int *ints) {
  if (nb <= 8) return small_chol_reg(G, nb, shift, ints);
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


// The same Cholesky for nb <= 8 with G in registers: lane x + nb y of
// wavefront 0 holds G[x][y]; a step reads the pivot and row j across lanes.
// Writes the same entries as the LDS version (the upper triangle) and the
// same failure flag.
__device__ __forceinline__ int small_chol_reg(double *G, int nb, double shift, int *ints) {
  const int t = threadIdx.x;
  constexpr int L = WLRA_BMAX;
  if (t < 64) {
    const bool in = t < nb * nb;
    const int x = in ? t % nb : 0, y = in ? t / nb : 0;
    double g = in ? G[x + y * L] : 0.0;
    if (in && x == y) g += shift;
    int bad = 0;
    for (int j = 0; j < nb; ++j) {
      double p = __shfl(g, j + j * nb, 64);
      if (!(p > 0.0)) {
        bad = 1;
        p = 1.0;
      }
      const double rjj = sqrt(p);
      if (in && x == j) g = (y == j) ? rjj : ((y > j) ? g / rjj : g);
      const double rx = __shfl(g, j + x * nb, 64), ry = __shfl(g, j + y * nb, 64);
      if (in && x > j && x <= y) g -= rx * ry;
    }
    if (in && x <= y) G[x + y * L] = g;
    if (t == 0) ints[0] = bad;
  }
  __syncthreads();
  return ints[0];
}

// The same Jacobi for nb <= 8 with H and S in registers: lane x + nb y of
// wavefront 0 holds H[x][y] and S[x][y]; a round's rotation parameters and
// its J^T H J, S J updates use cross-lane reads (ds_bpermute) only, and each
// lane below the diagonal takes its entry from the mirrored lane so that H
// stays exactly symmetric.  Same pairing, rotation formulas, stopping test
// and output (th descending, ties by index; S's columns) as below.
__device__ __forceinline__ void small_jacobi_reg(double *H, double *S, double *th, int *rk,
                                                 int nb) {
  const int t = threadIdx.x;
  constexpr int L = WLRA_BMAX;
  if (t < 64) {
    const int nn = nb * nb;
    const bool in = t < nn;
    const int x = in ? t % nb : 0, y = in ? t / nb : 0;
    double h = in ? ((x == y) ? H[x + y * L] : 0.5 * (H[x + y * L] + H[y + x * L])) : 0.0;
    double sv = (in && x == y) ? 1.0 : 0.0;
    const int nbp = nb + (nb & 1), per = nbp - 1;
    for (int sweep = 0; sweep < 40; ++sweep) {
      const double v2 = h * h;
      const double off = wave_sum((in && x != y) ? v2 : 0.0);
      const double tot = wave_sum(v2);
      if (!(off > 1e-28 * tot)) break;
      for (int round = 0; round < per; ++round) {
        // partner of an index in this round's circle arrangement (nb is the
        // dummy of an odd nb)
        // (i - 1 - round lies in (-per, per), pp - 1 + round in [0, 2 per))
        auto partner = [&](int i) {
          const int v = i - 1 - round;
          const int pos = (i == 0) ? 0 : 1 + (v < 0 ? v + per : v);
          const int pp = nbp - 1 - pos, w = pp - 1 + round;
          return (pp == 0) ? 0 : 1 + (w >= per ? w - per : w);
        };
        const int px = partner(x), py = partner(y);
        const bool paired = px < nb && px != x;
        const int p = paired ? min(x, px) : x, q = paired ? max(x, px) : x;
        const double hpp = __shfl(h, p + p * nb, 64), hqq = __shfl(h, q + q * nb, 64);
        const double hpq = __shfl(h, p + q * nb, 64);
        double c = 1.0, sn = 0.0;
        if (paired && fabs(hpq) > 1e-300) jacobi_cs(hpp, hqq, hpq, c, sn);
        const double ax = paired ? c : 1.0, bx = paired ? ((x == p) ? -sn : sn) : 0.0;
        // lane y holds index y as its x (y < nb), so its coefficients are y's
        const double ay = __shfl(ax, y, 64), by = __shfl(bx, y, 64);
        const int pxe = paired ? px : x, pye = (py < nb && py != y) ? py : y;
        const double h_xpy = __shfl(h, x + pye * nb, 64), h_pxy = __shfl(h, pxe + y * nb, 64);
        const double h_pxpy = __shfl(h, pxe + pye * nb, 64);
        const double s_xpy = __shfl(sv, x + pye * nb, 64);
        const double hn = (ax * ay * h + ax * by * h_xpy) + (bx * ay * h_pxy + bx * by * h_pxpy);
        const double hm = __shfl(hn, y + x * nb, 64);  // the upper entry, for x > y
        const double sn2 = ay * sv + by * s_xpy;
        if (in) {
          h = (x <= y) ? hn : hm;
          sv = sn2;
        }
      }
    }
    // eigenvalues descending (ties by index): the diagonal goes through H
    // (no longer needed), ranks per index, S's columns to their ranks
    if (in && x == y) H[x + x * L] = h;
    wave_sync();
    if (t < nb) {
      int r = 0;
      for (int c = 0; c < nb; ++c)
        r += (H[c + c * L] > H[t + t * L]) || (H[c + c * L] == H[t + t * L] && c < t);
      rk[t] = r;
      th[r] = H[t + t * L];
    }
    wave_sync();
    if (in) S[x + rk[y] * L] = sv;
  }
  __syncthreads();
}

// Symmetric eigendecomposition of H (nb x nb) by parallel cyclic Jacobi on
// wavefront 0 (round-robin pairing, nb/2 disjoint rotations per round).
// A round applies all of its rotations from both sides in one pass,
// H' = J^T H J and S' = S J, reading H, S and writing H2, S2 (the buffers
// then swap): index x of pair (p, q) maps to al[x] * row x + be[x] * row
// pt[x].  On return th[0..nb) is descending (ties by index) and S holds the
// eigenvectors; H2 and S2 are scratch (WLRA_BMAX^2 doubles each), rk holds
// nb ints of scratch.
__device__ __forceinline__ void small_jacobi_wave(double *H, double *S, double *H2, double *S2,
                                                  double *th, double *al, double *be, int *pt,
                                                  int *rk, int nb) {
  if (nb <= 8) {
    small_jacobi_reg(H, S, th, rk, nb);
    return;
  }
  const int t = threadIdx.x;
  constexpr int L = WLRA_BMAX;
  if (t < 64) {
    for (int e = t; e < L * L; e += 64) S[e] = ((e % L) == (e / L)) ? 1.0 : 0.0;
    // H = Y^T (M Y) is symmetric only to rounding: average the two triangles
    // so that the rotations can drive the off-diagonal mass to zero
    for (int e = t; e < nb * nb; e += 64) {
      const int a = e % nb, c = e / nb;
      if (a < c) {
        const double v = 0.5 * (H[a + c * L] + H[c + a * L]);
        H[a + c * L] = v;
        H[c + a * L] = v;
      }
    }
    const int nbp = nb + (nb & 1);
    const int half = nbp / 2;
    double *Hc = H, *Hn = H2, *Sc = S, *Sn = S2;
    wave_sync();
    for (int sweep = 0; sweep < 40; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int e = t; e < nb * nb; e += 64) {
        const int a = e % nb, c = e / nb;
        const double v = Hc[a + c * L];
        tot += v * v;
        if (a != c) off += v * v;
      }
      off = wave_sum(off);
      tot = wave_sum(tot);
      // converged once the off-diagonal mass is at the rounding level of H
      if (!(off > 1e-28 * tot)) break;
      for (int round = 0; round < nbp - 1; ++round) {
        if (t < half) {
          const int x0 = t, x1 = nbp - 1 - t, per = nbp - 1;
          const int w0 = x0 - 1 + round, w1 = x1 - 1 + round;  // in [0, 2 per)
          int p = (x0 == 0) ? 0 : 1 + (w0 >= per ? w0 - per : w0);
          int q = (x1 == 0) ? 0 : 1 + (w1 >= per ? w1 - per : w1);
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q < nb) {
            double c = 1.0, sn = 0.0;
            const double apq = Hc[p + q * L];
            if (fabs(apq) > 1e-300) jacobi_cs(Hc[p + p * L], Hc[q + q * L], apq, c, sn);
            al[p] = c;
            be[p] = -sn;
            pt[p] = q;
            al[q] = c;
            be[q] = sn;
            pt[q] = p;
          } else {  // paired with the dummy index: identity
            al[p] = 1.0;
            be[p] = 0.0;
            pt[p] = p;
          }
        }
        wave_sync();
        // upper triangle of J^T H J, mirrored (the result stays symmetric)
        for (int e = t; e < nb * nb; e += 64) {
          const int x = e % nb, y = e / nb;
          if (x > y) continue;
          const int px = pt[x], py = pt[y];
          const double ax = al[x], bx = be[x], ay = al[y], by = be[y];
          const double v = (ax * ay * Hc[x + y * L] + ax * by * Hc[x + py * L]) +
                           (bx * ay * Hc[px + y * L] + bx * by * Hc[px + py * L]);
          Hn[x + y * L] = v;
          Hn[y + x * L] = v;
        }
        for (int e = t; e < nb * nb; e += 64) {
          const int x = e % nb, y = e / nb;
          Sn[x + y * L] = al[y] * Sc[x + y * L] + be[y] * Sc[x + pt[y] * L];
        }
        wave_sync();
        double *tp = Hc;
        Hc = Hn;
        Hn = tp;
        tp = Sc;
        Sc = Sn;
        Sn = tp;
      }
    }
    // eigenvalues descending (ties by index): rank of each, then the
    // eigenvector columns move to their ranks, into S
    for (int a = t; a < nb; a += 64) al[a] = Hc[a + a * L];
    wave_sync();
    for (int a = t; a < nb; a += 64) {
      int r = 0;
      for (int c = 0; c < nb; ++c) r += (al[c] > al[a]) || (al[c] == al[a] && c < a);
      rk[a] = r;
      th[r] = al[a];
    }
    wave_sync();
    double *dst = (Sc == S) ? S2 : S;
    for (int e = t; e < nb * nb; e += 64) {
      const int x = e % nb, a = e / nb;
      dst[x + rk[a] * L] = Sc[x + a * L];
    }
    wave_sync();
    if (dst != S)
      for (int e = t; e < nb * nb; e += 64) S[(e % nb) + (e / nb) * L] = dst[(e % nb) + (e / nb) * L];
  }
  __syncthreads();
}
