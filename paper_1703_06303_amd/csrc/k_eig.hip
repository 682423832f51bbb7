// Top-(r-k) eigenpairs of M = (P^perp A2)^T (P^perp A2) (n2 x n2, double):
// the right singular vectors V and squared singular values of P^perp A2 that
// define D_p = H_{r-k}(P^perp A2) = (P^perp A2) V V^T (eq. (2), Algorithm 1
// steps 4 and 6).
//
// Method: Chebyshev-filtered subspace iteration on a block of b = r-k+guard
// vectors, warm-started from the previous sweep's block.  Each round filters
// the active vectors with a degree-d Chebyshev polynomial that damps [0, c]
// (c = smallest Ritz value of the block; M is positive semidefinite), using
// the three-term recurrence scaled so that values stay O(1).  Converged
// leading Ritz vectors are locked and deflated (M - L Theta L^T) so the filter
// cannot re-amplify them, and the degree is capped so the top active
// component grows at most ~1e6 times the others (the block is then safe for
// Cholesky QR).  Each round ends with CholeskyQR2 (shifted on failure) and a
// Rayleigh-Ritz step solved by parallel cyclic Jacobi.  A Ritz pair is
// converged when ||M y - theta y|| <= eig_floor.
//
// One workgroup of 1024 threads; vectors live in global memory (L2
// resident); the block being multiplied is staged through LDS.
#include "common.h"
#include "launch.h"

#define ET 1024
#define B_ WLRA_BMAX

struct EigLDS {
  double sx[8192];      // staged block (n2 x 8) for M * X
  double sp[8192];      // partial sums
  double H[B_ * B_];    // Gram / Rayleigh quotient / Cholesky factor
  double S[B_ * B_];    // Jacobi rotations (eigenvectors of H)
  double G[B_ * B_];    // L^T X for projections
  double th[B_];
  double res[B_];
  double red[16];
  double rc[32], rs[32];
  int rp[32], rq[32];
  int ints[4];
};

// Out[:, 0:nc] = M X[:, 0:nc] - L diag(thL) (L^T X)   (L = first `locked`
// columns of Lb); all blocks n2 x *, ld n2.
__device__ void blk_op(EigLDS &s, const double *__restrict__ M, int n2, const double *X, int nc,
                       double *Out, const double *Lb, const double *thL, int locked) {
  const int t = threadIdx.x;
  const int S = max(1, min(8, ET / n2));
  for (int c0 = 0; c0 < nc; c0 += 8) {
    const int cw = min(8, nc - c0);
    for (int e = t; e < n2 * 8; e += ET) {
      const int l = e >> 3, q = e & 7;
      s.sx[e] = (q < cw) ? X[l + (int64_t)(c0 + q) * n2] : 0.0;
    }
    __syncthreads();
    if (t < S * n2) {
      const int i = t % n2, sl = t / n2;
      const int l0 = sl * n2 / S, l1 = (sl + 1) * n2 / S;
      double acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
      for (int l = l0; l < l1; ++l) {
        const double mv = M[i + (int64_t)l * n2];
        const double *xr = s.sx + l * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(mv, xr[q], acc[q]);
      }
      if (S == 1) {
        for (int q = 0; q < cw; ++q) Out[i + (int64_t)(c0 + q) * n2] = acc[q];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) s.sp[(sl * n2 + i) * 8 + q] = acc[q];
      }
    }
    __syncthreads();
    if (S > 1) {
      for (int i = t; i < n2; i += ET)
        for (int q = 0; q < cw; ++q) {
          double v = 0.0;
          for (int sl = 0; sl < S; ++sl) v += s.sp[(sl * n2 + i) * 8 + q];
          Out[i + (int64_t)(c0 + q) * n2] = v;
        }
    }
    __syncthreads();
  }
  if (locked > 0) {
    // G = L^T X  (locked x nc)
    const int pairs = locked * nc;
    const int Sg = max(1, min(8, ET / pairs));
    for (int e = t; e < pairs * Sg; e += ET) {
      const int pr = e % pairs, sl = e / pairs;
      const int a = pr % locked, c = pr / locked;
      const int i0 = sl * n2 / Sg, i1 = (sl + 1) * n2 / Sg;
      double acc = 0.0;
      for (int i = i0; i < i1; ++i) acc = fma(Lb[i + (int64_t)a * n2], X[i + (int64_t)c * n2], acc);
      s.sp[e] = acc;
    }
    __syncthreads();
    for (int pr = t; pr < pairs; pr += ET) {
      double v = 0.0;
      for (int sl = 0; sl < Sg; ++sl) v += s.sp[sl * pairs + pr];
      s.G[(pr % locked) + (pr / locked) * B_] = v * thL[pr % locked];
    }
    __syncthreads();
    for (int i = t; i < n2; i += ET)
      for (int c = 0; c < nc; ++c) {
        double v = Out[i + (int64_t)c * n2];
        for (int a = 0; a < locked; ++a) v -= Lb[i + (int64_t)a * n2] * s.G[a + c * B_];
        Out[i + (int64_t)c * n2] = v;
      }
    __syncthreads();
  }
}

// G (p x q, ld B_) = X^T Y over n2 rows; fixed-order sums.
__device__ void blk_gram(EigLDS &s, int n2, const double *X, int p, const double *Y, int q,
                         double *G) {
  const int t = threadIdx.x;
  const int pairs = p * q;
  const int Sg = max(1, min(8, ET / pairs));
  for (int e = t; e < pairs * Sg; e += ET) {
    const int pr = e % pairs, sl = e / pairs;
    const int a = pr % p, c = pr / p;
    const int i0 = sl * n2 / Sg, i1 = (sl + 1) * n2 / Sg;
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) acc = fma(X[i + (int64_t)a * n2], Y[i + (int64_t)c * n2], acc);
    s.sp[e] = acc;
  }
  __syncthreads();
  for (int pr = t; pr < pairs; pr += ET) {
    double v = 0.0;
    for (int sl = 0; sl < Sg; ++sl) v += s.sp[sl * pairs + pr];
    G[(pr % p) + (pr / p) * B_] = v;
  }
  __syncthreads();
}

// Upper Cholesky in place of G (nb x nb, ld B_) by wavefront 0, with an
// optional diagonal shift.  Returns nonzero on a non-positive pivot.
__device__ int blk_chol(EigLDS &s, double *G, int nb, double shift) {
  const int t = threadIdx.x;
  if (t < 64) {
    if (t == 0) s.ints[0] = 0;
    if (shift != 0.0)
      for (int a = t; a < nb; a += 64) G[a + a * B_] += shift;
    wave_sync();
    for (int j = 0; j < nb; ++j) {
      if (t == 0) {
        double p = G[j + j * B_];
        if (!(p > 0.0)) {
          s.ints[0] = 1;
          p = 1.0;
        }
        G[j + j * B_] = sqrt(p);
      }
      wave_sync();
      const double rjj = G[j + j * B_];
      for (int c = j + 1 + t; c < nb; c += 64) G[j + c * B_] /= rjj;
      wave_sync();
      const int rem = nb - j - 1;
      for (int e = t; e < rem * rem; e += 64) {
        const int aa = j + 1 + e % rem, cc = j + 1 + e / rem;
        if (aa <= cc) G[aa + cc * B_] -= G[j + aa * B_] * G[j + cc * B_];
      }
      wave_sync();
    }
  }
  __syncthreads();
  return s.ints[0];
}

// X (n2 x nb) <- X R^-1, R upper in LDS; one row per thread.
__device__ void blk_trsm(int n2, double *X, int nb, const double *R) {
  for (int i = threadIdx.x; i < n2; i += ET) {
    double x[B_];
#pragma unroll
    for (int c = 0; c < B_; ++c) x[c] = (c < nb) ? X[i + (int64_t)c * n2] : 0.0;
#pragma unroll
    for (int c = 0; c < B_; ++c) {
      if (c < nb) {
        double v = x[c];
#pragma unroll
        for (int a = 0; a < c; ++a) v -= x[a] * R[a + c * B_];
        x[c] = v / R[c + c * B_];
      }
    }
#pragma unroll
    for (int c = 0; c < B_; ++c)
      if (c < nb) X[i + (int64_t)c * n2] = x[c];
  }
  __syncthreads();
}

// X (n2 x nb) <- X S (S nb x nb in LDS, ld B_); one row per thread.
__device__ void blk_rot(int n2, double *X, int nb, const double *S) {
  for (int i = threadIdx.x; i < n2; i += ET) {
    double x[B_];
#pragma unroll
    for (int c = 0; c < B_; ++c) x[c] = (c < nb) ? X[i + (int64_t)c * n2] : 0.0;
    for (int c = 0; c < nb; ++c) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < B_; ++a)
        if (a < nb) v = fma(x[a], S[a + c * B_], v);
      X[i + (int64_t)c * n2] = v;
    }
  }
  __syncthreads();
}

// Symmetric eigendecomposition of H (nb x nb) by parallel cyclic Jacobi on
// wavefront 0 (round-robin pairing, nb/2 disjoint rotations per round).
// On return th[0..nb) is descending and S holds the eigenvectors.
__device__ void blk_jacobi(EigLDS &s, int nb) {
  const int t = threadIdx.x;
  if (t < 64) {
    double *H = s.H, *S = s.S;
    for (int e = t; e < B_ * B_; e += 64) S[e] = ((e % B_) == (e / B_)) ? 1.0 : 0.0;
    const int nbp = nb + (nb & 1);
    const int half = nbp / 2;
    wave_sync();
    for (int sweep = 0; sweep < 40; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int e = t; e < nb * nb; e += 64) {
        const int a = e % nb, c = e / nb;
        const double v = H[a + c * B_];
        tot += v * v;
        if (a != c) off += v * v;
      }
      off = wave_sum(off);
      tot = wave_sum(tot);
      if (!(off > 1e-32 * tot)) break;
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
            const double apq = H[p + q * B_];
            if (fabs(apq) > 1e-300) {
              const double tau = (H[q + q * B_] - H[p + p * B_]) / (2.0 * apq);
              const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + tt * tt);
              sn = tt * c;
            }
          } else {
            q = p;  // dummy partner: identity
          }
          s.rp[t] = p;
          s.rq[t] = q;
          s.rc[t] = c;
          s.rs[t] = sn;
        }
        wave_sync();
        // rows p, q
        for (int e = t; e < half * nb; e += 64) {
          const int pr = e % half, x = e / half;
          const int p = s.rp[pr], q = s.rq[pr];
          if (p == q) continue;
          const double c = s.rc[pr], sn = s.rs[pr];
          const double hp = H[p + x * B_], hq = H[q + x * B_];
          H[p + x * B_] = c * hp - sn * hq;
          H[q + x * B_] = sn * hp + c * hq;
        }
        wave_sync();
        // columns p, q of H and of S
        for (int e = t; e < half * nb; e += 64) {
          const int pr = e % half, x = e / half;
          const int p = s.rp[pr], q = s.rq[pr];
          if (p == q) continue;
          const double c = s.rc[pr], sn = s.rs[pr];
          const double hp = H[x + p * B_], hq = H[x + q * B_];
          H[x + p * B_] = c * hp - sn * hq;
          H[x + q * B_] = sn * hp + c * hq;
          const double vp = S[x + p * B_], vq = S[x + q * B_];
          S[x + p * B_] = c * vp - sn * vq;
          S[x + q * B_] = sn * vp + c * vq;
        }
        wave_sync();
      }
    }
    // eigenvalues, sorted descending (selection sort with column swaps)
    for (int a = t; a < nb; a += 64) s.th[a] = H[a + a * B_];
    wave_sync();
    for (int a = 0; a < nb; ++a) {
      if (t == 0) {
        int best = a;
        for (int c = a + 1; c < nb; ++c)
          if (s.th[c] > s.th[best]) best = c;
        s.ints[1] = best;
      }
      wave_sync();
      const int best = s.ints[1];
      if (best != a) {
        for (int x = t; x < nb; x += 64) {
          const double v = S[x + a * B_];
          S[x + a * B_] = S[x + best * B_];
          S[x + best * B_] = v;
        }
        if (t == 0) {
          const double v = s.th[a];
          s.th[a] = s.th[best];
          s.th[best] = v;
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
}

// Orthonormalise the nb columns of X against the `locked` columns of L and
// among themselves: CholeskyQR2, shifted CholeskyQR3 if the Gram is not
// numerically positive definite.
__device__ void blk_orth(EigLDS &s, int n2, double *X, int nb, const double *L, int locked,
                         int *flags) {
  const int t = threadIdx.x;
  int shifted = 0;
  for (int rep = 0; rep < 3; ++rep) {
    if (rep == 2 && !shifted) break;
    if (locked > 0) {
      blk_gram(s, n2, L, locked, X, nb, s.G);
      for (int i = t; i < n2; i += ET)
        for (int c = 0; c < nb; ++c) {
          double v = X[i + (int64_t)c * n2];
          for (int a = 0; a < locked; ++a) v -= L[i + (int64_t)a * n2] * s.G[a + c * B_];
          X[i + (int64_t)c * n2] = v;
        }
      __syncthreads();
    }
    // normalise columns
    blk_gram(s, n2, X, nb, X, nb, s.H);
    for (int c = t; c < nb; c += ET) s.res[c] = s.H[c + c * B_];
    __syncthreads();
    for (int i = t; i < n2; i += ET)
      for (int c = 0; c < nb; ++c) {
        const double d = s.res[c];
        X[i + (int64_t)c * n2] *= (d > 0 ? 1.0 / sqrt(d) : 0.0);
      }
    __syncthreads();
    blk_gram(s, n2, X, nb, X, nb, s.H);
    if (blk_chol(s, s.H, nb, 0.0)) {
      blk_gram(s, n2, X, nb, X, nb, s.H);
      double fro = 0.0;
      for (int e = 0; e < nb * nb; ++e) fro += s.H[(e % nb) + (e / nb) * B_] * s.H[(e % nb) + (e / nb) * B_];
      const double sh = 11.0 * ((double)n2 * nb + (double)nb * (nb + 1)) * 2.220446049250313e-16 * sqrt(fro);
      shifted = 1;
      if (blk_chol(s, s.H, nb, sh)) {
        if (t == 0) atomicOr(flags, DEV_EIG_MAXIT);
        return;
      }
    }
    blk_trsm(n2, X, nb, s.H);
  }
}

__global__ __launch_bounds__(ET) void k_eig(SmallArgs a) {
  SmallState *st = a.st;
  if (st->done) return;
  __shared__ EigLDS s;
  const int n2 = a.n2, l = a.l, b = a.b, t = threadIdx.x;
  const double *M = a.M;
  double *Y = a.Y, *W = a.Wb;
  const double floor_ = st->eig_floor;
  const double maxamp = 1e6;

  if (st->eig_first) {
    for (int e = t; e < n2 * b; e += ET) Y[e] = hash_unit((uint32_t)(e % n2), (uint32_t)(e / n2));
    __syncthreads();
  }
  blk_orth(s, n2, Y, b, Y, 0, a.flags);
  blk_op(s, M, n2, Y, b, W, Y, s.th, 0);
  blk_gram(s, n2, Y, b, W, b, s.H);
  blk_jacobi(s, b);
  blk_rot(n2, Y, b, s.S);
  blk_rot(n2, W, b, s.S);

  int locked = 0, it = 0, nmv = b;
  while (true) {
    // residuals ||W_q - th_q Y_q|| for q in [locked, l)
    const int nq = l - locked;
    const int Sg = max(1, min(8, ET / max(nq, 1)));
    for (int e = t; e < nq * Sg; e += ET) {
      const int q = locked + e % nq, sl = e / nq;
      const int i0 = sl * n2 / Sg, i1 = (sl + 1) * n2 / Sg;
      const double th = s.th[q];
      double acc = 0.0;
      for (int i = i0; i < i1; ++i) {
        const double r = W[i + (int64_t)q * n2] - th * Y[i + (int64_t)q * n2];
        acc = fma(r, r, acc);
      }
      s.sp[e] = acc;
    }
    __syncthreads();
    if (t == 0) {
      int lk = locked;
      while (lk < l) {
        double v = 0.0;
        for (int sl = 0; sl < Sg; ++sl) v += s.sp[sl * nq + (lk - locked)];
        if (sqrt(v) <= floor_) ++lk;
        else break;
      }
      s.ints[2] = lk;
    }
    __syncthreads();
    locked = s.ints[2];
    if (locked >= l || it >= a.eig_maxit) break;

    const int act = b - locked;
    double *Ya = Y + (int64_t)locked * n2;
    double *Wa = W + (int64_t)locked * n2;
    // filter interval [0, c] damped; normalised at th[locked]
    const double cc = s.th[b - 1];
    const double e0 = 0.5 * cc;
    double h = 0.5 * cc;
    const double top = s.th[locked];
    if (!(h > 1e-15 * fabs(top))) h = 1e-15 * fabs(top) + 1e-300;
    const double x = (top - e0) / h;
    int d = a.eig_deg;
    if (x > 1.0) {
      const int dmax = max(2, (int)(log(2.0 * maxamp) / acosh(x)));
      d = min(d, dmax);
    }
    const double sigma = h / (top - e0), tau = 2.0 / sigma;
    double s1 = sigma;
    double *F0 = a.F0, *F1 = a.F1, *F2 = a.F2;
    for (int e = t; e < n2 * act; e += ET) F0[e] = Ya[e];
    __syncthreads();
    blk_op(s, M, n2, F0, act, F1, Y, s.th, locked);
    for (int e = t; e < n2 * act; e += ET) F1[e] = (F1[e] - e0 * F0[e]) * (s1 / h);
    __syncthreads();
    nmv += act * (d + 1);
    for (int j = 2; j <= d; ++j) {
      const double s2 = 1.0 / (tau - s1);
      blk_op(s, M, n2, F1, act, F2, Y, s.th, locked);
      for (int e = t; e < n2 * act; e += ET)
        F2[e] = 2.0 * (s2 / h) * (F2[e] - e0 * F1[e]) - (s1 * s2) * F0[e];
      __syncthreads();
      double *tmp = F0;
      F0 = F1;
      F1 = F2;
      F2 = tmp;
      s1 = s2;
    }
    for (int e = t; e < n2 * act; e += ET) Ya[e] = F1[e];
    __syncthreads();
    blk_orth(s, n2, Ya, act, Y, locked, a.flags);
    blk_op(s, M, n2, Ya, act, Wa, Y, s.th, 0);
    blk_gram(s, n2, Ya, act, Wa, act, s.H);
    // keep the locked Ritz values while Jacobi overwrites th[0..act)
    for (int q = t; q < locked; q += ET) s.res[q] = s.th[q];
    __syncthreads();
    blk_jacobi(s, act);
    blk_rot(n2, Ya, act, s.S);
    blk_rot(n2, Wa, act, s.S);
    if (t == 0) {
      for (int q = act - 1; q >= 0; --q) s.th[locked + q] = s.th[q];
      for (int q = 0; q < locked; ++q) s.th[q] = s.res[q];
    }
    __syncthreads();
    ++it;
  }
  for (int q = t; q < b; q += ET) a.theta[q] = s.th[q];
  if (t == 0) {
    st->eig_iters += it;
    st->eig_matvecs += nmv;
    st->eig_first = 0;
    if (it >= a.eig_maxit && locked < l) atomicOr(a.flags, DEV_EIG_MAXIT);
  }
}

void launch_eig(hipStream_t s, const SmallArgs &a) {
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(ET), 0, s, a);
}
