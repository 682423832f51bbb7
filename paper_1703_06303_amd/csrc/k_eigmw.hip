// Top-(r-k) eigenpairs of M = (P^perp A2)^T (P^perp A2) for larger n2, on
// several workgroups (eq. (2), Algorithm 1 steps 4 and 6).  Same method as
// the one-workgroup kernel k_eig (Chebyshev-filtered subspace iteration with
// locking, Hotelling deflation, CholeskyQR2 and Rayleigh-Ritz by Jacobi), laid
// out for a cooperative launch:
//
//  * workgroup g owns rows [16 g, 16 g + 16) of M (cached in its LDS when they
//    fit) and of every n2 x b block, which live in global memory;
//  * a block product Out = M X reads X straight from L2 into registers (all
//    of a wavefront's share at once) and multiplies on the FP64 matrix
//    cores, the four wavefronts splitting the inner index (their partial
//    16 x 16 tiles are added in a fixed order);
//  * locked Ritz pairs are deflated once per locking event, each workgroup
//    updating its own rows of M (M <- M - L Theta L^T);
//  * a Gram X^T Y is formed from per-workgroup partial sums written to one of
//    two alternating global buffers and, after a grid barrier, added in
//    workgroup order by every workgroup;
//  * the small dense steps (Cholesky, Jacobi, locking decisions) run
//    redundantly in every workgroup on identical inputs, so every workgroup
//    takes the same branches and reaches the same grid barriers.
//
// Grid barriers separate every write of a block by row slices from the next
// read of all its rows (a block product, a Gram).
#include <hip/hip_cooperative_groups.h>

#include "common.h"
#include "eig_small.h"
#include "launch.h"

namespace cg = cooperative_groups;

#define MW_T 256      // threads per workgroup (4 wavefronts)
#define MW_R 16       // rows per workgroup
#define MW_B WLRA_BMAX
#define MW_PART (MW_B * MW_B)
#define MW_DYN 15360  // doubles of dynamic LDS (this workgroup's rows of M)

typedef double mw_d4 __attribute__((ext_vector_type(4)));

struct MwShared {
  double H[MW_B * MW_B];
  double S[MW_B * MW_B];
  double G[MW_B * MW_B];
  double Xr[MW_R * MW_B];    // this workgroup's rows of a block (triangular solve)
  double th[MW_B], res[MW_B], sc[MW_B], keep[MW_B];
  double rc[32], rs[32];
  int rp[32], rq[32];
  int ints[4];
  double rmax;
  double tile[4][16 * 16];
};

struct Mw {
  int n2, G, g, r0, r1;
  double *M;     // global M (this workgroup's rows are deflated in place
                 // when they are not cached)
  double *part;  // 2 x G x MW_PART doubles
  int pb;
  double *Ml;    // 16 x n2 rows of M (ld 16) in LDS, or nullptr
};

__device__ __forceinline__ void mw_sync() { cg::this_grid().sync(); }

// Out (p x q, ld MW_B, LDS) = X^T Y over all n2 rows (X, Y global, ld n2).
__device__ void mw_gram(Mw &c, const double *X, int p, const double *Y, int q, double *Out) {
  const int t = threadIdx.x, n2 = c.n2;
  double *mine = c.part + ((size_t)c.pb * c.G + c.g) * MW_PART;
  for (int e = t; e < p * q; e += MW_T) {
    const int u = e % p, v = e / p;
    const double *xu = X + (size_t)u * n2, *yv = Y + (size_t)v * n2;
    double acc = 0.0;
    // all 2 x 16 reads issued together (clamped; rows past r1 weigh 0)
#pragma unroll
    for (int ii = 0; ii < MW_R; ++ii) {
      const int i = min(c.r0 + ii, n2 - 1);
      const double w = (c.r0 + ii < c.r1) ? 1.0 : 0.0;
      acc = fma(xu[i] * w, yv[i], acc);
    }
    mine[u + v * MW_B] = acc;
  }
  mw_sync();
  const double *all = c.part + (size_t)c.pb * c.G * MW_PART;
  for (int e = t; e < p * q; e += MW_T) {
    const int u = e % p, v = e / p;
    double acc = 0.0;
#pragma unroll 8
    for (int w = 0; w < c.G; ++w) acc += all[(size_t)w * MW_PART + u + v * MW_B];
    Out[u + v * MW_B] = acc;
  }
  c.pb ^= 1;
  __syncthreads();
}

// res[q - q0] = ||W_q - th_q Y_q|| for q in [q0, q1).
__device__ void mw_resid(Mw &c, MwShared &s, const double *W, const double *Y, int q0, int q1) {
  const int t = threadIdx.x, n2 = c.n2, nq = q1 - q0;
  double *mine = c.part + ((size_t)c.pb * c.G + c.g) * MW_PART;
  for (int q = t; q < nq; q += MW_T) {
    const double th = s.th[q0 + q];
    const double *wq = W + (size_t)(q0 + q) * n2, *yq = Y + (size_t)(q0 + q) * n2;
    double acc = 0.0;
#pragma unroll
    for (int ii = 0; ii < MW_R; ++ii) {
      const int i = min(c.r0 + ii, n2 - 1);
      const double w = (c.r0 + ii < c.r1) ? 1.0 : 0.0;
      const double r = (wq[i] - th * yq[i]) * w;
      acc = fma(r, r, acc);
    }
    mine[q] = acc;
  }
  mw_sync();
  const double *all = c.part + (size_t)c.pb * c.G * MW_PART;
  for (int q = t; q < nq; q += MW_T) {
    double acc = 0.0;
    for (int w = 0; w < c.G; ++w) acc += all[(size_t)w * MW_PART + q];
    s.res[q] = sqrt(acc);
  }
  c.pb ^= 1;
  __syncthreads();
}

// Out[:, 0:nc] = M X on this workgroup's rows (M as deflated so far).  The
// caller has written this workgroup's rows of X; the grid barrier at the
// start completes X.  Each wavefront takes a quarter of the inner index and
// loads its whole share of X (up to MW_KB k-steps of 4 per lane) into
// registers before the first multiply; reads are clamped to stay in bounds
// and masked by multiplying with zero, so none of them is waited for alone.
#define MW_KB 40
__device__ void mw_op(Mw &c, MwShared &s, const double *X, int nc, double *Out) {
  const int t = threadIdx.x, n2 = c.n2;
  const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int li = lane & 15, lk = lane >> 4;
  mw_sync();
  const int kq = (n2 + 3) / 4;
  const int kw = (kq + 3) / 4;
  const int ks0 = wv * kw, ks1 = min(kq, ks0 + kw);
  const int rcl = min(c.r0 + li, n2 - 1);
  for (int c0 = 0; c0 < nc; c0 += 16) {
    const int cwn = min(16, nc - c0);
    const double *xc = X + (size_t)(c0 + min(li, cwn - 1)) * n2;
    const double cm = (li < cwn) ? 1.0 : 0.0;
    mw_d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kb = ks0; kb < ks1; kb += MW_KB) {
      const int nk = min(MW_KB, ks1 - kb);
      double bb[MW_KB];
#pragma unroll
      for (int u0 = 0; u0 < MW_KB; u0 += 8) {
        if (u0 < nk) {
#pragma unroll
          for (int u = u0; u < u0 + 8; ++u) bb[u] = xc[min(4 * (kb + u) + lk, n2 - 1)];
        }
      }
#pragma unroll
      for (int u0 = 0; u0 < MW_KB; u0 += 8) {
        if (u0 < nk) {
          double av[8], bv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int kk = 4 * (kb + u0 + u) + lk;
            const int kc = min(kk, n2 - 1);
            av[u] = c.Ml ? c.Ml[kc * MW_R + li] : c.M[mf_idx(n2, rcl, kc)];
            bv[u] = bb[u0 + u] * ((u0 + u < nk && kk < n2) ? cm : 0.0);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) s.tile[wv][(lk + 4 * v) * 16 + li] = acc[v];
    __syncthreads();
    for (int e = t; e < MW_R * cwn; e += MW_T) {
      const int rr = e % MW_R, cc = e / MW_R;
      const int row = c.r0 + rr;
      if (row < c.r1)
        Out[row + (size_t)(c0 + cc) * n2] =
            ((s.tile[0][rr * 16 + cc] + s.tile[1][rr * 16 + cc]) + s.tile[2][rr * 16 + cc]) +
            s.tile[3][rr * 16 + cc];
    }
    __syncthreads();
  }
}

// Deflation of newly locked Ritz pairs [q0, q1) on this workgroup's rows of
// M: M[i, j] -= sum_a th_a Y[i, a] Y[j, a].  Y is complete (a grid barrier
// separates its last write from the locking decision).
__device__ __noinline__ void mw_deflate(Mw &c, MwShared &s, const double *Y, int q0, int q1) {
  const int t = threadIdx.x, n2 = c.n2, tot = MW_R * n2;
  for (int e0 = t; e0 < tot; e0 += 8 * MW_T) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * MW_T, tot - 1);
      const int li = e % MW_R, j = e / MW_R;
      v[u] = c.Ml ? c.Ml[e] : c.M[mf_idx(n2, min(c.r0 + li, n2 - 1), j)];
    }
    for (int a = q0; a < q1; ++a) {
      const double th = s.th[a];
      const double *ya = Y + (size_t)a * n2;
      double yi[8], yj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + u * MW_T, tot - 1);
        yi[u] = ya[min(c.r0 + e % MW_R, n2 - 1)];
        yj[u] = ya[e / MW_R];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] -= th * yi[u] * yj[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * MW_T;
      if (e < tot) {
        const int li = e % MW_R, j = e / MW_R;
        if (c.Ml)
          c.Ml[e] = v[u];
        else if (c.r0 + li < c.r1)
          c.M[mf_idx(n2, c.r0 + li, j)] = v[u];
      }
    }
  }
  __syncthreads();
}

// X <- X R^-1 on this workgroup's rows (R upper in s.H): R^-1 into s.G by
// wavefront 0 (column c on lane c), rows staged in s.Xr.
__device__ void mw_trsm(Mw &c, MwShared &s, double *X, int nb) {
  const int t = threadIdx.x, n2 = c.n2, nr = c.r1 - c.r0;
  double *Ri = s.G;
  if (t < 64) {
    for (int e = t; e < MW_B * MW_B; e += 64) Ri[e] = 0.0;
    wave_sync();
    if (t < nb) {
      const int cc = t;
      for (int a = cc; a >= 0; --a) {
        double v = (a == cc) ? 1.0 : 0.0;
        for (int q = a + 1; q <= cc; ++q) v -= s.H[a + q * MW_B] * Ri[q + cc * MW_B];
        Ri[a + cc * MW_B] = v / s.H[a + a * MW_B];
      }
    }
  }
  for (int e = t; e < nr * nb; e += MW_T) {
    const int i = e % nr, q = e / nr;
    s.Xr[i + q * MW_R] = X[c.r0 + i + (size_t)q * n2];
  }
  __syncthreads();
  for (int e = t; e < nr * nb; e += MW_T) {
    const int i = e % nr, q = e / nr;
    double v = 0.0;
    for (int a = 0; a <= q; ++a) v = fma(s.Xr[i + a * MW_R], Ri[a + q * MW_B], v);
    X[c.r0 + i + (size_t)q * n2] = v;
  }
  __syncthreads();
}

// X (own rows) <- X S for the nb x nb matrix S in LDS.
__device__ void mw_rot(Mw &c, MwShared &s, double *X, int nb, const double *S) {
  const int t = threadIdx.x, n2 = c.n2, nr = c.r1 - c.r0;
  for (int e = t; e < nr * nb; e += MW_T) {
    const int i = e % nr, q = e / nr;
    s.Xr[i + q * MW_R] = X[c.r0 + i + (size_t)q * n2];
  }
  __syncthreads();
  for (int e = t; e < nr * nb; e += MW_T) {
    const int i = e % nr, q = e / nr;
    double v = 0.0;
    for (int a = 0; a < nb; ++a) v = fma(s.Xr[i + a * MW_R], S[a + q * MW_B], v);
    X[c.r0 + i + (size_t)q * n2] = v;
  }
  __syncthreads();
}

// Orthonormalise the nb columns of X against the `locked` columns of L and
// among themselves (CholeskyQR2, shifted CholeskyQR3 if needed).  Returns
// nonzero when even the shifted factorisation fails (the same in every
// workgroup).
__device__ int mw_orth(Mw &c, MwShared &s, double *X, int nb, const double *L, int locked) {
  const int t = threadIdx.x, n2 = c.n2, nr = c.r1 - c.r0;
  int shifted = 0;
  for (int rep = 0; rep < 3; ++rep) {
    if (rep == 2 && !shifted) break;
    if (locked > 0) {
      mw_gram(c, L, locked, X, nb, s.G);
      for (int e = t; e < nr * nb; e += MW_T) {
        const int i = c.r0 + e % nr, q = e / nr;
        double v = X[i + (size_t)q * n2];
        for (int a0 = 0; a0 < locked; a0 += 8) {
          double lv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) lv[u] = L[i + (size_t)min(a0 + u, locked - 1) * n2];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (a0 + u < locked) v -= lv[u] * s.G[a0 + u + q * MW_B];
        }
        X[i + (size_t)q * n2] = v;
      }
      __syncthreads();
    }
    mw_gram(c, X, nb, X, nb, s.H);
    for (int q = t; q < nb; q += MW_T) {
      const double d = s.H[q + q * MW_B];
      s.sc[q] = d > 0 ? 1.0 / sqrt(d) : 1.0;
    }
    __syncthreads();
    for (int e = t; e < nb * nb; e += MW_T) s.H[(e % nb) + (e / nb) * MW_B] *= s.sc[e % nb] * s.sc[e / nb];
    __syncthreads();
    if (small_chol_wave(s.H, nb, 0.0, s.ints)) {
      mw_gram(c, X, nb, X, nb, s.H);
      for (int e = t; e < nb * nb; e += MW_T) s.H[(e % nb) + (e / nb) * MW_B] *= s.sc[e % nb] * s.sc[e / nb];
      __syncthreads();
      double fro = 0.0;
      for (int e = 0; e < nb * nb; ++e) fro += s.H[(e % nb) + (e / nb) * MW_B] * s.H[(e % nb) + (e / nb) * MW_B];
      const double sh = 11.0 * ((double)n2 * nb + (double)nb * (nb + 1)) * 2.220446049250313e-16 * sqrt(fro);
      shifted = 1;
      if (small_chol_wave(s.H, nb, sh, s.ints)) return 1;
    }
    // R = R' D^1/2 so that X R^-1 is the orthonormal factor of X itself
    for (int e = t; e < nb * nb; e += MW_T) {
      const int a = e % nb, q = e / nb;
      if (a <= q) s.H[a + q * MW_B] /= s.sc[q];
    }
    __syncthreads();
    mw_trsm(c, s, X, nb);
  }
  return 0;
}

__global__ __launch_bounds__(MW_T) void k_eig_mw(SmallArgs a) {
  SmallState *st = a.st;
  if (st->done) return;  // read before any barrier, the same in every workgroup
  __shared__ MwShared s;
  extern __shared__ double dyn[];
  const int n2 = a.n2, l = a.l, b = a.b, t = threadIdx.x;
  Mw c;
  c.n2 = n2;
  c.G = gridDim.x;
  c.g = blockIdx.x;
  c.r0 = c.g * MW_R;
  c.r1 = min(n2, c.r0 + MW_R);
  c.M = a.M;
  c.part = a.epart;
  c.pb = 0;
  const bool cacheM = MW_R * n2 <= MW_DYN;
  c.Ml = cacheM ? dyn : nullptr;
  if (cacheM)
    for (int e = t; e < MW_R * n2; e += MW_T) {
      const int li = e % MW_R, kk = e / MW_R, r = c.r0 + li;
      c.Ml[e] = (r < c.r1) ? a.M[mf_idx(n2, r, kk)] : 0.0;
    }
  const double floor_ = st->eig_floor;
  const double maxamp = 1e6;
  double *Y = a.Y, *F0 = a.F0, *F1 = a.F1, *F2 = a.F2;
  double *W = F0;
  const int nr = c.r1 - c.r0;
  const bool first = st->eig_first != 0;  // 2: a given start block in Y
  if (st->eig_first == 1) {
    // start from the columns of M with the largest diagonal entries
    if (t < 64) {
      for (int q = 0; q < b; ++q) {
        double best = -1.0;
        int bi = 0;
        for (int i = t; i < n2; i += 64) {
          bool used = false;
          for (int u = 0; u < q; ++u) used = used || (s.rp[u] == i);
          const double v = used ? -1.0 : a.M[mf_idx(n2, i, i)];
          if (v > best) {
            best = v;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (t == 0) s.rp[q] = bi;
        wave_sync();
      }
    }
    __syncthreads();
    for (int e = t; e < nr * b; e += MW_T) {
      const int i = c.r0 + e % nr, q = e / nr, j = s.rp[q];
      const double mjj = a.M[mf_idx(n2, j, j)];
      Y[i + (size_t)q * n2] = a.M[mf_idx(n2, i, j)] +
                              1e-6 * fabs(mjj) * hash_unit((uint32_t)i, (uint32_t)q) + 1e-300;
    }
    __syncthreads();
  }
  // each round: re-orthonormalisation (after a filter, or of a cold start),
  // Rayleigh-Ritz on the active columns, residuals and locking, then the
  // filter (a single copy of each step keeps the kernel's register use down)
  int locked = 0, it = 0, nmv = 0;
  bool orth = first;  // a cold start orthonormalises its columns first
  while (true) {
    if (orth && mw_orth(c, s, Y + (size_t)locked * n2, b - locked, Y, locked)) {
      if (c.g == 0 && t == 0) atomicOr(a.flags, DEV_EIG_ORTH);
      if (it == 0 && first) return;  // nothing valid to report
      break;
    }
    const int act = b - locked;
    double *Ya = Y + (size_t)locked * n2;
    double *Wa = W + (size_t)locked * n2;
    mw_op(c, s, Ya, act, Wa);
    nmv += act;
    mw_gram(c, Ya, act, Wa, act, s.H);
    for (int q = t; q < locked; q += MW_T) s.keep[q] = s.th[q];
    __syncthreads();
    small_jacobi_wave(s.H, s.S, s.G, &s.tile[0][0], s.th, s.rc, s.rs, s.rp, s.rq, act);
    mw_rot(c, s, Ya, act, s.S);
    mw_rot(c, s, Wa, act, s.S);
    if (t == 0) {
      for (int q = act - 1; q >= 0; --q) s.th[locked + q] = s.th[q];
      for (int q = 0; q < locked; ++q) s.th[q] = s.keep[q];
    }
    __syncthreads();

    mw_resid(c, s, W, Y, locked, l);
    if (t == 0) {
      int lk = locked;
      while (lk < l && s.res[lk - locked] <= floor_) ++lk;
      s.ints[2] = lk;
      double rm = 0.0;
      for (int q = lk; q < l; ++q) rm = fmax(rm, s.res[q - locked]);
      s.rmax = rm;
    }
    __syncthreads();
    const int newl = s.ints[2];
    if (newl >= l || it >= a.eig_maxit) {
      locked = newl;
      break;
    }
    if (newl > locked) mw_deflate(c, s, Y, locked, newl);
    locked = newl;

    const int actf = b - locked;
    double *Yf = Y + (size_t)locked * n2;
    const double cc = s.th[b - 1];
    const double e0 = 0.5 * cc;
    double h = 0.5 * cc;
    const double top = s.th[locked];
    if (!(h > 1e-15 * fabs(top))) h = 1e-15 * fabs(top) + 1e-300;
    const double x = (top - e0) / h;
    int d = a.eig_deg;
    if (x > 1.0) d = min(d, max(2, (int)(log(2.0 * maxamp) / acosh(x))));
    {
      const double xl = (s.th[l - 1] - e0) / h;
      if (xl > 1.0 && s.rmax > 0.0) {
        const double need = 4.0 * s.rmax / floor_;
        const int dn = (need > 1.0) ? (int)ceil(acosh(need) / acosh(xl)) : 2;
        d = min(d, max(2, dn));
      }
    }
    const double sigma = h / (top - e0), tau = 2.0 / sigma;
    double s1 = sigma;
    double *P0 = F0, *P1 = F1, *P2 = F2;
    for (int e = t; e < nr * actf; e += MW_T) {
      const int i = c.r0 + e % nr, q = e / nr;
      P0[i + (size_t)q * n2] = Yf[i + (size_t)q * n2];
    }
    mw_op(c, s, P0, actf, P1);
    for (int e = t; e < nr * actf; e += MW_T) {
      const size_t o = c.r0 + e % nr + (size_t)(e / nr) * n2;
      P1[o] = (P1[o] - e0 * P0[o]) * (s1 / h);
    }
    nmv += actf * d;
    for (int j = 2; j <= d; ++j) {
      const double s2 = 1.0 / (tau - s1);
      mw_op(c, s, P1, actf, P2);
      for (int e = t; e < nr * actf; e += MW_T) {
        const size_t o = c.r0 + e % nr + (size_t)(e / nr) * n2;
        P2[o] = 2.0 * (s2 / h) * (P2[o] - e0 * P1[o]) - (s1 * s2) * P0[o];
      }
      double *tmp = P0;
      P0 = P1;
      P1 = P2;
      P2 = tmp;
      s1 = s2;
    }
    for (int e = t; e < nr * actf; e += MW_T) {
      const size_t o = c.r0 + e % nr + (size_t)(e / nr) * n2;
      Yf[o] = P1[o];
    }
    __syncthreads();
    orth = true;
    ++it;
  }
  if (c.g == 0) {
    for (int q = t; q < b; q += MW_T) a.theta[q] = s.th[q];
    if (t == 0) {
      st->eig_iters += it;
      st->eig_matvecs += nmv;
      st->eig_first = 0;
      st->eig_fail = (it >= a.eig_maxit && locked < l) ? 1 : 0;
    }
  }
}

// Workgroups of the cooperative eigen kernel for n2 (0: use k_eig).
int eig_mw_groups(int n2) {
  if (n2 < EIG_MW_MIN) return 0;
  return (n2 + MW_R - 1) / MW_R;
}

hipError_t launch_eig_mw(hipStream_t s, const SmallArgs &a) {
  const int G = eig_mw_groups(a.n2);
  if (G < 1 || G > 64 || a.epart == nullptr) return hipErrorInvalidValue;
  const size_t shm = (size_t)MW_DYN * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_eig_mw,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  SmallArgs args = a;
  void *kargs[] = {&args};
  return hipLaunchCooperativeKernel((const void *)k_eig_mw, dim3(G), dim3(MW_T), kargs,
                                    (unsigned)shm, s);
}
