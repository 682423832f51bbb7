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
// leading Ritz vectors are locked and deflated (M <- M - L Theta L^T, in
// place, once per locking event) so the filter cannot re-amplify them, and
// the degree is capped so the top active
// component grows at most ~1e6 times the others (the block is then safe for
// Cholesky QR).  Each round ends with CholeskyQR2 (shifted on failure) and a
// Rayleigh-Ritz step solved by parallel cyclic Jacobi.  A Ritz pair is
// converged when ||M y - theta y|| <= eig_floor.
//
// One workgroup of 1024 threads.  Every filter step is a barrier-separated
// sequence of short phases, so the design keeps data on chip: M is read from
// L2 with 8 loads in flight per thread, and the blocks Y (basis), W = M Y and
// the three filter blocks live in LDS when they fit (W shares storage with a
// filter block: it is only needed between the Rayleigh-Ritz step and the next
// filter), else in global memory with LDS staging.  Blocks are addressed
// through a handle that is either an offset into the LDS pool or a global
// pointer, fixed at compile time, so LDS blocks compile to ds_* accesses.
#include "common.h"
#include "launch.h"
#include "eig_small.h"

#define ET 512
#define B_ WLRA_BMAX
#define EIG_POOL 17152     // doubles of LDS for blocks / staging / partial sums
#define EIG_PART 4096      // doubles reserved for matvec partial sums

struct EigLDS {
  double pool[EIG_POOL];
  double H[B_ * B_];    // Gram / Rayleigh quotient / Cholesky factor
  double S[B_ * B_];    // Jacobi rotations (eigenvectors of H)
  double G[B_ * B_];    // L^T X, R^-1
  double th[B_];
  double res[B_];
  double rc[32], rs[32];
  int rp[32], rq[32];
  int ints[4];
  double rmax;  // largest residual of the wanted vectors still unlocked
};

// Block handle: an offset into the LDS pool (RES) or a global pointer.
template <bool RES>
struct Blk;
template <>
struct Blk<true> {
  int off;
  __device__ __forceinline__ double &at(EigLDS &s, int i) const { return s.pool[off + i]; }
  __device__ __forceinline__ Blk<true> plus(int d) const { return Blk<true>{off + d}; }
  __device__ __forceinline__ bool same(const Blk<true> &o) const { return off == o.off; }
};
template <>
struct Blk<false> {
  double *p;
  __device__ __forceinline__ double &at(EigLDS &, int i) const { return p[i]; }
  __device__ __forceinline__ Blk<false> plus(int d) const { return Blk<false>{p + d}; }
  __device__ __forceinline__ bool same(const Blk<false> &o) const { return p == o.p; }
};

#define STAGE_OFF 0                      // staging (global mode), 8192 doubles
#define PART_OFF (EIG_POOL - EIG_PART)   // partial sums / row scratch

struct EigCtx {
  int n2, S, sl, row;    // slices of the matvec, this thread's slice and row
  int l0, l1;            // column range of M owned by this thread
  const double *M;
  double *Mw;            // the same matrix, written by the deflation
  int xs;                // LDS offset of the padded copy of a 16-column block (blocks in LDS)
};

template <bool RES>
__device__ __forceinline__ void blk_gram(EigLDS &s, const EigCtx &cx, Blk<RES> X, int p, Blk<RES> Y,
                                         int q, double *G, bool diag = false);

// Out[:, 0:nc] = M X[:, 0:nc], blocks n2 x * (ld n2), M as deflated so far,
// in passes of 8 columns.  On the FP64 matrix cores with
// v_mfma_f64_4x4x4_4b_f64 (a 16 x 4 slab of M times a 4 x 4 slab of X per
// instruction, so the few columns of the eigen block are not padded to 16).
// The waves form two groups that each take half of the inner index; a wave
// owns every fourth 16-row tile of the output and, per tile, issues all of
// its reads of M (16 bytes per lane per two k-steps, from the fragment-major
// storage) before its first multiply.  The second group writes its partial
// tiles to the output and the first group's, parked in LDS, are added after
// a barrier (a fixed order).
//
// The columns are first copied to an LDS buffer zero-padded to whole groups
// of 8 k-steps, with an odd leading dimension, so that the loop needs no
// clamps or masks and its LDS reads take immediate offsets.  When the
// buffer holds fewer than 8 columns, lanes past them read a zero column.
// epi(f, v) gives the value stored for entry f (row + column n2) of Out
// from v = (M X)[f]; the filter's three-term recurrence runs there.
typedef double eig_d4 __attribute__((ext_vector_type(4)));
#define OP_KH 24   // k-steps of 4 per register batch of M
#define OP_TPW 4   // row tiles per wave per round (4 waves per group: 16 tiles)
struct EpiCopy {
  __device__ __forceinline__ double operator()(int, double v) const { return v; }
};
template <bool RES, typename Epi = EpiCopy>
__device__ __forceinline__ void blk_op(EigLDS &s, const EigCtx &cx, Blk<RES> X, int nc,
                                       Blk<RES> Out, Epi epi = Epi()) {
  const int t = threadIdx.x, n2 = cx.n2;
  const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int grp = wv >> 2, wq = wv & 3;
  const int rtiles = (n2 + 15) / 16;
  const int kq = (n2 + 3) / 4;
  const int kq2 = (int)mf_kq2(n2);  // pairs of k-steps, padded to groups of 8 steps
  const int kq8 = 2 * kq2;
  const int xld = (4 * kq8) | 1;
  // staged columns per pass (8); with fewer, the next column is zero
  const int fbase = RES ? cx.xs : STAGE_OFF;
  const int cwf = RES ? 8 : min(8, 8192 / xld - 1);
  const int ncopy = min(8, cwf + 1);
  // group 0 takes k-steps [0, kh), group 1 [kh, kq8): whole groups of 8
  const int kh = ((kq + 1) / 2 + 7) & ~7;
  const int ks0 = grp * kh, ks1 = min(kq8, ks0 + kh);
  double *part = s.pool + PART_OFF;  // 16 partial tiles of 16 x 16
  for (int c0 = 0; c0 < nc; c0 += cwf) {
    const int cw = min(cwf, nc - c0);
    const Blk<RES> Xc = X.plus(c0 * n2);
    for (int e = t; e < ncopy * xld; e += ET) {
      const int i = e % xld, c = e / xld;
      s.pool[fbase + e] = (i < n2 && c < cw) ? Xc.at(s, i + c * n2) : 0.0;
    }
    __syncthreads();
    // v_mfma_f64_4x4x4_4b_f64: four 4 x 4 blocks (rows 4b..4b+3) per
    // instruction, one instruction per 4 columns.  Its A operand is the
    // same fragment as the 16 x 16 x 4 one (lane l: row l % 16, k l / 16);
    // B[k][j] sits at lane 16k + 4b + j and D[i][j] at lane 16i + 4b + j.
    // Even and odd k-steps go to separate accumulators (four chains).
    const double *xq0 = s.pool + fbase + 4 * ks0 + lk + min(li & 3, cwf) * xld;
    const double *xq1 = s.pool + fbase + 4 * ks0 + lk + min(4 + (li & 3), cwf) * xld;
    // M's fragments of k-steps [ks0 + kb, ks0 + kb + nk) of row tile rt
    auto load_m = [&](double *a, int rt, int kb, int nk) __attribute__((always_inline)) {
      const double2 *mt =
          reinterpret_cast<const double2 *>(cx.M) + ((int64_t)rt * kq2 + ks0 / 2) * 64 + lane;
#pragma unroll
      for (int u0 = 0; u0 < OP_KH; u0 += 8) {
        if (u0 < nk) {
#pragma unroll
          for (int u = u0; u < u0 + 8; u += 2) {
            const double2 v = mt[(int64_t)((kb + u) >> 1) * 64];
            a[u] = v.x;
            a[u + 1] = v.y;
          }
        }
      }
    };
    auto mul = [&](const double *a, int kb, int nk, double &c00, double &c01, double &c10,
                   double &c11) __attribute__((always_inline)) {
#pragma unroll
      for (int u0 = 0; u0 < OP_KH; u0 += 8) {
        if (u0 < nk) {
          double b0[8], b1[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            b0[u] = xq0[4 * (kb + u0 + u)];
            b1[u] = xq1[4 * (kb + u0 + u)];
          }
#pragma unroll
          for (int u = 0; u < 8; u += 2) {
            c00 = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u0 + u], b0[u], c00, 0, 0, 0);
            c10 = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u0 + u], b1[u], c10, 0, 0, 0);
            c01 = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u0 + u + 1], b0[u + 1], c01, 0, 0, 0);
            c11 = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u0 + u + 1], b1[u + 1], c11, 0, 0, 0);
          }
        }
      }
    };
    // group 1 writes its half of tile rt to Out, group 0 parks its half
    auto emit = [&](int rt, int rp0, double d0, double d1) __attribute__((always_inline)) {
      const int row_t = 4 * ((lane >> 2) & 3) + (lane >> 4), col = lane & 3;
      if (grp == 0) {
        part[(rt - rp0) * 256 + row_t * 16 + col] = d0;
        part[(rt - rp0) * 256 + row_t * 16 + 4 + col] = d1;
      } else {
        const int row = rt * 16 + row_t;
        if (row < n2) {
          if (col < cw) Out.at(s, row + (c0 + col) * n2) = d0;
          if (4 + col < cw) Out.at(s, row + (c0 + 4 + col) * n2) = d1;
        }
      }
    };
    for (int rp0 = 0; rp0 < rtiles; rp0 += 4 * OP_TPW) {
#pragma unroll 1
      for (int j = 0; j < OP_TPW; ++j) {
        const int rt = rp0 + wq + 4 * j;
        if (rt >= rtiles) break;
        double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
        for (int kb = 0; kb < ks1 - ks0; kb += OP_KH) {
          const int nk = min(OP_KH, ks1 - ks0 - kb);
          double a[OP_KH];
          load_m(a, rt, kb, nk);
          mul(a, kb, nk, c00, c01, c10, c11);
        }
        emit(rt, rp0, c00 + c01, c10 + c11);
      }
      __syncthreads();
      // Out = epi(group 1's half + group 0's half), a fixed order
      const int pr0 = rp0 * 16, prn = min(n2, (rp0 + 4 * OP_TPW) * 16) - pr0;
      for (int e = t; e < prn * cw; e += ET) {
        const int i = e % prn, c = e / prn;
        const int f = pr0 + i + (c0 + c) * n2;
        Out.at(s, f) = epi(f, Out.at(s, f) + part[(i >> 4) * 256 + (i & 15) * 16 + c]);
      }
      __syncthreads();
    }
  }
}

// G (p x q, ld B_) = X^T Y over n2 rows.  Global blocks are staged through
// LDS first when they fit.  On the FP64 matrix cores: the output is cut into
// 16 x 16 tiles (at most 4) and the inner index into chunks, one (tile,
// chunk) per wavefront; the partial tiles are added in chunk order
// (deterministic).  Column indices are clamped into the blocks (a clamped
// column only feeds an output entry that is not stored) and the last k-step
// is masked.  `diag` stores only a == c (p == q).
__device__ __forceinline__ void gram_pairs(EigLDS &s, int n2, int xoff, int p, int yoff, int q,
                                           double *G, bool diag) {
  const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int tp = (p + 15) / 16, tq = (q + 15) / 16, T = tp * tq;
  const int K = (ET / 64) / T;
  double *part = s.pool + PART_OFF;  // (ET / 64) partial tiles
  if (wv < T * K) {
    const int tile = wv % T, kc = wv / T;
    const int ti = tile % tp, tj = tile / tp;
    const int ks = (n2 + 3) / 4, per = (ks + K - 1) / K;
    const int s0 = kc * per, s1 = min(ks, s0 + per);
    const double *xa = s.pool + xoff + min(16 * ti + li, p - 1) * n2;
    const double *yb = s.pool + yoff + min(16 * tj + li, q - 1) * n2;
    eig_d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int st = s0; st < s1; ++st) {
      const int kk = 4 * st + lk;
      const double av = xa[min(kk, n2 - 1)];
      const double bv = (kk < n2) ? yb[kk] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wv * 256 + (lk + 4 * v) * 16 + li] = acc[v];
  }
  __syncthreads();
  for (int e = t; e < p * q; e += ET) {
    const int a = e % p, c = e / p;
    if (diag && a != c) continue;
    const int tile = (a >> 4) + (c >> 4) * tp;
    double sum = 0.0;
    for (int kc = 0; kc < K; ++kc) sum += part[(tile + kc * T) * 256 + (a & 15) * 16 + (c & 15)];
    G[a + c * B_] = sum;
  }
  __syncthreads();
}

template <bool RES>
__device__ __forceinline__ void blk_gram(EigLDS &s, const EigCtx &cx, Blk<RES> X, int p, Blk<RES> Y,
                                         int q, double *G, bool diag) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, n2 = cx.n2;
  if (RES) {
    gram_pairs(s, n2, reinterpret_cast<const Blk<true> &>(X).off, p,
               reinterpret_cast<const Blk<true> &>(Y).off, q, G, diag);
    return;
  }
  const bool same = X.same(Y) && (p == q);
  if ((int64_t)n2 * (same ? p : p + q) <= 8192) {
    for (int e = t; e < n2 * p; e += ET) s.pool[STAGE_OFF + e] = X.at(s, e);
    if (!same)
      for (int e = t; e < n2 * q; e += ET) s.pool[STAGE_OFF + n2 * p + e] = Y.at(s, e);
    __syncthreads();
    gram_pairs(s, n2, STAGE_OFF, p, same ? STAGE_OFF : STAGE_OFF + n2 * p, q, G, diag);
    return;
  }
  const int pairs = diag ? p : p * q;
  for (int pr = wv; pr < pairs; pr += ET / 64) {
    const int a = diag ? pr : pr % p, c = diag ? pr : pr / p;
    double acc = 0.0;
    for (int i = lane; i < n2; i += 64) acc = fma(X.at(s, i + a * n2), Y.at(s, i + c * n2), acc);
    acc = wave_sum(acc);
    if (lane == 0) G[a + c * B_] = acc;
  }
  __syncthreads();
}

// res[q - q0] = ||W_q - th_q Y_q|| for q in [q0, q1): wave per column.
template <bool RES>
__device__ __forceinline__ void blk_resid(EigLDS &s, int n2, Blk<RES> W, Blk<RES> Y, int q0, int q1) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int q = q0 + wv; q < q1; q += ET / 64) {
    const double th = s.th[q];
    double acc = 0.0;
    for (int i = lane; i < n2; i += 64) {
      const double r = W.at(s, i + q * n2) - th * Y.at(s, i + q * n2);
      acc = fma(r, r, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) s.res[q - q0] = sqrt(acc);
  }
  __syncthreads();
}
// Upper Cholesky in place of G (nb x nb, ld B_) by wavefront 0, with an
// optional diagonal shift.  Returns nonzero on a non-positive pivot.
__device__ __forceinline__ int blk_chol(EigLDS &s, double *G, int nb, double shift) {
  return small_chol_wave(G, nb, shift, s.ints);
}

// X (n2 x nb) <- X S (S nb x nb in LDS, ld B_).  Rows are copied to LDS
// scratch in chunks, column-major (consecutive threads touch consecutive
// words), then each thread forms one output entry.
template <bool RES>
__device__ __forceinline__ void blk_rot(EigLDS &s, int n2, Blk<RES> X, int nb, const double *S) {
  const int t = threadIdx.x;
  const int tmp = RES ? PART_OFF : STAGE_OFF;
  const int cap = RES ? EIG_PART : 8192;
  const int rows = max(1, cap / nb);
  for (int r0 = 0; r0 < n2; r0 += rows) {
    const int nr = min(rows, n2 - r0);
    for (int e = t; e < nr * nb; e += ET) {
      const int i = e % nr, c = e / nr;
      s.pool[tmp + e] = X.at(s, r0 + i + c * n2);
    }
    __syncthreads();
    for (int e = t; e < nr * nb; e += ET) {
      const int i = e % nr, c = e / nr;
      double v = 0.0;
      for (int a = 0; a < nb; ++a) v = fma(s.pool[tmp + i + a * nr], S[a + c * B_], v);
      X.at(s, r0 + i + c * n2) = v;
    }
    __syncthreads();
  }
}

// The small steps of one CholeskyQR pass, from the Gram H of the nb columns
// of X (nb x nb, ld B_): with D = diag(H), R'^T R' = D^-1/2 H D^-1/2 (plus
// a diagonal shift of shift_coef ||D^-1/2 H D^-1/2||_F when shift_coef > 0),
// R = R' D^1/2 and G = R^-1 (upper), so that X G is the orthonormal factor
// of X.  For nb <= 8 all of it runs on wavefront 0 between two barriers,
// the Gram entry (x, y) in lane x + nb y and column c of R^-1 in lane c;
// larger blocks take the steps one by one.  Returns nonzero on a
// non-positive pivot.
__device__ __forceinline__ int cqr_small(EigLDS &s, int nb, double shift_coef) {
  const int t = threadIdx.x;
  if (nb > 8) {
    for (int c = t; c < nb; c += ET) {
      const double d = s.H[c + c * B_];
      s.res[c] = d > 0 ? 1.0 / sqrt(d) : 1.0;  // a zero column is left to the shift
    }
    __syncthreads();
    for (int e = t; e < nb * nb; e += ET) {
      const int a2 = e % nb, c = e / nb;
      s.H[a2 + c * B_] *= s.res[a2] * s.res[c];
    }
    __syncthreads();
    double sh = 0.0;
    if (shift_coef > 0.0) {
      double fro = 0.0;
      for (int e = 0; e < nb * nb; ++e) fro += s.H[(e % nb) + (e / nb) * B_] * s.H[(e % nb) + (e / nb) * B_];
      sh = shift_coef * sqrt(fro);
    }
    if (blk_chol(s, s.H, nb, sh)) return 1;
    for (int e = t; e < nb * nb; e += ET) {
      const int a2 = e % nb, c = e / nb;
      if (a2 <= c) s.H[a2 + c * B_] /= s.res[c];
    }
    __syncthreads();
    double *Ri = s.G;
    if (t < 64) {
      for (int e = t; e < B_ * B_; e += 64) Ri[e] = 0.0;
      wave_sync();
      if (t < nb) {
        const int c = t;
        for (int a = c; a >= 0; --a) {
          double v = (a == c) ? 1.0 : 0.0;
          for (int q = a + 1; q <= c; ++q) v -= s.H[a + q * B_] * Ri[q + c * B_];
          Ri[a + c * B_] = v / s.H[a + a * B_];
        }
      }
    }
    __syncthreads();
    return 0;
  }
  if (t < 64) {
    const bool in = t < nb * nb;
    const int x = in ? t % nb : 0, y = in ? t / nb : 0;
    const double h = in ? s.H[x + y * B_] : 0.0;
    const double dx = __shfl(h, x + x * nb, 64), dy = __shfl(h, y + y * nb, 64);
    const double sx = dx > 0 ? rsq_nr(dx) : 1.0, sy = dy > 0 ? rsq_nr(dy) : 1.0;
    double g = h * (sx * sy);
    if (shift_coef > 0.0) {
      const double fro = wave_sum(in ? g * g : 0.0);
      if (in && x == y) g += shift_coef * sqrt(fro);
    }
    int bad = 0;
    for (int j = 0; j < nb; ++j) {
      double p = __shfl(g, j + j * nb, 64);
      if (!(p > 0.0)) {
        bad = 1;
        p = 1.0;
      }
      const double ir = rsq_nr(p), rjj = p * ir;
      if (in && x == j) g = (y == j) ? rjj : ((y > j) ? g * ir : g);
      const double rx = __shfl(g, j + x * nb, 64), ry = __shfl(g, j + y * nb, 64);
      if (in && x > j && x <= y) g -= rx * ry;
    }
    // R = R' D^1/2 to LDS (upper triangle), then column t of R^-1 by back
    // substitution in registers
    if (in && x <= y) s.H[x + y * B_] = g / sy;
    wave_sync();
    if (t < nb) {
      const int c = t;
      double ri[8];
#pragma unroll
      for (int a = 7; a >= 0; --a) {
        double v = (a == c) ? 1.0 : 0.0;
#pragma unroll
        for (int q = a + 1; q < 8; ++q)
          if (q <= c) v = fma(-s.H[min(a, nb - 1) + min(q, nb - 1) * B_], ri[q], v);
        ri[a] = (a <= c && a < nb) ? v * rcp_nr(s.H[min(a, nb - 1) + min(a, nb - 1) * B_]) : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (a < nb) s.G[a + c * B_] = ri[a];
    }
    if (t == 0) s.ints[0] = bad;
  }
  __syncthreads();
  return s.ints[0];
}

// Hotelling deflation of newly locked Ritz pairs, once per locking event:
// M <- M - sum_{a in [q0, q1)} th_a y_a y_a^T, in place in global memory (M
// is formed afresh for every eigen step and read by nothing else), walking
// the fragment-major storage in order.  The
// filter steps then multiply by the deflated matrix directly.  Reads go in
// batches of DF_U per thread, clamped to stay in bounds, so that they are in
// flight together.
#define DF_U 16
template <bool RES>
__device__ __forceinline__ void blk_deflate(EigLDS &s, const EigCtx &cx, Blk<RES> Y, int q0, int q1) {
  const int t = threadIdx.x, n2 = cx.n2;
  const int nn = (int)mf_size(n2), kq2 = (int)mf_kq2(n2);
  // offset f = e0 + u * ET: its lane/pair bits are fixed by t, its 128-double
  // block advances by 4 per u (no division in the loop)
  const int h = t & 1, lane = (t >> 1) & 63;
  const int ri = lane & 15, cj = 4 * h + (lane >> 4);
  double *M = cx.Mw;
  for (int e0 = t; e0 < nn; e0 += DF_U * ET) {
    double v[DF_U];
#pragma unroll
    for (int u = 0; u < DF_U; ++u) v[u] = M[min(e0 + u * ET, nn - 1)];
    const int T0 = e0 >> 7;
    int rt = T0 / kq2, q2 = T0 - rt * kq2;
#pragma unroll
    for (int u = 0; u < DF_U; ++u) {
      const int i = rt * 16 + ri, j = 8 * q2 + cj;
      if (e0 + u * ET < nn && i < n2 && j < n2)
        for (int a = q0; a < q1; ++a) v[u] -= s.th[a] * Y.at(s, i + a * n2) * Y.at(s, j + a * n2);
      q2 += 4;
      if (q2 >= kq2) {
        q2 -= kq2;
        ++rt;
      }
    }
#pragma unroll
    for (int u = 0; u < DF_U; ++u)
      if (e0 + u * ET < nn) M[e0 + u * ET] = v[u];
  }
  __syncthreads();
}

// Symmetric eigendecomposition of H (nb x nb) by parallel cyclic Jacobi on
// wavefront 0, with G and the partial-sum region of the pool as scratch.  On
// return th[0..nb) is descending and S holds the eigenvectors.
__device__ __forceinline__ void blk_jacobi(EigLDS &s, int nb) {
  small_jacobi_wave(s.H, s.S, s.G, s.pool + PART_OFF, s.th, s.rc, s.rs, s.rp, s.rq, nb);
}

// X (n2 x nb) <- X S - L F (S nb x nb, F locked x nb, both ld B_, in LDS;
// L n2 x locked): X's and L's rows staged column-major in LDS scratch by
// chunks, then one output entry per thread.
template <bool RES>
__device__ __forceinline__ void blk_rot_proj(EigLDS &s, int n2, Blk<RES> X, int nb,
                                             const double *S, Blk<RES> L, int locked,
                                             const double *F) {
  const int t = threadIdx.x;
  const int tmp = RES ? PART_OFF : STAGE_OFF;
  const int cap = RES ? EIG_PART : 8192;
  const int wd = nb + locked;
  const int rows = max(1, cap / wd);
  for (int r0 = 0; r0 < n2; r0 += rows) {
    const int nr = min(rows, n2 - r0);
    for (int e = t; e < nr * wd; e += ET) {
      const int i = e % nr, c = e / nr;
      s.pool[tmp + e] = c < nb ? X.at(s, r0 + i + c * n2) : L.at(s, r0 + i + (c - nb) * n2);
    }
    __syncthreads();
    for (int e = t; e < nr * nb; e += ET) {
      const int i = e % nr, c = e / nr;
      double v = 0.0;
      for (int a = 0; a < nb; ++a) v = fma(s.pool[tmp + i + a * nr], S[a + c * B_], v);
      for (int q = 0; q < locked; ++q) v = fma(-s.pool[tmp + i + (nb + q) * nr], F[q + c * B_], v);
      X.at(s, r0 + i + c * n2) = v;
    }
    __syncthreads();
  }
}

// H = X^T X - G^T G for the Gram of [L X] against X in s.S (rows 0 .. locked-1
// G = L^T X, rows locked .. X^T X): the Gram of X - L L^T X for orthonormal L.
__device__ __forceinline__ void proj_gram(EigLDS &s, int locked, int nb) {
  for (int e = threadIdx.x; e < nb * nb; e += ET) {
    const int a2 = e % nb, c = e / nb;
    double v = s.S[locked + a2 + c * B_];
    for (int q = 0; q < locked; ++q) v = fma(-s.S[q + a2 * B_], s.S[q + c * B_], v);
    s.H[a2 + c * B_] = v;
  }
  __syncthreads();
}

// Orthonormalise the nb columns of X against the `locked` columns of L and
// among themselves: CholeskyQR2, shifted CholeskyQR3 if the Gram is not
// numerically positive definite.  With locked columns (which must directly
// precede X's in the same block) each pass forms one Gram of [L X] against X,
// takes the projected Gram X^T X - (L^T X)^T (L^T X), and applies
// X <- (X - L L^T X) R^-1 = X R^-1 - L (L^T X R^-1) in one rotation pass: the
// filter has shrunk X's components along the locked (deflated) vectors, so
// the subtraction cancels little.
template <bool RES>
__device__ __forceinline__ void blk_orth(EigLDS &s, const EigCtx &cx, Blk<RES> X, int nb,
                                         Blk<RES> L, int locked, int *flags) {
  const int t = threadIdx.x, n2 = cx.n2;
  const double shift_coef = 11.0 * ((double)n2 * nb + (double)nb * (nb + 1)) * 2.220446049250313e-16;
  int shifted = 0;
  for (int rep = 0; rep < 3; ++rep) {
    if (rep == 2 && !shifted) break;
    if (locked > 0) {
      blk_gram<RES>(s, cx, L, locked + nb, X, nb, s.S);
      proj_gram(s, locked, nb);
      if (cqr_small(s, nb, 0.0)) {
        proj_gram(s, locked, nb);
        shifted = 1;
        if (cqr_small(s, nb, shift_coef)) {
          if (t == 0) atomicOr(flags, DEV_EIG_ORTH);
          return;
        }
      }
      // F = (L^T X) R^-1 (locked x nb) into s.H, free once R^-1 is formed
      for (int e = t; e < locked * nb; e += ET) {
        const int q = e % locked, c = e / locked;
        double v = 0.0;
        for (int a2 = 0; a2 <= c; ++a2) v = fma(s.S[q + a2 * B_], s.G[a2 + c * B_], v);
        s.H[q + c * B_] = v;
      }
      __syncthreads();
      blk_rot_proj<RES>(s, n2, X, nb, s.G, L, locked, s.H);
      continue;
    }
    // Gram, scaled to unit diagonal (D^-1/2 G D^-1/2 = R'^T R'), so that
    // X R^-1 = X D^-1/2 R'^-1: the normalisation costs no pass over X
    blk_gram<RES>(s, cx, X, nb, X, nb, s.H);
    if (cqr_small(s, nb, 0.0)) {
      blk_gram<RES>(s, cx, X, nb, X, nb, s.H);
      shifted = 1;
      if (cqr_small(s, nb, shift_coef)) {
        if (t == 0) atomicOr(flags, DEV_EIG_ORTH);
        return;
      }
    }
    blk_rot<RES>(s, n2, X, nb, s.G);  // X R^-1
  }
}


template <bool RES>
__device__ __forceinline__ void eig_body(EigLDS &s, const SmallArgs &a, const EigCtx &cx,
                                         Blk<RES> Y, Blk<RES> F0, Blk<RES> F1, Blk<RES> F2) {
  SmallState *st = a.st;
  const int n2 = a.n2, l = a.l, b = a.b, t = threadIdx.x;
  const double floor_ = st->eig_floor;
  const double maxamp = 1e6;
  Blk<RES> W = F0;
  if (st->eig_first == 1) {
    // Start from the columns of M with the largest diagonal entries (the
    // frames whose residual energy is largest, on which the leading
    // eigenvectors concentrate), plus a small deterministic perturbation
    // that keeps the block of full rank.
    if (t < 64) {
      for (int q = 0; q < b; ++q) {
        double best = -1.0;
        int bi = 0;
        for (int i = t; i < n2; i += 64) {
          bool used = false;
          for (int u = 0; u < q; ++u) used = used || (s.rp[u] == i);
          const double v = used ? -1.0 : cx.M[mf_idx(n2, i, i)];
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
    for (int e = t; e < n2 * b; e += ET) {
      const int i = e % n2, q = e / n2, j = s.rp[q];
      const double mjj = cx.M[mf_idx(n2, j, j)];
      Y.at(s, e) = cx.M[mf_idx(n2, i, j)] +
                   1e-6 * fabs(mjj) * hash_unit((uint32_t)i, (uint32_t)q) + 1e-300;
    }
  } else if (RES) {
    for (int e = t; e < n2 * b; e += ET) Y.at(s, e) = a.Y[e];
  }
  __syncthreads();
  // a warm start is the previous sweep's Ritz block, orthonormal already; a
  // cold start or a given start (eig_first 2) is orthonormalised first
  if (st->eig_first) blk_orth<RES>(s, cx, Y, b, Y, 0, a.flags);
  blk_op<RES>(s, cx, Y, b, W);
  blk_gram<RES>(s, cx, Y, b, W, b, s.H);
  blk_jacobi(s, b);
  blk_rot<RES>(s, n2, Y, b, s.S);
  blk_rot<RES>(s, n2, W, b, s.S);
  int locked = 0, it = 0, nmv = b;
  while (true) {
    // residuals ||W_q - th_q Y_q|| for q in [locked, l); lock the converged prefix
    blk_resid<RES>(s, n2, W, Y, locked, l);
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
    if (newl > locked) blk_deflate<RES>(s, cx, Y, locked, newl);
    locked = newl;

    const int act = b - locked;
    const Blk<RES> Ya = Y.plus(locked * n2);
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
    // no higher than the residual reduction still needed asks for: the
    // l-th Ritz vector's error shrinks by about T_d((th_l - e0) / h)
    {
      const double rmax = s.rmax;
      const double xl = (s.th[l - 1] - e0) / h;
      if (xl > 1.0 && rmax > 0.0) {
        const double need = 4.0 * rmax / floor_;
        const int dn = (need > 1.0) ? (int)ceil(acosh(need) / acosh(xl)) : 2;
        d = min(d, max(2, dn));
      }
    }
    const double sigma = h / (top - e0), tau = 2.0 / sigma;
    double s1 = sigma;
    // the recurrence's three blocks rotate through Ya (the filter's input,
    // not needed once the first step has read it), F1 and F2
    Blk<RES> P0 = Ya, P1 = F1, P2 = F2;
    {
      const double f1 = s1 / h;
      blk_op<RES>(s, cx, P0, act, P1, [&](int f, double v) { return (v - e0 * P0.at(s, f)) * f1; });
    }
    nmv += act * (d + 1);
    for (int j = 2; j <= d; ++j) {
      const double s2 = 1.0 / (tau - s1);
      const double f2 = 2.0 * (s2 / h), f0 = s1 * s2;
      blk_op<RES>(s, cx, P1, act, P2, [&](int f, double v) {
        return f2 * (v - e0 * P1.at(s, f)) - f0 * P0.at(s, f);
      });
      const Blk<RES> tmp = P0;
      P0 = P1;
      P1 = P2;
      P2 = tmp;
      s1 = s2;
    }
    if (!P1.same(Ya)) {
      for (int e = t; e < n2 * act; e += ET) Ya.at(s, e) = P1.at(s, e);
      __syncthreads();
    }
    blk_orth<RES>(s, cx, Ya, act, Y, locked, a.flags);
    // W (active columns) in F0: free once the filter is done
    const Blk<RES> Wa = W.plus(locked * n2);
    blk_op<RES>(s, cx, Ya, act, Wa);
    blk_gram<RES>(s, cx, Ya, act, Wa, act, s.H);
    // keep the locked Ritz values while Jacobi overwrites th[0..act)
    for (int q = t; q < locked; q += ET) s.res[q] = s.th[q];
    __syncthreads();
    blk_jacobi(s, act);
    blk_rot<RES>(s, n2, Ya, act, s.S);
    blk_rot<RES>(s, n2, Wa, act, s.S);
    if (t == 0) {
      for (int q = act - 1; q >= 0; --q) s.th[locked + q] = s.th[q];
      for (int q = 0; q < locked; ++q) s.th[q] = s.res[q];
    }
    __syncthreads();
    ++it;
  }
  if (RES)
    for (int e = t; e < n2 * b; e += ET) a.Y[e] = Y.at(s, e);
  for (int q = t; q < b; q += ET) a.theta[q] = s.th[q];
  if (t == 0) {
    st->eig_iters += it;
    st->eig_matvecs += nmv;
    st->eig_first = 0;
    st->eig_fail = (it >= a.eig_maxit && locked < l) ? 1 : 0;
  }
}

__device__ __forceinline__ void eig_kernel_body(const SmallArgs &a) {
  if (a.st->done) return;
  __shared__ EigLDS s;
  const int n2 = a.n2, b = a.b, t = threadIdx.x;
  EigCtx cx;
  cx.n2 = n2;
  cx.M = a.M;
  cx.Mw = a.M;
  cx.S = max(1, min(8, ET / n2));
  cx.sl = t / n2;
  cx.row = (t < cx.S * n2) ? t % n2 : -1;
  cx.l0 = cx.sl * n2 / cx.S;
  cx.l1 = (cx.sl + 1) * n2 / cx.S;
  // the blocks live in LDS when they fit with room after them for the padded
  // copy of a 16-column block (the product's B operand)
  const int xld = (8 * (int)mf_kq2(n2)) | 1;
  cx.xs = 4 * n2 * b;
  if (4 * n2 * b + 16 * xld <= PART_OFF) {
    eig_body<true>(s, a, cx, Blk<true>{0}, Blk<true>{n2 * b}, Blk<true>{2 * n2 * b},
                   Blk<true>{3 * n2 * b});
  } else {
    eig_body<false>(s, a, cx, Blk<false>{a.Y}, Blk<false>{a.F0}, Blk<false>{a.F1},
                    Blk<false>{a.F2});
  }
}
__global__ __launch_bounds__(ET) void k_eig(SmallArgs a) { eig_kernel_body(a); }
// one workgroup per instance of a batch
__global__ __launch_bounds__(ET) void k_eig_b(const SmallArgs *__restrict__ av) {
  eig_kernel_body(av[blockIdx.x]);
}

void launch_eig_b(hipStream_t s, int count, const SmallArgs *av) {
  if (count > 0) hipLaunchKernelGGL(k_eig_b, dim3(count), dim3(ET), 0, s, av);
}

// Start block of the first eigen step from a given V (v0 x l, ld ldv):
// Y(i, q) = V(i, q) for i < v0 and q < l, zero for the other rows, and the
// b - l guard columns small pseudo-random vectors that keep the block of full
// rank (the eigen step orthonormalises it).
__global__ __launch_bounds__(256) void k_eig_seed(int n2, int l, int b, const double *V,
                                                  int64_t ldv, int v0, double *Y) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n2 * b; e += gridDim.x * 256) {
    const int i = e % n2, q = e / n2;
    double v;
    if (q < l)
      v = (i < v0) ? V[i + (int64_t)q * ldv] : 0.0;
    else
      v = hash_unit((uint32_t)i, (uint32_t)q) / sqrt((double)n2);
    Y[e] = v;
  }
}

void launch_eig_seed(hipStream_t s, int n2, int l, int b, const double *V, int64_t ldv, int v0,
                     double *Y) {
  const int grid = std::max(1, std::min(64, (n2 * b + 255) / 256));
  hipLaunchKernelGGL(k_eig_seed, dim3(grid), dim3(256), 0, s, n2, l, b, V, ldv, v0, Y);
}

void launch_eig(hipStream_t s, const SmallArgs &a) {
  // larger n2: the multi-workgroup kernel; the one-workgroup kernel serves
  // small n2 and any case the cooperative launch is refused
  // (a.eig_one_wg, a handle option, forces the one-workgroup kernel)
  if (eig_mw_groups(a.n2) > 0 && !a.eig_one_wg && launch_eig_mw(s, a) == hipSuccess)
    return;
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(ET), 0, s, a);
}
