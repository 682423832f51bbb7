// Streaming kernels of the sWLR sweep: passes over the m rows of A.
//
// All matrices are column-major.  Row i of a matrix is strided by its leading
// dimension, so a wavefront whose 64 lanes take 64 consecutive rows reads
// 64 consecutive elements of each column: every global load below is
// coalesced.  Sums over rows accumulate in double in every precision.
#include "common.h"

// ---------------------------------------------------------------------------
// Input checks (problem (5) needs finite A and W1 > 0; Theorem 2 assumes
// (W1)_ij > 0).  flags |= DEV_BAD_A / DEV_BAD_W.
template <typename T>
__global__ __launch_bounds__(256) void k_validate(int64_t m, int64_t n, const T *__restrict__ A,
                                                  int64_t lda, int64_t k, const T *__restrict__ W1,
                                                  int64_t ldw, int *flags) {
  int bad_a = 0, bad_w = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
      const T v = A[i + j * lda];
      if (!isfinite(v)) bad_a = 1;
      if (W1 != nullptr && j < k) {
        const T w = W1[i + j * ldw];
        if (!(w > T(0)) || !isfinite(w)) bad_w = 1;
      }
    }
  }
  bad_a = __syncthreads_or(bad_a);
  bad_w = __syncthreads_or(bad_w);
  if (threadIdx.x == 0) {
    if (bad_a) atomicOr(flags, DEV_BAD_A);
    if (bad_w) atomicOr(flags, DEV_BAD_W);
  }
}

// ---------------------------------------------------------------------------
// X1_0: mode 0 = iid N(0,1) (Philox4x32-10 + Box-Muller), 1 = copy of a given
// matrix, 2 = copy of A1.  Non-finite given entries set DEV_BAD_A.
template <typename T>
__global__ __launch_bounds__(256) void k_init_x1(int64_t m, int64_t k, int mode, uint64_t seed,
                                                 const T *__restrict__ src, int64_t lds,
                                                 T *__restrict__ X1, int *flags) {
  const int64_t total = m * k;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / m, i = e - c * m;
    T v;
    if (mode == 0) {
      double z0, z1;
      philox_normal2(seed, (uint64_t)(e >> 1), z0, z1);
      v = (T)((e & 1) ? z1 : z0);
    } else {
      v = src[i + c * lds];
      if (!isfinite(v)) bad = 1;
    }
    X1[e] = v;
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flags, DEV_BAD_A);
}

// ---------------------------------------------------------------------------
// Tall-skinny transposed product:  part[s] = X[rows of split s]^T Y[rows of s]
// (k1 x k2, double).  32 x 32 output tile per workgroup, 2 x 2 per thread;
// row chunks of 32 are staged through LDS as double.  `sym` computes only the
// tiles on or above the diagonal (X == Y).
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tsgemm(int64_t m, const TX *__restrict__ X, int64_t ldx,
                                                int k1, const TY *__restrict__ Y, int64_t ldy,
                                                int k2, int sym, int64_t rows_per_split,
                                                double *__restrict__ part, const int *skip) {
  if (skip != nullptr && *skip) return;
  const int ti = blockIdx.x, tj = blockIdx.y, s = blockIdx.z;
  if (sym && ti > tj) return;
  __shared__ double sX[32][33];
  __shared__ double sY[32][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = ti * 32, j0 = tj * 32;
  const int64_t r0 = (int64_t)s * rows_per_split;
  const int64_t r1 = min(m, r0 + rows_per_split);
  double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
  for (int64_t rb = r0; rb < r1; rb += 32) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int rr = e & 31, cc = e >> 5;
      const int64_t row = rb + rr;
      const bool rin = row < r1;
      sX[cc][rr] = (rin && i0 + cc < k1) ? (double)X[row + (int64_t)(i0 + cc) * ldx] : 0.0;
      sY[cc][rr] = (rin && j0 + cc < k2) ? (double)Y[row + (int64_t)(j0 + cc) * ldy] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) {
      const double x0 = sX[2 * tx][rr], x1 = sX[2 * tx + 1][rr];
      const double y0 = sY[2 * ty][rr], y1 = sY[2 * ty + 1][rr];
      a00 = fma(x0, y0, a00);
      a01 = fma(x0, y1, a01);
      a10 = fma(x1, y0, a10);
      a11 = fma(x1, y1, a11);
    }
    __syncthreads();
  }
  double *out = part + (int64_t)s * k1 * k2;
  const int i = i0 + 2 * tx, j = j0 + 2 * ty;
  if (i < k1 && j < k2) out[i + (int64_t)j * k1] = a00;
  if (i < k1 && j + 1 < k2) out[i + (int64_t)(j + 1) * k1] = a01;
  if (i + 1 < k1 && j < k2) out[i + 1 + (int64_t)j * k1] = a10;
  if (i + 1 < k1 && j + 1 < k2) out[i + 1 + (int64_t)(j + 1) * k1] = a11;
}

// Sum of the split partials in a fixed order (deterministic).  For `sym`
// the lower tiles are mirrored from the upper ones.
__global__ __launch_bounds__(256) void k_reduce_parts(int k1, int k2, int splits, int sym,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ out,
                                                      const int *skip) {
  if (skip != nullptr && *skip) return;
  const int64_t total = (int64_t)k1 * k2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e % k1), j = (int)(e / k1);
    int64_t src = e;
    if (sym && (i >> 5) > (j >> 5)) src = j + (int64_t)i * k1;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += part[(int64_t)s * total + src];
    out[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// f1 = ||(A1 - X1) o W1||^2 for the start matrix; partial per workgroup,
// written as (f1, 0) pairs in the same layout k_update uses.
template <typename T>
__global__ __launch_bounds__(256) void k_f1(int64_t m, int k, const T *__restrict__ A, int64_t lda,
                                            const T *__restrict__ W1, int64_t ldw, double wc,
                                            const T *__restrict__ X1, double *__restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / m, i = e - c * m;
    const double w = W1 ? (double)W1[i + c * ldw] : wc;
    const double d = (double)A[i + c * lda] - (double)X1[e];
    acc += d * d * w * w;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// The X1 update of Algorithm 1 (steps 7-9), one row per lane, 64 rows per
// workgroup (one wavefront).  Row i of X1_{p+1} is E_p(i,:) K_i^-1 with
// K_i = diag(W1(i,:)^2) + C C^T and E_p = A1 o W1 o W1 + (A2 - D_p) C_p^T.
// Since D_p = (A2 - X1 C) V V^T,  (A2 - D_p) C^T = A2 Z + X1 T  with
// Z = (I - V V^T) C^T and T = (CV)(CV)^T.  The kernel solves for the
// deviation from A1 instead of X1 itself:
//     y_i = (a2_i Z + x1_i T - a1_i S) K_i^-1,     x1_i' = a1_i + y_i,
// which is the same row (E - A1 K = (A2 - D) C^T - A1 S) without the
// a1 o w^2 term whose size (w^2 up to 1e8) would otherwise swamp the rounding
// of x1' once the objective weighs it again by w^2.
// When W1 is one constant w, K = w^2 I + S is shared: the small step
// pre-multiplies Z, T and S by K^-1 and no per-row solve is needed.
// Layouts (row-major, input index first): Zt[j*k + c], Tt[c'*k + c],
// St[c'*k + c] (S, or S K^-1 when CONSTW).
// Per-row Cholesky factors live in LDS, lane-interleaved (element e of lane l
// at [e*nl + l]), for `nl` lanes at a time.
// Partials per workgroup: (||(A1 - X1') o W1||^2, ||X1' - X1||^2).
template <typename T, int KMAX, bool CONSTW>
__global__ __launch_bounds__(64) void k_update(int64_t m, int k, int n2, const T *__restrict__ A,
                                               int64_t lda, const T *__restrict__ W1, int64_t ldw,
                                               T wc, const T *__restrict__ X1o,
                                               T *__restrict__ X1n, const T *__restrict__ Zt,
                                               const T *__restrict__ Tt, const T *__restrict__ St,
                                               double *__restrict__ part, int nl,
                                               const SmallState *__restrict__ st, int *flags) {
  if (st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);

  T e[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) e[c] = T(0);

  for (int cp = 0; cp < k; ++cp) {
    const T xv = X1o[ir + (int64_t)cp * m];
    const T *row = Tt + cp * k;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) e[c] = fma(xv, row[c], e[c]);
  }
  for (int cp = 0; cp < k; ++cp) {
    const T av = A[ir + (int64_t)cp * lda];
    const T *row = St + cp * k;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) e[c] = fma(-av, row[c], e[c]);
  }
  const T *A2 = A + (int64_t)k * lda;
  int j = 0;
  for (; j + 4 <= n2; j += 4) {
    const T v0 = A2[ir + (int64_t)j * lda];
    const T v1 = A2[ir + (int64_t)(j + 1) * lda];
    const T v2 = A2[ir + (int64_t)(j + 2) * lda];
    const T v3 = A2[ir + (int64_t)(j + 3) * lda];
    const T *z0 = Zt + (int64_t)j * k;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) {
        T t = e[c];
        t = fma(v0, z0[c], t);
        t = fma(v1, z0[k + c], t);
        t = fma(v2, z0[2 * k + c], t);
        t = fma(v3, z0[3 * k + c], t);
        e[c] = t;
      }
  }
  for (; j < n2; ++j) {
    const T v0 = A2[ir + (int64_t)j * lda];
    const T *z0 = Zt + (int64_t)j * k;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) e[c] = fma(v0, z0[c], e[c]);
  }

  int bad = 0;
  if (!CONSTW) {
    const int tri = k * (k + 1) / 2;
    for (int round = 0; round < 64; round += nl) {
      const int sl = lane - round;
      if (sl >= 0 && sl < nl) {
        T *L = sm + sl;
        T *E = sm + (int64_t)tri * nl + sl;
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
          if (c < k) E[c * nl] = e[c];
        for (int jj = 0; jj < k; ++jj) {
          const int bj = jj * (jj + 1) / 2;
          const T w = W1[ir + (int64_t)jj * ldw];
          T s = fma(w, w, St[jj * k + jj]);
          for (int p = 0; p < jj; ++p) {
            const T l = L[(bj + p) * nl];
            s -= l * l;
          }
          if (!(s > T(0))) {
            bad = 1;
            s = T(1);
          }
          const T ljj = sqrt(s);
          L[(bj + jj) * nl] = ljj;
          const T inv = T(1) / ljj;
          for (int ii = jj + 1; ii < k; ++ii) {
            const int bi = ii * (ii + 1) / 2;
            T t = St[ii * k + jj];
            for (int p = 0; p < jj; ++p) t -= L[(bi + p) * nl] * L[(bj + p) * nl];
            L[(bi + jj) * nl] = t * inv;
          }
        }
        for (int ii = 0; ii < k; ++ii) {
          const int bi = ii * (ii + 1) / 2;
          T t = E[ii * nl];
          for (int p = 0; p < ii; ++p) t -= L[(bi + p) * nl] * E[p * nl];
          E[ii * nl] = t / L[(bi + ii) * nl];
        }
        for (int ii = k - 1; ii >= 0; --ii) {
          T t = E[ii * nl];
          for (int p = ii + 1; p < k; ++p) t -= L[(p * (p + 1) / 2 + ii) * nl] * E[p * nl];
          E[ii * nl] = t / L[(ii * (ii + 1) / 2 + ii) * nl];
        }
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
          if (c < k) e[c] = E[c * nl];
      }
    }
  }

  double f1 = 0.0, dx = 0.0;
  if (act) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) {
        const T x = A[i + (int64_t)c * lda] + e[c];
        X1n[i + (int64_t)c * m] = x;
        const double w = CONSTW ? (double)wc : (double)W1[i + (int64_t)c * ldw];
        const double d = (double)A[i + (int64_t)c * lda] - (double)x;
        f1 += d * d * w * w;
        const double dd = (double)x - (double)X1o[i + (int64_t)c * m];
        dx += dd * dd;
      }
  }
  f1 = wave_sum(f1);
  dx = wave_sum(dx);
  if (lane == 0) {
    part[2 * blockIdx.x] = f1;
    part[2 * blockIdx.x + 1] = dx;
  }
  if (bad) atomicOr(flags, DEV_ROWSOLVE);
}

// ---------------------------------------------------------------------------
// Dense output X2 = X1 C + D = a2 V V^T + x1 Z^T row by row (one row per
// lane): u = a2_i V, then x2_ij = u . V(j,:) + x1_i . Z(j,:).
// Vr is n2 x l row-major, Zt n2 x k row-major (same as k_update).
template <typename T, int KMAX, int LMAX>
__global__ __launch_bounds__(64) void k_x2(int64_t m, int k, int n2, int l,
                                           const T *__restrict__ A, int64_t lda,
                                           const T *__restrict__ X1, const T *__restrict__ Zt,
                                           const T *__restrict__ Vr, T *__restrict__ X2,
                                           int64_t ldx2) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  const T *A2 = A + (int64_t)k * lda;
  T u[LMAX];
  T x[KMAX];
#pragma unroll
  for (int q = 0; q < LMAX; ++q) u[q] = T(0);
  for (int j = 0; j < n2; ++j) {
    const T v = A2[ir + (int64_t)j * lda];
    const T *vr = Vr + (int64_t)j * l;
#pragma unroll
    for (int q = 0; q < LMAX; ++q)
      if (q < l) u[q] = fma(v, vr[q], u[q]);
  }
#pragma unroll
  for (int c = 0; c < KMAX; ++c) x[c] = (c < k) ? X1[ir + (int64_t)c * m] : T(0);
  for (int j = 0; j < n2; ++j) {
    const T *vr = Vr + (int64_t)j * l;
    const T *zr = Zt + (int64_t)j * k;
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < LMAX; ++q)
      if (q < l) acc = fma(u[q], vr[q], acc);
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) acc = fma(x[c], zr[c], acc);
    if (act) X2[i + (int64_t)j * ldx2] = acc;
  }
}

// ---------------------------------------------------------------------------
// Error_p of Section 4.1, unweighted block: ||X2_p - X2_{p-1}||_F^2 summed
// row by row in double, with x2_i = a2_i V V^T + x1_i Z^T for both sweeps.
// Each row difference is formed directly, so no large Gram terms cancel and
// changes far below sqrt(eps) ||X|| stay resolved.  One partial per
// workgroup.  Zp/Zq: n2 x k, Vp/Vq: n2 x l, all row-major double.
template <typename T, int KMAX, int LMAX>
__global__ __launch_bounds__(64) void k_change(int64_t m, int k, int n2, int l,
                                               const T *__restrict__ A, int64_t lda,
                                               const T *__restrict__ X1p, const T *__restrict__ X1q,
                                               const double *__restrict__ Zp,
                                               const double *__restrict__ Zq,
                                               const double *__restrict__ Vp,
                                               const double *__restrict__ Vq,
                                               double *__restrict__ part,
                                               const SmallState *__restrict__ st) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  const T *A2 = A + (int64_t)k * lda;
  double up[LMAX], uq[LMAX], xp[KMAX], xq[KMAX];
#pragma unroll
  for (int q = 0; q < LMAX; ++q) up[q] = uq[q] = 0.0;
  for (int j = 0; j < n2; ++j) {
    const double v = (double)A2[ir + (int64_t)j * lda];
    const double *vp = Vp + (int64_t)j * l, *vq = Vq + (int64_t)j * l;
#pragma unroll
    for (int q = 0; q < LMAX; ++q)
      if (q < l) {
        up[q] = fma(v, vp[q], up[q]);
        uq[q] = fma(v, vq[q], uq[q]);
      }
  }
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    xp[c] = (c < k) ? (double)X1p[ir + (int64_t)c * m] : 0.0;
    xq[c] = (c < k) ? (double)X1q[ir + (int64_t)c * m] : 0.0;
  }
  double acc = 0.0;
  for (int j = 0; j < n2; ++j) {
    const double *vp = Vp + (int64_t)j * l, *vq = Vq + (int64_t)j * l;
    const double *zp = Zp + (int64_t)j * k, *zq = Zq + (int64_t)j * k;
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < LMAX; ++q)
      if (q < l) d = fma(up[q], vp[q], fma(-uq[q], vq[q], d));
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) d = fma(xp[c], zp[c], fma(-xq[c], zq[c], d));
    acc = fma(d, d, acc);
  }
  acc = wave_sum(act ? acc : 0.0);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Copy an m x k matrix (ld m) into a caller buffer with leading dimension ld.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_out(int64_t m, int64_t k, const T *__restrict__ src,
                                                  T *__restrict__ dst, int64_t ld) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / m, i = e - c * m;
    dst[i + c * ld] = src[e];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by wlra_api.hip).
#include "launch.h"

template <typename T>
void launch_validate(hipStream_t s, int64_t m, int64_t n, const T *A, int64_t lda, int64_t k,
                     const T *W1, int64_t ldw, int *flags) {
  dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)std::min<int64_t>(n, 1024));
  hipLaunchKernelGGL(k_validate<T>, grid, dim3(256), 0, s, m, n, A, lda, k, W1, ldw, flags);
}

template <typename T>
void launch_init_x1(hipStream_t s, int64_t m, int64_t k, int mode, uint64_t seed, const T *src,
                    int64_t lds, T *X1, int *flags) {
  const int64_t total = m * k;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
  hipLaunchKernelGGL(k_init_x1<T>, dim3(g), dim3(256), 0, s, m, k, mode, seed, src, lds, X1, flags);
}

template <typename TX, typename TY>
void launch_tsgemm(hipStream_t s, int64_t m, const TX *X, int64_t ldx, int k1, const TY *Y,
                   int64_t ldy, int k2, int sym, int splits, int64_t rows_per_split, double *part,
                   double *out, const int *skip) {
  const int ti = (k1 + 31) / 32, tj = (k2 + 31) / 32;
  hipLaunchKernelGGL((k_tsgemm<TX, TY>), dim3(ti, tj, splits), dim3(256), 0, s, m, X, ldx, k1, Y,
                     ldy, k2, sym, rows_per_split, part, skip);
  const int64_t total = (int64_t)k1 * k2;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1024));
  hipLaunchKernelGGL(k_reduce_parts, dim3(g), dim3(256), 0, s, k1, k2, splits, sym, part, out, skip);
}

template <typename T>
void launch_f1(hipStream_t s, int64_t m, int k, const T *A, int64_t lda, const T *W1, int64_t ldw,
               double wc, const T *X1, double *part, int nwg) {
  hipLaunchKernelGGL(k_f1<T>, dim3(nwg), dim3(256), 0, s, m, k, A, lda, W1, ldw, wc, X1, part);
}

template <typename T, int KMAX>
static void launch_update_k(hipStream_t s, const UpdateArgs<T> &a) {
  const unsigned grid = (unsigned)((a.m + 63) / 64);
  if (a.constw) {
    hipLaunchKernelGGL((k_update<T, KMAX, true>), dim3(grid), dim3(64), 0, s, a.m, a.k, a.n2, a.A,
                       a.lda, a.W1, a.ldw, a.wc, a.X1o, a.X1n, a.Zt, a.Tt, a.St, a.part, 64, a.st,
                       a.flags);
  } else {
    const size_t shm = (size_t)(a.k * (a.k + 1) / 2 + a.k) * a.nl * sizeof(T);
    hipLaunchKernelGGL((k_update<T, KMAX, false>), dim3(grid), dim3(64), shm, s, a.m, a.k, a.n2,
                       a.A, a.lda, a.W1, a.ldw, a.wc, a.X1o, a.X1n, a.Zt, a.Tt, a.St, a.part, a.nl,
                       a.st, a.flags);
  }
}

template <typename T>
void launch_update(hipStream_t s, const UpdateArgs<T> &a) {
  if (a.k <= 8) launch_update_k<T, 8>(s, a);
  else if (a.k <= 16) launch_update_k<T, 16>(s, a);
  else if (a.k <= 32) launch_update_k<T, 32>(s, a);
  else launch_update_k<T, 64>(s, a);
}

template <typename T, int KMAX>
static void launch_x2_k(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
                        const T *X1, const T *Zt, const T *Vr, T *X2, int64_t ldx2) {
  const unsigned grid = (unsigned)((m + 63) / 64);
  if (l <= 8)
    hipLaunchKernelGGL((k_x2<T, KMAX, 8>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A, lda, X1, Zt,
                       Vr, X2, ldx2);
  else
    hipLaunchKernelGGL((k_x2<T, KMAX, WLRA_BMAX>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A, lda,
                       X1, Zt, Vr, X2, ldx2);
}

template <typename T>
void launch_x2(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
               const T *X1, const T *Zt, const T *Vr, T *X2, int64_t ldx2) {
  if (k <= 8) launch_x2_k<T, 8>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2);
  else if (k <= 16) launch_x2_k<T, 16>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2);
  else if (k <= 32) launch_x2_k<T, 32>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2);
  else launch_x2_k<T, 64>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2);
}

template <typename T, int KMAX>
static void launch_change_k(hipStream_t s, int64_t m, int k, int n2, int l, const T *A,
                            int64_t lda, const T *X1p, const T *X1q, const double *Zp,
                            const double *Zq, const double *Vp, const double *Vq, double *part,
                            const SmallState *st) {
  const unsigned grid = (unsigned)((m + 63) / 64);
  if (l <= 8)
    hipLaunchKernelGGL((k_change<T, KMAX, 8>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A, lda,
                       X1p, X1q, Zp, Zq, Vp, Vq, part, st);
  else
    hipLaunchKernelGGL((k_change<T, KMAX, WLRA_BMAX>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A,
                       lda, X1p, X1q, Zp, Zq, Vp, Vq, part, st);
}

template <typename T>
void launch_change(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
                   const T *X1p, const T *X1q, const double *Zp, const double *Zq,
                   const double *Vp, const double *Vq, double *part, const SmallState *st) {
  if (k <= 8) launch_change_k<T, 8>(s, m, k, n2, l, A, lda, X1p, X1q, Zp, Zq, Vp, Vq, part, st);
  else if (k <= 16) launch_change_k<T, 16>(s, m, k, n2, l, A, lda, X1p, X1q, Zp, Zq, Vp, Vq, part, st);
  else if (k <= 32) launch_change_k<T, 32>(s, m, k, n2, l, A, lda, X1p, X1q, Zp, Zq, Vp, Vq, part, st);
  else launch_change_k<T, 64>(s, m, k, n2, l, A, lda, X1p, X1q, Zp, Zq, Vp, Vq, part, st);
}

template <typename T>
void launch_copy_out(hipStream_t s, int64_t m, int64_t k, const T *src, T *dst, int64_t ld) {
  const int64_t total = m * k;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
  hipLaunchKernelGGL(k_copy_out<T>, dim3(g), dim3(256), 0, s, m, k, src, dst, ld);
}

#define INST(T)                                                                                   \
  template void launch_validate<T>(hipStream_t, int64_t, int64_t, const T *, int64_t, int64_t,    \
                                   const T *, int64_t, int *);                                    \
  template void launch_init_x1<T>(hipStream_t, int64_t, int64_t, int, uint64_t, const T *,        \
                                  int64_t, T *, int *);                                           \
  template void launch_tsgemm<T, T>(hipStream_t, int64_t, const T *, int64_t, int, const T *,     \
                                    int64_t, int, int, int, int64_t, double *, double *,          \
                                    const int *);                                                 \
  template void launch_f1<T>(hipStream_t, int64_t, int, const T *, int64_t, const T *, int64_t,   \
                             double, const T *, double *, int);                                   \
  template void launch_update<T>(hipStream_t, const UpdateArgs<T> &);                             \
  template void launch_x2<T>(hipStream_t, int64_t, int, int, int, const T *, int64_t, const T *,  \
                             const T *, const T *, T *, int64_t);                                 \
  template void launch_copy_out<T>(hipStream_t, int64_t, int64_t, const T *, T *, int64_t);     \
  template void launch_change<T>(hipStream_t, int64_t, int, int, int, const T *, int64_t,         \
                                 const T *, const T *, const double *, const double *,            \
                                 const double *, const double *, double *, const SmallState *);
INST(float)
INST(double)
