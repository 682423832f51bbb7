// Streaming kernels of the sWLR sweep: passes over the m rows of A.
//
// All matrices are column-major.  Row i of a matrix is strided by its leading
// dimension, so a wavefront whose 64 lanes take 64 consecutive rows reads
// 64 consecutive elements of each column: every global load below is
// coalesced.  Sums over rows accumulate in double in every precision.
#include <type_traits>

#include "common.h"
#include "launch.h"

// Element (i, j) of [A1 A2] as T.  A2 is either part of A (A + k lda, same
// type) or a separate copy in BF16 (mixed precision).
template <typename T, typename TA2>
__device__ __forceinline__ T a_elem(const T *__restrict__ A, int64_t lda,
                                    const TA2 *__restrict__ A2, int64_t lda2, int k, int64_t i,
                                    int j) {
  if constexpr (std::is_same<T, TA2>::value) {
    return A[i + (int64_t)j * lda];
  } else {
    return j < k ? A[i + (int64_t)j * lda] : (T)to_f(A2[i + (int64_t)(j - k) * lda2]);
  }
}

// ---------------------------------------------------------------------------
// Input checks (problem (5) needs finite A and W1 > 0; Theorem 2 assumes
// (W1)_ij > 0).  flags |= DEV_BAD_A / DEV_BAD_W.  When A2b is given, the
// same read also stages A2 in BF16 (m x (n - k), leading dimension m) for the
// mixed-precision sweeps.
// Column weights of the unweighted block (eq. (6) with W2(i, j) = w2_j): the
// same read writes As = [A1, A2 diag(w2)] (m x n, leading dimension m), the
// matrix of the equivalent problem (5) that the sweeps then run on, and the
// BF16 copy is taken of the scaled columns; a w2_j that is not > 0 and
// finite sets DEV_BAD_W.
template <typename T>
__global__ __launch_bounds__(256) void k_validate(int64_t m, int64_t n, const T *__restrict__ A,
                                                  int64_t lda, int64_t k, const T *__restrict__ W1,
                                                  int64_t ldw, int *flags, bf16s *__restrict__ A2b,
                                                  const T *__restrict__ W2, T *__restrict__ As) {
  int bad_a = 0, bad_w = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    const T sc = (W2 != nullptr && j >= k) ? W2[j - k] : T(1);
    if (W2 != nullptr && j >= k && !(sc > T(0) && isfinite(sc))) bad_w = 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
      T v = A[i + j * lda];
      if (!isfinite(v)) bad_a = 1;
      if (W2 != nullptr) {
        v *= sc;
        As[i + j * m] = v;
      }
      if (A2b != nullptr && j >= k) A2b[i + (j - k) * m] = bf16_rne((float)v);
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

// The same checks (and BF16 staging) for float storage without column weights
// when rows come in aligned groups of four (m, lda, ldw multiples of 4,
// 16-byte aligned A and W1): 16-byte reads of A and W1, 8-byte writes of the
// BF16 copy, four rows per thread and a column per grid row.
__global__ __launch_bounds__(256) void k_validate4(int64_t m, int64_t n, const float *__restrict__ A,
                                                   int64_t lda, int64_t k,
                                                   const float *__restrict__ W1, int64_t ldw,
                                                   int *flags, bf16s *__restrict__ A2b) {
  int bad_a = 0, bad_w = 0;
  const int64_t m4 = m / 4, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m4; g += stride) {
      const float4 v = *reinterpret_cast<const float4 *>(A + 4 * g + j * lda);
      if (!isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w)) bad_a = 1;
      if (A2b != nullptr && j >= k) {
        const uint32_t lo = (uint32_t)bf16_rne(v.x).u | ((uint32_t)bf16_rne(v.y).u << 16);
        const uint32_t hi = (uint32_t)bf16_rne(v.z).u | ((uint32_t)bf16_rne(v.w).u << 16);
        *reinterpret_cast<uint2 *>(A2b + 4 * g + (j - k) * m) = make_uint2(lo, hi);
      }
      if (W1 != nullptr && j < k) {
        const float4 w = *reinterpret_cast<const float4 *>(W1 + 4 * g + j * ldw);
        if (!(w.x > 0.f) || !isfinite(w.x) || !(w.y > 0.f) || !isfinite(w.y) ||
            !(w.z > 0.f) || !isfinite(w.z) || !(w.w > 0.f) || !isfinite(w.w))
          bad_w = 1;
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
// matrix, 2 = copy of A1.  Non-finite given entries set DEV_BAD_A.  With a
// gate, nothing is written unless *gate is nonzero.
template <typename T>
__global__ __launch_bounds__(256) void k_init_x1(int64_t m, int64_t k, int mode, uint64_t seed,
                                                 const T *__restrict__ src, int64_t lds,
                                                 T *__restrict__ X1, int *flags,
                                                 const int *__restrict__ gate) {
  // a start that replaces a learned one is written only if that one failed
  if (gate != nullptr && *gate == 0) return;
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
// (k1 x k2, double), on the FP64 matrix cores.  A workgroup owns a 32 x 32
// output tile; its four wavefronts own 16 x 16 quadrants and multiply with
// v_mfma_f64_16x16x4f64 (products of float inputs are exact in double, sums
// in double).  Row chunks of 32 are staged through LDS as double
// (column-major, padded), the next chunk being loaded into registers while
// the current one multiplies.  `sym` computes only the tiles on or above the
// diagonal (X == Y).  With Y2 given, Y's columns ky1 .. k2 - 1 are Y2's
// columns 0 .. k2 - ky1 - 1 (ld ldy2): one product X^T [Y Y2].  Fragment
// layouts (lane l): A[l % 16][l / 16], B[l / 16][l % 16], accumulator v
// holds D[l / 16 + 4 v][l % 16].
typedef double ts_d4 __attribute__((ext_vector_type(4)));
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_tsgemm(int64_t m, const TX *__restrict__ X, int64_t ldx,
                                                int k1, const TY *__restrict__ Y, int64_t ldy,
                                                int k2, int sym, int64_t rows_per_split,
                                                double *__restrict__ part, const int *skip,
                                                const TY *__restrict__ Y2, int64_t ldy2, int ky1) {
  if (skip != nullptr && *skip) return;
  const int ti = blockIdx.x, tj = blockIdx.y, s = blockIdx.z;
  if (sym && ti > tj) return;
  __shared__ double sX[32][33];  // [column of X][row in chunk]
  __shared__ double sY[32][33];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int qi = w & 1, qj = w >> 1;
  const int i0 = ti * 32, j0 = tj * 32;
  const int64_t r0 = (int64_t)s * rows_per_split;
  const int64_t r1 = min(m, r0 + rows_per_split);
  TX px[4];  // raw reads of the next chunk, converted when stored
  TY py[4];
  // reads clamped into the operands (never skipped: a skipped read would be
  // waited for on its own) and masked by multiplying with zero (finite)
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e & 31, cc = e >> 5;
      const int64_t rowc = min(rb + rr, r1 - 1);
      px[u] = X[rowc + (int64_t)min(i0 + cc, k1 - 1) * ldx];
      const int jc = min(j0 + cc, k2 - 1);
      const TY *yc = jc < ky1 ? Y + (int64_t)jc * ldy : Y2 + (int64_t)(jc - ky1) * ldy2;
      py[u] = yc[rowc];
    }
  };
  ts_d4 acc = {0.0, 0.0, 0.0, 0.0};
  if (r0 < r1) fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += 32) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e & 31, cc = e >> 5;
      const bool rin = rb + rr < r1;
      sX[cc][rr] = (double)to_f(px[u]) * ((rin && i0 + cc < k1) ? 1.0 : 0.0);
      sY[cc][rr] = (double)to_f(py[u]) * ((rin && j0 + cc < k2) ? 1.0 : 0.0);
    }
    __syncthreads();
    if (rb + 32 < r1) fetch(rb + 32);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = 4 * u + lk;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[16 * qi + li][kk], sY[16 * qj + li][kk], acc,
                                                 0, 0, 0);
    }
    __syncthreads();
  }
  double *out = part + (int64_t)s * k1 * k2;
  const int j = j0 + 16 * qj + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 16 * qi + lk + 4 * v;
    if (i < k1 && j < k2) out[i + (int64_t)j * k1] = acc[v];
  }
}

// Sum of the split partials in a fixed order (deterministic).  A workgroup
// takes 32 consecutive outputs; its RP_G thread groups each sum every RP_G-th
// split (loads coalesced over the 32 outputs, several in flight per thread),
// then the group sums are added in order.  For `sym` the lower tiles are
// mirrored from the upper ones.
#define RP_G 8
__global__ __launch_bounds__(256) void k_reduce_parts(int k1, int k2, int splits, int sym,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ out,
                                                      const int *skip) {
  if (skip != nullptr && *skip) return;
  __shared__ double sp[RP_G][32];
  const int64_t total = (int64_t)k1 * k2;
  const int o = threadIdx.x & 31, g = threadIdx.x >> 5;
  for (int64_t e0 = (int64_t)blockIdx.x * 32; e0 < total; e0 += (int64_t)gridDim.x * 32) {
    const int64_t e = e0 + o;
    double acc = 0.0;
    if (e < total) {
      const int i = (int)(e % k1), j = (int)(e / k1);
      int64_t src = e;
      if (sym && (i >> 5) > (j >> 5)) src = j + (int64_t)i * k1;
#pragma unroll 4
      for (int sp_ = g; sp_ < splits; sp_ += RP_G) acc += part[(int64_t)sp_ * total + src];
    }
    sp[g][o] = acc;
    __syncthreads();
    if (g == 0 && e < total) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < RP_G; ++q) t += sp[q][o];
      out[e] = t;
    }
    __syncthreads();
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
// The X1 update of Algorithm 1 (steps 7-9), one row per lane.  Row i of X1_{p+1} is E_p(i,:) K_i^-1 with
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
//
// Work split: a workgroup owns 64 rows; E (64 x k) = [A1 A2 X1] [-S; Z; T]
// is a product with inner dimension n + k, run on the matrix cores
// (v_mfma_f32_16x16x4f32 for float, v_mfma_f64_16x16x4f64 for double; BF16
// entries of A2 are widened exactly): wavefront w owns rows 16w..16w+15 and
// all 16-column tiles of E.  Rows of B = [-S; Z; T] (input index first) are
// staged through LDS in chunks, zero past k; each wavefront reads its A
// operand straight from global memory, UB k-steps of 4 at a time with all
// reads in flight (clamped, so never masked), and sums in a fixed order.
// E goes through LDS to wavefront 0, one row per lane, which finishes as
// before: with a constant weight it writes X1' = A1 + e directly; otherwise
// it stores the right-hand sides e for k_rowsolve.
// Partials per workgroup: (||(A1 - X1') o W1||^2, ||X1' - X1||^2).
// MFMA fragment layouts (lane l): A[l % 16][l / 16], B[l / 16][l % 16];
// accumulator v holds D[4 (l / 16) + v][l % 16] (float) or
// D[l / 16 + 4 v][l % 16] (double).
#define UPD_T 256
template <typename T>
struct UpdMma;
template <>
struct UpdMma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct UpdMma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <int KMAX>
constexpr int upd_kp() { return ((KMAX + 15) / 16) * 16; }
template <typename T, int KMAX, bool CONSTW, typename TA2>
__global__ __launch_bounds__(UPD_T) void k_update(
    int64_t m, int k, int n, const T *__restrict__ A, int64_t lda, const TA2 *__restrict__ A2,
    int64_t lda2, const T *__restrict__ W1,
    int64_t ldw, T wc, const T *__restrict__ X1o, T *__restrict__ X1n, const T *__restrict__ Gt,
    const T *__restrict__ Tt, const T *__restrict__ St, double *__restrict__ part,
    T *__restrict__ Eb, int grows, const SmallState *__restrict__ st) {
  if (st->done) return;
  constexpr int KP = upd_kp<KMAX>(), NT = KP / 16, UB = 32;
  typedef typename UpdMma<T>::acc_t acc_t;
  // LDS: [B chunk: grows x KP] [E: 64 x (KP + 1)]
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sB = reinterpret_cast<T *>(smem_raw);
  T *sE = sB + (size_t)grows * KP;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int ntot = n + k;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int64_t ra = min(r0 + 16 * w + li, m - 1);  // this lane's A-operand row (clamped)
  acc_t acc[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) acc[ct] = acc_t{0, 0, 0, 0};
  // the inner index in three segments of one source each (A1, A2, X1), so
  // that every read is a plain load (a choice between sources per element
  // would make the compiler wait for each read on its own); a segment's last
  // k-step is padded with zero rows of B and clamped reads
  // (brow: row ja of B = [-S; Z; T], k entries per row)
  auto segment = [&](const auto *src, int64_t ld, int ja, int jb, const T *brow0) {
    for (int j0 = ja; j0 < jb; j0 += grows) {
      const int jl = min(grows, jb - j0);
      const int nsteps = (jl + 3) / 4;
      __syncthreads();
      for (int e = t; e < 4 * nsteps * KP; e += UPD_T) {
        const int jr = e / KP, c = e - jr * KP;
        const T v = brow0[(int64_t)(j0 - ja + min(jr, jl - 1)) * k + min(c, k - 1)];
        sB[e] = v * ((jr < jl && c < k) ? T(1) : T(0));
      }
      __syncthreads();
      for (int s0 = 0; s0 < nsteps; s0 += UB) {
        T av[UB];
#pragma unroll
        for (int u0 = 0; u0 < UB; u0 += 8) {
          if (s0 + u0 < nsteps) {
#pragma unroll
            for (int u = u0; u < u0 + 8; ++u) {
              const int jc = min(j0 + 4 * (s0 + u) + lk, jb - 1);
              av[u] = (T)to_f(src[ra + (int64_t)(jc - ja) * ld]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          if (s0 + u < nsteps) {
            const T *brow = sB + (4 * (s0 + u) + lk) * KP + li;
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) acc[ct] = UpdMma<T>::mma(av[u], brow[16 * ct], acc[ct]);
          }
        }
      }
    }
  };
  segment(A, lda, 0, k, Gt);
  segment(A2, lda2, k, n, Gt + (int64_t)k * k);
  segment(X1o, m, n, ntot, Tt);
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      sE[(16 * w + UpdMma<T>::row(lk, v)) * (KP + 1) + 16 * ct + li] = acc[ct][v];
  __syncthreads();
  if (w > 0) return;
  const int64_t i = r0 + lane;
  const bool act = i < m;
  T e[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) e[c] = (c < k) ? sE[lane * (KP + 1) + c] : T(0);

  if (!CONSTW) {
    // right-hand sides for the per-row solve (k_rowsolve)
    if (act) {
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c < k) Eb[i + (int64_t)c * m] = e[c];
    }
    return;
  }
  double f1 = 0.0, dx = 0.0;
  // reads first, all in flight (row and column clamped), then the sums
  const int64_t ic = act ? i : (m - 1);
  T av[KMAX], xo[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    const int cc = min(c, k - 1);
    av[c] = A[ic + (int64_t)cc * lda];
    xo[c] = X1o[ic + (int64_t)cc * m];
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) {
        const T x = av[c] + e[c];
        X1n[i + (int64_t)c * m] = x;
        const double d = (double)av[c] - (double)x;
        f1 += d * d * (double)wc * (double)wc;
        const double dd = (double)x - (double)xo[c];
        dx += dd * dd;
      }
  }
  f1 = wave_sum(f1);
  dx = wave_sum(dx);
  if (lane == 0) {
    part[2 * blockIdx.x] = f1;
    part[2 * blockIdx.x + 1] = dx;
  }
}

// ---------------------------------------------------------------------------
// Row update for float storage, tiled: E = [A1 A2 X1] [-S; Z; T] for 128
// rows per workgroup (four wavefronts of 32 rows, each two 16-row MFMA tiles
// by KP output columns).  The inner index runs in chunks of 32 columns: the
// chunk of A (128 rows x 32 columns) is read with 16-byte loads (a column's
// 128 rows are 512 contiguous bytes, so every load of a wavefront covers two
// whole columns), staged in LDS, and the next chunk's loads are issued before
// the current chunk is multiplied.
//  * float segments (A1, A2 in float, X1): LDS [column][row], products on
//    v_mfma_f32_16x16x4f32, the 32 rows of B = [-S; Z; T] of the chunk in
//    LDS too;
//  * the BF16 copy of A2 (mixed precision): the chunk is transposed into LDS
//    [row][column] as it is stored, and multiplied on v_mfma_f32_16x16x32_bf16
//    against Z split into two BF16 terms, Z ~ Zh + Zl (|Z - Zh - Zl| <=
//    2^-17 |Z|), so the product of the BF16 data with Z loses no more than
//    the FP32 products do; Zh and Zl are stored [column][row] with rows
//    padded to n2p (a multiple of 32, zero rows and columns beyond).
// The epilogue is the one of k_update: for a constant W1 the panel already
// holds K^-1 and X1' = A1 + E is written with the objective and change
// partials (one pair per 64 rows); otherwise E goes to the per-row solve.
// Requires m % 8 == 0, lda % 4 == 0 and 16-byte aligned A, X1 (checked by the
// launcher).
#define UT_T 256
#define UT_R 128
#define UT_KC 32
#define UT_SLD (UT_R + 16)  // floats per staged column of A
#define UT_BKS 40           // bf16 per staged row of the BF16 chunk (32 + pad)
typedef __bf16 ut_bf8 __attribute__((ext_vector_type(8)));
typedef float ut_f4 __attribute__((ext_vector_type(4)));

template <int KMAX, bool CONSTW, bool A2BF>
__global__ __launch_bounds__(UT_T) void k_update_t(
    int64_t m, int k, int n, const float *__restrict__ A, int64_t lda,
    const bf16s *__restrict__ A2b, int64_t ldb, const float *__restrict__ W1, int64_t ldw,
    float wc, const float *__restrict__ X1o, float *__restrict__ X1n,
    const float *__restrict__ Gt, const float *__restrict__ Tt, const bf16s *__restrict__ Zh,
    const bf16s *__restrict__ Zl, int n2p, double *__restrict__ part, float *__restrict__ Eb,
    const SmallState *__restrict__ st) {
  if (st->done) return;
  constexpr int KP = upd_kp<KMAX>(), NT = KP / 16, KPL = KP + 16;
  constexpr int SM1 = UT_KC * UT_SLD + UT_KC * KPL, SM2 = UT_R * (KP + 1);
  __shared__ __align__(16) float smem[SM1 > SM2 ? SM1 : SM2];
  float *sA = smem;                       // [32][UT_SLD] float chunk
  float *sB = smem + UT_KC * UT_SLD;      // [32][KPL] rows of B
  bf16s *sAb = reinterpret_cast<bf16s *>(smem);  // [128][UT_BKS] BF16 chunk
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * UT_R;
  const int n2 = n - k;
  ut_f4 acc[2][NT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = ut_f4{0.f, 0.f, 0.f, 0.f};

  // float segment: nj columns of src (ld), rows of B from brow0 (k per row)
  auto fseg = [&](const float *src, int64_t ld, int nj, const float *brow0) {
    if (nj <= 0) return;
    // thread t stages rows 4 (t % 32) .. + 3 of columns t / 32 + 8 p
    const int q = t & 31, cq = t >> 5;
    const int64_t g = min(r0 / 4 + q, m / 4 - 1);  // clamped 4-row group
    float4 ra[4];
    float rb[UT_KC * KP / UT_T];
#define UT_FLOAD(J0)                                                                \
  do {                                                                              \
    _Pragma("unroll") for (int p = 0; p < 4; ++p) {                                 \
      const int jc = min((J0) + cq + 8 * p, nj - 1);                                \
      ra[p] = *reinterpret_cast<const float4 *>(src + 4 * g + (int64_t)jc * ld);    \
    }                                                                               \
    _Pragma("unroll") for (int u = 0; u < UT_KC * KP / UT_T; ++u) {                 \
      const int e = t + u * UT_T, jr = e / KP, c = e - jr * KP;                     \
      const int jj = min((J0) + jr, nj - 1);                                        \
      const float v = brow0[(int64_t)jj * k + min(c, k - 1)];                       \
      rb[u] = ((J0) + jr < nj && c < k) ? v : 0.f;                                  \
    }                                                                               \
  } while (0)
    UT_FLOAD(0);
    for (int j0 = 0; j0 < nj; j0 += UT_KC) {
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 4; ++p)
        *reinterpret_cast<float4 *>(sA + (cq + 8 * p) * UT_SLD + 4 * q) = ra[p];
#pragma unroll
      for (int u = 0; u < UT_KC * KP / UT_T; ++u) {
        const int e = t + u * UT_T, jr = e / KP, c = e - jr * KP;
        sB[jr * KPL + c] = rb[u];
      }
      __syncthreads();
      if (j0 + UT_KC < nj) UT_FLOAD(j0 + UT_KC);
      const int nk = min(UT_KC, nj - j0);
#pragma unroll
      for (int kk = 0; kk < UT_KC / 4; ++kk) {
        if (4 * kk < nk) {
          const float a0 = sA[(4 * kk + lg) * UT_SLD + 32 * w + li];
          const float a1 = sA[(4 * kk + lg) * UT_SLD + 32 * w + 16 + li];
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            const float b = sB[(4 * kk + lg) * KPL + 16 * ct + li];
            acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b, acc[0][ct], 0, 0, 0);
            acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b, acc[1][ct], 0, 0, 0);
          }
        }
      }
    }
  };
  // BF16 segment: the n2 columns of A2b against Zh + Zl
  auto bseg = [&]() {
    if (n2 <= 0) return;
    // thread t stages rows 8 (t % 16) .. + 7 of columns t / 16 + 16 p
    const int q = t & 15, cq = t >> 4;
    const int64_t g = min(r0 / 8 + q, m / 8 - 1);  // clamped 8-row group
    uint4 ra[2];
#define UT_BLOAD(J0)                                                                \
  do {                                                                              \
    _Pragma("unroll") for (int p = 0; p < 2; ++p) {                                 \
      const int jc = min((J0) + cq + 16 * p, n2 - 1);                               \
      ra[p] = *reinterpret_cast<const uint4 *>(A2b + 8 * g + (int64_t)jc * ldb);    \
    }                                                                               \
  } while (0)
    UT_BLOAD(0);
    for (int j0 = 0; j0 < n2; j0 += UT_KC) {
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int col = cq + 16 * p;
        const uint32_t w0 = ra[p].x, w1 = ra[p].y, w2 = ra[p].z, w3 = ra[p].w;
        bf16s *d = sAb + (8 * q) * UT_BKS + col;
        d[0 * UT_BKS] = bf16s{(uint16_t)(w0 & 0xffffu)};
        d[1 * UT_BKS] = bf16s{(uint16_t)(w0 >> 16)};
        d[2 * UT_BKS] = bf16s{(uint16_t)(w1 & 0xffffu)};
        d[3 * UT_BKS] = bf16s{(uint16_t)(w1 >> 16)};
        d[4 * UT_BKS] = bf16s{(uint16_t)(w2 & 0xffffu)};
        d[5 * UT_BKS] = bf16s{(uint16_t)(w2 >> 16)};
        d[6 * UT_BKS] = bf16s{(uint16_t)(w3 & 0xffffu)};
        d[7 * UT_BKS] = bf16s{(uint16_t)(w3 >> 16)};
      }
      __syncthreads();
      if (j0 + UT_KC < n2) UT_BLOAD(j0 + UT_KC);
      // columns j0 + 32 .. of the chunk past n2 meet zero rows of Zh, Zl
      const ut_bf8 a0 = *reinterpret_cast<const ut_bf8 *>(sAb + (32 * w + li) * UT_BKS + 8 * lg);
      const ut_bf8 a1 =
          *reinterpret_cast<const ut_bf8 *>(sAb + (32 * w + 16 + li) * UT_BKS + 8 * lg);
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        const int64_t zo = (int64_t)(16 * ct + li) * n2p + j0 + 8 * lg;
        const ut_bf8 bh = *reinterpret_cast<const ut_bf8 *>(Zh + zo);
        const ut_bf8 bl = *reinterpret_cast<const ut_bf8 *>(Zl + zo);
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bh, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bh, acc[1][ct], 0, 0, 0);
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bl, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bl, acc[1][ct], 0, 0, 0);
      }
    }
  };
  fseg(A, lda, k, Gt);
  if constexpr (A2BF)
    bseg();
  else
    fseg(A + (int64_t)k * lda, lda, n2, Gt + (int64_t)k * k);
  fseg(X1o, m, k, Tt);

  // E tile to LDS (rows of the workgroup x KP), then one row per thread
  __syncthreads();
  float *sE = smem;  // [128][KP + 1]
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sE[(32 * w + 16 * rt + 4 * lg + v) * (KP + 1) + 16 * ct + li] = acc[rt][ct][v];
  __syncthreads();
  if (t >= UT_R) return;
  const int64_t i = r0 + t;
  const bool act = i < m;
  const float *er = sE + t * (KP + 1);
  if (!CONSTW) {
    if (act)
      for (int c = 0; c < k; ++c) Eb[i + (int64_t)c * m] = er[c];
    return;
  }
  // eight columns at a time: their reads in flight together, few registers
  double f1 = 0.0, dx = 0.0;
  const int64_t ic = act ? i : (m - 1);
  for (int c0 = 0; c0 < k; c0 += 8) {
    float av[8], xo[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int cc = min(c0 + u, k - 1);
      av[u] = A[ic + (int64_t)cc * lda];
      xo[u] = X1o[ic + (int64_t)cc * m];
    }
    if (act) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < k) {
          const float x = av[u] + er[c0 + u];
          X1n[i + (int64_t)(c0 + u) * m] = x;
          const double d = (double)av[u] - (double)x;
          f1 += d * d * (double)wc * (double)wc;
          const double dd = (double)x - (double)xo[u];
          dx += dd * dd;
        }
    }
  }
  f1 = wave_sum(f1);
  dx = wave_sum(dx);
  // one (f1, dx) pair per 64 rows, as k_update writes them
  const int64_t pidx = 2 * (int64_t)blockIdx.x + (t >> 6);
  if (lane == 0 && pidx * 64 < m) {
    part[2 * pidx] = f1;
    part[2 * pidx + 1] = dx;
  }
}

#undef UT_FLOAD
#undef UT_BLOAD

// Zh + Zl ~ Z (rows k .. n - 1 of the panel Gt = [-S; Z], k per row) in BF16,
// stored [column c][row j] with rows padded to n2p and columns to kp (zeros).
__device__ __forceinline__ void panel_body(int n2, int k, int kp, int n2p,
                                           const float *__restrict__ Gt, bf16s *__restrict__ Zh,
                                           bf16s *__restrict__ Zl,
                                           const SmallState *__restrict__ st) {
  if (st->done) return;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < kp * n2p; e += gridDim.x * 256) {
    const int c = e / n2p, j = e - c * n2p;
    const float z = (c < k && j < n2) ? Gt[(int64_t)(k + j) * k + c] : 0.f;
    const bf16s h = bf16_rne(z);
    Zh[e] = h;
    Zl[e] = bf16_rne(z - to_f(h));
  }
}
__global__ __launch_bounds__(256) void k_panel_bf16(int n2, int k, int kp, int n2p,
                                                     const float *__restrict__ Gt,
                                                     bf16s *__restrict__ Zh,
                                                     bf16s *__restrict__ Zl,
                                                     const SmallState *__restrict__ st) {
  panel_body(n2, k, kp, n2p, Gt, Zh, Zl, st);
}
// batch: blockIdx.y = instance
__global__ __launch_bounds__(256) void k_panel_bf16_b(const PanelArgs *__restrict__ av) {
  const PanelArgs &a = av[blockIdx.y];
  panel_body(a.n2, a.k, a.kp, a.n2p, a.Gt, a.Zh, a.Zl, a.st);
}

// ---------------------------------------------------------------------------
// Per-row solve of the X1 update: x1_i' = a1_i + e_i (diag(w_i^2) + S)^-1,
// one row per lane.  Register version: the lower Cholesky factor of the
// row's k x k matrix lives in registers (all indices compile-time after
// unrolling; k <= KMAX), S is read through uniform (scalar) loads.
template <typename T, int KMAX>
__global__ __launch_bounds__(64) void k_rowsolve_reg(
    int64_t m, int k, const T *__restrict__ A, int64_t lda, const T *__restrict__ W1, int64_t ldw,
    const T *__restrict__ X1o, T *__restrict__ X1n, const T *__restrict__ Eb,
    const T *__restrict__ St, double *__restrict__ part, const SmallState *__restrict__ st,
    int *flags, const int *__restrict__ cgflag) {
  if (st->done) return;
  // after the CG solve, only when it left rows unsolved in this sweep
  if (cgflag != nullptr && *cgflag != st->sweep + 1) return;
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  T e[KMAX], q[KMAX], L[KMAX * (KMAX + 1) / 2];
  // clamped reads, all in flight; past k: e = 0 and q = 1 by arithmetic
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    const int cc = min(c, k - 1);
    const T mf = (c < k) ? T(1) : T(0);
    e[c] = Eb[ir + (int64_t)cc * m] * mf;
    const T wv = W1[ir + (int64_t)cc * ldw];
    q[c] = wv * wv * mf + (T(1) - mf);
  }
  int bad = 0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k) {
      T sv = q[j] + St[j * k + j];
#pragma unroll
      for (int p = 0; p < j; ++p) sv -= L[j * (j + 1) / 2 + p] * L[j * (j + 1) / 2 + p];
      if (!(sv > T(0))) {
        bad = 1;
        sv = T(1);
      }
      const T ljj = sqrt(sv);
      L[j * (j + 1) / 2 + j] = ljj;
      const T inv = T(1) / ljj;
#pragma unroll
      for (int r = j + 1; r < KMAX; ++r) {
        if (r < k) {
          T t = St[r * k + j];
#pragma unroll
          for (int p = 0; p < j; ++p) t -= L[r * (r + 1) / 2 + p] * L[j * (j + 1) / 2 + p];
          L[r * (r + 1) / 2 + j] = t * inv;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < KMAX; ++r)
    if (r < k) {
      T t = e[r];
#pragma unroll
      for (int p = 0; p < r; ++p) t -= L[r * (r + 1) / 2 + p] * e[p];
      e[r] = t / L[r * (r + 1) / 2 + r];
    }
#pragma unroll
  for (int r = KMAX - 1; r >= 0; --r)
    if (r < k) {
      T t = e[r];
#pragma unroll
      for (int p = r + 1; p < KMAX; ++p)
        if (p < k) t -= L[p * (p + 1) / 2 + r] * e[p];
      e[r] = t / L[r * (r + 1) / 2 + r];
    }
  double f1 = 0.0, dx = 0.0;
  if (act) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) {
        const T a1 = A[i + (int64_t)c * lda];
        const T x = a1 + e[c];
        X1n[i + (int64_t)c * m] = x;
        const double d = (double)a1 - (double)x;
        f1 += d * d * (double)q[c];
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

// Per-row solves by preconditioned conjugate gradients (float storage): one
// row per thread, K_i = diag(w_i^2) + S with S = C C^T shared (in LDS,
// zero-padded to KP x KP, read by every lane at once), the Jacobi
// preconditioner diag(K_i).  With P_i = diag(K_i), P_i^-1/2 K_i P_i^-1/2 =
// I + E_i with ||E_i|| <= ||S|| / min w^2, so the iteration contracts fast
// when the weights dominate C C^T (on the 19200 x 200 workload ||S|| = 17
// against min w^2 = 100; rows where ||S||_F > min w^2 / 2 are not
// attempted).  A row stops when ||r|| <= 2^-21 ||e||; a row still
// above it after CG_MAXIT iterations marks the sweep in *cgflag (sweep + 1),
// and the direct per-row Cholesky kernel launched after this one then
// solves every row again.  Reads and epilogue as k_rowsolve_reg.
#define CG_MAXIT 40
template <int KP>
__global__ __launch_bounds__(256) void k_rowsolve_cg(
    int64_t m, int k, const float *__restrict__ A, int64_t lda, const float *__restrict__ W1,
    int64_t ldw, const float *__restrict__ X1o, float *__restrict__ X1n,
    const float *__restrict__ Eb, const float *__restrict__ St, double *__restrict__ part,
    const SmallState *__restrict__ st, int *cgflag) {
  if (st->done) return;
  __shared__ __align__(16) float sS[KP * KP];
  __shared__ double red[4];
  const int t = threadIdx.x, lane = t & 63;
  double s2 = 0.0;
  for (int e2 = t; e2 < KP * KP; e2 += 256) {
    const int r2 = e2 / KP, c2 = e2 - r2 * KP;
    const float v = (r2 < k && c2 < k) ? St[r2 * k + c2] : 0.f;
    sS[e2] = v;
    s2 += (double)v * v;
  }
  // ||S||_F (>= ||S||_2): a row is left to the direct solve unless
  // ||S||_F <= min w^2 / 2, which bounds the preconditioned matrix's
  // eigenvalues to [1/2, 3/2]
  const float snorm = (float)sqrt(block_sum(s2, red));
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  // x, r, p, q and w^2 per row in registers; the Jacobi preconditioner
  // diag(K) = w^2 + diag(S) is re-read from LDS where it is needed (1 in the
  // padding, where r stays 0)
  float x[KP], r[KP], p[KP], q[KP], wq[KP];
  auto dinv = [&](int c) { return 1.f / (wq[c] + sS[c * KP + c] + (c < k ? 0.f : 1.f)); };
  float ee = 0.f;
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const int cc = min(c, k - 1);
    const float mf = (c < k) ? 1.f : 0.f;
    r[c] = Eb[ir + (int64_t)cc * m] * mf;  // r = e - K x with x = 0
    const float wv = W1[ir + (int64_t)cc * ldw];
    wq[c] = wv * wv * mf;
    x[c] = 0.f;
    ee = fmaf(r[c], r[c], ee);
  }
  const float stop = ee * (1.f / 4398046511104.f);  // (2^-21)^2 ||e||^2
  float rz = 0.f;
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    p[c] = r[c] * dinv(c);
    rz = fmaf(r[c], p[c], rz);
  }
  float wmin = wq[0];
#pragma unroll
  for (int c = 1; c < KP; ++c)
    if (c < k) wmin = fminf(wmin, wq[c]);
  const bool handled = snorm <= 0.5f * wmin;
  bool done_row = !(ee > 0.f) || !handled;
  for (int it = 0; it < CG_MAXIT; ++it) {
    if (__all(done_row)) break;
    // q = K p = w^2 o p + S p; S row by row from LDS (a compiler barrier per
    // row keeps its KP entries from being hoisted out of the iteration)
    float pq = 0.f;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      __asm__ volatile("" ::: "memory");
      float acc = wq[c] * p[c];
#pragma unroll
      for (int j4 = 0; j4 < KP; j4 += 4) {
        const float4 sv = *reinterpret_cast<const float4 *>(sS + c * KP + j4);
        acc = fmaf(sv.x, p[j4], acc);
        acc = fmaf(sv.y, p[j4 + 1], acc);
        acc = fmaf(sv.z, p[j4 + 2], acc);
        acc = fmaf(sv.w, p[j4 + 3], acc);
      }
      q[c] = acc;
      pq = fmaf(p[c], acc, pq);
    }
    const float alpha = (pq > 0.f && !done_row) ? rz / pq : 0.f;
    float rr = 0.f, rzn = 0.f;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      x[c] = fmaf(alpha, p[c], x[c]);
      r[c] = fmaf(-alpha, q[c], r[c]);
      rr = fmaf(r[c], r[c], rr);
      q[c] = r[c] * dinv(c);  // z = P^-1 r, in q's registers
      rzn = fmaf(r[c], q[c], rzn);
    }
    if (!done_row && rr <= stop) done_row = true;
    const float beta = (rz > 0.f && !done_row) ? rzn / rz : 0.f;
#pragma unroll
    for (int c = 0; c < KP; ++c) p[c] = fmaf(beta, p[c], q[c]);
    rz = rzn;
  }
  if (act && (!done_row || !handled)) atomicMax(cgflag, st->sweep + 1);
  double f1 = 0.0, dx = 0.0;
  if (act) {
#pragma unroll
    for (int c = 0; c < KP; ++c)
      if (c < k) {
        const float a1 = A[i + (int64_t)c * lda];
        const float xn = a1 + x[c];
        X1n[i + (int64_t)c * m] = xn;
        const double d = (double)a1 - (double)xn;
        f1 += d * d * (double)wq[c];
        const double dd = (double)xn - (double)X1o[i + (int64_t)c * m];
        dx += dd * dd;
      }
  }
  f1 = wave_sum(f1);
  dx = wave_sum(dx);
  // one (f1, dx) pair per 64 rows, as k_update writes them
  const int64_t pidx = 4 * (int64_t)blockIdx.x + (t >> 6);
  if (lane == 0 && pidx * 64 < m) {
    part[2 * pidx] = f1;
    part[2 * pidx + 1] = dx;
  }
}

// LDS version for any k <= WLRA_KMAX: the factor of each lane's matrix is
// lane-interleaved in LDS (element e of lane l at [e*nl + l]), `nl` lanes at
// a time.
template <typename T, int KMAX>
__global__ __launch_bounds__(64) void k_rowsolve_lds(
    int64_t m, int k, const T *__restrict__ A, int64_t lda, const T *__restrict__ W1, int64_t ldw,
    const T *__restrict__ X1o, T *__restrict__ X1n, const T *__restrict__ Eb,
    const T *__restrict__ St, double *__restrict__ part, int nl,
    const SmallState *__restrict__ st, int *flags, const int *__restrict__ cgflag) {
  if (st->done) return;
  if (cgflag != nullptr && *cgflag != st->sweep + 1) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sS = reinterpret_cast<T *>(smem_raw);  // k x k
  T *sm = sS + k * k;
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  for (int e2 = lane; e2 < k * k; e2 += 64) sS[e2] = St[e2];
  // all reads in flight first (clamped columns; entries past k are never used)
  T e[KMAX], wq[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    const int cc = min(c, k - 1);
    e[c] = Eb[ir + (int64_t)cc * m];
    const T wv = W1[ir + (int64_t)cc * ldw];
    wq[c] = wv * wv;
  }
  __syncthreads();
  int bad = 0;
  {
    const int tri = k * (k + 1) / 2;
    for (int round = 0; round < 64; round += nl) {
      const int sl = lane - round;
      if (sl >= 0 && sl < nl) {
        T *L = sm + sl;
        T *E = sm + (int64_t)tri * nl + sl;
        T *Q = E + (int64_t)k * nl;  // w^2 of this row
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
          if (c < k) {
            E[c * nl] = e[c];
            Q[c * nl] = wq[c];
          }
        for (int jj = 0; jj < k; ++jj) {
          const int bj = jj * (jj + 1) / 2;
          T sv = Q[jj * nl] + sS[jj * k + jj];
          {
            T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
            int p = 0;
            for (; p + 4 <= jj; p += 4) {
              const T l0 = L[(bj + p) * nl], l1 = L[(bj + p + 1) * nl];
              const T l2 = L[(bj + p + 2) * nl], l3 = L[(bj + p + 3) * nl];
              a0 = fma(l0, l0, a0); a1 = fma(l1, l1, a1);
              a2 = fma(l2, l2, a2); a3 = fma(l3, l3, a3);
            }
            for (; p < jj; ++p) { const T l0 = L[(bj + p) * nl]; a0 = fma(l0, l0, a0); }
            sv -= (a0 + a1) + (a2 + a3);
          }
          if (!(sv > T(0))) {
            bad = 1;
            sv = T(1);
          }
          const T ljj = sqrt(sv);
          L[(bj + jj) * nl] = ljj;
          const T inv = T(1) / ljj;
          for (int ii = jj + 1; ii < k; ++ii) {
            const int bi = ii * (ii + 1) / 2;
            T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
            int p = 0;
            for (; p + 4 <= jj; p += 4) {
              a0 = fma(L[(bi + p) * nl], L[(bj + p) * nl], a0);
              a1 = fma(L[(bi + p + 1) * nl], L[(bj + p + 1) * nl], a1);
              a2 = fma(L[(bi + p + 2) * nl], L[(bj + p + 2) * nl], a2);
              a3 = fma(L[(bi + p + 3) * nl], L[(bj + p + 3) * nl], a3);
            }
            for (; p < jj; ++p) a0 = fma(L[(bi + p) * nl], L[(bj + p) * nl], a0);
            L[(bi + jj) * nl] = (sS[ii * k + jj] - ((a0 + a1) + (a2 + a3))) * inv;
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
        const T a1 = A[i + (int64_t)c * lda];
        const T x = a1 + e[c];
        X1n[i + (int64_t)c * m] = x;
        const double wd = (double)W1[i + (int64_t)c * ldw];
        const double d = (double)a1 - (double)x;
        f1 += d * d * wd * wd;
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
// Output pass over the rows of the returned X_p.  Dense X2 = X1 C + D =
// a2 V V^T + x1 Z^T row by row (one row per lane): u = a2_i V, then
// x2_ij = u . V(j,:) + x1_i . Z(j,:).  Vr is n2 x l row-major, Zt n2 x k
// row-major (same as k_update).  X2 is written when given.
// Column weights (w2 given): the rows are those of the scaled problem, so
// x2_ij is divided by w2_j on the way out, and the residual of entry (i, j)
// is |a2s_ij - x2s_ij| / w2_j.
// Foreground mask (mask given): byte (i, j) is 1 where |A(i, j) - X(i, j)| >
// tau, else 0, for all n columns (A1 - X1 included), decided in T.
template <typename T, int KMAX, int LMAX>
__global__ __launch_bounds__(64) void k_x2(int64_t m, int k, int n2, int l,
                                           const T *__restrict__ A, int64_t lda,
                                           const T *__restrict__ X1, const T *__restrict__ Zt,
                                           const T *__restrict__ Vr, T *__restrict__ X2,
                                           int64_t ldx2, const T *__restrict__ w2,
                                           uint8_t *__restrict__ mask, int64_t ldm, T tau) {
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
  if (mask != nullptr && act) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) mask[i + (int64_t)c * ldm] = fabs(A[i + (int64_t)c * lda] - x[c]) > tau ? 1 : 0;
  }
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
    const T sc = w2 != nullptr ? w2[j] : T(1);
    if (act && X2 != nullptr) X2[i + (int64_t)j * ldx2] = w2 != nullptr ? acc / sc : acc;
    if (act && mask != nullptr) {
      const T res = fabs(A2[i + (int64_t)j * lda] - acc);
      mask[i + (int64_t)(k + j) * ldm] = (w2 != nullptr ? res / sc : res) > tau ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Error_p through a Gram of aligned differences.  Row i of X2_p - X2_{p-1} is
//     d_i = a2_i (V_p V_p^T - V_q V_q^T) + x1p_i Z_p^T - x1q_i Z_q^T.
// V_q is first rotated onto V_p: V_q' = V_q O with O the orthogonal polar
// factor of V_q^T V_p (this leaves V_q V_q^T, hence X2_{p-1}, unchanged and
// undoes sign flips, swaps and rotations of near-equal eigenvectors).  With
// dV = V_q' - V_p and dZ = Z_q - Z_p,
//     d_i = g_i H^T,  H = [V_p, dV, Z_p, dZ],
//     g_i = [-a2_i dV, -a2_i V_q', x1p_i - x1q_i, -x1q_i],
// and every product g_ia H_ja is of the size of d_i itself (one factor of
// each pair is a difference), so ||d_i||^2 = g_i (H^T H) g_i^T loses only a
// few ulps of ||d_i||^2 -- unlike a Gram of the undifferenced basis, whose
// terms are ||x2_i||^2 in size.
//
// k_chgprep (one workgroup): O by Newton-Schulz iteration from V_q^T V_p,
// made exactly orthogonal by two-pass Gram-Schmidt (a column that vanishes
// is replaced by the unit vector farthest from the span of the others), the
// columns [V_p dV] of H column-major into Hb (n2 x 2l, what the row pass
// reads) and Kg = H^T H (K x K, K = 2l + 2k, symmetric).  Rows of V_p, V_q,
// Z_p and Z_q are read in chunks, contiguously, into LDS; both V_q^T V_p and
// H^T H are summed over the chunks on v_mfma_f64_16x16x4f64 (16 x 16 output
// tiles; for H^T H the tiles on or above the diagonal, a fixed set per
// wavefront, mirrored when written).
#define QR_T 512
#define CHG_NW 8    // wavefronts per workgroup of the change row pass
#define CHG_GLD 65  // leading dimension of g in LDS (padded against bank conflicts)
#define CHP_LDS 16384  // doubles of LDS for the staged rows
#define CHP_MAXT 10    // H^T H tiles per wavefront (78 tiles at K = 192)
typedef double chp_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void chgprep_body(int n2, int k, int l,
                                             const double *__restrict__ Vp,
                                             const double *__restrict__ Vq,
                                             const double *__restrict__ Zp,
                                             const double *__restrict__ Zq,
                                             double *__restrict__ Hb, double *__restrict__ Kg,
                                             const SmallState *__restrict__ st) {
  if (st->done || !st->have_prev) return;
  __shared__ double X[WLRA_BMAX * WLRA_BMAX];
  __shared__ double E[WLRA_BMAX * WLRA_BMAX];
  __shared__ __align__(16) double sH[CHP_LDS];
  const int K = 2 * l + 2 * k, t = threadIdx.x;
  const int lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int B_ = WLRA_BMAX;
  if (l > 0) {
    // X = V_q^T V_p: chunks of rows of V_q and V_p side by side in LDS;
    // wavefront w multiplies every eighth k-step of 4 rows into its own
    // partial tiles, which are summed in wavefront order at the end
    const int TL = (l + 15) / 16;
    const int ra = max(4, min((n2 + 3) & ~3, (CHP_LDS / (2 * l)) & ~3));
    double *sQ = sH, *sP = sH + ra * l;
    chp_d4 xa[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) xa[u][v] = chp_d4{0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < n2; i0 += ra) {
      const int nr = min(ra, n2 - i0), ne = nr * l;
      __syncthreads();
      for (int e0 = t; e0 < ne; e0 += 4 * QR_T) {
        double q4[4], p4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * QR_T, ne - 1);
          q4[u] = Vq[(int64_t)i0 * l + e];
          p4[u] = Vp[(int64_t)i0 * l + e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (e0 + u * QR_T < ne) {
            sQ[e0 + u * QR_T] = q4[u];
            sP[e0 + u * QR_T] = p4[u];
          }
      }
      __syncthreads();
      for (int ks = w; 4 * ks < nr; ks += QR_T / 64) {
        const int i = 4 * ks + lk;
        const bool ri = i < nr;
        const int ic = ri ? i : nr - 1;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (u < TL) {
            const int aa = 16 * u + li;
            const double av = (ri && aa < l) ? sQ[ic * l + min(aa, l - 1)] : 0.0;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
              if (v < TL) {
                const int bb = 16 * v + li;
                const double bv = (ri && bb < l) ? sP[ic * l + min(bb, l - 1)] : 0.0;
                xa[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, xa[u][v], 0, 0, 0);
              }
            }
          }
        }
      }
    }
    __syncthreads();
    // partial tile (u, v) of wavefront w at sH + ((w * 2 + u) * 2 + v) * 256,
    // entry (row, column) at row * 16 + column
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        if (u < TL && v < TL)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            sH[((w * 2 + u) * 2 + v) * 256 + (lk + 4 * q) * 16 + li] = xa[u][v][q];
    __syncthreads();
    for (int e = t; e < l * l; e += QR_T) {
      const int aa = e % l, bb = e / l, u = aa >> 4, v = bb >> 4;
      double sacc = 0.0;
      for (int ww = 0; ww < QR_T / 64; ++ww)
        sacc += sH[((ww * 2 + u) * 2 + v) * 256 + (aa & 15) * 16 + (bb & 15)];
      X[aa + bb * B_] = sacc;
    }
    __syncthreads();
    // Newton-Schulz on wavefront 0: X <- X (3 I - X^T X) / 2 until X^T X = I
    // to rounding (up to 16 entries of X per lane, l <= 32)
    if (t < 64) {
      for (int it = 0; it < 60; ++it) {
        double dev = 0.0;
        for (int e = lane; e < l * l; e += 64) {
          const int aa = e % l, bb = e / l;
          double sacc = 0.0;
          for (int q = 0; q < l; ++q) sacc = fma(X[q + aa * B_], X[q + bb * B_], sacc);
          E[aa + bb * B_] = sacc;
          const double d = sacc - (aa == bb ? 1.0 : 0.0);
          dev = fma(d, d, dev);
        }
        dev = wave_sum(dev);
        if (!(dev > 1e-28)) break;
        wave_sync();
        double xn[WLRA_BMAX * WLRA_BMAX / 64];
#pragma unroll
        for (int u = 0; u < WLRA_BMAX * WLRA_BMAX / 64; ++u) {
          const int e = lane + 64 * u;
          xn[u] = 0.0;
          if (e < l * l) {
            const int aa = e % l, bb = e / l;
            double sacc = 0.0;
            for (int q = 0; q < l; ++q)
              sacc = fma(X[aa + q * B_], (q == bb ? 3.0 : 0.0) - E[q + bb * B_], sacc);
            xn[u] = 0.5 * sacc;
          }
        }
        wave_sync();
#pragma unroll
        for (int u = 0; u < WLRA_BMAX * WLRA_BMAX / 64; ++u) {
          const int e = lane + 64 * u;
          if (e < l * l) X[(e % l) + (e / l) * B_] = xn[u];
        }
        wave_sync();
      }
      // two-pass Gram-Schmidt on the columns of X
      for (int c = 0; c < l; ++c) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int q = 0; q < c; ++q) {
            double dq = (lane < l) ? X[lane + q * B_] * X[lane + c * B_] : 0.0;
            dq = wave_sum(dq);
            if (lane < l) X[lane + c * B_] -= dq * X[lane + q * B_];
            wave_sync();
          }
        }
        double nn = (lane < l) ? X[lane + c * B_] * X[lane + c * B_] : 0.0;
        nn = wave_sum(nn);
        if (!(nn > 1e-20)) {
          // replace by the unit vector with the largest residual
          int best = 0;
          double bres = -1.0;
          for (int u = 0; u < l; ++u) {
            double res = 1.0;
            for (int q = 0; q < c; ++q) res -= X[u + q * B_] * X[u + q * B_];
            if (res > bres) {
              bres = res;
              best = u;
            }
          }
          if (lane < l) X[lane + c * B_] = (lane == best) ? 1.0 : 0.0;
          wave_sync();
          for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < c; ++q) {
              double dq = (lane < l) ? X[lane + q * B_] * X[lane + c * B_] : 0.0;
              dq = wave_sum(dq);
              if (lane < l) X[lane + c * B_] -= dq * X[lane + q * B_];
              wave_sync();
            }
          nn = (lane < l) ? X[lane + c * B_] * X[lane + c * B_] : 0.0;
          nn = wave_sum(nn);
        }
        const double inv = 1.0 / sqrt(nn);
        if (lane < l) X[lane + c * B_] *= inv;
        wave_sync();
      }
    }
    __syncthreads();
  }
  // H = [V_p, V_q O - V_p, Z_p, Z_q - Z_p] by chunks of rows: row i of the
  // chunk at sH + i * hld (columns K .. K16 - 1 and rows past the chunk zero),
  // the chunk's V_q rows after it
  const int K16 = (K + 15) & ~15, T16 = K16 / 16, ntile = T16 * (T16 + 1) / 2;
  const int hld = K16 + 16;  // 4 consecutive rows fall in distinct bank halves
  const int rb = max(4, min((n2 + 3) & ~3, (CHP_LDS / (hld + l)) & ~3));
  double *sVq = sH + rb * hld;
  chp_d4 ka[CHP_MAXT];
  int tr_[CHP_MAXT], tc_[CHP_MAXT];
#pragma unroll
  for (int u = 0; u < CHP_MAXT; ++u) {
    ka[u] = chp_d4{0.0, 0.0, 0.0, 0.0};
    // upper tile w + 8 u in row order: (0,0) (0,1) .. (0,T16-1) (1,1) ..
    int tt = w + (QR_T / 64) * u, r = 0;
    while (r < T16 && tt >= T16 - r) {
      tt -= T16 - r;
      ++r;
    }
    tr_[u] = r;
    tc_[u] = r + tt;
  }
  for (int i0 = 0; i0 < n2; i0 += rb) {
    const int nr = min(rb, n2 - i0), nr4 = (nr + 3) & ~3;
    __syncthreads();
    {
      const int nv = nr * l, nz = nr * k;
      // V_p into columns 0 .. l-1, V_q to its own block
      for (int e0 = t; e0 < nv; e0 += 4 * QR_T) {
        double p4[4], q4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * QR_T, nv - 1);
          p4[u] = Vp[(int64_t)i0 * l + e];
          q4[u] = Vq[(int64_t)i0 * l + e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * QR_T;
          if (e < nv) {
            sH[(e / l) * hld + (e % l)] = p4[u];
            sVq[e] = q4[u];
          }
        }
      }
      // Z_p into columns 2l .. 2l+k-1, Z_q - Z_p into 2l+k .. K-1
      for (int e0 = t; e0 < nz; e0 += 4 * QR_T) {
        double p4[4], q4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * QR_T, nz - 1);
          p4[u] = Zp[(int64_t)i0 * k + e];
          q4[u] = Zq[(int64_t)i0 * k + e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * QR_T;
          if (e < nz) {
            const int i = e / k, c = e % k;
            sH[i * hld + 2 * l + c] = p4[u];
            sH[i * hld + 2 * l + k + c] = q4[u] - p4[u];
          }
        }
      }
      // zero padding: columns K .. K16-1 of the chunk's rows, rows nr .. nr4-1
      const int padc = K16 - K;
      for (int e = t; e < nr * padc; e += QR_T) sH[(e / padc) * hld + K + (e % padc)] = 0.0;
      for (int e = t; e < (nr4 - nr) * K16; e += QR_T) sH[(nr + e / K16) * hld + (e % K16)] = 0.0;
    }
    __syncthreads();
    // dV = V_q O - V_p into columns l .. 2l-1
    for (int e = t; e < nr * l; e += QR_T) {
      const int i = e / l, bb = e % l;
      double sacc = 0.0;
      for (int aa = 0; aa < l; ++aa) sacc = fma(sVq[i * l + aa], X[aa + bb * B_], sacc);
      sH[i * hld + l + bb] = sacc - sH[i * hld + bb];
    }
    __syncthreads();
    // columns [V_p dV] for the row pass
    for (int e = t; e < nr * 2 * l; e += QR_T) {
      const int c = e / nr, i = e - c * nr;
      Hb[(int64_t)(i0 + i) + (int64_t)c * n2] = sH[i * hld + c];
    }
    // H^T H, this wavefront's tiles
    for (int ks = 0; 4 * ks < nr4; ++ks) {
      const double *row = sH + (4 * ks + lk) * hld + li;
#pragma unroll
      for (int u = 0; u < CHP_MAXT; ++u)
        if (w + (QR_T / 64) * u < ntile)
          ka[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * tr_[u]], row[16 * tc_[u]], ka[u],
                                                      0, 0, 0);
    }
  }
  // Kg, both triangles from the tiles on or above the diagonal (entries
  // below the diagonal of a diagonal tile are taken from above it)
#pragma unroll
  for (int u = 0; u < CHP_MAXT; ++u) {
    if (w + (QR_T / 64) * u < ntile) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * tr_[u] + lk + 4 * q, c = 16 * tc_[u] + li;
        if (r < K && c < K && (tr_[u] < tc_[u] || r <= c)) {
          Kg[r + (int64_t)c * K] = ka[u][q];
          Kg[c + (int64_t)r * K] = ka[u][q];
        }
      }
    }
  }
}
__global__ __launch_bounds__(QR_T) void k_chgprep(int n2, int k, int l,
                                                  const double *__restrict__ Vp,
                                                  const double *__restrict__ Vq,
                                                  const double *__restrict__ Zp,
                                                  const double *__restrict__ Zq,
                                                  double *__restrict__ Hb, double *__restrict__ Kg,
                                                  const SmallState *__restrict__ st) {
  chgprep_body(n2, k, l, Vp, Vq, Zp, Zq, Hb, Kg, st);
}
// one workgroup per instance of a batch
__global__ __launch_bounds__(QR_T) void k_chgprep_b(const ChgArgs *__restrict__ av) {
  const ChgArgs &c = av[blockIdx.x];
  chgprep_body(c.n2, c.k, c.l, c.Vp, c.Vq, c.Zp, c.Zq, c.Hb, c.Kg, c.st);
}

// Row pass: u_p = a2 V_p and u_d = a2 dV (wavefronts split the n2 columns,
// rows of [V_p dV] staged through LDS from H, fixed-order sum); then g per
// lane in LDS (K x 64, ld CHG_GLD, rows past m and entries past K zero) and
// the workgroup's sum of g Kg g^T as <Kg, G^T G>: the Gram G^T G of its 64
// rows in 16 x 16 tiles on v_mfma_f64_16x16x4f64 (tiles on or above the
// diagonal, split between the wavefronts), each tile contracted with the
// matching block of Kg.  One partial per workgroup.
template <typename T, int LMAX>
__global__ __launch_bounds__(64 * CHG_NW) void k_change_q(
    int64_t m, int k, int n2, int l, const T *__restrict__ A2, int64_t lda,
    const T *__restrict__ X1p, const T *__restrict__ X1q, const double *__restrict__ Hb,
    const double *__restrict__ Kg, int stage_rows, double *__restrict__ part,
    const SmallState *__restrict__ st) {
  if (st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *sR = reinterpret_cast<double *>(smem_raw);   // staged [V_p dV] rows, later g
  double *su = sR + (size_t)max(stage_rows * 2 * l, ((2 * l + 2 * k + 15) / 16) * 16 * CHG_GLD);
  __shared__ double sacc[CHG_NW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  const int rw = 2 * l, K = 2 * l + 2 * k;
  double up[LMAX], ud[LMAX];
#pragma unroll
  for (int q = 0; q < LMAX; ++q) up[q] = ud[q] = 0.0;
  if (l > 0) {
    for (int c0 = 0; c0 < n2; c0 += stage_rows) {
      const int c1 = min(n2, c0 + stage_rows), len = c1 - c0;
      __syncthreads();
      // columns 0..2l-1 of H: [V_p dV]; eight clamped reads in flight
      for (int e0 = threadIdx.x; e0 < len * rw; e0 += 8 * 64 * CHG_NW) {
        double hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = min(e0 + u * 64 * CHG_NW, len * rw - 1), r = e / rw, q = e - r * rw;
          hv[u] = Hb[c0 + r + (int64_t)q * n2];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (e0 + u * 64 * CHG_NW < len * rw) sR[e0 + u * 64 * CHG_NW] = hv[u];
      }
      __syncthreads();
      const int j0 = c0 + w * len / CHG_NW, j1 = c0 + (w + 1) * len / CHG_NW;
      // sixteen clamped column reads in flight, widened at the use
      for (int j = j0; j < j1; j += 16) {
        T raw[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) raw[u] = A2[ir + (int64_t)min(j + u, j1 - 1) * lda];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          if (j + u < j1) {
            const double v = (double)raw[u];
            const double *rr = sR + (j + u - c0) * rw;
#pragma unroll
            for (int q = 0; q < LMAX; ++q)
              if (q < l) {
                up[q] = fma(v, rr[q], up[q]);
                ud[q] = fma(v, rr[l + q], ud[q]);
              }
          }
        }
      }
    }
    // fixed-order sum of the wavefront slices
    for (int ww = 0; ww < CHG_NW; ++ww) {
      __syncthreads();
      if (w == ww) {
#pragma unroll
        for (int q = 0; q < LMAX; ++q)
          if (q < l) {
            const double a0 = (ww == 0) ? 0.0 : su[q * 64 + lane];
            const double b0 = (ww == 0) ? 0.0 : su[(LMAX + q) * 64 + lane];
            su[q * 64 + lane] = a0 + up[q];
            su[(LMAX + q) * 64 + lane] = b0 + ud[q];
          }
      }
    }
  }
  __syncthreads();
  // g = [-u_d, -(u_p + u_d), x1p - x1q, -x1q] per lane, zero past row m
  const double am = act ? 1.0 : 0.0;
  if (w == 0) {
#pragma unroll
    for (int q = 0; q < LMAX; ++q)
      if (q < l) {
        const double pu = su[q * 64 + lane], du = su[(LMAX + q) * 64 + lane];
        sR[q * CHG_GLD + lane] = -du * am;
        sR[(l + q) * CHG_GLD + lane] = -(pu + du) * am;
      }
  }
  for (int c0 = w; c0 < k; c0 += 4 * CHG_NW) {
    T xp[4], xq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = min(c0 + u * CHG_NW, k - 1);
      xp[u] = X1p[ir + (int64_t)c * m];
      xq[u] = X1q[ir + (int64_t)c * m];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * CHG_NW;
      if (c < k) {
        sR[(2 * l + c) * CHG_GLD + lane] = ((double)xp[u] - (double)xq[u]) * am;
        sR[(2 * l + k + c) * CHG_GLD + lane] = -(double)xq[u] * am;
      }
    }
  }
  const int nt = (K + 15) / 16;
  for (int a = K + w; a < 16 * nt; a += CHG_NW) sR[a * CHG_GLD + lane] = 0.0;
  __syncthreads();
  // sum over the 64 rows of g Kg g^T = sum_{a,b} Kg_ab (G^T G)_ab
  double acc = 0.0;
  {
    const int li = lane & 15, lk = lane >> 4;
    int p = 0;
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = ti; tj < nt; ++tj, ++p) {
        if (p % CHG_NW != w) continue;
        const double *ga = sR + (16 * ti + li) * CHG_GLD + lk;
        const double *gb = sR + (16 * tj + li) * CHG_GLD + lk;
        ts_d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i0 = 0; i0 < 64; i0 += 4)
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[i0], gb[i0], d, 0, 0, 0);
        // lane holds (G^T G)[16 ti + lk + 4 v][16 tj + li]
        const int b = 16 * tj + li;
        double kv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * ti + lk + 4 * v;
          kv[v] = Kg[(int64_t)min(a, K - 1) * K + min(b, K - 1)];
        }
        const double wt = (ti == tj) ? 1.0 : 2.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * ti + lk + 4 * v;
          acc = fma(wt * ((a < K && b < K) ? 1.0 : 0.0) * kv[v], d[v], acc);
        }
      }
  }
  acc = wave_sum(acc);
  if (lane == 0) sacc[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int ww = 0; ww < CHG_NW; ++ww) t += sacc[ww];
    part[blockIdx.x] = fmax(t, 0.0);
  }
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
                     const T *W1, int64_t ldw, int *flags, bf16s *A2b, const T *W2, T *As) {
  if constexpr (std::is_same<T, float>::value) {
    auto al = [](const void *p) { return ((uintptr_t)p & 15u) == 0; };
    if (W2 == nullptr && m % 4 == 0 && lda % 4 == 0 && al(A) &&
        (W1 == nullptr || (ldw % 4 == 0 && al(W1)))) {
      dim3 g4((unsigned)std::max<int64_t>(1, std::min<int64_t>((m / 4 + 255) / 256, 64)),
              (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 1024)));
      hipLaunchKernelGGL(k_validate4, g4, dim3(256), 0, s, m, n, A, lda, k, W1, ldw, flags, A2b);
      return;
    }
  }
  dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 64), (unsigned)std::min<int64_t>(n, 1024));
  hipLaunchKernelGGL(k_validate<T>, grid, dim3(256), 0, s, m, n, A, lda, k, W1, ldw, flags, A2b,
                     W2, As);
}

template <typename T>
void launch_init_x1(hipStream_t s, int64_t m, int64_t k, int mode, uint64_t seed, const T *src,
                    int64_t lds, T *X1, int *flags, const int *gate) {
  const int64_t total = m * k;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
  hipLaunchKernelGGL(k_init_x1<T>, dim3(g), dim3(256), 0, s, m, k, mode, seed, src, lds, X1, flags,
                     gate);
}

template <typename TX, typename TY>
void launch_tsgemm(hipStream_t s, int64_t m, const TX *X, int64_t ldx, int k1, const TY *Y,
                   int64_t ldy, int k2, int sym, int splits, int64_t rows_per_split, double *part,
                   double *out, const int *skip, const TY *Y2, int64_t ldy2, int ky1) {
  const int ti = (k1 + 31) / 32, tj = (k2 + 31) / 32;
  if (Y2 == nullptr) ky1 = k2;
  hipLaunchKernelGGL((k_tsgemm<TX, TY>), dim3(ti, tj, splits), dim3(256), 0, s, m, X, ldx, k1, Y,
                     ldy, k2, sym, rows_per_split, part, skip, Y2, ldy2, ky1);
  const int64_t total = (int64_t)k1 * k2;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 31) / 32, 4096));
  hipLaunchKernelGGL(k_reduce_parts, dim3(g), dim3(256), 0, s, k1, k2, splits, sym, part, out, skip);
}

template <typename T>
void launch_f1(hipStream_t s, int64_t m, int k, const T *A, int64_t lda, const T *W1, int64_t ldw,
               double wc, const T *X1, double *part, int nwg) {
  hipLaunchKernelGGL(k_f1<T>, dim3(nwg), dim3(256), 0, s, m, k, A, lda, W1, ldw, wc, X1, part);
}

// LDS plan of k_update: staged G elements (grows) and dynamic LDS bytes;
// and the lanes per round of k_rowsolve_lds.
template <typename T>
UpdatePlan update_plan(int k, bool constw) {
  UpdatePlan pl;
  // rows of B = [-S; Z; T] staged per chunk (a multiple of 4, 64 KiB of LDS)
  const int kp = ((k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64) + 15) / 16 * 16;
  pl.grows = (int)(65536 / ((size_t)kp * sizeof(T)));
  pl.shm = ((size_t)pl.grows * kp + (size_t)64 * (kp + 1)) * sizeof(T);
  const size_t per = (size_t)(k * (k + 1) / 2 + 2 * k) * sizeof(T);
  pl.nl = 64;
  while (pl.nl > 1 && per * pl.nl + (size_t)k * k * sizeof(T) > 65536) pl.nl >>= 1;
  (void)constw;
  return pl;
}

template <typename T, int KMAX, bool CONSTW, typename TA2>
static void launch_update_kernel(hipStream_t s, const UpdateArgs<T> &a, const TA2 *A2,
                                 int64_t lda2, const UpdatePlan &pl) {
  const unsigned grid = (unsigned)((a.m + 63) / 64);
  if (pl.shm > 65536)
    (void)hipFuncSetAttribute((const void *)k_update<T, KMAX, CONSTW, TA2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.shm);
  hipLaunchKernelGGL((k_update<T, KMAX, CONSTW, TA2>), dim3(grid), dim3(UPD_T), pl.shm, s,
                     a.m, a.k, a.n, a.A, a.lda, A2, lda2, a.W1, a.ldw, a.wc, a.X1o, a.X1n, a.Gt,
                     a.Tt, a.St, a.part, a.Eb, pl.grows, a.st);
}

// The tiled kernel's requirements: 8-row groups, 16-byte aligned columns.
template <typename T>
static bool update_tiled_ok(const UpdateArgs<T> &a) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    auto al = [](const void *p) { return ((uintptr_t)p & 15u) == 0; };
    if (a.m % 8 != 0 || a.lda % 4 != 0 || !al(a.A) || !al(a.X1o)) return false;
    if (a.A2b != nullptr && (a.ldb % 8 != 0 || !al(a.A2b) || !a.Zh || !a.Zl || a.n2p % 32 != 0))
      return false;
    return true;
  }
}

template <int KMAX, bool CONSTW, bool A2BF>
static void launch_update_tiled(hipStream_t s, const UpdateArgs<float> &a) {
  const unsigned grid = (unsigned)((a.m + UT_R - 1) / UT_R);
  hipLaunchKernelGGL((k_update_t<KMAX, CONSTW, A2BF>), dim3(grid), dim3(UT_T), 0, s, a.m, a.k,
                     a.n, a.A, a.lda, a.A2b, a.ldb, a.W1, a.ldw, a.wc, a.X1o, a.X1n, a.Gt, a.Tt,
                     a.Zh, a.Zl, a.n2p, a.part, a.Eb, a.st);
}

template <typename T, int KMAX, bool CONSTW>
static void launch_update_a2(hipStream_t s, const UpdateArgs<T> &a, const UpdatePlan &pl) {
  if constexpr (std::is_same<T, float>::value) {
    if (update_tiled_ok(a)) {
      if (a.A2b != nullptr)
        launch_update_tiled<KMAX, CONSTW, true>(s, a);
      else
        launch_update_tiled<KMAX, CONSTW, false>(s, a);
      return;
    }
    if (a.A2b != nullptr) {
      launch_update_kernel<T, KMAX, CONSTW, bf16s>(s, a, a.A2b, a.ldb, pl);
      return;
    }
  }
  launch_update_kernel<T, KMAX, CONSTW, T>(s, a, a.A + (int64_t)a.k * a.lda, a.lda, pl);
}

template <typename T>
static void launch_rowsolve_reg(hipStream_t s, const UpdateArgs<T> &a, unsigned grid,
                                const int *cgflag) {
  if (a.k <= 8)
    hipLaunchKernelGGL((k_rowsolve_reg<T, 8>), dim3(grid), dim3(64), 0, s, a.m, a.k, a.A, a.lda,
                       a.W1, a.ldw, a.X1o, a.X1n, a.Eb, a.St, a.part, a.st, a.flags, cgflag);
  else if (a.k <= 16)
    hipLaunchKernelGGL((k_rowsolve_reg<T, 16>), dim3(grid), dim3(64), 0, s, a.m, a.k, a.A, a.lda,
                       a.W1, a.ldw, a.X1o, a.X1n, a.Eb, a.St, a.part, a.st, a.flags, cgflag);
  else
    hipLaunchKernelGGL((k_rowsolve_reg<T, 24>), dim3(grid), dim3(64), 0, s, a.m, a.k, a.A, a.lda,
                       a.W1, a.ldw, a.X1o, a.X1n, a.Eb, a.St, a.part, a.st, a.flags, cgflag);
}

// CG per-row solves (float, k <= 48); false when k is beyond them.
static bool launch_rowsolve_cg(hipStream_t s, const UpdateArgs<float> &a, int *cgflag) {
  const unsigned grid = (unsigned)((a.m + 255) / 256);
#define RS_CG(KP)                                                                               \
  hipLaunchKernelGGL((k_rowsolve_cg<KP>), dim3(grid), dim3(256), 0, s, a.m, a.k, a.A, a.lda,     \
                     a.W1, a.ldw, a.X1o, a.X1n, a.Eb, a.St, a.part, a.st, cgflag)
  if (a.k <= 16) RS_CG(16);
  else if (a.k <= 24) RS_CG(24);
  else if (a.k <= 32) RS_CG(32);
  else if (a.k <= 40) RS_CG(40);
  else if (a.k <= 48) RS_CG(48);
  else return false;
#undef RS_CG
  return true;
}

template <typename T, int KMAX>
static void launch_update_k(hipStream_t s, const UpdateArgs<T> &a) {
  const unsigned grid = (unsigned)((a.m + 63) / 64);
  const UpdatePlan pl = update_plan<T>(a.k, a.constw);
  if (a.constw) {
    launch_update_a2<T, KMAX, true>(s, a, pl);
    return;
  }
  launch_update_a2<T, KMAX, false>(s, a, pl);
  // float: conjugate gradients per row, the direct solves below only for a
  // sweep in which some row did not converge (a flag word of its own)
  const int *cgflag = nullptr;
  if constexpr (sizeof(T) == 4) {
    if (a.flags != nullptr && launch_rowsolve_cg(s, a, a.flags + 2)) cgflag = a.flags + 2;
  }
  // register-resident per-row solves for fp32 up to k = 24 (the fp64 factor would not fit)
  if constexpr (sizeof(T) == 4) {
    if (a.k <= 24) {
      launch_rowsolve_reg<T>(s, a, grid, cgflag);
      return;
    }
  }
  {
    const size_t shm = (size_t)a.k * a.k * sizeof(T) +
                       (size_t)(a.k * (a.k + 1) / 2 + 2 * a.k) * pl.nl * sizeof(T);
    hipLaunchKernelGGL((k_rowsolve_lds<T, KMAX>), dim3(grid), dim3(64), shm, s, a.m, a.k, a.A,
                       a.lda, a.W1, a.ldw, a.X1o, a.X1n, a.Eb, a.St, a.part, pl.nl, a.st, a.flags,
                       cgflag);
  }
}

int update_panel_kp(int k) { return ((k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64) + 15) / 16 * 16; }

void launch_panel_bf16(hipStream_t s, int n2, int k, int n2p, const float *Gt, bf16s *Zh,
                       bf16s *Zl, const SmallState *st) {
  const int kp = update_panel_kp(k);
  const int grid = std::max(1, std::min(256, (kp * n2p + 255) / 256));
  hipLaunchKernelGGL(k_panel_bf16, dim3(grid), dim3(256), 0, s, n2, k, kp, n2p, Gt, Zh, Zl, st);
}

void launch_panel_bf16_b(hipStream_t s, int count, const PanelArgs *av) {
  if (count > 0) hipLaunchKernelGGL(k_panel_bf16_b, dim3(64, count), dim3(256), 0, s, av);
}

template <typename T>
void launch_update(hipStream_t s, const UpdateArgs<T> &a) {
  // refuse to launch with a missing operand (the kernels have no null checks)
  if (!a.A || !a.X1o || !a.X1n || !a.Gt || !a.Tt || !a.St || !a.part || !a.st || !a.flags ||
      (!a.constw && (!a.Eb || !a.W1)))
    return;
  if (a.k <= 8) launch_update_k<T, 8>(s, a);
  else if (a.k <= 16) launch_update_k<T, 16>(s, a);
  else if (a.k <= 32) launch_update_k<T, 32>(s, a);
  else launch_update_k<T, 64>(s, a);
}

template <typename T, int KMAX>
static void launch_x2_k(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
                        const T *X1, const T *Zt, const T *Vr, T *X2, int64_t ldx2, const T *w2,
                        uint8_t *mask, int64_t ldm, T tau) {
  const unsigned grid = (unsigned)((m + 63) / 64);
  if (l <= 8)
    hipLaunchKernelGGL((k_x2<T, KMAX, 8>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A, lda, X1, Zt,
                       Vr, X2, ldx2, w2, mask, ldm, tau);
  else
    hipLaunchKernelGGL((k_x2<T, KMAX, WLRA_BMAX>), dim3(grid), dim3(64), 0, s, m, k, n2, l, A, lda,
                       X1, Zt, Vr, X2, ldx2, w2, mask, ldm, tau);
}

template <typename T>
void launch_x2(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
               const T *X1, const T *Zt, const T *Vr, T *X2, int64_t ldx2, const T *w2,
               uint8_t *mask, int64_t ldm, T tau) {
  if (k <= 8) launch_x2_k<T, 8>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2, w2, mask, ldm, tau);
  else if (k <= 16)
    launch_x2_k<T, 16>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2, w2, mask, ldm, tau);
  else if (k <= 32)
    launch_x2_k<T, 32>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2, w2, mask, ldm, tau);
  else launch_x2_k<T, 64>(s, m, k, n2, l, A, lda, X1, Zt, Vr, X2, ldx2, w2, mask, ldm, tau);
}

void launch_chgprep_b(hipStream_t s, int count, const ChgArgs *av) {
  if (count > 0) hipLaunchKernelGGL(k_chgprep_b, dim3(count), dim3(QR_T), 0, s, av);
}

void launch_chgprep(hipStream_t s, int n2, int k, int l, const double *Vp, const double *Vq,
                    const double *Zp, const double *Zq, double *Hb, double *Kg,
                    const SmallState *st) {
  hipLaunchKernelGGL(k_chgprep, dim3(1), dim3(QR_T), 0, s, n2, k, l, Vp, Vq, Zp, Zq, Hb, Kg, st);
}

template <typename T, int LMAX>
static void launch_change_qr_k(hipStream_t s, int64_t m, int k, int n2, int l, const T *A2,
                               int64_t lda2, const T *X1p, const T *X1q, const double *Hb,
                               const double *Kg, double *part, const SmallState *st) {
  const unsigned grid = (unsigned)((m + 63) / 64);
  const int K = 2 * l + 2 * k;
  int rows = n2;
  if (l > 0) rows = std::min(n2, std::max(1, 8192 / (2 * l)));
  const size_t stage = (size_t)std::max(rows * 2 * l, ((K + 15) / 16) * 16 * CHG_GLD);
  const size_t shm = (stage + (size_t)2 * LMAX * 64) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void *)k_change_q<T, LMAX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((k_change_q<T, LMAX>), dim3(grid), dim3(64 * CHG_NW), shm, s, m, k,
                     n2, l, A2, lda2, X1p, X1q, Hb, Kg, rows, part, st);
}

template <typename T>
void launch_change_qr(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
                      const T *X1p, const T *X1q, const double *Hb, const double *Kg,
                      double *part, const SmallState *st) {
  const T *A2 = A + (int64_t)k * lda;
  // the row pass's per-lane products are unrolled over LMAX >= l
  if (l <= 8)
    launch_change_qr_k<T, 8>(s, m, k, n2, l, A2, lda, X1p, X1q, Hb, Kg, part, st);
  else if (l <= 16)
    launch_change_qr_k<T, 16>(s, m, k, n2, l, A2, lda, X1p, X1q, Hb, Kg, part, st);
  else
    launch_change_qr_k<T, WLRA_BMAX>(s, m, k, n2, l, A2, lda, X1p, X1q, Hb, Kg, part, st);
}

template <typename T>
void launch_copy_out(hipStream_t s, int64_t m, int64_t k, const T *src, T *dst, int64_t ld) {
  const int64_t total = m * k;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
  hipLaunchKernelGGL(k_copy_out<T>, dim3(g), dim3(256), 0, s, m, k, src, dst, ld);
}

#define INST(T)                                                                                   \
  template void launch_validate<T>(hipStream_t, int64_t, int64_t, const T *, int64_t, int64_t,    \
                                   const T *, int64_t, int *, bf16s *, const T *, T *);           \
  template void launch_init_x1<T>(hipStream_t, int64_t, int64_t, int, uint64_t, const T *,        \
                                  int64_t, T *, int *, const int *);                              \
  template void launch_tsgemm<T, T>(hipStream_t, int64_t, const T *, int64_t, int, const T *,     \
                                    int64_t, int, int, int, int64_t, double *, double *,          \
                                    const int *, const T *, int64_t, int);                        \
  template void launch_f1<T>(hipStream_t, int64_t, int, const T *, int64_t, const T *, int64_t,   \
                             double, const T *, double *, int);                                   \
  template void launch_update<T>(hipStream_t, const UpdateArgs<T> &);                             \
  template UpdatePlan update_plan<T>(int, bool);                                                 \
  template void launch_x2<T>(hipStream_t, int64_t, int, int, int, const T *, int64_t, const T *,  \
                             const T *, const T *, T *, int64_t, const T *, uint8_t *, int64_t,  \
                             T);                                                                  \
  template void launch_copy_out<T>(hipStream_t, int64_t, int64_t, const T *, T *, int64_t);     \
  template void launch_change_qr<T>(hipStream_t, int64_t, int, int, int, const T *, int64_t,      \
                                    const T *, const T *, const double *, const double *,         \
                                    double *, const SmallState *);
INST(float)
INST(double)
