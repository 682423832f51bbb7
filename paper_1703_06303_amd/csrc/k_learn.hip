// Learned warm start: Gaussian sketch of A, the MLP 512 -> 256 -> 256 -> n r
// (forward, backward, Adam) and the decode of the predicted row basis Y into
// X1_0 (k_ldecode, then the row-update kernels).  Not part of the paper
// (which starts Algorithm 1 from a random X1_0); the sweep that follows is
// unchanged.
//
// Network matrices are row-major float: activations B x features, weights
// out x in.  Sums over the m rows of A use the tall-skinny product kernel
// (double partials); the small solves run in double.
#include "common.h"
#include "launch.h"

// ---------------------------------------------------------------------------
// out[e] = scale * z_e, z the N(0,1) Philox draws keyed by seed in element
// order (pair e/2, cos for even e and sin for odd e).
template <typename T>
__global__ __launch_bounds__(256) void k_gauss_fill(int64_t count, uint64_t seed, double scale,
                                                    T *__restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; 2 * p < count;
       p += (int64_t)gridDim.x * blockDim.x) {
    double z0, z1;
    philox_normal2(seed, (uint64_t)p, z0, z1);
    out[2 * p] = (T)(scale * z0);
    if (2 * p + 1 < count) out[2 * p + 1] = (T)(scale * z1);
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(int64_t count, float *__restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = 0.f;
}

// s = vec(P1 Ps) / ||P1 Ps||_F with P1 = Om^T A (16 x n, double, ld 16) and
// Ps (n x 32, column-major); s[a + 16 b].
template <typename T>
__global__ __launch_bounds__(256) void k_sketch_finish(int n, const double *__restrict__ P1,
                                                       const T *__restrict__ Ps,
                                                       float *__restrict__ out) {
  // chunks of the n columns of P1 (16 x n) and rows of Psi (n x 32) in LDS
  constexpr int CH = 256;
  __shared__ double sP[LEARN_SK_ROWS * CH];
  __shared__ double sQ[CH * LEARN_SK_COLS];
  __shared__ double red[4];
  double v[2] = {0.0, 0.0};
  for (int j0 = 0; j0 < n; j0 += CH) {
    const int nj = min(CH, n - j0);
    __syncthreads();
    // eight clamped reads in flight per thread
    const int np = LEARN_SK_ROWS * nj, nq = nj * LEARN_SK_COLS;
    for (int e0 = threadIdx.x; e0 < np; e0 += 8 * 256) {
      double v8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v8[u] = P1[(int64_t)j0 * LEARN_SK_ROWS + min(e0 + 256 * u, np - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e0 + 256 * u < np) sP[e0 + 256 * u] = v8[u];
    }
    for (int e0 = threadIdx.x; e0 < nq; e0 += 8 * 256) {
      T q8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + 256 * u, nq - 1), jj = e % nj, b = e / nj;
        q8[u] = Ps[j0 + jj + (int64_t)b * n];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 256 * u, jj = e % nj, b = e / nj;
        if (e < nq) sQ[jj * LEARN_SK_COLS + b] = (double)q8[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int o = threadIdx.x + 256 * u;  // 0..511
      const int a = o % LEARN_SK_ROWS, b = o / LEARN_SK_ROWS;
      double acc = v[u];
      for (int jj = 0; jj < nj; ++jj)
        acc = fma(sP[a + jj * LEARN_SK_ROWS], sQ[jj * LEARN_SK_COLS + b], acc);
      v[u] = acc;
    }
  }
  double ss = v[0] * v[0] + v[1] * v[1];
  ss = block_sum(ss, red);
  const double inv = ss > 0 ? 1.0 / sqrt(ss) : 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) out[threadIdx.x + 256 * u] = (float)(v[u] * inv);
}

// ---------------------------------------------------------------------------
// C (M x N) = op(A) op(B) (+ bias per column) (relu) (* [mask > 0]), row-major.
//   MODE 0: C = A B^T, A M x K, B N x K
//   MODE 1: C = A B,   A M x K, B K x N
//   MODE 2: C = A^T B, A K x M, B K x N
// 64 x 64 tile per workgroup, 4 x 4 per thread, K in chunks of 16 in LDS.
#define GT 64
#define GK 16
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A,
                                              int lda, const float *__restrict__ B, int ldb,
                                              float *__restrict__ C, int ldc,
                                              const float *__restrict__ bias, int relu,
                                              const float *__restrict__ mask, int ldm) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row0 = blockIdx.y * GT, col0 = blockIdx.x * GT;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (MODE == 2) {
        const int rr = e % GT, kk = e / GT;
        const int gr = row0 + rr, gk = k0 + kk;
        As[kk][rr] = (gr < M && gk < K) ? A[(int64_t)gk * lda + gr] : 0.f;
      } else {
        const int kk = e % GK, rr = e / GK;
        const int gr = row0 + rr, gk = k0 + kk;
        As[kk][rr] = (gr < M && gk < K) ? A[(int64_t)gr * lda + gk] : 0.f;
      }
      if (MODE == 0) {
        const int kk = e % GK, cc = e / GK;
        const int gc = col0 + cc, gk = k0 + kk;
        Bs[kk][cc] = (gc < N && gk < K) ? B[(int64_t)gc * ldb + gk] : 0.f;
      } else {
        const int cc = e % GT, kk = e / GT;
        const int gc = col0 + cc, gk = k0 + kk;
        Bs[kk][cc] = (gc < N && gk < K) ? B[(int64_t)gk * ldb + gc] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + ty * 4 + i;
    if (row >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = col0 + tx * 4 + j;
      if (col >= N) continue;
      float v = acc[i][j];
      if (bias) v += bias[col];
      if (relu) v = fmaxf(v, 0.f);
      if (mask && !(mask[(int64_t)row * ldm + col] > 0.f)) v = 0.f;
      C[(int64_t)row * ldc + col] = v;
    }
  }
}

// out[c] = sum over rows of A (M x N, row-major), summed in double.
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float *__restrict__ A,
                                                float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double s = 0.0;
  for (int r = 0; r < M; ++r) s += (double)A[(int64_t)r * N + c];
  out[c] = (float)s;
}

// ---------------------------------------------------------------------------
// Subspace loss of one sample per workgroup.  Y, T: n x r column-major
// (sample stride n r).  With G = T^T T and M1 = G^-1 T^T Y (so that
// T M1 = Q Q^T Y for an orthonormal basis Q of span T) and E = Y^T Y - I:
//     loss_b = ||Y - T M1||^2 + lam ||E||^2,  gy = (2 (Y - T M1) + 4 lam Y E) / B.
__global__ __launch_bounds__(256) void k_subspace_loss(int n, int r, int batch,
                                                       const float *__restrict__ y,
                                                       const float *__restrict__ Tg, double lam,
                                                       float *__restrict__ gy,
                                                       double *__restrict__ loss_part,
                                                       int *flags) {
  __shared__ double G[LEARN_RMAX * LEARN_RMAX];
  __shared__ double TY[LEARN_RMAX * LEARN_RMAX];
  __shared__ double E[LEARN_RMAX * LEARN_RMAX];
  __shared__ double red[4];
  __shared__ int bad;
  const int b = blockIdx.x, t = threadIdx.x;
  const float *Y = y + (int64_t)b * n * r;
  const float *T = Tg + (int64_t)b * n * r;
  if (t == 0) bad = 0;
  for (int e = t; e < 3 * r * r; e += 256) {
    const int which = e / (r * r), q = e % (r * r);
    const int a = q % r, c = q / r;
    const float *X = (which == 2) ? Y : T;
    const float *Z = (which == 0) ? T : Y;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s = fma((double)X[j + (int64_t)a * n], (double)Z[j + (int64_t)c * n], s);
    if (which == 0) G[a + c * LEARN_RMAX] = s;
    else if (which == 1) TY[a + c * LEARN_RMAX] = s;
    else E[a + c * LEARN_RMAX] = s - (a == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // Cholesky G = L L^T (lower, in place), one thread: r <= 32
  if (t == 0) {
    for (int j = 0; j < r; ++j) {
      double d = G[j + j * LEARN_RMAX];
      for (int q = 0; q < j; ++q) d -= G[j + q * LEARN_RMAX] * G[j + q * LEARN_RMAX];
      if (!(d > 0.0)) {
        bad = 1;
        d = 1.0;
      }
      const double ljj = sqrt(d);
      G[j + j * LEARN_RMAX] = ljj;
      for (int i = j + 1; i < r; ++i) {
        double s = G[i + j * LEARN_RMAX];
        for (int q = 0; q < j; ++q) s -= G[i + q * LEARN_RMAX] * G[j + q * LEARN_RMAX];
        G[i + j * LEARN_RMAX] = s / ljj;
      }
    }
  }
  __syncthreads();
  // M1 = G^-1 TY column by column (in place in TY)
  for (int c = t; c < r; c += 256) {
    double *x = TY + c * LEARN_RMAX;
    for (int i = 0; i < r; ++i) {
      double s = x[i];
      for (int q = 0; q < i; ++q) s -= G[i + q * LEARN_RMAX] * x[q];
      x[i] = s / G[i + i * LEARN_RMAX];
    }
    for (int i = r - 1; i >= 0; --i) {
      double s = x[i];
      for (int q = i + 1; q < r; ++q) s -= G[q + i * LEARN_RMAX] * x[q];
      x[i] = s / G[i + i * LEARN_RMAX];
    }
  }
  __syncthreads();
  double acc = 0.0;
  const double sc = 1.0 / (double)batch;
  for (int e = t; e < n * r; e += 256) {
    const int j = e % n, q = e / n;
    double proj = 0.0, ye = 0.0;
    for (int c = 0; c < r; ++c) {
      proj = fma((double)T[j + (int64_t)c * n], TY[c + q * LEARN_RMAX], proj);
      ye = fma((double)Y[j + (int64_t)c * n], E[c + q * LEARN_RMAX], ye);
    }
    const double rm = (double)Y[e] - proj;
    acc = fma(rm, rm, acc);
    gy[(int64_t)b * n * r + e] = (float)(sc * (2.0 * rm + 4.0 * lam * ye));
  }
  double ee = 0.0;
  for (int e = t; e < r * r; e += 256) {
    const double v = E[(e % r) + (e / r) * LEARN_RMAX];
    ee = fma(v, v, ee);
  }
  acc = block_sum(acc, red);
  ee = block_sum(ee, red);
  if (t == 0) {
    loss_part[b] = acc + lam * ee;
    if (bad) atomicOr(flags, DEV_LEARN_FAIL);
  }
}

// Adam (Kingma & Ba): bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.  The
// complements c1 = 1 - beta1 and c2 = 1 - beta2 come from the host, formed in
// double and rounded once: 1.f - 0.999f would be off by 1.3e-5 relative.
__global__ __launch_bounds__(256) void k_adam(int64_t P, float *__restrict__ p,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float c1,
                                              float b2, float c2, float eps, float bc1,
                                              float bc2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < P;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + c1 * gg;
    const float vv = b2 * v[e] + c2 * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  }
}

// ---------------------------------------------------------------------------
// Lane `lane`'s value of x, in every lane.
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(v & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Solve M X = B in place of B (M: SPD nn x nn, B: nn x cols, both in LDS
// with leading dimension ld; nn <= LEARN_RMAX, nn + cols <= 64) by
// Gauss-Jordan elimination without pivoting on wavefront 0, lane c holding
// column c of [M B] in registers: per pivot j, column j is read from lane j
// (v_readlane) and row j is divided by the pivot p, every other row losing
// M[i][j] / p times it; no workgroup barriers between the steps.  On SPD
// input the pivots are the Schur complements of the leading blocks (the
// squared Cholesky pivots); one below 1e-13 of the largest diagonal entry
// sets *bad and is replaced by 1.  M is left as it was.  Entered and left
// with a barrier.
__device__ __forceinline__ void ld_gj_solve(const double *M, double *B, int nn, int cols, int ld,
                                            int *bad) {
  constexpr int L = LEARN_RMAX;
  const int t = threadIdx.x, nc = nn + cols;
  if (t < 64) {
    double dmax = 0.0;
    for (int j = 0; j < nn; ++j) dmax = fmax(dmax, M[j + j * ld]);
    const int c = min(t, max(nc - 1, 0));
    // rows past nn are zero and stay zero: every step updates all L rows
    // without a branch
    double m[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int ic = min(i, max(nn - 1, 0));
      const double v = (c < nn) ? M[ic + c * ld] : B[ic + (c - nn) * ld];
      m[i] = (i < nn) ? v : 0.0;
    }
#pragma unroll
    for (int j = 0; j < L; ++j) {
      if (j < nn) {
        double p = readlane_d(m[j], j);
        if (!(p > 1e-13 * dmax)) {
          if (t == 0) *bad = 1;
          p = 1.0;
        }
        const double mj = m[j] / p;
#pragma unroll
        for (int i = 0; i < L; ++i)
          if (i != j) m[i] = fma(-readlane_d(m[i], j), mj, m[i]);
        m[j] = mj;
      }
    }
    if (t >= nn && t < nc) {
#pragma unroll
      for (int i = 0; i < L; ++i)
        if (i < nn) B[i + (t - nn) * ld] = m[i];
    }
  }
  __syncthreads();
}

// epi(a, c, v) for every entry (a, c) of X Y (rows, cols <= 32, inner <=
// LEARN_RMAX), operands in LDS with leading dimension ld, XT / YT reading
// them transposed.  On the FP64 matrix cores: 16 x 16 output tiles dealt to
// wavefronts [w0, w0 + nw) of the workgroup, the inner index in k-steps of 4
// (every read issued before the first multiply); indices clamped, the
// excess masked.  No barrier.
template <bool XT, bool YT, typename Epi>
__device__ __forceinline__ void ld_mm(const double *X, const double *Y, int rows, int cols,
                                      int inner, int ld, int w0, int nw, Epi epi) {
  typedef double pd4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6) - w0;
  const int li = lane & 15, lk = lane >> 4, tr = (rows + 15) / 16, tc = (cols + 15) / 16;
  if (w < 0 || w >= nw) return;
  for (int tile = w; tile < tr * tc; tile += nw) {
    const int r0 = 16 * (tile % tr), c0 = 16 * (tile / tr);
    const int a = min(r0 + li, rows - 1), c = min(c0 + li, cols - 1);
    double av[LEARN_RMAX / 4], bv[LEARN_RMAX / 4];
#pragma unroll
    for (int u = 0; u < LEARN_RMAX / 4; ++u) {
      const int bi = 4 * u + lk, bc = min(bi, inner - 1);
      const double x = XT ? X[bc + a * ld] : X[a + bc * ld];
      av[u] = (bi < inner) ? x : 0.0;
      bv[u] = YT ? Y[c + bc * ld] : Y[bc + c * ld];
    }
    pd4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < LEARN_RMAX / 4; ++u)
      if (4 * u < inner) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = r0 + lk + 4 * v, cb = c0 + li;  // output row lk + 4 v, column li
      if (ra < rows && cb < cols) epi(ra, cb, acc[v]);
    }
  }
}

// Decode of the predicted row basis Y (n x r, Y[j + n q], r <= LEARN_RMAX).
// With the row space fixed, problem (5) separates over rows; row i of the
// start is the weighted least-squares fit z_i Y^T.  Writing the rows of
// span(Y^T) as [x1, x1 C + u W^T] (C^T = Y2 F^T with F = (Y1 Y1^T)^-1 Y1,
// Y1 = Y[:k], Y2 = Y[k:]; W = Y2 P_b, P_b = I - Y1^T F the projector on
// null(Y1)), the fit of u is a plain projection and what is left for x1 is
// the k x k problem
//     x1 (diag(w_i^2) + S) = a1 diag(w_i^2) + a2 Z,
// Z = (I - P_W) C^T, S = C Z: the row update of Algorithm 1 (steps 7-9)
// with these S and Z and no X1 term.  Y2 enters only through its r x r Gram
// Gy = Y2^T Y2 and the final product Z = Y2 Q:
//   N = P_b Gy P_b + (I - P_b)   (SPD when W has rank r - k; N^-1 on
//                                  range(W^T) is the pseudo-inverse of W^T W)
//   Q = F^T - P_b N^-1 P_b Gy F^T,   Z = Y2 Q,   S = F Gy Q (symmetrised).
// Output as the row update's operands: Gt = [-S; Z] ((k + n2) x k,
// row-major), St = S, Tt = 0.  One workgroup, all in double (Gy and Z on
// the FP64 matrix cores, the two SPD inverses by ld_inverse); Y is scaled to
// ||Y||_F^2 = r (the row space does not change).  A zero Y, a
// pivot of Y1 Y1^T or N below 1e-13 of its largest diagonal entry, or a
// non-finite result sets DEV_LEARN_FAIL.
template <typename T>
__global__ __launch_bounds__(1024) void k_ldecode(int n, int k, int r, const float *__restrict__ yv,
                                                  T *__restrict__ Gt, T *__restrict__ Tt,
                                                  T *__restrict__ St, int *flags) {
  typedef double pd4 __attribute__((ext_vector_type(4)));
  constexpr int L = LEARN_RMAX, LP = L + 1, NT = 1024, NW = NT / 64;  // LP odd: no bank conflicts
  // Y2 is staged through sY in chunks of crow rows (float, column stride
  // crow = 20 mod 64: the Gram's matrix-core reads are free of bank
  // conflicts, those of Z at most two-way)
  constexpr int YST = 16384;
  __shared__ float sY[YST];
  __shared__ double pool[8 * L * LP];
  __shared__ double red[NW];
  __shared__ int bad;
  // Y1 and Gy stay unscaled; the scale of Y (||Y||_F^2 = r) enters the
  // products that read them
  double *sY1 = pool, *sG = pool + L * LP, *sK = pool + 2 * L * LP, *sF = pool + 3 * L * LP;
  double *sP = pool + 4 * L * LP, *sN = pool + 5 * L * LP, *sT = pool + 6 * L * LP;
  double *sU = pool + 7 * L * LP;
  double *park = sK;  // 16 partial Gram tiles (4096 doubles) before sK..sU are used
  const int t = threadIdx.x, n2 = n - k;
  const int lane = t & 63, w = t >> 6, li = lane & 15, lk = lane >> 4;
  const int crow = (((YST / r) - 20) & ~63) + 20;  // <= YST / r since r <= LEARN_RMAX
  const int nchunk = (n2 + crow - 1) / crow;
  if (t == 0) bad = 0;
  // rows [j0, j0 + cl) of Y2 to sY (coalesced, eight reads in flight)
  auto stage = [&](int j0, int cl) {
    for (int e0 = t; e0 < cl * r; e0 += 8 * NT) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + u * NT, cl * r - 1);
        v[u] = yv[k + j0 + (e % cl) + (int64_t)n * (e / cl)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * NT;
        if (e < cl * r) sY[(e % cl) + (e / cl) * crow] = v[u];
      }
    }
  };
  // Y1 = Y[:k] to LDS; its squared entries towards ||Y||_F^2
  double ss = 0.0;
  for (int e = t; e < k * r; e += NT) {
    const int a = e % k, q = e / k;
    const double v = (double)yv[a + (int64_t)n * q];
    sY1[a + q * LP] = v;
    ss = fma(v, v, ss);
  }
  // Gy = Y2^T Y2 on the FP64 matrix cores: 16 x 16 output tiles (r <= 32:
  // at most 4), four wavefronts per tile taking every fourth group of 8
  // k-steps (4 rows each); the partial tiles are added in a fixed order
  {
    const int tile = w & 3, part = w >> 2;
    const int r0 = 16 * (tile & 1), c0 = 16 * (tile >> 1);
    const bool act = r0 < r && c0 < r;
    const int qa = min(r0 + li, r - 1), qb = min(c0 + li, r - 1);
    const double ma = (r0 + li < r) ? 1.0 : 0.0, mb = (c0 + li < r) ? 1.0 : 0.0;
    pd4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int j0 = ch * crow, cl = min(crow, n2 - j0);
      if (ch > 0) __syncthreads();  // the previous chunk has been read
      stage(j0, cl);
      __syncthreads();
      if (act) {
        for (int s0 = 32 * part; s0 < cl; s0 += 128) {
          double av[8], bv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int jj = s0 + 4 * u + lk, jc = min(jj, cl - 1);
            const double mj = (jj < cl) ? ma : 0.0;
            av[u] = (double)sY[jc + qa * crow] * mj;
            bv[u] = (double)sY[jc + qb * crow] * mb;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) park[(part * 4 + tile) * 256 + (lk + 4 * v) * 16 + li] = acc[v];
  }
  ss = wave_sum(ss);
  if (lane == 0) red[w] = ss;
  __syncthreads();
  {
    const int tile = t >> 8, el = t & 255;  // output row el / 16, column el % 16
    const int rr = 16 * (tile & 1) + el / 16, cc = 16 * (tile >> 1) + el % 16;
    if (rr < r && cc < r)
      sG[rr + cc * LP] = ((park[tile * 256 + el] + park[(4 + tile) * 256 + el]) +
                          park[(8 + tile) * 256 + el]) + park[(12 + tile) * 256 + el];
  }
  __syncthreads();
  ss = 0.0;
  for (int i = 0; i < NW; ++i) ss += red[i];
  for (int q = 0; q < r; ++q) ss += sG[q + q * LP];
  if (!(ss > 0.0) || !isfinite(ss)) {
    if (t == 0) atomicOr(flags, DEV_LEARN_FAIL);
    return;
  }
  const double sc = sqrt((double)r / ss), sc2 = (double)r / ss;
  // K = Y1 Y1^T (scaled) and the right-hand side Y1 of F = K^-1 Y1
  ld_mm<false, true>(sY1, sY1, k, k, r, LP, 0, 4, [&](int a, int c, double v) { sK[a + c * LP] = sc2 * v; });
  for (int e = t; e < k * r; e += NT) sF[(e % k) + (e / k) * LP] = sc * sY1[(e % k) + (e / k) * LP];
  __syncthreads();
  ld_gj_solve(sK, sF, k, r, LP, &bad);  // F (k x r)
  // P_b = I - Y1^T F (r x r, symmetric) and Gy F^T (r x k)
  ld_mm<true, false>(sY1, sF, r, r, k, LP, 0, 4, [&](int a, int c, double v) {
    sP[a + c * LP] = ((a == c) ? 1.0 : 0.0) - sc * v;
  });
  ld_mm<false, true>(sG, sF, r, k, r, LP, 4, 4, [&](int a, int c, double v) { sU[a + c * LP] = sc2 * v; });
  __syncthreads();
  ld_mm<false, false>(sG, sP, r, r, r, LP, 0, 4, [&](int a, int c, double v) { sT[a + c * LP] = sc2 * v; });
  ld_mm<false, false>(sP, sU, r, k, r, LP, 4, 4, [&](int a, int c, double v) { sK[a + c * LP] = v; });
  __syncthreads();
  // N = P_b (Gy P_b) + I - P_b; then N^-1 U with U = P_b Gy F^T (in sK)
  ld_mm<false, false>(sP, sT, r, r, r, LP, 0, 4, [&](int a, int c, double v) {
    sN[a + c * LP] = v + ((a == c) ? 1.0 : 0.0) - sP[a + c * LP];
  });
  __syncthreads();
  ld_gj_solve(sN, sK, r, k, LP, &bad);
  // Q = F^T - P_b N^-1 U (r x k)
  ld_mm<false, false>(sP, sK, r, k, r, LP, 0, 4, [&](int a, int c, double v) {
    sT[a + c * LP] = sF[c + a * LP] - v;
  });
  __syncthreads();
  ld_mm<false, false>(sG, sT, r, k, r, LP, 0, 4, [&](int a, int c, double v) { sU[a + c * LP] = sc2 * v; });
  // Z = sc Y2 Q (n2 x k, row-major below S) on the FP64 matrix cores while
  // wavefronts 0-3 form Gy Q: 16 x 16 tiles of each chunk dealt round-robin
  // to wavefronts 4.., the r columns of Y2 as the inner index (at most 8
  // k-steps, all reads issued first); a single chunk is still in sY from
  // the Gram
  int nb = 0;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int j0 = ch * crow, cl = min(crow, n2 - j0);
    if (nchunk > 1) {
      __syncthreads();
      stage(j0, cl);
      __syncthreads();
    }
    const int nti = (cl + 15) / 16, ntj = (k + 15) / 16;
    for (int tile = w - 4; tile >= 0 && tile < nti * ntj; tile += NW - 4) {
      const int jt = 16 * (tile % nti), c0 = 16 * (tile / nti);
      const int ja = min(jt + li, cl - 1), cb = min(c0 + li, k - 1);
      const double mc = (c0 + li < k) ? 1.0 : 0.0;
      double av[L / 4], bv[L / 4];
#pragma unroll
      for (int u = 0; u < L / 4; ++u) {
        const int q = 4 * u + lk, qc = min(q, r - 1);
        av[u] = (double)sY[ja + qc * crow];
        bv[u] = (q < r) ? sT[qc + cb * LP] * mc : 0.0;
      }
      pd4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < L / 4; ++u)
        if (4 * u < r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jt + lk + 4 * v, c = c0 + li;
        if (j < cl && c < k) {
          const double z = sc * acc[v];
          nb |= !isfinite(z);
          Gt[(int64_t)(k + j0 + j) * k + c] = (T)z;
        }
      }
    }
  }
  if (nb) bad = 1;
  __syncthreads();
  // S = F (Gy Q), symmetrised; Gt's first k rows are -S; T = 0
  ld_mm<false, false>(sF, sU, k, k, r, LP, 0, 4, [&](int a, int c, double v) { sP[a + c * LP] = v; });
  __syncthreads();
  for (int e = t; e < k * k; e += NT) {
    const int a = e % k, c = e / k;
    const double sv = 0.5 * (sP[a + c * LP] + sP[c + a * LP]);
    if (!isfinite(sv)) bad = 1;
    St[a * k + c] = (T)sv;
    Gt[a * k + c] = (T)(-sv);
    Tt[a * k + c] = T(0);
  }
  __syncthreads();
  if (t == 0 && bad) atomicOr(flags, DEV_LEARN_FAIL);
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(int64_t count, T *__restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = T(0);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
static unsigned grid_for(int64_t n, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

template <typename T>
void launch_gauss_fill(hipStream_t s, int64_t count, uint64_t seed, double scale, T *out) {
  hipLaunchKernelGGL(k_gauss_fill<T>, dim3(grid_for((count + 1) / 2, 4096)), dim3(256), 0, s,
                     count, seed, scale, out);
}

void launch_fill_zero(hipStream_t s, int64_t count, float *out) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(count, 4096)), dim3(256), 0, s, count, out);
}

template <typename T>
void launch_sketch_finish(hipStream_t s, int n, const double *P1, const T *Ps, float *out) {
  hipLaunchKernelGGL(k_sketch_finish<T>, dim3(1), dim3(256), 0, s, n, P1, Ps, out);
}

// One row (inference): y (1 x N) = x B^T (+ bias) (relu), B N x K row-major;
// a wavefront per output, lanes over K, a fixed xor-tree sum.
__global__ __launch_bounds__(256) void k_gemv0(int N, int K, const float *__restrict__ x,
                                               const float *__restrict__ B, int ldb,
                                               float *__restrict__ y, const float *__restrict__ bias,
                                               int relu) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  const float *row = B + (int64_t)n * ldb;
  float acc = 0.f;
  for (int k = lane; k < K; k += 64) acc = fmaf(x[k], row[k], acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    float v = acc;
    if (bias) v += bias[n];
    if (relu) v = fmaxf(v, 0.f);
    y[n] = v;
  }
}

void launch_gemm(hipStream_t s, int mode, int M, int N, int K, const float *A, int lda,
                 const float *B, int ldb, float *C, int ldc, const float *bias, int relu,
                 const float *mask, int ldm) {
  if (mode == 0 && M == 1 && mask == nullptr) {
    hipLaunchKernelGGL(k_gemv0, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, N, K, A, B, ldb, C,
                       bias, relu);
    return;
  }
  dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
  if (mode == 0)
    hipLaunchKernelGGL(k_gemm<0>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       relu, mask, ldm);
  else if (mode == 1)
    hipLaunchKernelGGL(k_gemm<1>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       relu, mask, ldm);
  else
    hipLaunchKernelGGL(k_gemm<2>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       relu, mask, ldm);
}

void launch_colsum(hipStream_t s, int M, int N, const float *A, float *out) {
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, M, N, A, out);
}

void launch_subspace_loss(hipStream_t s, int n, int r, int batch, const float *y, const float *T,
                          double lam, float *gy, double *loss_part, int *flags) {
  hipLaunchKernelGGL(k_subspace_loss, dim3((unsigned)batch), dim3(256), 0, s, n, r, batch, y, T,
                     lam, gy, loss_part, flags);
}

void launch_adam(hipStream_t s, int64_t P, float *p, const float *g, float *m, float *v, float lr,
                 double b1, double b2, float eps, float bc1, float bc2) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(P, 4096)), dim3(256), 0, s, P, p, g, m, v, lr,
                     (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), eps, bc1, bc2);
}

template <typename T>
void launch_ldecode(hipStream_t s, int n, int k, int r, const float *yv, T *Gt, T *Tt, T *St,
                    int *flags) {
  hipLaunchKernelGGL(k_ldecode<T>, dim3(1), dim3(1024), 0, s, n, k, r, yv, Gt, Tt, St, flags);
}

template <typename T>
void launch_zero(hipStream_t s, int64_t count, T *out) {
  hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(count, 4096)), dim3(256), 0, s, count, out);
}

#define INST_L(T)                                                                               \
  template void launch_gauss_fill<T>(hipStream_t, int64_t, uint64_t, double, T *);            \
  template void launch_sketch_finish<T>(hipStream_t, int, const double *, const T *, float *); \
  template void launch_ldecode<T>(hipStream_t, int, int, int, const float *, T *, T *, T *,     \
                                  int *);                                                      \
  template void launch_zero<T>(hipStream_t, int64_t, T *);
INST_L(float)
INST_L(double)
template void launch_zero<int>(hipStream_t, int64_t, int *);

