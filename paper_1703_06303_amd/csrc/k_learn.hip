// Learned warm start: Gaussian sketch of A, the MLP 512 -> 256 -> 256 -> n r
// (forward, backward, Adam) and the decode X1_0 = L0 (L0^T L0)^-1 L0^T A1 with
// L0 = A Y.  Not part of the paper (which starts Algorithm 1 from a random
// X1_0); the sweep that follows is unchanged.
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
    for (int e = threadIdx.x; e < LEARN_SK_ROWS * nj; e += 256) sP[e] = P1[(int64_t)j0 * LEARN_SK_ROWS + e];
    for (int e = threadIdx.x; e < nj * LEARN_SK_COLS; e += 256) {
      const int jj = e % nj, b = e / nj;
      sQ[jj * LEARN_SK_COLS + b] = (double)Ps[j0 + jj + (int64_t)b * n];
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

// Adam (Kingma & Ba): bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void k_adam(int64_t P, float *__restrict__ p,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < P;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  }
}

// ---------------------------------------------------------------------------
// Decode.  out (m x c, column-major, ld ldo) = A (m x kin, ld lda) times a
// small kin x c matrix S with element (j, q) at S[j rs + q cs]; one row per
// lane, rows of S staged through LDS.
#define TS_STAGE_BYTES 32768
template <typename T, typename TS, int CMAX>
__global__ __launch_bounds__(64) void k_tall_small(int64_t m, int kin, int c,
                                                   const T *__restrict__ A, int64_t lda,
                                                   const TS *__restrict__ S, int64_t rs,
                                                   int64_t cs, T *__restrict__ out, int64_t ldo) {
  constexpr int TS_STAGE = TS_STAGE_BYTES / sizeof(T);
  __shared__ T sS[TS_STAGE];
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool act = i < m;
  const int64_t ir = act ? i : (m - 1);
  T acc[CMAX];
#pragma unroll
  for (int q = 0; q < CMAX; ++q) acc[q] = T(0);
  const int rows = max(1, TS_STAGE / max(c, 1));
  for (int j0 = 0; j0 < kin; j0 += rows) {
    const int nr = min(rows, kin - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * c; e += 64) {
      const int jj = e / c, q = e - jj * c;
      sS[e] = (T)S[(int64_t)(j0 + jj) * rs + (int64_t)q * cs];
    }
    __syncthreads();
    int jj = 0;
    for (; jj + 8 <= nr; jj += 8) {  // 8 reads of A in flight
      T a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = A[ir + (int64_t)(j0 + jj + u) * lda];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const T *srow = sS + (jj + u) * c;
#pragma unroll
        for (int q = 0; q < CMAX; ++q)
          if (q < c) acc[q] = fma(a[u], srow[q], acc[q]);
      }
    }
    for (; jj < nr; ++jj) {
      const T a = A[ir + (int64_t)(j0 + jj) * lda];
      const T *srow = sS + jj * c;
#pragma unroll
      for (int q = 0; q < CMAX; ++q)
        if (q < c) acc[q] = fma(a, srow[q], acc[q]);
    }
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < CMAX; ++q)
      if (q < c) out[i + (int64_t)q * ldo] = acc[q];
  }
}

// Y = G^-1 H (G r x r SPD, H r x k, both column-major double) by Cholesky in
// LDS (lower, right-looking, by wavefront 0); then one thread per column of
// H solves L L^T y = h with the column in registers.  Y is stored typed,
// row-major r x k (element (q, c) at Y[q k + c]).  A pivot below 1e-13 of
// the largest diagonal entry or a non-finite entry sets DEV_LEARN_FAIL.
template <typename T>
__global__ __launch_bounds__(256) void k_decode_solve(int r, int k, const double *__restrict__ Gg,
                                                      const double *__restrict__ H,
                                                      T *__restrict__ Y, int *flags) {
  constexpr int L = LEARN_RMAX;
  __shared__ double G[L * L];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < L * L; e += 256) {
    const int a = e % L, b = e / L;
    G[e] = (a < r && b < r) ? Gg[a + b * r] : 0.0;
  }
  __syncthreads();
  double dmax = 0.0;
  for (int j = 0; j < r; ++j) dmax = fmax(dmax, G[j + j * L]);
  if (t < 64) {
    for (int j = 0; j < r; ++j) {
      if (t == 0) {
        double d = G[j + j * L];
        if (!(d > 1e-13 * dmax)) {
          bad = 1;
          d = 1.0;
        }
        G[j + j * L] = sqrt(d);
      }
      wave_sync();
      const double ljj = G[j + j * L];
      for (int i = j + 1 + t; i < r; i += 64) G[i + j * L] /= ljj;
      wave_sync();
      const int rem = r - j - 1;
      for (int e = t; e < rem * rem; e += 64) {
        const int i = j + 1 + e % rem, q = j + 1 + e / rem;
        if (q <= i) G[i + q * L] -= G[i + j * L] * G[q + j * L];
      }
      wave_sync();
    }
    // the strict upper triangle is never read below; keep it zero
    for (int e = t; e < r * r; e += 64)
      if ((e % r) < (e / r)) G[(e % r) + (e / r) * L] = 0.0;
  }
  __syncthreads();
  for (int c = t; c < k; c += 256) {
    double x[L];
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = (i < r) ? H[i + (int64_t)c * r] : 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      if (i < r) {
        double s = x[i];
#pragma unroll
        for (int q = 0; q < i; ++q) s -= G[i + q * L] * x[q];
        x[i] = s / G[i + i * L];
      }
      asm volatile("" ::: "memory");  // keep each row's reads of L in place
    }
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
      if (i < r) {
        double s = x[i];
#pragma unroll
        for (int q = i + 1; q < L; ++q) s -= G[q + i * L] * x[q];
        x[i] = s / G[i + i * L];
      }
      asm volatile("" ::: "memory");
    }
    int nb = 0;
#pragma unroll
    for (int i = 0; i < L; ++i)
      if (i < r) {
        nb |= !isfinite(x[i]);
        Y[(int64_t)i * k + c] = (T)x[i];
      }
    if (nb) bad = 1;
  }
  __syncthreads();
  if (t == 0 && bad) atomicOr(flags, DEV_LEARN_FAIL);
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
                 float b1, float b2, float eps, float bc1, float bc2) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(P, 4096)), dim3(256), 0, s, P, p, g, m, v, lr, b1, b2,
                     eps, bc1, bc2);
}

template <typename T, typename TS>
void launch_tall_small(hipStream_t s, int64_t m, int kin, int c, const T *A, int64_t lda,
                       const TS *S, int64_t rs, int64_t cs, T *out, int64_t ldo) {
  if (c < 1 || c > 64) return;  // the kernel holds at most 64 accumulators
  const unsigned grid = (unsigned)((m + 63) / 64);
  if (c <= 32)
    hipLaunchKernelGGL((k_tall_small<T, TS, 32>), dim3(grid), dim3(64), 0, s, m, kin, c, A, lda, S,
                       rs, cs, out, ldo);
  else
    hipLaunchKernelGGL((k_tall_small<T, TS, 64>), dim3(grid), dim3(64), 0, s, m, kin, c, A, lda, S,
                       rs, cs, out, ldo);
}

template <typename T>
void launch_decode_solve(hipStream_t s, int r, int k, const double *G, const double *H, T *Y,
                         int *flags) {
  hipLaunchKernelGGL(k_decode_solve<T>, dim3(1), dim3(256), 0, s, r, k, G, H, Y, flags);
}

#define INST_L(T)                                                                               \
  template void launch_gauss_fill<T>(hipStream_t, int64_t, uint64_t, double, T *);            \
  template void launch_sketch_finish<T>(hipStream_t, int, const double *, const T *, float *); \
  template void launch_tall_small<T, T>(hipStream_t, int64_t, int, int, const T *, int64_t,    \
                                        const T *, int64_t, int64_t, T *, int64_t);            \
  template void launch_decode_solve<T>(hipStream_t, int, int, const double *, const double *,   \
                                       T *, int *);
INST_L(float)
INST_L(double)
template void launch_tall_small<double, float>(hipStream_t, int64_t, int, int, const double *,
                                               int64_t, const float *, int64_t, int64_t, double *,
                                               int64_t);
