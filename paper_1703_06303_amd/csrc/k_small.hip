// Small-step kernels of the sWLR sweep, all in double on the device:
//   k_coef   Cholesky R of X1^T X1 (the R of X1 = QR, Algorithm 1 step 4),
//            B = R^-T X1^T A2 = Q^T A2 and C = R^-1 B (step 5)
//   k_formM  M = A2^T A2 - B^T B = (P^perp A2)^T (P^perp A2), whose top r-k
//            eigenpairs give D = H_{r-k}(P^perp A2) (steps 4 and 6)
//   k_post   S = C C^T, T = (CV)(CV)^T, Z = (I - VV^T) C^T for the row pass
//            (step 7) and the objective F(X_p)
//   k_decide Error_p of Section 4.1 (from the row pass k_change_q) and
//            the stopping decision.
// One workgroup each except k_formM.
#include "common.h"
#include "launch.h"

// -----------------------------------------------------------------------------
// Trace and Frobenius norm of G_A = A2^T A2 (one workgroup; 8 reads in
// flight per thread, the trace from the diagonal alone).
__global__ __launch_bounds__(1024) void k_gastats(int n2, const double *__restrict__ GA,
                                                  SmallState *st) {
  __shared__ double red[16];
  const int64_t nn = (int64_t)n2 * n2;
  double tr = 0, f = 0;
  for (int64_t e0 = threadIdx.x; e0 < nn; e0 += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = GA[min(e0 + u * 1024, nn - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + u * 1024 < nn) f += v[u] * v[u];
  }
  for (int i = threadIdx.x; i < n2; i += 1024) tr += GA[i + (int64_t)i * n2];
  tr = block_sum(tr, red);
  f = block_sum(f, red);
  if (threadIdx.x == 0) {
    st->trGA = tr;
    st->nrmGA = sqrt(f);
    st->eig_floor *= sqrt(f);  // relative target -> absolute residual
  }
}

// Lane `lane`'s x (lane uniform).
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(v & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// -----------------------------------------------------------------------------
// Cholesky of G1 = X1^T X1 by wavefront 0 (rank check on the pivots): lane c
// holds column c in registers, and at step j the scaled row j of R goes
// through LDS to every lane.  Then one thread per column of P: forward
// substitution with R^T gives that column of B, backward substitution with
// R gives the column of C, the column held in registers (k <= KMAX) and R
// read from LDS (every thread reads the same entry at once).
// Several workgroups per instance when n2 > 256 (wg of nwg): each one
// factors G1 (the same arithmetic in every workgroup) and solves its own
// 256-column slice of P; workgroup 0 alone writes R and the sweep state, and
// every workgroup writes its share of ||B||^2 to coef_part[wg] (summed in
// order by k_post).
#define COEF_LD 65  // odd leading dimension: a lane per column hits distinct banks
template <int KMAX>
__device__ __forceinline__ void coef_body(const SmallArgs &a, int wg, int nwg) {
  SmallState *st = a.st;
  if (st->done) return;
  constexpr int LD = COEF_LD;
  __shared__ double sG[64 * LD];   // G1, then R (upper), column-major, ld LD
  __shared__ double sR[64 * 64];   // R for the substitutions (ld 64: aligned pairs)
  __shared__ double sRow[2][64];   // row j of R during the factorisation
  __shared__ double red[4];
  __shared__ int fail;
  const int k = a.k, n2 = a.n2, t = threadIdx.x;

  double f1 = 0, dx = 0;
  for (int i = t; i < a.nparts; i += 256) {
    f1 += a.upd_part[2 * i];
    dx += a.upd_part[2 * i + 1];
  }
  f1 = block_sum(f1, red);
  dx = block_sum(dx, red);
  if (t == 0) {
    if (wg == 0) {
      st->f1 = f1;
      st->dx1 = dx;
    }
    fail = 0;
  }
  {
    // clamped reads, all in flight; entries outside k x k are zero (and
    // nothing is read for k = 0)
    const int k1 = max(k, 1);
    double gv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u, r = e % 64, c = e / 64;
      gv[u] = (k > 0) ? a.G1[min(r, k1 - 1) + min(c, k1 - 1) * k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u, r = e % 64, c = e / 64;
      sG[r + c * LD] = (r < k && c < k) ? gv[u] : 0.0;
    }
  }
  __syncthreads();
  double gmax = 0, tr = 0;
  for (int i = 0; i < k; ++i) {
    gmax = fmax(gmax, sG[i + i * LD]);
    tr += sG[i + i * LD];
  }
  // A pivot below k * eps * max diag(X1^T X1) means X1 is numerically
  // rank deficient (cond(X1) > 1 / sqrt(k eps)).
  const double thr = (double)k * 2.220446049250313e-16 * gmax;
  if (t < 64) {
    // Entries below the diagonal are updated too (they stay the symmetric
    // Schur complement) and are discarded at the end; columns past k hold
    // zeros, so their updates change nothing.
    double g[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) g[i] = sG[i + t * LD];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        double p = readlane_d(g[j], j);
        if (!(p > thr)) {
          if (t == 0) fail = 1;
          p = gmax > 0 ? gmax : 1.0;
        }
        const double ir = rsq_nr(p), rjj = p * ir;
        g[j] = (t == j) ? rjj : g[j] * ir;
        sRow[j & 1][t] = g[j];
        wave_sync();
#pragma unroll
        for (int aa = j + 1; aa < KMAX; ++aa) g[aa] = fma(-sRow[j & 1][aa], g[j], g[aa]);
      }
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) sG[i + t * LD] = (i <= t) ? g[i] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < 64 * 64; e += 256) sR[e] = sG[(e & 63) + (e >> 6) * LD];
  __syncthreads();
  if (fail) {
    if (t == 0 && wg == 0) {
      atomicOr(a.flags, DEV_RANK);
      st->done = 1;
    }
    return;
  }
  if (wg == 0)
    for (int e = t; e < k * k; e += 256) {
      const int r = e % k, c = e / k;
      a.R[e] = (r <= c) ? sR[r + c * 64] : 0.0;
    }
  double nb2 = 0.0;
  for (int jj = wg * 256 + t; k > 0 && jj < n2; jj += nwg * 256) {
    const double *pc = a.P + (int64_t)jj * k;
    double x[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) x[i] = pc[min(i, k - 1)];  // clamped; past k never used
    // B = R^-T P
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      if (i < k) {
        double s = x[i];
#pragma unroll
        for (int q = 0; q < i; ++q) s -= sR[q + i * 64] * x[q];
        x[i] = s * rcp_nr(sR[i + i * 64]);
      }
      // keep the reads of R inside their row (unrolled, the compiler would
      // otherwise hoist all of R into registers)
      asm volatile("" ::: "memory");
    }
    double *bc = a.B + (int64_t)jj * k;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < k) {
        bc[i] = x[i];
        nb2 += x[i] * x[i];
      }
    // C = R^-1 B (entries past k are zero on both sides)
#pragma unroll
    for (int i = KMAX - 1; i >= 0; --i) {
      if (i < k) {
        double s = x[i];
#pragma unroll
        for (int q = i + 1; q < KMAX; ++q) s -= sR[i + q * 64] * x[q];
        x[i] = s * rcp_nr(sR[i + i * 64]);
      }
      asm volatile("" ::: "memory");
    }
    double *cc = a.C + (int64_t)jj * k;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < k) cc[i] = x[i];
  }
  nb2 = block_sum(nb2, red);
  if (t == 0) {
    a.coef_part[wg] = nb2;
    if (wg == 0) st->trG1 = tr;
  }
}
// workgroups per instance of the coefficient step
__host__ __device__ inline int coef_groups(int n2) { return n2 > 256 ? (n2 + 255) / 256 : 1; }
template <int KMAX>
__global__ __launch_bounds__(256) void k_coef(SmallArgs a) {
  coef_body<KMAX>(a, blockIdx.x, gridDim.x);
}
// batch: blockIdx.y = instance; workgroups past an instance's count exit
template <int KMAX>
__global__ __launch_bounds__(256) void k_coef_b(const SmallArgs *__restrict__ av) {
  const SmallArgs &a = av[blockIdx.y];
  const int ng = coef_groups(a.n2);
  if ((int)blockIdx.x >= ng) return;
  coef_body<KMAX>(a, blockIdx.x, ng);
}

// -----------------------------------------------------------------------------
// M in the fragment-major layout of the eigen step (padding entries zero).
__device__ __forceinline__ void formM_body(int n2, int k, const double *__restrict__ GA,
                                           const double *__restrict__ B, double *__restrict__ M,
                                           const SmallState *st) {
  if (st->done) return;
  const int64_t total = mf_size(n2);
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < total;
       f += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    mf_rc(n2, (int)f, i, j);
    double v = 0.0;
    if (i < n2 && j < n2) {
      const double *bi = B + (int64_t)i * k, *bj = B + (int64_t)j * k;
      double s = 0.0;
      for (int c = 0; c < k; ++c) s = fma(bi[c], bj[c], s);
      v = GA[i + (int64_t)j * n2] - s;
    }
    M[f] = v;
  }
}
__global__ __launch_bounds__(256) void k_formM(int n2, int k, const double *__restrict__ GA,
                                               const double *__restrict__ B,
                                               double *__restrict__ M, const SmallState *st) {
  formM_body(n2, k, GA, B, M, st);
}
// batch: blockIdx.y = instance
__global__ __launch_bounds__(256) void k_formM_b(const SmallArgs *__restrict__ av) {
  const SmallArgs &a = av[blockIdx.y];
  formM_body(a.n2, a.k, a.GA, a.B, a.M, a.st);
}

// -----------------------------------------------------------------------------
// k_post (1024 threads).  The two long sums over n2 (CV = C V and S = C C^T)
// stage column chunks of C and row chunks of V through LDS, each thread
// owning fixed output entries; everything else is elementwise with short
// inner products.  Small matrices are column-major in the global scratch
// (CV, S, T, K^-1); the n2-row outputs are left to k_postz.

// In-place Cholesky (upper, K = R^T R) of a symmetric k x k matrix in LDS
// (ld 64) by wavefront 0: at step j lane c forms R_jc = K_cj / R_jj from
// column j (consecutive words), passes it to every lane through `row` (64
// doubles of LDS), writes it into row j, and then updates row c of the
// trailing block, both triangles (for each column the lanes touch
// consecutive words).  The pivot's reciprocal square root is the refined
// hardware estimate.
__device__ int small_chol64(double *K, int k, int *fail, double *row) {
  const int t = threadIdx.x;
  if (t == 0) *fail = 0;
  __syncthreads();
  if (t < 64) {
    for (int j = 0; j < k; ++j) {
      double p = K[j + j * 64];
      if (!(p > 0)) {
        if (t == 0) *fail = 1;
        p = 1.0;
      }
      const double ir = rsq_nr(p);
      const bool own = t > j && t < k;
      const double r = own ? K[t + j * 64] * ir : 0.0;
      row[t] = r;
      wave_sync();
      if (t == j) K[j + j * 64] = p * ir;
      if (own) {
        K[j + t * 64] = r;
        for (int c = j + 1; c < k; ++c) K[t + c * 64] -= r * row[c];
      }
      wave_sync();
    }
  }
  __syncthreads();
  return *fail;
}

#define POST_CH 7680
template <typename T>
__device__ __forceinline__ void post_body(const SmallArgs &a, const SmallOut<T> &o) {
  SmallState *st = a.st;
  if (st->done) return;
  __shared__ double sC[POST_CH];     // C chunk, k x cw (ld k)
  __shared__ double sV[4096];        // V chunk, cw x l (row-major)
  __shared__ double sK[64 * 64];     // K = w^2 I + S, then its Cholesky factor
  __shared__ double sKi[64 * 64];    // R^-1, then K^-1
  __shared__ int fail;
  const int k = a.k, n2 = a.n2, l = a.l, b = a.b, t = threadIdx.x;
  const double *V = a.Y;  // first l columns, ld n2
  double *ws = a.scratch;
  double *CV = ws;                       // k x l
  double *S = CV + 64 * 32;              // k x k
  double *Tm = S + 64 * 64;              // k x k
  double *Ki = Tm + 64 * 64;             // K^-1, k x k (constant weight)

  // ---- CV = C V and S = C C^T ----------------------------------------------
  // on the FP64 matrix cores: 16 x 16 output tiles (S: ceil(k/16)^2, CV:
  // ceil(k/16) x ceil(l/16)), one wavefront per tile, the inner index (the
  // n2 columns of C) in k-steps of 4, sixteen steps' reads in flight at once;
  // C (k x n2, ld k) and V (n2 x l, ld n2) are read from L2, clamped and
  // masked by zero factors.
  {
    typedef double pd4 __attribute__((ext_vector_type(4)));
    const int lane = t & 63, w = t >> 6, li = lane & 15, lk = lane >> 4;
    const int tk = (k + 15) / 16, tl = (l + 15) / 16;
    const int ntile = tk * tk + tk * tl;
    for (int tile = w; tile < ntile; tile += 16) {
      const bool isS = tile < tk * tk;
      const int tt = isS ? tile : tile - tk * tk;
      const int r0 = 16 * (tt % tk), c0 = 16 * (tt / tk);
      const int ra = min(r0 + li, max(k - 1, 0));
      const double ma = (r0 + li < k) ? 1.0 : 0.0;
      const int cb = isS ? min(c0 + li, max(k - 1, 0)) : min(c0 + li, max(l - 1, 0));
      const double mb = isS ? ((c0 + li < k) ? 1.0 : 0.0) : ((c0 + li < l) ? 1.0 : 0.0);
      pd4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int j0 = 0; j0 < n2; j0 += 64) {
        double av[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int jj = j0 + 4 * u + lk, jc = min(jj, n2 - 1);
          const double mj = (jj < n2) ? 1.0 : 0.0;
          av[u] = a.C[(int64_t)jc * k + ra] * (ma * mj);
          bv[u] = isS ? a.C[(int64_t)jc * k + cb] * mb : V[jc + (int64_t)cb * n2] * mb;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + lk + 4 * v, cc = c0 + li;  // output row lk + 4 v, column li
        if (isS) {
          if (rr < k && cc < k) S[rr + cc * k] = acc[v];
        } else if (rr < k && cc < l) {
          CV[rr + cc * k] = acc[v];
          sK[rr + cc * k] = acc[v];  // LDS copy of CV for T (k l <= 2048)
        }
      }
    }
  }
  __syncthreads();
  // ---- T = (CV)(CV)^T, Z = C^T - V (CV)^T --------------------------------------
  for (int e = t; e < k * k; e += 1024) {
    const int c = e % k, d = e / k;
    double s_ = 0.0;
    for (int q = 0; q < l; ++q) s_ = fma(sK[c + q * k], sK[d + q * k], s_);
    Tm[e] = s_;
  }
  __syncthreads();
  const bool constw = a.wconst > 0;
  if (constw) {
    // K^-1 = R^-1 R^-T with K = w^2 I + S = R^T R
    const double w2 = a.wconst * a.wconst;
    for (int e = t; e < k * k; e += 1024) {
      const int r = e % k, c = e / k;
      sK[r + c * 64] = S[e] + (r == c ? w2 : 0.0);
    }
    __syncthreads();
    small_chol64(sK, k, &fail, sKi);  // sKi is free until R^-1
    if (t < k) {
      const int c = t;
      for (int r = 0; r < k; ++r) sKi[r + c * 64] = 0.0;
      for (int r = c; r >= 0; --r) {
        double v = (r == c) ? 1.0 : 0.0;
        for (int q = r + 1; q <= c; ++q) v -= sK[r + q * 64] * sKi[q + c * 64];
        sKi[r + c * 64] = v / sK[r + r * 64];
      }
    }
    __syncthreads();
    for (int e = t; e < k * k; e += 1024) {  // K^-1 into sK (symmetric)
      const int r = e % k, c = e / k;
      double v = 0.0;
      for (int q = max(r, c); q < k; ++q) v = fma(sKi[r + q * 64], sKi[c + q * 64], v);
      sK[r + c * 64] = v;
    }
    __syncthreads();
    // S K^-1, T K^-1 (col-major k x k), each factor staged in LDS (sC is
    // free now; k*k <= 4096); Z K^-1 is formed by k_postz
    for (int e = t; e < k * k; e += 1024) {
      sC[e] = S[e];
      Ki[e] = sK[(e % k) + (e / k) * 64];
    }
    __syncthreads();
    for (int e = t; e < k * k; e += 1024) {
      const int r = e % k, c = e / k;
      double vs = 0.0;
      for (int q = 0; q < k; ++q) vs = fma(sC[r + q * k], sK[q + c * 64], vs);
      sKi[r + c * 64] = vs;      // S K^-1
    }
    __syncthreads();
    for (int e = t; e < k * k; e += 1024) sC[e] = Tm[e];
    __syncthreads();
    for (int e = t; e < k * k; e += 1024) {
      const int r = e % k, c = e / k;
      double vt = 0.0;
      for (int q = 0; q < k; ++q) vt = fma(sC[r + q * k], sK[q + c * 64], vt);
      sV[r + c * 64] = vt;       // T K^-1 (sV is free now)
    }
    __syncthreads();
    for (int e = t; e < k * k; e += 1024) {
      const int r = e % k, c = e / k;
      S[e] = sKi[r + c * 64];
      Tm[e] = sV[r + c * 64];
    }
    __syncthreads();
  }
  // typed copies for the row pass (row-major, input index first)
  for (int e = t; e < k * k; e += 1024) {
    const int r = e % k, c = e / k;  // S, Tm are col-major; store [r][c] row-major
    o.St[r * k + c] = (T)S[e];
    o.Tt[r * k + c] = (T)Tm[e];
    o.Gt[r * k + c] = (T)(-S[e]);
  }
  if (t == 0) {
    // F(X_p) = ||(A1 - X1) o W1||^2 + ||P^perp A2||^2 - sum of the top r-k
    // eigenvalues of M, with ||P^perp A2||^2 = ||A2||^2 - ||B||^2.
    double sth = 0.0;
    for (int q = 0; q < l; ++q) sth += a.theta[q];
    double nb2 = 0.0;  // ||B||^2 from the coefficient step's workgroups, in order
    const int ng = coef_groups(a.n2);
    for (int w = 0; w < ng; ++w) nb2 += a.coef_part[w];
    st->nB2 = nb2;
    st->F = st->f1 + st->trGA - st->nB2 - sth;
    st->nrmX2sq = st->nB2 + sth;
    st->nrmX = sqrt(st->trG1 + st->nB2 + sth);
    if (l == 0 || b <= l)
      st->gap = __builtin_inf();
    else
      st->gap = sqrt(fmax(a.theta[l - 1], 0.0)) - sqrt(fmax(a.theta[l], 0.0));
  }
}
template <typename T>
__global__ __launch_bounds__(1024) void k_post(SmallArgs a, SmallOut<T> o) { post_body<T>(a, o); }
template <typename T>
__global__ __launch_bounds__(1024) void k_post_b(const SmallArgs *__restrict__ av,
                                                 const SmallOut<T> *__restrict__ ov) {
  post_body<T>(av[blockIdx.x], ov[blockIdx.x]);
}

// The n2-row part of the small step, one workgroup per PZ_R rows j: the
// row-major copy of V, Z = (I - V V^T) C^T = C^T - V (CV)^T (kept in double
// for the change pass, typed for the X2 output), and the rows of the row-pass
// panel: Z K^-1 with a constant weight (K^-1 from k_post), else Z.  CV and
// K^-1 are staged in LDS; every product has k or l terms.
#define PZ_R 16
template <typename T>
__device__ __forceinline__ void postz_body(const SmallArgs &a, const SmallOut<T> &o, int bx) {
  SmallState *st = a.st;
  if (st->done) return;
  __shared__ double sCV[64 * 32];
  __shared__ double sKi[64 * 64];
  __shared__ double sVr[PZ_R * 32];
  __shared__ double sZ[PZ_R * 65];
  const int k = a.k, n2 = a.n2, l = a.l, t = threadIdx.x;
  const int j0 = bx * PZ_R, nr = min(PZ_R, n2 - j0);
  const double *CV = a.scratch;
  const double *Ki = a.scratch + 64 * 32 + 2 * 64 * 64;
  const bool constw = a.wconst > 0;
  for (int e = t; e < k * l; e += 256) sCV[e] = CV[e];
  if (constw)
    for (int e = t; e < k * k; e += 256) sKi[e] = Ki[e];
  const double *V = a.Y;  // first l columns, ld n2
  for (int e = t; e < nr * l; e += 256) {
    const int r = e % nr, q = e / nr, j = j0 + r;
    const double v = V[j + (int64_t)q * n2];
    sVr[r * 32 + q] = v;
    a.Vcur[(int64_t)j * l + q] = v;
    o.Vr[(int64_t)j * l + q] = (T)v;
  }
  __syncthreads();
  for (int e = t; e < nr * k; e += 256) {
    const int r = e / k, c = e - r * k, j = j0 + r;
    double s_ = a.C[(int64_t)j * k + c];
    for (int q = 0; q < l; ++q) s_ -= sVr[r * 32 + q] * sCV[c + q * k];
    sZ[r * 65 + c] = s_;
    a.Zcur[(int64_t)j * k + c] = s_;
    o.Zx[(int64_t)j * k + c] = (T)s_;
  }
  __syncthreads();
  for (int e = t; e < nr * k; e += 256) {
    const int r = e / k, c = e - r * k, j = j0 + r;
    double v = sZ[r * 65 + c];
    if (constw) {
      v = 0.0;
      for (int q = 0; q < k; ++q) v = fma(sZ[r * 65 + q], sKi[q + c * k], v);
    }
    o.Gt[(int64_t)k * k + (int64_t)j * k + c] = (T)v;
  }
}
template <typename T>
__global__ __launch_bounds__(256) void k_postz(SmallArgs a, SmallOut<T> o) {
  postz_body<T>(a, o, blockIdx.x);
}
// batch: blockIdx.y = instance; blocks past an instance's n2 rows exit
template <typename T>
__global__ __launch_bounds__(256) void k_postz_b(const SmallArgs *__restrict__ av,
                                                 const SmallOut<T> *__restrict__ ov) {
  const SmallArgs &a = av[blockIdx.y];
  if ((int)blockIdx.x * PZ_R >= a.n2) return;
  postz_body<T>(a, ov[blockIdx.y], blockIdx.x);
}

// Error_p and the stopping rule of Section 4.1:
//   Error_p = ||X_p - X_{p-1}||_F,  stop when Error_p < tol or
//   Error_p / ||X_{p-1}||_F < tol, or when p = max_sweeps.
// ||X1_p - X1_{p-1}||^2 comes from the row update (dx1), ||X2_p - X2_{p-1}||^2
// from the row pass k_change_q (partials in chg_part).
__device__ __forceinline__ void decide_body(const SmallArgs &a) {
  SmallState *st = a.st;
  if (st->done) return;
  __shared__ double red[4];
  double d2 = 0.0;
  if (st->have_prev)
    for (int i = threadIdx.x; i < a.nchg; i += 256) d2 += a.chg_part[i];
  d2 = block_sum(d2, red);
  if (threadIdx.x == 0) {
    int done = 0;
    if (st->have_prev) {
      const double err = sqrt(st->dx1 + d2);
      st->err = err;
      st->rel = st->nrmX_q > 0 ? err / st->nrmX_q : __builtin_inf();
      if (st->tol > 0 && (err < st->tol || st->rel < st->tol)) {
        done = 1;
        st->status = 0;
      }
    } else {
      st->err = 0.0;
      st->rel = 0.0;
    }
    if (!done && st->sweep >= st->max_sweeps) {
      done = 1;
      st->status = 1;
    }
    st->nrmX_q = st->nrmX;
    st->done = done;
    st->have_prev = 1;
    if (!done) st->sweep += 1;
  }
}
__global__ __launch_bounds__(256) void k_decide(SmallArgs a) { decide_body(a); }
// batch: then every instance's state is copied to stall[i] (one read-back)
__global__ __launch_bounds__(256) void k_decide_b(const SmallArgs *__restrict__ av,
                                                  SmallState *__restrict__ stall) {
  const SmallArgs &a = av[blockIdx.x];
  decide_body(a);
  __syncthreads();
  if (threadIdx.x == 0) __threadfence();
  __syncthreads();
  const int nw = (int)(sizeof(SmallState) / sizeof(int32_t));
  const int32_t *src = reinterpret_cast<const int32_t *>(a.st);
  int32_t *dst = reinterpret_cast<int32_t *>(stall + blockIdx.x);
  for (int e = threadIdx.x; e < nw; e += 256) dst[e] = src[e];
}

// -----------------------------------------------------------------------------
void launch_gastats(hipStream_t s, int n2, const double *GA, SmallState *st) {
  hipLaunchKernelGGL(k_gastats, dim3(1), dim3(1024), 0, s, n2, GA, st);
}

void launch_coef(hipStream_t s, const SmallArgs &a) {
  const dim3 g(coef_groups(a.n2));
  if (a.k <= 8) hipLaunchKernelGGL(k_coef<8>, g, dim3(256), 0, s, a);
  else if (a.k <= 16) hipLaunchKernelGGL(k_coef<16>, g, dim3(256), 0, s, a);
  else if (a.k <= 32) hipLaunchKernelGGL(k_coef<32>, g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_coef<64>, g, dim3(256), 0, s, a);
}

void launch_formM(hipStream_t s, const SmallArgs &a) {
  const int64_t total = mf_size(a.n2);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1024));
  hipLaunchKernelGGL(k_formM, dim3(g), dim3(256), 0, s, a.n2, a.k, a.GA, a.B, a.M, a.st);
}

void launch_decide(hipStream_t s, const SmallArgs &a) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, a);
}

template <typename T>
void launch_post(hipStream_t s, const SmallArgs &a, const SmallOut<T> &o) {
  hipLaunchKernelGGL(k_post<T>, dim3(1), dim3(1024), 0, s, a, o);
  if (a.n2 > 0)
    hipLaunchKernelGGL(k_postz<T>, dim3((a.n2 + PZ_R - 1) / PZ_R), dim3(256), 0, s, a, o);
}
template void launch_post<float>(hipStream_t, const SmallArgs &, const SmallOut<float> &);
template void launch_post<double>(hipStream_t, const SmallArgs &, const SmallOut<double> &);

// Batched launches: `count` instances whose argument blocks are consecutive
// in device memory (av); kmax: the common k class of the instances (8, 16,
// 32 or 64) for the coefficient kernel; n2max, the largest n2.
void launch_coef_b(hipStream_t s, int kmax, int count, int n2max, const SmallArgs *av) {
  if (count <= 0) return;
  const dim3 g(coef_groups(n2max), count);
  if (kmax <= 8) hipLaunchKernelGGL(k_coef_b<8>, g, dim3(256), 0, s, av);
  else if (kmax <= 16) hipLaunchKernelGGL(k_coef_b<16>, g, dim3(256), 0, s, av);
  else if (kmax <= 32) hipLaunchKernelGGL(k_coef_b<32>, g, dim3(256), 0, s, av);
  else hipLaunchKernelGGL(k_coef_b<64>, g, dim3(256), 0, s, av);
}

void launch_formM_b(hipStream_t s, int count, int n2max, const SmallArgs *av) {
  if (count <= 0) return;
  const int64_t total = mf_size(n2max);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 256));
  hipLaunchKernelGGL(k_formM_b, dim3(g, count), dim3(256), 0, s, av);
}

template <typename T>
void launch_post_b(hipStream_t s, int count, int n2max, const SmallArgs *av,
                   const SmallOut<T> *ov) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_post_b<T>, dim3(count), dim3(1024), 0, s, av, ov);
  if (n2max > 0)
    hipLaunchKernelGGL(k_postz_b<T>, dim3((n2max + PZ_R - 1) / PZ_R, count), dim3(256), 0, s, av,
                       ov);
}
template void launch_post_b<float>(hipStream_t, int, int, const SmallArgs *,
                                   const SmallOut<float> *);
template void launch_post_b<double>(hipStream_t, int, int, const SmallArgs *,
                                    const SmallOut<double> *);

void launch_decide_b(hipStream_t s, int count, const SmallArgs *av, SmallState *stall) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_decide_b, dim3(count), dim3(256), 0, s, av, stall);
}
