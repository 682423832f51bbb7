// Shared device helpers and the workspace layout of libwlra (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WLRA_KMAX 64      // largest k (columns of A1) the row kernels hold in registers
#define WLRA_BMAX 32      // largest eigen block (r - k + guard)
#define WLRA_NMAX 4096    // largest n - k

// Device status bits (ws.flags[0]).
#define DEV_BAD_A 1
#define DEV_BAD_W 2
#define DEV_RANK 4
#define DEV_EIG_ORTH 8     // the eigen step's block orthonormalisation failed
#define DEV_ROWSOLVE 16    // a per-row system of the X1 update had a pivot <= 0
#define DEV_LEARN_FAIL 32

// Learned warm start: sketch Om^T A Ps with Om m x 16 and Ps n x 32 (Philox
// N(0,1) draws under fixed keys), network 512 -> 256 -> 256 -> n r.
#define LEARN_SK_ROWS 16
#define LEARN_SK_COLS 32
#define LEARN_D_IN 512
#define LEARN_HID 256
#define LEARN_RMAX 32
#define LEARN_SEED_OMEGA 0x5EEDA001ull
#define LEARN_SEED_PSI 0x5EEDA002ull

// BF16 storage of A2 in mixed precision: the bit pattern of the upper half of
// an IEEE float.  Widening to float is exact; narrowing rounds to nearest
// even (inputs are checked finite before it matters).
struct bf16s {
  uint16_t u;
};

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ double to_f(double x) { return x; }
__device__ __forceinline__ float to_f(bf16s x) { return __uint_as_float((uint32_t)x.u << 16); }
__device__ __forceinline__ bf16s bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16s{(uint16_t)(u >> 16)};
}

// 1 / x and 1 / sqrt(x) to a few ulps: the hardware estimates (about 23
// correct bits) refined by two Newton steps each.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Per-solve device state shared by the small-step kernels (all double).
// Index p below is the sweep of Algorithm 1: X_p = [X1_p, X1_p C_p + D_p].
struct SmallState {
  double f1;          // ||(A1 - X1_p) o W1||^2
  double dx1;         // ||X1_p - X1_{p-1}||^2
  double trGA;        // trace(A2^T A2) = ||A2||_F^2
  double nrmGA;       // ||A2^T A2||_F
  double nB2;         // ||B_p||_F^2 = ||P_{X1_p} A2||_F^2
  double trG1;        // ||X1_p||_F^2
  double F;           // objective F(X_p) of problem (5)
  double err;         // Error_p = ||X_p - X_{p-1}||_F
  double rel;         // Error_p / ||X_{p-1}||_F
  double nrmX;        // ||X_p||_F
  double nrmX2sq;     // ||X2_p||_F^2
  double nrmX2sq_q;   // ||X2_{p-1}||_F^2
  double nrmX_q;      // ||X_{p-1}||_F
  double gap;         // sigma_l - sigma_{l+1} of P^perp A2
  double tol;         // stopping threshold (Section 4.1)
  double eig_floor;   // absolute residual target of the eigen step
  int32_t sweep;      // p
  int32_t done;       // 1 once X_p is final
  int32_t status;     // 0 converged, 1 max sweeps
  int32_t max_sweeps;
  int32_t eig_iters;  // filter rounds, summed over sweeps
  int32_t have_prev;  // 1 when the (p-1) quantities are valid
  int32_t eig_first;  // 1 until the eigen block holds a warm start
  int32_t eig_matvecs;  // products M y (single vectors), summed over sweeps
  int32_t eig_fail;   // 1 when this sweep's eigen step stopped at its round
                      // limit with a wanted Ritz pair above its residual target
  int32_t pad_;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum; `red` is LDS of at least blockDim.x/64 doubles.  All
// threads get the result.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based generator.
__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t key[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * ctr[0];
    const uint64_t p1 = (uint64_t)M1 * ctr[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    const uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    ctr[0] = n0; ctr[1] = lo1; ctr[2] = n2; ctr[3] = lo0;
    key[0] += W0; key[1] += W1;
  }
}

// Two N(0,1) draws for element pair `idx` (Box-Muller on Philox output).
__device__ __forceinline__ void philox_normal2(uint64_t seed, uint64_t idx, double &z0, double &z1) {
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), 0u, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  philox4x32_10(ctr, key);
  const double inv = 1.0 / 4294967296.0;
  double u0 = ((double)ctr[0] + 0.5) * inv + ((double)ctr[1]) * inv * inv;
  double u1 = ((double)ctr[2] + 0.5) * inv + ((double)ctr[3]) * inv * inv;
  const double rad = sqrt(-2.0 * log(u0));
  const double ang = 6.283185307179586476925 * u1;
  z0 = rad * cos(ang);
  z1 = rad * sin(ang);
}

// Deterministic value in [-1, 1) from (i, j) for eigen-block starts.
__device__ __forceinline__ double hash_unit(uint32_t i, uint32_t j) {
  uint32_t h = i * 0x9E3779B1u ^ (j + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}
