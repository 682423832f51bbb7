// Host-side launcher prototypes shared by the kernel files and the API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"

template <typename T>
struct UpdateArgs {
  int64_t m;
  int k, n;
  const T *A;
  int64_t lda;
  const T *W1;
  int64_t ldw;
  T wc;
  bool constw;
  const T *X1o;
  T *X1n;
  const T *Gt, *Tt, *St;   // Gt = [-S; Z] (n x k), Tt = T, St = S (row-major)
  T *Eb;                   // m x k right-hand sides of the per-row solve
  const bf16s *A2b;        // mixed precision: A2 in BF16 (ld ldb); NULL: A2 = A + k lda
  int64_t ldb;
  const bf16s *Zh, *Zl;    // with A2b: Z ~ Zh + Zl in BF16, [column][row], rows padded to n2p
  int n2p;
  double *part;
  const SmallState *st;
  int *flags;
};

template <typename T>
void launch_validate(hipStream_t s, int64_t m, int64_t n, const T *A, int64_t lda, int64_t k,
                     const T *W1, int64_t ldw, int *flags, bf16s *A2b, const T *W2 = nullptr,
                     T *As = nullptr);
template <typename T>
void launch_init_x1(hipStream_t s, int64_t m, int64_t k, int mode, uint64_t seed, const T *src,
                    int64_t lds, T *X1, int *flags, const int *gate = nullptr);
// part[split] = X[rows]^T Y[rows] (k1 x k2), then out = the sum of the
// splits in order.  With Y2, Y's columns from ky1 on are Y2's (ld ldy2).
template <typename TX, typename TY>
void launch_tsgemm(hipStream_t s, int64_t m, const TX *X, int64_t ldx, int k1, const TY *Y,
                   int64_t ldy, int k2, int sym, int splits, int64_t rows_per_split, double *part,
                   double *out, const int *skip, const TY *Y2 = nullptr, int64_t ldy2 = 0,
                   int ky1 = 0);
template <typename T>
void launch_f1(hipStream_t s, int64_t m, int k, const T *A, int64_t lda, const T *W1, int64_t ldw,
               double wc, const T *X1, double *part, int nwg);
template <typename T>
void launch_update(hipStream_t s, const UpdateArgs<T> &a);
struct UpdatePlan {
  int nl;      // Cholesky lanes per round
  int grows;   // G elements staged per chunk
  size_t shm;  // dynamic LDS bytes
};
template <typename T>
UpdatePlan update_plan(int k, bool constw);
// Output columns of the row update's tiles for k (16, 32 or 64): the column
// count of the BF16 panel Zh, Zl.
int update_panel_kp(int k);
// Zh + Zl ~ Z from the panel Gt = [-S; Z] (float), for the BF16 row update.
void launch_panel_bf16(hipStream_t s, int n2, int k, int n2p, const float *Gt, bf16s *Zh,
                       bf16s *Zl, const SmallState *st);
template <typename T>
void launch_x2(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
               const T *X1, const T *Zt, const T *Vr, T *X2, int64_t ldx2, const T *w2,
               uint8_t *mask, int64_t ldm, T tau);
template <typename T>
void launch_copy_out(hipStream_t s, int64_t m, int64_t k, const T *src, T *dst, int64_t ld);

// Small-step kernels (k_small.hip, k_eig.hip).
// The eigen step's matrix M (n2 x n2, symmetric, double) is stored
// fragment-major for v_mfma_f64_16x16x4f64: 16-row tiles, then pairs of
// 4-column k-steps, then the 64 lanes of a wavefront, then the pair, so that
// the A operand of two consecutive k-steps is one contiguous 16-byte read per
// lane (lane = 16 * (column % 4) + row % 16).  The k-steps are padded to a
// multiple of 8; entries past n2 are zero.
__host__ __device__ inline int64_t mf_kq2(int n2) { return (((n2 + 3) / 4 + 7) & ~7) / 2; }
__host__ __device__ inline int64_t mf_size(int n2) {
  return (int64_t)((n2 + 15) / 16) * mf_kq2(n2) * 128;
}
__host__ __device__ inline int64_t mf_idx(int n2, int i, int j) {
  const int q = j >> 2;
  return ((((int64_t)(i >> 4) * mf_kq2(n2) + (q >> 1)) * 64 + (j & 3) * 16 + (i & 15)) << 1) + (q & 1);
}
// (row, column) of fragment-major offset f (< 2^31 for n2 <= WLRA_NMAX)
__host__ __device__ inline void mf_rc(int n2, int f, int &i, int &j) {
  const int h = f & 1, lane = (f >> 1) & 63;
  const int T = f >> 7, kq2 = (int)mf_kq2(n2);
  const int rt = T / kq2;
  i = rt * 16 + (lane & 15);
  j = 4 * (2 * (T - rt * kq2) + h) + (lane >> 4);
}

struct SmallArgs {
  int k, n2, l, b;
  int nparts;              // workgroups of the last row pass (f1, dx1 pairs)
  const double *upd_part;  // [nparts][2]
  int nchg;                // workgroups of the last change pass
  const double *chg_part;  // [nchg]
  const double *G1, *P, *GA;
  double *R, *B, *C, *M;
  double *Y, *Wb, *F0, *F1, *F2, *theta;
  double *Zcur, *Vcur;     // this sweep's Z (n2 x k) and V (n2 x l), row-major double
  double *scratch;         // k_post workspace
  SmallState *st;
  int *flags;
  double wconst;           // > 0: constant W1
  int eig_maxit, eig_deg;
  int eig_one_wg;          // 1: the one-workgroup eigen kernel for every n2
  double *epart;           // partial Grams of the multi-workgroup eigen kernel
  double *coef_part;       // ||B||^2 per coefficient workgroup (WLRA_NMAX / 256 + 1)
};

template <typename T>
struct SmallOut {
  T *Gt, *Tt, *St, *Vr;  // row-pass operands (K^-1 folded in when W1 is constant):
                         // Gt = [-S; Z] is n x k row-major
  T *Zx;                 // plain Z = (I - V V^T) C^T for the dense X2 output
};

// Arguments of the change pass's small step (k_chgprep), one per instance
// of a batch.
struct ChgArgs {
  int n2, k, l;
  const double *Vp, *Vq, *Zp, *Zq;
  double *Hb, *Kg;
  const SmallState *st;
};

// Batched small steps: one launch for `count` instances whose argument
// blocks are consecutive in device memory.
void launch_coef_b(hipStream_t s, int kmax, int count, int n2max, const SmallArgs *av);
void launch_formM_b(hipStream_t s, int count, int n2max, const SmallArgs *av);
void launch_eig_b(hipStream_t s, int count, const SmallArgs *av);
template <typename T>
void launch_post_b(hipStream_t s, int count, int n2max, const SmallArgs *av, const SmallOut<T> *ov);
void launch_decide_b(hipStream_t s, int count, const SmallArgs *av, SmallState *stall);
void launch_chgprep_b(hipStream_t s, int count, const ChgArgs *av);
// The BF16 panel of one instance of a batch (k_panel_bf16).
struct PanelArgs {
  int n2, k, kp, n2p;
  const float *Gt;
  bf16s *Zh, *Zl;
  const SmallState *st;
};
void launch_panel_bf16_b(hipStream_t s, int count, const PanelArgs *av);


void launch_coef(hipStream_t s, const SmallArgs &a);
void launch_formM(hipStream_t s, const SmallArgs &a);
void launch_eig(hipStream_t s, const SmallArgs &a);
// Multi-workgroup eigen kernel (k_eigmw.hip) for n2 >= EIG_MW_MIN: 16 rows of
// M per workgroup; partial Grams need 2 x workgroups x WLRA_BMAX^2 doubles.
#define EIG_MW_MIN 256
int eig_mw_groups(int n2);
hipError_t launch_eig_mw(hipStream_t s, const SmallArgs &a);
template <typename T>
void launch_post(hipStream_t s, const SmallArgs &a, const SmallOut<T> &o);
void launch_gastats(hipStream_t s, int n2, const double *GA, SmallState *st);
void launch_decide(hipStream_t s, const SmallArgs &a);
// Learned warm start (k_learn.hip).
template <typename T>
void launch_gauss_fill(hipStream_t s, int64_t count, uint64_t seed, double scale, T *out);
void launch_fill_zero(hipStream_t s, int64_t count, float *out);
template <typename T>
void launch_sketch_finish(hipStream_t s, int n, const double *P1, const T *Ps, float *out);
void launch_gemm(hipStream_t s, int mode, int M, int N, int K, const float *A, int lda,
                 const float *B, int ldb, float *C, int ldc, const float *bias, int relu,
                 const float *mask, int ldm);
void launch_colsum(hipStream_t s, int M, int N, const float *A, float *out);
void launch_subspace_loss(hipStream_t s, int n, int r, int batch, const float *y, const float *T,
                          double lam, float *gy, double *loss_part, int *flags);
void launch_eig_seed(hipStream_t s, int n2, int l, int b, const double *V, int64_t ldv, int v0,
                     double *Y);
void launch_adam(hipStream_t s, int64_t P, float *p, const float *g, float *m, float *v, float lr,
                 double b1, double b2, float eps, float bc1, float bc2);
template <typename T>
void launch_ldecode(hipStream_t s, int n, int k, int r, const float *yv, T *Gt, T *Tt, T *St,
                    int *flags);
template <typename T>
void launch_zero(hipStream_t s, int64_t count, T *out);

// Error_p through a Gram of aligned factor differences (k_stream.hip): the
// aligned basis's columns [V_p dV] into Hb and its Gram Kg in one workgroup.
void launch_chgprep(hipStream_t s, int n2, int k, int l, const double *Vp, const double *Vq,
                    const double *Zp, const double *Zq, double *Hb, double *Kg,
                    const SmallState *st);
template <typename T>
void launch_change_qr(hipStream_t s, int64_t m, int k, int n2, int l, const T *A, int64_t lda,
                      const T *X1p, const T *X1q, const double *Hb, const double *Kg,
                      double *part, const SmallState *st);
