// C-ABI of libwlra: argument checks, workspace, and the sweep loop of
// Algorithm 1 driven from the host with one small device-to-host read of the
// sweep state per sweep.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/wlra.h"
#include "common.h"
#include "launch.h"

#define WLRA_VERSION 200
#define EIG_GUARD 3
#define EIG_DEG 20
#define EIG_MAXIT 60
// Mixed precision: the sweeps whose X1 update takes its A2 product from the
// BF16 copy stop at max(tol, MIXED_TOL) before the exact refinement sweep.
// Every small step (eigen step included, at the full tolerance) is exact, so
// X_p at the end of that phase needs no re-evaluation.
#define MIXED_TOL 1e-5
#define WLRA_BATCH_LANES_DEFAULT 4
#define WLRA_BATCH_LANES_MAX 16

// Workspace of wlra_solve_noalloc (for callers that cannot allocate): one
// copy of this array per device, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: it uses the device
// address that hipGetSymbolAddress returned for that device (kept in
// g_scratch_dev, set up by wlra_create with the device current).
#define WLRA_NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) char scratch[WLRA_NOALLOC_SCRATCH_BYTES];
static void *g_scratch_dev[WLRA_NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Look up (once per device, with `device` current) the address of `scratch`.
static void scratch_setup(int device) {
  if (device < 0 || device >= WLRA_NOALLOC_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device] != nullptr) return;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr != nullptr)
    g_scratch_dev[device] = ptr;
  else
    (void)hipGetLastError();  // wlra_solve_noalloc reports WLRA_E_HIP
}

static void *scratch_ptr(int device) {
  if (device < 0 || device >= WLRA_NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

enum KernelKind {
  KK_VALIDATE, KK_INIT, KK_GRAM, KK_GAST, KK_XTA, KK_F1, KK_COEF, KK_FORMM, KK_EIG,
  KK_POST, KK_CHANGE, KK_DECIDE, KK_UPDATE, KK_X2, KK_COPY, KK_LEARN, KK_CHGQR, KK_COUNT
};
static const char *kKernelNames[KK_COUNT] = {
    "validate", "init_x1", "gram_A2", "gram_stats", "gram_X1", "objective_f1",
    "coef", "form_M", "eig", "post", "change", "decide", "update", "x2_out", "copy_out",
    "learned_init", "change_qr"};

struct ProfEvent {
  int kind;
  hipEvent_t e0, e1;
  double bytes, flops;  // algorithmic HBM bytes and flops of the launch
};

struct wlra_ctx {
  int device = 0;
  // batched solves: streams used by wlra_solve_batched (the handle's and extra ones)
  int batch_lanes = WLRA_BATCH_LANES_DEFAULT;
  // batch engine: streams besides the handle's, events, workspace slices
  // and pinned argument/state blocks (grown at the start of a batch call)
  std::vector<hipStream_t> bstreams;
  std::vector<hipEvent_t> bjoin, bdone;
  char *bws = nullptr;
  size_t bws_bytes = 0;
  char *bhost = nullptr;
  size_t bhost_bytes = 0;
  bool owns_stream = false;
  hipStream_t stream = nullptr;
  int precision = 0;
  uint32_t flags = 0;
  // options (wlra_set_option)
  int eig_maxit = EIG_MAXIT;
  int eig_one_wg = 0;
  // autotuner (WLRA_OPT_AUTOTUNE): workgroup targets of the tall-skinny
  // products per (m, n2, k, element size, BF16 copy), measured once
  int autotune = 1;
  std::map<std::array<int64_t, 5>, std::pair<int, int>> tune;
  hipEvent_t tev0 = nullptr, tev1 = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  uint64_t ws_epoch = 0;  // counts the allocations of ws
  // the learned start's Gaussian sketch matrices (fixed seeds) in ws, kept
  // from the last solve on ws while its layout (hence their place) is the
  // same and ws has not been reallocated; any other solve on ws drops them
  bool sk_valid = false;
  const void *sk_om = nullptr;
  int64_t sk_m = -1, sk_n = -1;
  size_t sk_total = 0;
  uint64_t sk_epoch = 0;
  char *lws = nullptr;  // learned warm start: sketch and training buffers
  size_t lws_bytes = 0;
  SmallState *st_host = nullptr;  // pinned
  int *flags_host = nullptr;      // pinned
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // profiling (WLRA_FLAG_PROFILE)
  std::vector<hipEvent_t> pool;
  std::vector<ProfEvent> pending;
  int64_t launches[KK_COUNT] = {};
  double ms[KK_COUNT] = {};
  double bytes[KK_COUNT] = {};
  double flops[KK_COUNT] = {};
};

static hipEvent_t prof_event(wlra_ctx *h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold finished event pairs into the totals (call after a stream sync).
static void prof_collect(wlra_ctx *h) {
  for (auto &pe : h->pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pe.e0, pe.e1) == hipSuccess) {
      h->ms[pe.kind] += t;
      h->launches[pe.kind] += 1;
      h->bytes[pe.kind] += pe.bytes;
      h->flops[pe.kind] += pe.flops;
    }
    h->pool.push_back(pe.e0);
    h->pool.push_back(pe.e1);
  }
  h->pending.clear();
}

// Run `stmt` (one kernel launch) between two events when profiling, and
// tally the launch's algorithmic bytes and flops.
#define PROFW(h, kind, nbytes, nflops, stmt)                       \
  do {                                                             \
    if ((h)->flags & WLRA_FLAG_PROFILE) {                          \
      ProfEvent pe{kind, prof_event(h), prof_event(h), (double)(nbytes), (double)(nflops)}; \
      if (pe.e0 && pe.e1) hipEventRecord(pe.e0, (h)->stream);       \
      stmt;                                                        \
      if (pe.e0 && pe.e1) {                                        \
        hipEventRecord(pe.e1, (h)->stream);                        \
        (h)->pending.push_back(pe);                                \
      }                                                            \
    } else {                                                       \
      stmt;                                                        \
    }                                                              \
  } while (0)
#define PROF(h, kind, stmt) PROFW(h, kind, 0, 0, stmt)
// The same on a given stream (events recorded on `strm`).
#define PROFWS(h, strm, kind, nbytes, nflops, stmt)                \
  do {                                                             \
    if ((h)->flags & WLRA_FLAG_PROFILE) {                          \
      ProfEvent pe{kind, prof_event(h), prof_event(h), (double)(nbytes), (double)(nflops)}; \
      if (pe.e0 && pe.e1) hipEventRecord(pe.e0, (strm));           \
      stmt;                                                        \
      if (pe.e0 && pe.e1) {                                        \
        hipEventRecord(pe.e1, (strm));                             \
        (h)->pending.push_back(pe);                                \
      }                                                            \
    } else {                                                       \
      stmt;                                                        \
    }                                                              \
  } while (0)

namespace {

struct Layout {
  size_t off[40];
  size_t total;
  int n = 0;
  size_t add(size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct Sizes {
  int64_t m, n, k, r, n2, l, b;
  int splits_ga, splits_p;
  int64_t rows_ga, rows_p;
  int tiles_ga, tiles_p;          // output tiles of A2^T A2 and X1^T A2
  int splits_ga_max, splits_p_max;  // at the largest autotuner target
  int nwg_upd, nwg_f1;
  size_t elt;
  bool mixed;
  bool learned;
  bool colw;  // column weights of the unweighted block: A staged scaled
  int splits_l1;  // Om^T A of the learned start's sketch
  int64_t rows_l1;
};

struct Ptrs {
  void *X1[2];
  double *part, *GA, *P, *G1, *R, *B, *C, *M;
  double *Y, *Wb, *F0, *F1, *F2, *theta, *scratch, *upd_part, *chg_part;
  double *Zd[2], *Vd[2];
  void *Gt, *Tt, *St, *Vr, *Zx, *Eb;
  bf16s *Ab;  // mixed precision: BF16 copy of A2 (m x n2), else NULL
  bf16s *Zh, *Zl;  // mixed precision: the row update's panel Z in two BF16 terms
  void *As;   // column weights: [A1, A2 diag(W2)] (m x n), else NULL
  double *Hb, *Rh;  // change pass: aligned basis [V_p dV Z_p dZ] and its Gram
  double *epart;    // multi-workgroup eigen kernel: partial Grams
  double *coef_part;  // ||B||^2 per workgroup of the coefficient step
  // learned warm start (NULL unless the start is learned)
  void *Om, *Ps;
  double *P1, *lpart;
  float *sk, *lh1, *lh2, *yv;
  SmallState *st;
  int *flags;
};

// Row splits of a tall-skinny product: about `target` workgroups in all
// (2048 by default: eight per CU, so that each walks few row chunks), at
// least 256 rows each.  The autotuner picks the target per shape.
#define TUNE_TARGET_MAX 4096
int choose_splits(int64_t m, int tiles, int64_t *rows, int target = 2048) {
  int s = (int)std::max<int64_t>(1, std::min<int64_t>((target + tiles - 1) / tiles, (m + 255) / 256));
  int64_t r = (m + s - 1) / s;
  r = (r + 31) / 32 * 32;
  s = (int)((m + r - 1) / r);
  *rows = r;
  return std::max(1, s);
}

Sizes make_sizes(int64_t m, int64_t n, int64_t k, int64_t r, size_t elt, bool mixed,
                 bool learned = false, bool colw = false) {
  Sizes z;
  z.mixed = mixed;
  z.learned = learned;
  z.colw = colw;
  z.m = m; z.n = n; z.k = k; z.r = r; z.n2 = n - k; z.l = r - k;
  z.b = z.l > 0 ? std::min<int64_t>(z.n2, z.l + EIG_GUARD) : 0;
  const int tga = (int)(((z.n2 + 31) / 32) * ((z.n2 + 31) / 32 + 1) / 2);
  z.tiles_ga = std::max(1, tga);
  z.splits_ga = choose_splits(m, z.tiles_ga, &z.rows_ga);
  const int tp = (int)(((std::max<int64_t>(k, 1) + 31) / 32) * ((z.n2 + 31) / 32));
  z.tiles_p = std::max(1, tp);
  z.splits_p = choose_splits(m, z.tiles_p, &z.rows_p);
  {
    int64_t rr;
    z.splits_ga_max = std::max(z.splits_ga, choose_splits(m, z.tiles_ga, &rr, TUNE_TARGET_MAX));
    z.splits_p_max = std::max(z.splits_p, choose_splits(m, z.tiles_p, &rr, TUNE_TARGET_MAX));
  }
  z.splits_l1 = choose_splits(m, (int)((n + 31) / 32), &z.rows_l1);
  z.nwg_upd = (int)((m + 63) / 64);
  z.nwg_f1 = 256;
  z.elt = elt;
  return z;
}

// Rows of the BF16 panel: n2 padded to the row update's chunk of 32.
inline int64_t panel_rows(int64_t n2) { return (std::max<int64_t>(n2, 1) + 31) / 32 * 32; }

// Device workspace of one solve, in allocation order (256-byte aligned).
Layout make_layout(const Sizes &z, Ptrs *P, char *base) {
  Layout L{};
  L.total = 0;
  const size_t d = sizeof(double);
  const int64_t m = z.m, k = z.k, n2 = z.n2, l = z.l;
  const int64_t kk = std::max<int64_t>(k, 1), ll = std::max<int64_t>(l, 1);
  const size_t part = std::max<size_t>((size_t)z.splits_ga_max * n2 * n2,
                                       (size_t)z.splits_p_max * kk * (kk + n2));
  struct Item { void **dst; size_t bytes; };
  Ptrs p{};
  Item items[] = {
      {&p.X1[0], (size_t)(m * kk) * z.elt},
      {&p.X1[1], (size_t)(m * kk) * z.elt},
      {(void **)&p.part, part * d},
      {(void **)&p.GA, (size_t)(n2 * n2) * d},
      // X1^T [X1 A2] = [G1 P]: G1 (k x k) and P (k x n2), both ld k, in one
      // block (one product forms both)
      {(void **)&p.G1, (size_t)(kk * (kk + n2)) * d},
      {(void **)&p.R, (size_t)(kk * kk) * d},
      {(void **)&p.B, (size_t)(kk * n2) * d},
      {(void **)&p.C, (size_t)(kk * n2) * d},
      {(void **)&p.M, (size_t)mf_size((int)n2) * d},
      {(void **)&p.Y, (size_t)(n2 * WLRA_BMAX) * d},
      {(void **)&p.Wb, (size_t)(n2 * WLRA_BMAX) * d},
      {(void **)&p.F0, (size_t)(n2 * WLRA_BMAX) * d},
      {(void **)&p.F1, (size_t)(n2 * WLRA_BMAX) * d},
      {(void **)&p.F2, (size_t)(n2 * WLRA_BMAX) * d},
      {(void **)&p.theta, (size_t)WLRA_BMAX * d},
      {(void **)&p.scratch, (size_t)(2048 + 3 * 4096) * d},
      {(void **)&p.upd_part, (size_t)2 * std::max(z.nwg_upd, z.nwg_f1) * d},
      {(void **)&p.chg_part, (size_t)z.nwg_upd * d},
      {(void **)&p.Zd[0], (size_t)(n2 * kk) * d},
      {(void **)&p.Zd[1], (size_t)(n2 * kk) * d},
      {(void **)&p.Vd[0], (size_t)(n2 * ll) * d},
      {(void **)&p.Vd[1], (size_t)(n2 * ll) * d},
      {&p.Gt, (size_t)((n2 + kk) * kk) * z.elt},
      {&p.Eb, (size_t)(m * kk) * z.elt},
      {&p.Tt, (size_t)(kk * kk) * z.elt},
      {&p.St, (size_t)(kk * kk) * z.elt},
      {&p.Vr, (size_t)(n2 * ll) * z.elt},
      {&p.Zx, (size_t)(n2 * kk) * z.elt},
      {(void **)&p.st, sizeof(SmallState)},
      {(void **)&p.flags, 64},
      {(void **)&p.Ab, z.mixed ? (size_t)(m * n2) * sizeof(bf16s) : 0},
      {(void **)&p.Zh, z.mixed ? (size_t)update_panel_kp((int)kk) * panel_rows(n2) * sizeof(bf16s) : 0},
      {(void **)&p.Zl, z.mixed ? (size_t)update_panel_kp((int)kk) * panel_rows(n2) * sizeof(bf16s) : 0},
      {&p.As, z.colw ? (size_t)(m * z.n) * z.elt : 0},
      {(void **)&p.Hb, (size_t)(n2 * (2 * l + 2 * k)) * d},
      {(void **)&p.coef_part, (size_t)(WLRA_NMAX / 256 + 1) * d},
      {(void **)&p.Rh, (size_t)((2 * l + 2 * k) * (2 * l + 2 * k)) * d},
      {(void **)&p.epart,
       (l > 0 && eig_mw_groups((int)n2) > 0)
           ? (size_t)2 * eig_mw_groups((int)n2) * WLRA_BMAX * WLRA_BMAX * d
           : 0},
      {&p.Om, z.learned ? (size_t)(m * LEARN_SK_ROWS) * z.elt : 0},
      {&p.Ps, z.learned ? (size_t)(z.n * LEARN_SK_COLS) * z.elt : 0},
      {(void **)&p.P1, z.learned ? (size_t)(LEARN_SK_ROWS * z.n) * d : 0},
      {(void **)&p.lpart,
       z.learned ? (size_t)z.splits_l1 * LEARN_SK_ROWS * z.n * d : 0},
      {(void **)&p.sk, z.learned ? (size_t)LEARN_D_IN * sizeof(float) : 0},
      {(void **)&p.lh1, z.learned ? (size_t)LEARN_HID * sizeof(float) : 0},
      {(void **)&p.lh2, z.learned ? (size_t)LEARN_HID * sizeof(float) : 0},
      {(void **)&p.yv, z.learned ? (size_t)(z.n * z.r) * sizeof(float) : 0},
  };
  for (auto &it : items) {
    const size_t off = L.add(it.bytes);
    *it.dst = (base && it.bytes) ? (void *)(base + off) : nullptr;
  }
  p.P = p.G1 ? p.G1 + kk * kk : nullptr;
  if (P) *P = p;
  return L;
}

int ensure_ws(wlra_ctx *h, size_t bytes) {
  if (bytes <= h->ws_bytes) return WLRA_OK;
  if (h->ws) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return WLRA_E_HIP;
    hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  const size_t want = bytes + bytes / 4;
  ++h->ws_epoch;
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    h->ws = nullptr;
    return WLRA_E_NOMEM;
  }
  h->ws_bytes = want;
  return WLRA_OK;
}

size_t workspace_bytes(const wlra_problem &p, int precision) {
  const Sizes z = make_sizes(p.m, p.n, p.k, p.r, precision == WLRA_FP64 ? 8 : 4,
                             precision == WLRA_MIXED_BF16,
                             p.k > 0 && p.init == WLRA_INIT_LEARNED,
                             p.W2 != nullptr && p.n > p.k);
  return make_layout(z, nullptr, nullptr).total;
}

int check_problem(const wlra_problem *p, int precision) {
  if (p == nullptr) return WLRA_E_ARG;
  if (precision < WLRA_FP64 || precision > WLRA_MIXED_BF16) return WLRA_E_ARG;
  const int64_t m = p->m, n = p->n, k = p->k, r = p->r;
  if (m < 1 || n < 1 || k < 0 || r < k || r > std::min(m, n)) return WLRA_E_ARG;
  if (k > WLRA_KMAX) return WLRA_E_ARG;
  const int64_t l = r - k, n2 = n - k;
  if (l > WLRA_BMAX - EIG_GUARD) return WLRA_E_ARG;
  if (l > 0 && n2 > 1024) return WLRA_E_ARG;
  if (n2 > WLRA_NMAX) return WLRA_E_ARG;
  if (p->A == nullptr || p->lda < m) return WLRA_E_ARG;
  if (k > 0 && p->W1 != nullptr && p->ldw < m) return WLRA_E_ARG;
  if (k > 0 && p->W1 == nullptr && !(p->w1_const > 0 && isfinite(p->w1_const))) return WLRA_E_WEIGHT;
  if (p->max_sweeps < 0) return WLRA_E_ARG;
  if (k > 0 && (p->X1_out == nullptr || p->ldx1 < m)) return WLRA_E_ARG;
  if (p->X2_out != nullptr && p->ldx2 < m) return WLRA_E_ARG;
  if (p->init < WLRA_INIT_RANDOM || p->init > WLRA_INIT_LEARNED) return WLRA_E_ARG;
  if (k > 0 && p->init == WLRA_INIT_LEARNED && (p->model == nullptr || r > LEARN_RMAX))
    return WLRA_E_ARG;
  if (k > 0 && p->init == WLRA_INIT_GIVEN && (p->X1_init == nullptr || p->ldx0 < m)) return WLRA_E_ARG;
  if (!(p->tol == p->tol)) return WLRA_E_ARG;
  if (p->mask_out != nullptr && (p->ldm < m || !(p->mask_tau >= 0 && isfinite(p->mask_tau))))
    return WLRA_E_ARG;
  if (p->V_init != nullptr && l > 0 &&
      (p->v0_rows < 1 || p->v0_rows > n2 || p->ldv0 < p->v0_rows))
    return WLRA_E_ARG;
  return WLRA_OK;
}

#define HIPCHK(x)                         \
  do {                                    \
    if ((x) != hipSuccess) return WLRA_E_HIP; \
  } while (0)

// Batch resources, grown before a batch's first kernel (never during its
// sweeps): `ns - 1` extra streams (default priority) and their join events.
int ensure_batch_streams(wlra_ctx *h, int ns) {
  while ((int)h->bstreams.size() < ns - 1) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return WLRA_E_HIP;
    h->bstreams.push_back(st);
  }
  while ((int)h->bjoin.size() < ns) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return WLRA_E_HIP;
    h->bjoin.push_back(e);
  }
  return WLRA_OK;
}

int ensure_batch_ws(wlra_ctx *h, size_t bytes) {
  if (bytes <= h->bws_bytes) return WLRA_OK;
  if (h->bws) {
    if (hipDeviceSynchronize() != hipSuccess) return WLRA_E_HIP;
    (void)hipFree(h->bws);
    h->bws = nullptr;
    h->bws_bytes = 0;
  }
  const size_t want = bytes + bytes / 8;
  if (hipMalloc(&h->bws, want) != hipSuccess) {
    h->bws = nullptr;
    return WLRA_E_NOMEM;
  }
  h->bws_bytes = want;
  return WLRA_OK;
}

// Pinned host blocks of a batch and one completion event per instance.
int ensure_batch_host(wlra_ctx *h, size_t bytes, int count) {
  if (bytes > h->bhost_bytes) {
    if (h->bhost) {
      if (hipDeviceSynchronize() != hipSuccess) return WLRA_E_HIP;
      (void)hipHostFree(h->bhost);
      h->bhost = nullptr;
      h->bhost_bytes = 0;
    }
    if (hipHostMalloc((void **)&h->bhost, bytes, hipHostMallocDefault) != hipSuccess) {
      h->bhost = nullptr;
      return WLRA_E_NOMEM;
    }
    h->bhost_bytes = bytes;
  }
  while ((int)h->bdone.size() < count) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return WLRA_E_HIP;
    h->bdone.push_back(e);
  }
  return WLRA_OK;
}

// Per-instance state of one solve of Algorithm 1 and the steps that enqueue
// its kernels.  A single solve (wlra_solve) drives one Run from the host,
// reading the sweep state once per sweep; the batch engine
// (wlra_solve_batched) drives many Runs in lockstep, with the single-workgroup
// small steps of all of them in one launch each.
template <typename T>
struct Run {
  wlra_ctx *h = nullptr;
  const wlra_problem *pr = nullptr;
  wlra_result *res = nullptr;
  hipStream_t s = nullptr;     // stream of this instance's own launches
  SmallState *sh = nullptr;    // host copy of the sweep state (pinned)
  bool mixed = false, learned = false, colw = false, constw = false;
  Sizes z{};
  Ptrs P{};
  int64_t m = 0, k = 0, n2 = 0, l = 0, b = 0, lda = 0;
  const T *A = nullptr, *A2 = nullptr, *W1 = nullptr, *W2 = nullptr;
  double wc = 0.0, eig_tol = 0.0, es = 0.0, md = 0.0, kd = 0.0, n2d = 0.0;
  T *X1c = nullptr;
  int cur = 0, nparts = 0, p = 0, max_sweeps = 0, mixed_status = 0, rc_tune = 0;
  bool may_tune = true;  // false: no new autotuner entries (nothing allocates)
  bool on_bf16 = false;  // the X1 update's A2 product on the BF16 copy
  SmallArgs sa{};
  SmallOut<T> so{};

  // Validation, start, the one-time Gram and the sums of sweep 0.  Returns
  // a negative status on a launch failure.
  int begin(wlra_ctx *h_, const wlra_problem *pr_, wlra_result *res_, char *ws, hipStream_t s_,
            SmallState *sh_) {
    h = h_; pr = pr_; res = res_; s = s_; sh = sh_;
    mixed = (h->precision == WLRA_MIXED_BF16);
    learned = (pr->k > 0 && pr->init == WLRA_INIT_LEARNED);
    colw = (pr->W2 != nullptr && pr->n > pr->k);
    z = make_sizes(pr->m, pr->n, pr->k, pr->r, sizeof(T), mixed, learned, colw);
    const size_t total = make_layout(z, &P, ws).total;
    // the sketch matrices survive in the handle's own workspace from the
    // last solve of the same layout; every other solve there drops them
    bool sketch_kept = false;
    if (ws == h->ws) {
      sketch_kept = learned && h->sk_valid && h->sk_om == P.Om && h->sk_m == pr->m &&
                    h->sk_n == pr->n && h->sk_total == total && h->sk_epoch == h->ws_epoch;
      h->sk_valid = false;  // set again once this solve's sketch matrices are enqueued
      h->sk_om = P.Om; h->sk_m = pr->m; h->sk_n = pr->n; h->sk_total = total;
      h->sk_epoch = h->ws_epoch;
    }
    m = z.m; k = z.k; n2 = z.n2; l = z.l; b = z.b;
    // with column weights every pass after validation reads the staged
    // [A1, A2 diag(W2)] (leading dimension m) in place of A
    A = colw ? static_cast<const T *>(P.As) : static_cast<const T *>(pr->A);
    lda = colw ? m : pr->lda;
    A2 = A + k * lda;
    W2 = colw ? static_cast<const T *>(pr->W2) : nullptr;
    W1 = (k > 0) ? static_cast<const T *>(pr->W1) : nullptr;
    constw = (k > 0 && W1 == nullptr);
    wc = constw ? pr->w1_const : 0.0;
    es = (double)sizeof(T); md = (double)m; kd = (double)k; n2d = (double)n2;

    launch_zero<int>(s, 16, P.flags);  // a fill kernel, no memset node
    memset(sh, 0, sizeof(SmallState));
    // Mixed precision runs the sweeps on the BF16 copy of A2 with a looser
    // threshold and one sweep fewer, then refines in exact arithmetic.
    max_sweeps = (k > 0) ? pr->max_sweeps : 0;
    sh->tol = (mixed && pr->tol > 0) ? std::max(pr->tol, MIXED_TOL) : pr->tol;
    sh->max_sweeps = mixed ? std::max(max_sweeps - 1, 0) : max_sweeps;
    sh->eig_first = 1;
    if (pr->V_init != nullptr && l > 0) {
      // the first eigen step starts from the given block (orthonormalised there)
      launch_eig_seed(s, (int)n2, (int)l, (int)b, pr->V_init, pr->ldv0, (int)pr->v0_rows, P.Y);
      sh->eig_first = 2;
    }
    eig_tol = pr->eig_tol > 0 ? pr->eig_tol
                              : (h->precision == WLRA_FP64 ? 64.0 * 2.220446049250313e-16 : 1e-10);
    sh->eig_floor = eig_tol;
    HIPCHK(hipMemcpyAsync(P.st, sh, sizeof(SmallState), hipMemcpyHostToDevice, s));

    // algorithmic bytes per launch of the streaming kernels (each operand
    // read or written once)
    PROFWS(h, s, KK_VALIDATE,
           md * (double)pr->n * es + (W1 ? md * kd * es : 0.0) + (mixed ? md * n2d * 2.0 : 0.0), 0,
           launch_validate<T>(s, m, pr->n, static_cast<const T *>(pr->A), pr->lda, k, W1, pr->ldw,
                              P.flags, P.Ab, W2, static_cast<T *>(P.As)));
    X1c = static_cast<T *>(P.X1[0]);
    int *lflag = nullptr;  // learned start: the random start is its fallback
    if (learned) {
      // Y = network(sketch of A), the predicted row basis; X1_0 is the
      // per-row weighted least-squares fit in span(Y^T): k_ldecode forms the
      // row update's operands, the row-update kernels solve the k x k systems.
      const int64_t n = pr->n;
      const float *W1m = pr->model, *b1 = W1m + LEARN_HID * LEARN_D_IN;
      const float *W2m = b1 + LEARN_HID, *b2 = W2m + LEARN_HID * LEARN_HID;
      const float *W3m = b2 + LEARN_HID, *b3 = W3m + n * z.r * LEARN_HID;
      T *Om = static_cast<T *>(P.Om), *Ps = static_cast<T *>(P.Ps);
      T *Gt = static_cast<T *>(P.Gt), *Tt = static_cast<T *>(P.Tt), *St = static_cast<T *>(P.St);
      T *X1z = static_cast<T *>(P.X1[1]);
      // the decode's failures (k_ldecode, or a per-row solve) go to a flag
      // word of their own, which gates the random start that replaces it
      lflag = P.flags + 1;
      auto seq = [&]() {
        if (!sketch_kept) {
          launch_gauss_fill<T>(s, m * LEARN_SK_ROWS, LEARN_SEED_OMEGA, 1.0, Om);
          launch_gauss_fill<T>(s, n * LEARN_SK_COLS, LEARN_SEED_PSI, 1.0, Ps);
        }
        launch_tsgemm<T, T>(s, m, Om, m, LEARN_SK_ROWS, A, lda, (int)n, 0, z.splits_l1,
                            z.rows_l1, P.lpart, P.P1, nullptr);
        launch_sketch_finish<T>(s, (int)n, P.P1, Ps, P.sk);
        launch_gemm(s, 0, 1, LEARN_HID, LEARN_D_IN, P.sk, LEARN_D_IN, W1m, LEARN_D_IN, P.lh1,
                    LEARN_HID, b1, 1, nullptr, 0);
        launch_gemm(s, 0, 1, LEARN_HID, LEARN_HID, P.lh1, LEARN_HID, W2m, LEARN_HID, P.lh2,
                    LEARN_HID, b2, 1, nullptr, 0);
        launch_gemm(s, 0, 1, (int)(n * z.r), LEARN_HID, P.lh2, LEARN_HID, W3m, LEARN_HID, P.yv,
                    (int)(n * z.r), b3, 0, nullptr, 0);
        launch_ldecode<T>(s, (int)n, (int)k, (int)z.r, P.yv, Gt, Tt, St, lflag);
        // the fit's X1 term multiplies T = 0, so any finite m x k matrix
        // (ld m) serves as its X1: A1 itself when A's leading dimension is m
        // (a non-finite A is rejected by the validation pass), zeros else
        const T *X1fit = X1z;
        if (lda == m)
          X1fit = A;
        else
          launch_zero<T>(s, m * k, X1z);
        UpdateArgs<T> ua{};
        ua.m = m; ua.k = (int)k; ua.n = (int)n; ua.A = A; ua.lda = lda; ua.W1 = W1;
        ua.ldw = pr->ldw; ua.wc = (T)wc; ua.constw = constw; ua.X1o = X1fit; ua.X1n = X1c;
        ua.Gt = Gt; ua.Tt = Tt; ua.St = St; ua.part = P.upd_part; ua.st = P.st;
        ua.Eb = static_cast<T *>(P.Eb);
        ua.A2b = nullptr;
        ua.ldb = m;
        ua.flags = lflag;
        launch_update<T>(s, ua);
      };
      PROFWS(h, s, KK_LEARN, 0, 0, seq());
      if (ws == h->ws) h->sk_valid = true;
    }
    if (k > 0) {
      const int mode = (pr->init == WLRA_INIT_RANDOM || pr->init == WLRA_INIT_LEARNED) ? 0 : 1;
      const T *src = pr->init == WLRA_INIT_GIVEN ? static_cast<const T *>(pr->X1_init) : A;
      const int64_t lds = pr->init == WLRA_INIT_GIVEN ? pr->ldx0 : lda;
      PROFWS(h, s, KK_INIT, 0, 0,
             launch_init_x1<T>(s, m, k, mode, pr->seed, src, lds, X1c, P.flags, lflag));
    }
    on_bf16 = mixed;  // the mixed phase: BF16 in the X1 update's A2 product only
    rc_tune = tune_products();
    if (rc_tune != WLRA_OK) return rc_tune;
    gram_A2();
    // eig_floor is relative to ||A2^T A2||_F; k_gastats scales it.
    PROFWS(h, s, KK_GAST, 0, 0, launch_gastats(s, (int)n2, P.GA, P.st));
    if (k > 0) {
      gram_X1(X1c);
      PROFWS(h, s, KK_F1, 0, 0,
             launch_f1<T>(s, m, (int)k, A, lda, W1, pr->ldw, wc, X1c, P.upd_part, z.nwg_f1));
      nparts = z.nwg_f1;
    }
    sa = SmallArgs{};
    sa.k = (int)k; sa.n2 = (int)n2; sa.l = (int)l; sa.b = (int)b;
    sa.G1 = P.G1; sa.P = P.P; sa.GA = P.GA;
    sa.R = P.R; sa.B = P.B; sa.C = P.C; sa.M = P.M;
    sa.Y = P.Y; sa.Wb = P.Wb; sa.F0 = P.F0; sa.F1 = P.F1; sa.F2 = P.F2; sa.theta = P.theta;
    sa.scratch = P.scratch; sa.st = P.st; sa.flags = P.flags; sa.wconst = constw ? wc : 0.0;
    sa.eig_maxit = h->eig_maxit; sa.eig_deg = EIG_DEG;
    sa.eig_one_wg = h->eig_one_wg;
    sa.epart = P.epart;
    sa.coef_part = P.coef_part;
    sa.upd_part = P.upd_part; sa.chg_part = P.chg_part; sa.nchg = z.nwg_upd;
    so = SmallOut<T>{static_cast<T *>(P.Gt), static_cast<T *>(P.Tt), static_cast<T *>(P.St),
                     static_cast<T *>(P.Vr), static_cast<T *>(P.Zx)};
    cur = 0;
    p = 0;
    mixed_status = 0;
    return WLRA_OK;
  }

  // Autotuner: the workgroup target (512 .. 4096) of the X1^T A2 product
  // and of the A2^T A2 Gram, each timed once per shape on this instance's own
  // operands (the products' results are overwritten by the solve), then
  // reused for every later solve of that shape on the handle.  Different
  // targets sum the rows in different orders, so results are reproducible
  // per handle.
  int tune_products() {
    if (!h->autotune || n2 == 0) return WLRA_OK;
    const std::array<int64_t, 5> key{m, n2, k, (int64_t)sizeof(T), 0};
    auto it = h->tune.find(key);
    int tp = 0, tg = 0;
    if (it != h->tune.end()) {
      tp = it->second.first;
      tg = it->second.second;
    } else {
      if (!may_tune) return WLRA_OK;
      static const int cand[4] = {512, 1024, 2048, TUNE_TARGET_MAX};
      float best_p = 1e30f, best_g = 1e30f;
      for (int c : cand) {
        int64_t rp, rg;
        const int sp = choose_splits(m, z.tiles_p, &rp, c);
        const int sg = choose_splits(m, z.tiles_ga, &rg, c);
        float tms_p = 0.f, tms_g = 0.f;
        if (k > 0) {
          auto xta = [&]() {
            launch_tsgemm<T, T>(s, m, X1c, m, (int)k, A2, lda, (int)n2, 0, sp, rp, P.part, P.P,
                                nullptr);
          };
          xta();
          HIPCHK(hipEventRecord(h->tev0, s));
          for (int rep = 0; rep < 3; ++rep) xta();
          HIPCHK(hipEventRecord(h->tev1, s));
          HIPCHK(hipEventSynchronize(h->tev1));
          HIPCHK(hipEventElapsedTime(&tms_p, h->tev0, h->tev1));
          if (tms_p < best_p) { best_p = tms_p; tp = c; }
        }
        auto gram = [&]() {
          launch_tsgemm<T, T>(s, m, A2, lda, (int)n2, A2, lda, (int)n2, 1, sg, rg, P.part, P.GA,
                              nullptr);
        };
        gram();
        HIPCHK(hipEventRecord(h->tev0, s));
        gram();
        HIPCHK(hipEventRecord(h->tev1, s));
        HIPCHK(hipEventSynchronize(h->tev1));
        HIPCHK(hipEventElapsedTime(&tms_g, h->tev0, h->tev1));
        if (tms_g < best_g) { best_g = tms_g; tg = c; }
      }
      h->tune[key] = {tp, tg};
    }
    if (tp > 0) z.splits_p = choose_splits(m, z.tiles_p, &z.rows_p, tp);
    if (tg > 0) z.splits_ga = choose_splits(m, z.tiles_ga, &z.rows_ga, tg);
    return WLRA_OK;
  }

  // Input checks of the validation pass (after a synchronisation).
  static int input_status(int dflags) {
    if (dflags & DEV_BAD_W) return WLRA_E_WEIGHT;
    if (dflags & DEV_BAD_A) return WLRA_E_NONFINITE;
    return WLRA_OK;
  }

  // One-time Gram of the unweighted block: A2^T A2 (always of A2 itself:
  // M = G_A - B^T B subtracts two numbers of the size of the background
  // energy, so both come from the same data in every precision).
  void gram_A2() {
    PROFWS(h, s, KK_GRAM, md * n2d * es, md * n2d * n2d,
           (launch_tsgemm<T, T>(s, m, A2, lda, (int)n2, A2, lda, (int)n2, 1, z.splits_ga,
                                z.rows_ga, P.part, P.GA, nullptr)));
  }
  // X1^T [X1 A2] = [G1 P] (k x (k + n2)) for the next small step: one
  // product over the rows of X1 and A2 (X1 read once for both).
  void gram_X1(const T *X1) {
    PROFWS(h, s, KK_XTA, md * (kd + n2d) * es, 2.0 * md * kd * (kd + n2d),
           (launch_tsgemm<T, T>(s, m, X1, m, (int)k, X1, m, (int)(k + n2), 0, z.splits_p,
                                z.rows_p, P.part, P.G1, nullptr, A2, lda, (int)k)));
  }

  // Arguments of sweep p's small step.
  void small_args() {
    sa.nparts = nparts;
    sa.Zcur = P.Zd[p & 1];
    sa.Vcur = P.Vd[p & 1];
  }
  // Small step for sweep p on this instance's stream: R, B, C from the Grams
  // of X1_p; the top r-k eigenpairs of (P^perp A2)^T (P^perp A2); Z, T, S
  // and F(X_p).
  void small_single() {
    PROFWS(h, s, KK_COEF, 0, 0, launch_coef(s, sa));
    if (l > 0) {
      PROFWS(h, s, KK_FORMM, 0, 0, launch_formM(s, sa));
      PROFWS(h, s, KK_EIG, 0, 0, launch_eig(s, sa));
    }
    PROFWS(h, s, KK_POST, 0, 0, launch_post<T>(s, sa, so));
  }
  // BF16 phase: Z ~ Zh + Zl for the row update's BF16 products.
  void panel() {
    if constexpr (std::is_same<T, float>::value) {
      if (on_bf16 && k > 0)
        PROFWS(h, s, KK_POST, 0, 0,
               launch_panel_bf16(s, (int)n2, (int)k, (int)panel_rows(n2), so.Gt, P.Zh, P.Zl,
                                 P.st));
    }
  }
  bool panel_needed() const { return std::is_same<T, float>::value && on_bf16 && k > 0; }
  PanelArgs panel_args() const {
    return PanelArgs{(int)n2, (int)k, update_panel_kp((int)k), (int)panel_rows(n2),
                     reinterpret_cast<const float *>(so.Gt), P.Zh, P.Zl, P.st};
  }
  bool change_needed() const { return p > 0; }
  ChgArgs chg_args() const {
    return ChgArgs{(int)n2, (int)k, (int)l, P.Vd[p & 1], P.Vd[(p & 1) ^ 1], P.Zd[p & 1],
                   P.Zd[(p & 1) ^ 1], P.Hb, P.Rh, P.st};
  }
  // Error_p: the aligned basis and its Gram (one workgroup), then the row
  // pass.  batched_prep: the one-workgroup part ran in a batch launch.
  void change(bool batched_prep) {
    if (!batched_prep)
      PROFWS(h, s, KK_CHGQR, 0, 0,
             launch_chgprep(s, (int)n2, (int)k, (int)l, P.Vd[p & 1], P.Vd[(p & 1) ^ 1],
                            P.Zd[p & 1], P.Zd[(p & 1) ^ 1], P.Hb, P.Rh, P.st));
    PROFWS(h, s, KK_CHANGE, md * (n2d * es + 2.0 * kd * es),
           md * (4.0 * (double)l * n2d +
                 (2.0 * (double)l + 2.0 * kd) * (2.0 * (double)l + 2.0 * kd)),
           launch_change_qr<T>(s, m, (int)k, (int)n2, (int)l, A, lda, X1c,
                               static_cast<const T *>(P.X1[cur ^ 1]), P.Hb, P.Rh, P.chg_part,
                               P.st));
  }

  // Host side of sweep p after its state is in *sh: the trace, and the end
  // of the mixed phase.  Returns 1 when X_p is final, 0 when the X1 update
  // follows.
  int after_decide() {
    if (pr->trace && p <= pr->max_sweeps) {
      pr->trace[p] = sh->F;
      pr->trace[pr->max_sweeps + 1 + p] = sh->err;
    }
    if (sh->done && on_bf16) {
      // End of the mixed phase at X1_p.  Its small step was exact already
      // (only the X1 updates used the BF16 copy), so one more X1 update in
      // exact arithmetic (the refinement sweep) follows within max_sweeps.
      mixed_status = sh->status;
      on_bf16 = false;
      if (p >= max_sweeps) return 1;
      sh->done = 0;
      sh->sweep = p + 1;  // the decision did not count the sweep it ended on
      sh->tol = pr->tol;
      sh->max_sweeps = p + 1;
      (void)hipMemcpyAsync(P.st, sh, sizeof(SmallState), hipMemcpyHostToDevice, s);
      return 0;
    }
    return sh->done ? 1 : 0;
  }

  // X1_{p+1} from X1_p (Algorithm 1 steps 7-9), then the sums for p+1.
  void update() {
    T *X1n = static_cast<T *>(P.X1[cur ^ 1]);
    UpdateArgs<T> ua{};
    ua.m = m; ua.k = (int)k; ua.n = (int)pr->n; ua.A = A; ua.lda = lda; ua.W1 = W1;
    ua.ldw = pr->ldw; ua.wc = (T)wc; ua.constw = constw; ua.X1o = X1c; ua.X1n = X1n;
    ua.Gt = so.Gt; ua.Tt = so.Tt; ua.St = so.St; ua.part = P.upd_part; ua.st = P.st;
    ua.Eb = static_cast<T *>(P.Eb);
    ua.A2b = on_bf16 ? P.Ab : nullptr;
    ua.ldb = m;
    ua.Zh = on_bf16 ? P.Zh : nullptr;
    ua.Zl = on_bf16 ? P.Zl : nullptr;
    ua.n2p = (int)panel_rows(n2);
    ua.flags = P.flags;
    // reads A1, A2, X1_p (and W1), writes X1_{p+1}; the product
    // [A1 A2 X1] [-S; Z; T] and, for a matrix W1, the per-row SPD solves
    PROFWS(h, s, KK_UPDATE,
           md * (n2d * (on_bf16 ? 2.0 : es) + (3.0 + (constw ? 0.0 : 1.0)) * kd * es),
           2.0 * md * ((double)pr->n + kd) * kd +
               (constw ? 0.0 : md * (kd * kd * kd / 3.0 + 2.0 * kd * kd)),
           launch_update<T>(s, ua));
    gram_X1(X1n);
    nparts = z.nwg_upd;
    cur ^= 1;
    X1c = X1n;
    ++p;
  }

  // Failure flags of the device (after a synchronisation).
  static int device_status(int dflags) {
    // a failed row solve first: a rank-deficient X1 can follow from it
    if (dflags & DEV_ROWSOLVE) return WLRA_E_ROWSOLVE;
    if (dflags & DEV_RANK) return WLRA_E_RANK;
    if (dflags & DEV_EIG_ORTH) return WLRA_E_EIG;
    return WLRA_OK;
  }
  // Outputs of the returned X_p.
  int outputs() {
    if (k > 0)
      PROFWS(h, s, KK_COPY, 0, 0,
             launch_copy_out<T>(s, m, k, X1c, static_cast<T *>(pr->X1_out), pr->ldx1));
    if (pr->factors_out != nullptr) {
      // R (k x k), C (k x n2), V (n2 x l), theta (l): the returned X_p's factors
      double *f = pr->factors_out;
      const size_t d = sizeof(double);
      if (k > 0) {
        HIPCHK(hipMemcpyAsync(f, P.R, (size_t)(k * k) * d, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(f + k * k, P.C, (size_t)(k * n2) * d, hipMemcpyDeviceToDevice, s));
      }
      if (l > 0) {
        HIPCHK(hipMemcpyAsync(f + k * k + k * n2, P.Y, (size_t)(n2 * l) * d,
                              hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(f + k * k + k * n2 + n2 * l, P.theta, (size_t)l * d,
                              hipMemcpyDeviceToDevice, s));
      }
    }
    if (pr->X2_out != nullptr || pr->mask_out != nullptr)
      PROFWS(h, s, KK_X2, 0, 0,
             launch_x2<T>(s, m, (int)k, (int)n2, (int)l, A, lda, X1c, so.Zx, so.Vr,
                          static_cast<T *>(pr->X2_out), pr->ldx2, W2, pr->mask_out, pr->ldm,
                          (T)pr->mask_tau));
    return WLRA_OK;
  }
  // The result record (ms: the caller's measurement).
  int result(float ms) {
    int status = (k == 0) ? WLRA_OK : (mixed ? mixed_status : sh->status);
    // the eigen step of the returned X_p's sweep (each step sets eig_fail)
    if (sh->eig_fail) status = WLRA_INEXACT;
    if (res) {
      res->status = status;
      res->sweeps = sh->sweep;
      res->objective = sh->F;
      res->abs_change = sh->err;
      res->rel_change = sh->rel;
      res->gap = sh->gap;
      res->ms = ms;
      res->eig_iters = sh->eig_iters;
      res->eig_matvecs = sh->eig_matvecs;
    }
    return status;
  }
};

// One solve.  ws: a workspace of at least make_layout(...).total bytes.
template <typename T>
int solve_impl(wlra_ctx *h, const wlra_problem *pr, wlra_result *res, char *ws,
               bool may_tune = true) {
  hipStream_t s = h->stream;
  HIPCHK(hipEventRecord(h->ev0, s));
  Run<T> r;
  r.may_tune = may_tune;
  int rc = r.begin(h, pr, res, ws, s, h->st_host);
  if (rc != WLRA_OK) return rc;
  // the input checks' flags come back with the first sweep's state (one
  // synchronisation fewer; the sweep's kernels are harmless on bad input)
  bool inputs_checked = false;
  for (;;) {
    r.small_args();
    r.small_single();
    r.panel();
    if (r.change_needed()) r.change(false);
    PROFWS(h, s, KK_DECIDE, 0, 0, launch_decide(s, r.sa));
    HIPCHK(hipMemcpyAsync(h->st_host, r.P.st, sizeof(SmallState), hipMemcpyDeviceToHost, s));
    if (!inputs_checked)
      HIPCHK(hipMemcpyAsync(h->flags_host, r.P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!inputs_checked) {
      inputs_checked = true;
      rc = Run<T>::input_status(*h->flags_host);
      if (rc != WLRA_OK) return rc;
    }
    prof_collect(h);
    const int d = r.after_decide();
    if (d == 1) break;
    r.update();
  }
  // outputs, the device flags and the end event under one synchronisation;
  // a failure status then means the outputs must not be used
  rc = r.outputs();
  if (rc != WLRA_OK) return rc;
  HIPCHK(hipMemcpyAsync(h->flags_host, r.P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(h->ev1, s));
  HIPCHK(hipEventSynchronize(h->ev1));
  rc = Run<T>::device_status(*h->flags_host);
  if (rc != WLRA_OK) return rc;
  prof_collect(h);
  float ms = 0.f;
  hipEventElapsedTime(&ms, h->ev0, h->ev1);
  return r.result(ms);
}

// ---------------------------------------------------------------------------
// Batch engine (wlra_solve_batched): every instance is a Run with its own
// workspace slice.  The instances advance one sweep per round in lockstep:
// the single-workgroup small steps of all active instances (coefficients,
// M, the eigen step, the post step, the change pass's basis, the decision)
// run as one launch each, one workgroup per instance, so that a batch of
// clips fills the device where one clip's small step uses one CU; the
// streaming passes of each instance are enqueued on the batch streams
// (round robin); one read-back of all sweep states per round drives the
// host side (trace, end of the mixed phase, which instances update).
template <typename T>
int batch_impl(wlra_ctx *h, int count, const wlra_problem *probs, wlra_result *res) {
  const int ns = std::max(1, std::min(h->batch_lanes, count));
  int rc = ensure_batch_streams(h, ns);
  if (rc != WLRA_OK) return rc;
  std::vector<hipStream_t> strm(ns);
  strm[0] = h->stream;
  for (int j = 1; j < ns; ++j) strm[j] = h->bstreams[j - 1];
  // workspace slices, argument blocks, state copies
  std::vector<size_t> off(count);
  size_t tot = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = tot;
    tot += (workspace_bytes(probs[i], h->precision) + 255) & ~(size_t)255;
  }
  const size_t a_sa = ((size_t)count * sizeof(SmallArgs) + 255) & ~(size_t)255;
  const size_t a_so = ((size_t)count * sizeof(SmallOut<T>) + 255) & ~(size_t)255;
  const size_t a_ch = ((size_t)count * sizeof(ChgArgs) + 255) & ~(size_t)255;
  const size_t a_st = ((size_t)count * sizeof(SmallState) + 255) & ~(size_t)255;
  const size_t a_pa = ((size_t)count * sizeof(PanelArgs) + 255) & ~(size_t)255;
  const size_t dev_bytes = tot + 2 * a_sa + a_so + a_ch + a_st + a_pa;
  rc = ensure_batch_ws(h, dev_bytes);
  if (rc != WLRA_OK) return rc;
  const size_t host_bytes = 2 * a_sa + a_so + a_ch + 2 * a_st + a_pa + (size_t)count * sizeof(int);
  rc = ensure_batch_host(h, host_bytes, count);
  if (rc != WLRA_OK) return rc;
  char *dws = h->bws;
  SmallArgs *av_d = reinterpret_cast<SmallArgs *>(dws + tot);
  SmallArgs *ae_d = reinterpret_cast<SmallArgs *>(dws + tot + a_sa);
  SmallOut<T> *ov_d = reinterpret_cast<SmallOut<T> *>(dws + tot + 2 * a_sa);
  ChgArgs *ch_d = reinterpret_cast<ChgArgs *>(dws + tot + 2 * a_sa + a_so);
  SmallState *stall_d = reinterpret_cast<SmallState *>(dws + tot + 2 * a_sa + a_so + a_ch);
  PanelArgs *pa_d = reinterpret_cast<PanelArgs *>(dws + tot + 2 * a_sa + a_so + a_ch + a_st);
  char *hb = h->bhost;
  SmallArgs *av_h = reinterpret_cast<SmallArgs *>(hb);
  SmallArgs *ae_h = reinterpret_cast<SmallArgs *>(hb + a_sa);
  SmallOut<T> *ov_h = reinterpret_cast<SmallOut<T> *>(hb + 2 * a_sa);
  ChgArgs *ch_h = reinterpret_cast<ChgArgs *>(hb + 2 * a_sa + a_so);
  SmallState *stall_h = reinterpret_cast<SmallState *>(hb + 2 * a_sa + a_so + a_ch);
  SmallState *sh_h = reinterpret_cast<SmallState *>(hb + 2 * a_sa + a_so + a_ch + a_st);
  PanelArgs *pa_h = reinterpret_cast<PanelArgs *>(hb + 2 * a_sa + a_so + a_ch + 2 * a_st);
  int *flags_h = reinterpret_cast<int *>(hb + 2 * a_sa + a_so + a_ch + 2 * a_st + a_pa);

  // ordering helpers: main waits for the other streams, or they for main
  auto join = [&]() -> int {
    for (int j = 1; j < ns; ++j) {
      HIPCHK(hipEventRecord(h->bjoin[j], strm[j]));
      HIPCHK(hipStreamWaitEvent(strm[0], h->bjoin[j], 0));
    }
    return WLRA_OK;
  };
  auto fork = [&]() -> int {
    HIPCHK(hipEventRecord(h->bjoin[0], strm[0]));
    for (int j = 1; j < ns; ++j) HIPCHK(hipStreamWaitEvent(strm[j], h->bjoin[0], 0));
    return WLRA_OK;
  };

  HIPCHK(hipEventRecord(h->ev0, strm[0]));
  rc = fork();
  if (rc != WLRA_OK) return rc;
  std::vector<Run<T>> runs(count);
  std::vector<int> state(count, 0);  // 0 active, 1 finished, -1 failed
  for (int i = 0; i < count; ++i) {
    rc = runs[i].begin(h, &probs[i], &res[i], dws + off[i], strm[i % ns], &sh_h[i]);
    if (rc != WLRA_OK) return rc;
    HIPCHK(hipMemcpyAsync(&flags_h[i], runs[i].P.flags, sizeof(int), hipMemcpyDeviceToHost,
                          runs[i].s));
  }
  for (int j = 0; j < ns; ++j) HIPCHK(hipStreamSynchronize(strm[j]));
  prof_collect(h);
  for (int i = 0; i < count; ++i) {
    const int st = Run<T>::input_status(flags_h[i]);
    if (st != WLRA_OK) {
      memset(&res[i], 0, sizeof(wlra_result));
      res[i].status = st;
      state[i] = -1;
    }
  }
  std::vector<int> order, eig_list, chg_list, pan_list;
  for (;;) {
    order.clear();
    for (int i = 0; i < count; ++i)
      if (state[i] == 0) order.push_back(i);
    if (order.empty()) break;
    // instances by coefficient class (the kernel's k bound), stable
    auto kcls = [&](int i) { const int64_t k = probs[i].k; return k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return kcls(a) < kcls(b); });
    const int na = (int)order.size();
    eig_list.clear();
    chg_list.clear();
    pan_list.clear();
    int n2max = 0;
    for (int q = 0; q < na; ++q) {
      Run<T> &r = runs[order[q]];
      r.small_args();
      av_h[q] = r.sa;
      ov_h[q] = r.so;
      n2max = std::max(n2max, (int)r.n2);
      if (r.l > 0) {
        ae_h[eig_list.size()] = r.sa;
        eig_list.push_back(order[q]);
      }
      if (r.change_needed()) {
        ch_h[chg_list.size()] = r.chg_args();
        chg_list.push_back(order[q]);
      }
      if (r.panel_needed()) {
        pa_h[pan_list.size()] = r.panel_args();
        pan_list.push_back(order[q]);
      }
    }
    rc = join();
    if (rc != WLRA_OK) return rc;
    hipStream_t s0 = strm[0];
    HIPCHK(hipMemcpyAsync(av_d, av_h, (size_t)na * sizeof(SmallArgs), hipMemcpyHostToDevice, s0));
    HIPCHK(hipMemcpyAsync(ov_d, ov_h, (size_t)na * sizeof(SmallOut<T>), hipMemcpyHostToDevice, s0));
    if (!eig_list.empty())
      HIPCHK(hipMemcpyAsync(ae_d, ae_h, eig_list.size() * sizeof(SmallArgs),
                            hipMemcpyHostToDevice, s0));
    if (!chg_list.empty())
      HIPCHK(hipMemcpyAsync(ch_d, ch_h, chg_list.size() * sizeof(ChgArgs),
                            hipMemcpyHostToDevice, s0));
    if (!pan_list.empty())
      HIPCHK(hipMemcpyAsync(pa_d, pa_h, pan_list.size() * sizeof(PanelArgs),
                            hipMemcpyHostToDevice, s0));
    for (int q0 = 0; q0 < na;) {
      int q1 = q0;
      while (q1 < na && kcls(order[q1]) == kcls(order[q0])) ++q1;
      int n2c = 0;
      for (int q = q0; q < q1; ++q) n2c = std::max(n2c, (int)runs[order[q]].n2);
      PROFWS(h, s0, KK_COEF, 0, 0, launch_coef_b(s0, kcls(order[q0]), q1 - q0, n2c, av_d + q0));
      q0 = q1;
    }
    if (!eig_list.empty()) {
      int n2e = 0;
      for (int i : eig_list) n2e = std::max(n2e, (int)runs[i].n2);
      PROFWS(h, s0, KK_FORMM, 0, 0, launch_formM_b(s0, (int)eig_list.size(), n2e, ae_d));
      PROFWS(h, s0, KK_EIG, 0, 0, launch_eig_b(s0, (int)eig_list.size(), ae_d));
    }
    PROFWS(h, s0, KK_POST, 0, 0, launch_post_b<T>(s0, na, n2max, av_d, ov_d));
    if (!pan_list.empty())
      PROFWS(h, s0, KK_POST, 0, 0, launch_panel_bf16_b(s0, (int)pan_list.size(), pa_d));
    if (!chg_list.empty()) {
      PROFWS(h, s0, KK_CHGQR, 0, 0, launch_chgprep_b(s0, (int)chg_list.size(), ch_d));
      rc = fork();
      if (rc != WLRA_OK) return rc;
      for (int i : chg_list) runs[i].change(true);
      rc = join();
      if (rc != WLRA_OK) return rc;
    }
    PROFWS(h, s0, KK_DECIDE, 0, 0, launch_decide_b(s0, na, av_d, stall_d));
    HIPCHK(hipMemcpyAsync(stall_h, stall_d, (size_t)na * sizeof(SmallState),
                          hipMemcpyDeviceToHost, s0));
    HIPCHK(hipStreamSynchronize(s0));
    prof_collect(h);
    rc = fork();
    if (rc != WLRA_OK) return rc;
    for (int q = 0; q < na; ++q) {
      const int i = order[q];
      Run<T> &r = runs[i];
      *r.sh = stall_h[q];
      const int d = r.after_decide();
      if (d == 1) {
        state[i] = 1;
        // the instance's solve is complete on the device here (its outputs
        // follow at the end of the batch)
        HIPCHK(hipEventRecord(h->bdone[i], s0));
        HIPCHK(hipMemcpyAsync(&flags_h[i], r.P.flags, sizeof(int), hipMemcpyDeviceToHost, r.s));
      } else if (d == 0) {
        r.update();
      }
    }
  }
  for (int j = 0; j < ns; ++j) HIPCHK(hipStreamSynchronize(strm[j]));
  prof_collect(h);
  // outputs of the finished instances, each timed from the batch's start to
  // the end of its outputs on its stream
  for (int i = 0; i < count; ++i) {
    if (state[i] != 1) continue;
    const int st = Run<T>::device_status(flags_h[i]);
    if (st != WLRA_OK) {
      memset(&res[i], 0, sizeof(wlra_result));
      res[i].status = st;
      state[i] = -1;
      continue;
    }
    rc = runs[i].outputs();
    if (rc != WLRA_OK) return rc;
  }
  rc = join();
  if (rc != WLRA_OK) return rc;
  for (int j = 0; j < ns; ++j) HIPCHK(hipStreamSynchronize(strm[j]));
  prof_collect(h);
  for (int i = 0; i < count; ++i) {
    if (state[i] != 1) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev0, h->bdone[i]);
    runs[i].result(ms);
  }
  return WLRA_OK;
}

}  // namespace

extern "C" {

int wlra_version(void) { return WLRA_VERSION; }

const char *wlra_strerror(int status) {
  switch (status) {
    case WLRA_OK: return "converged";
    case WLRA_MAX_SWEEPS: return "maximum number of sweeps reached";
    case WLRA_E_ARG: return "invalid argument";
    case WLRA_E_WEIGHT: return "W1 entry not positive or not finite";
    case WLRA_E_NONFINITE: return "non-finite entry in A or X1_init";
    case WLRA_E_RANK: return "X1 numerically rank deficient";
    case WLRA_E_NOMEM: return "out of device memory";
    case WLRA_E_HIP: return "HIP runtime error";
    case WLRA_E_NODEVICE: return "no usable gfx950 device";
    case WLRA_INEXACT: return "eigen step of the returned sweep stopped at its round limit";
    case WLRA_E_ROWSOLVE: return "per-row system of the X1 update not positive definite in the storage precision";
    case WLRA_E_EIG: return "eigen step could not orthonormalise its block";
    case WLRA_E_SCRATCH: return "problem needs more workspace than the no-allocation scratch holds";
    default: return "unknown status";
  }
}

int wlra_validate(const wlra_problem *prob, int precision) {
  const int rc = check_problem(prob, precision);
  return rc == WLRA_E_WEIGHT ? WLRA_E_ARG : rc;
}

int wlra_create(wlra_handle *out, int device, void *hip_stream, int precision, uint32_t flags) {
  if (out == nullptr) return WLRA_E_ARG;
  *out = nullptr;
  if (precision < WLRA_FP64 || precision > WLRA_MIXED_BF16) return WLRA_E_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return WLRA_E_NODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return WLRA_E_NODEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return WLRA_E_NODEVICE;
  if (hipSetDevice(device) != hipSuccess) return WLRA_E_HIP;
  wlra_ctx *h = new (std::nothrow) wlra_ctx();
  if (h == nullptr) return WLRA_E_NOMEM;
  h->device = device;
  scratch_setup(device);
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->precision = precision;
  h->flags = flags;
  if (hipHostMalloc((void **)&h->st_host, sizeof(SmallState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h->flags_host, 64, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipEventCreate(&h->tev0) != hipSuccess || hipEventCreate(&h->tev1) != hipSuccess) {
    wlra_destroy(h);
    return WLRA_E_HIP;
  }
  *out = h;
  return WLRA_OK;
}

int wlra_reserve(wlra_handle h, int64_t m, int64_t n, int64_t k, int64_t r) {
  if (h == nullptr || m < 1 || n < 1 || k < 0 || r < k || r > std::min(m, n)) return WLRA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  const Sizes z = make_sizes(m, n, k, r, h->precision == WLRA_FP64 ? 8 : 4,
                            h->precision == WLRA_MIXED_BF16);
  return ensure_ws(h, make_layout(z, nullptr, nullptr).total);
}

int wlra_solve(wlra_handle h, const wlra_problem *prob, wlra_result *res) {
  if (h == nullptr) return WLRA_E_ARG;
  int rc = check_problem(prob, h->precision);
  if (rc != WLRA_OK) {
    if (res) { memset(res, 0, sizeof(*res)); res->status = rc; }
    return rc;
  }
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  rc = ensure_ws(h, workspace_bytes(*prob, h->precision));
  if (rc == WLRA_OK)
    rc = (h->precision == WLRA_FP64) ? solve_impl<double>(h, prob, res, h->ws)
                                     : solve_impl<float>(h, prob, res, h->ws);
  if (rc < 0 && res) res->status = rc;
  return rc;
}

int wlra_solve_noalloc(wlra_handle h, const wlra_problem *prob, wlra_result *res) {
  if (h == nullptr) return WLRA_E_ARG;
  // a profiling handle records its events into a growing host list
  if (h->flags & WLRA_FLAG_PROFILE) return WLRA_E_ARG;
  int rc = check_problem(prob, h->precision);
  if (rc == WLRA_OK && workspace_bytes(*prob, h->precision) > (size_t)WLRA_NOALLOC_SCRATCH_BYTES)
    rc = WLRA_E_SCRATCH;
  if (rc != WLRA_OK) {
    if (res) { memset(res, 0, sizeof(*res)); res->status = rc; }
    return rc;
  }
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  char *ws = static_cast<char *>(scratch_ptr(h->device));
  if (ws == nullptr) return WLRA_E_HIP;
  // no new autotuner entries: inserting one would allocate host memory
  rc = (h->precision == WLRA_FP64) ? solve_impl<double>(h, prob, res, ws, false)
                                   : solve_impl<float>(h, prob, res, ws, false);
  if (rc < 0 && res) res->status = rc;
  return rc;
}

int wlra_set_option(wlra_handle h, int32_t option, int64_t value) {
  if (h == nullptr) return WLRA_E_ARG;
  switch (option) {
    case WLRA_OPT_EIG_MAXIT:
      if (value < 1 || value > 100000) return WLRA_E_ARG;
      h->eig_maxit = (int)value;
      break;
    case WLRA_OPT_EIG_ONE_WG:
      if (value != 0 && value != 1) return WLRA_E_ARG;
      h->eig_one_wg = (int)value;
      break;
    case WLRA_OPT_AUTOTUNE:
      if (value != 0 && value != 1) return WLRA_E_ARG;
      h->autotune = (int)value;
      break;
    default:
      return WLRA_E_ARG;
  }
  return WLRA_OK;
}

int wlra_set_batch_lanes(wlra_handle h, int32_t lanes) {
  if (h == nullptr || lanes < 1 || lanes > WLRA_BATCH_LANES_MAX) return WLRA_E_ARG;
  h->batch_lanes = lanes;
  return WLRA_OK;
}



int wlra_solve_batched(wlra_handle h, int32_t count, const wlra_problem *probs, wlra_result *res) {
  if (h == nullptr || count < 0 || (count > 0 && (probs == nullptr || res == nullptr)))
    return WLRA_E_ARG;
  for (int i = 0; i < count; ++i)
    if (check_problem(&probs[i], h->precision) == WLRA_E_ARG) return WLRA_E_ARG;
  if (count == 0) return WLRA_OK;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  for (int i = 0; i < count; ++i) {
    memset(&res[i], 0, sizeof(wlra_result));
    const int rc = check_problem(&probs[i], h->precision);
    res[i].status = rc;  // WLRA_E_WEIGHT (a bad constant weight) is per instance
  }
  std::vector<wlra_problem> ok;
  std::vector<int> idx;
  for (int i = 0; i < count; ++i)
    if (res[i].status == WLRA_OK) {
      ok.push_back(probs[i]);
      idx.push_back(i);
    }
  if (ok.empty()) return WLRA_OK;
  std::vector<wlra_result> rr(ok.size());
  const int rc = (h->precision == WLRA_FP64) ? batch_impl<double>(h, (int)ok.size(), ok.data(), rr.data())
                                             : batch_impl<float>(h, (int)ok.size(), ok.data(), rr.data());
  for (size_t q = 0; q < ok.size(); ++q) res[idx[q]] = rr[q];
  return rc < 0 ? rc : WLRA_OK;
}

// ---------------------------------------------------------------------------
// Learned warm start: training and inference entry points.
extern "C++" {
namespace {

int ensure_lws(wlra_ctx *h, size_t bytes) {
  if (bytes <= h->lws_bytes) return WLRA_OK;
  if (h->lws) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return WLRA_E_HIP;
    (void)hipFree(h->lws);
    h->lws = nullptr;
    h->lws_bytes = 0;
  }
  const size_t want = bytes + bytes / 4;
  if (hipMalloc(&h->lws, want) != hipSuccess) {
    h->lws = nullptr;
    return WLRA_E_NOMEM;
  }
  h->lws_bytes = want;
  return WLRA_OK;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename P>
void mlp_offsets(P *base, int64_t o, P **W1, P **b1, P **W2, P **b2, P **W3, P **b3) {
  *W1 = base;
  *b1 = *W1 + LEARN_HID * LEARN_D_IN;
  *W2 = *b1 + LEARN_HID;
  *b2 = *W2 + LEARN_HID * LEARN_HID;
  *W3 = *b2 + LEARN_HID;
  *b3 = *W3 + o * LEARN_HID;
}

template <typename T>
int sketch_impl(wlra_ctx *h, int64_t m, int64_t n, const T *A, int64_t lda, float *out) {
  int64_t rows = 0;
  const int splits = choose_splits(m, (int)((n + 31) / 32), &rows);
  const size_t b_om = al256((size_t)(m * LEARN_SK_ROWS) * sizeof(T));
  const size_t b_ps = al256((size_t)(n * LEARN_SK_COLS) * sizeof(T));
  const size_t b_p1 = al256((size_t)(LEARN_SK_ROWS * n) * sizeof(double));
  const size_t b_pt = al256((size_t)splits * LEARN_SK_ROWS * n * sizeof(double));
  int rc = ensure_lws(h, b_om + b_ps + b_p1 + b_pt);
  if (rc != WLRA_OK) return rc;
  T *Om = reinterpret_cast<T *>(h->lws);
  T *Ps = reinterpret_cast<T *>(h->lws + b_om);
  double *P1 = reinterpret_cast<double *>(h->lws + b_om + b_ps);
  double *part = reinterpret_cast<double *>(h->lws + b_om + b_ps + b_p1);
  hipStream_t s = h->stream;
  launch_gauss_fill<T>(s, m * LEARN_SK_ROWS, LEARN_SEED_OMEGA, 1.0, Om);
  launch_gauss_fill<T>(s, n * LEARN_SK_COLS, LEARN_SEED_PSI, 1.0, Ps);
  launch_tsgemm<T, T>(s, m, Om, m, LEARN_SK_ROWS, A, lda, (int)n, 0, splits, rows, part, P1,
                      nullptr);
  launch_sketch_finish<T>(s, (int)n, P1, Ps, out);
  return hipStreamSynchronize(s) == hipSuccess ? WLRA_OK : WLRA_E_HIP;
}

}  // namespace
}  // extern "C++"

int64_t wlra_mlp_param_count(int64_t n, int64_t r) {
  if (n < 1 || r < 1 || r > n || r > LEARN_RMAX || n > WLRA_NMAX + WLRA_KMAX) return -1;
  const int64_t o = n * r;
  return (int64_t)LEARN_HID * LEARN_D_IN + LEARN_HID + (int64_t)LEARN_HID * LEARN_HID +
         LEARN_HID + o * LEARN_HID + o;
}

int wlra_mlp_init(wlra_handle h, float *params, int64_t n, int64_t r, uint64_t seed) {
  if (h == nullptr || params == nullptr || wlra_mlp_param_count(n, r) < 0) return WLRA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  const int64_t o = n * r;
  float *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_offsets<float>(params, o, &W1, &b1, &W2, &b2, &W3, &b3);
  hipStream_t s = h->stream;
  launch_gauss_fill<float>(s, (int64_t)LEARN_HID * LEARN_D_IN, seed + 1, sqrt(2.0 / LEARN_D_IN), W1);
  launch_fill_zero(s, LEARN_HID, b1);
  launch_gauss_fill<float>(s, (int64_t)LEARN_HID * LEARN_HID, seed + 2, sqrt(2.0 / LEARN_HID), W2);
  launch_fill_zero(s, LEARN_HID, b2);
  launch_gauss_fill<float>(s, o * LEARN_HID, seed + 3, sqrt(2.0 / LEARN_HID), W3);
  launch_fill_zero(s, o, b3);
  return hipStreamSynchronize(s) == hipSuccess ? WLRA_OK : WLRA_E_HIP;
}

int wlra_sketch(wlra_handle h, int64_t m, int64_t n, const void *A, int64_t lda, float *out) {
  if (h == nullptr || A == nullptr || out == nullptr || m < 1 || n < 1 || lda < m)
    return WLRA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  if (h->precision == WLRA_FP64)
    return sketch_impl<double>(h, m, n, static_cast<const double *>(A), lda, out);
  return sketch_impl<float>(h, m, n, static_cast<const float *>(A), lda, out);
}

int wlra_mlp_forward(wlra_handle h, const float *params, int64_t n, int64_t r, int32_t batch,
                     const float *X, float *Y) {
  if (h == nullptr || params == nullptr || X == nullptr || Y == nullptr || batch < 1 ||
      wlra_mlp_param_count(n, r) < 0)
    return WLRA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  const int64_t o = n * r;
  const size_t bh = al256((size_t)batch * LEARN_HID * sizeof(float));
  int rc = ensure_lws(h, 2 * bh);
  if (rc != WLRA_OK) return rc;
  float *h1 = reinterpret_cast<float *>(h->lws), *h2 = reinterpret_cast<float *>(h->lws + bh);
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_offsets<const float>(params, o, &W1, &b1, &W2, &b2, &W3, &b3);
  hipStream_t s = h->stream;
  launch_gemm(s, 0, batch, LEARN_HID, LEARN_D_IN, X, LEARN_D_IN, W1, LEARN_D_IN, h1, LEARN_HID,
              b1, 1, nullptr, 0);
  launch_gemm(s, 0, batch, LEARN_HID, LEARN_HID, h1, LEARN_HID, W2, LEARN_HID, h2, LEARN_HID, b2,
              1, nullptr, 0);
  launch_gemm(s, 0, batch, (int)o, LEARN_HID, h2, LEARN_HID, W3, LEARN_HID, Y, (int)o, b3, 0,
              nullptr, 0);
  return hipStreamSynchronize(s) == hipSuccess ? WLRA_OK : WLRA_E_HIP;
}

int wlra_mlp_train_step(wlra_handle h, float *params, float *adam_m, float *adam_v,
                        int32_t step, int64_t n, int64_t r, int32_t batch, const float *X,
                        const float *T, double lr, double *loss, float *grad_out) {
  const int64_t P = wlra_mlp_param_count(n, r);
  if (h == nullptr || params == nullptr || X == nullptr || T == nullptr || batch < 1 ||
      batch > 65535 || P < 0 || (step > 0 && (adam_m == nullptr || adam_v == nullptr)))
    return WLRA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return WLRA_E_HIP;
  const int64_t o = n * r;
  const int B = batch;
  const size_t bh = al256((size_t)B * LEARN_HID * sizeof(float));
  const size_t bo = al256((size_t)B * o * sizeof(float));
  const size_t bp = al256((size_t)P * sizeof(float));
  const size_t bl = al256((size_t)B * sizeof(double));
  int rc = ensure_lws(h, 4 * bh + 2 * bo + bp + bl + 256);
  if (rc != WLRA_OK) return rc;
  char *w = h->lws;
  float *h1 = reinterpret_cast<float *>(w), *h2 = reinterpret_cast<float *>(w + bh);
  float *gh2 = reinterpret_cast<float *>(w + 2 * bh), *gh1 = reinterpret_cast<float *>(w + 3 * bh);
  float *y = reinterpret_cast<float *>(w + 4 * bh);
  float *gy = reinterpret_cast<float *>(w + 4 * bh + bo);
  float *g = reinterpret_cast<float *>(w + 4 * bh + 2 * bo);
  double *lp = reinterpret_cast<double *>(w + 4 * bh + 2 * bo + bp);
  int *dflag = reinterpret_cast<int *>(w + 4 * bh + 2 * bo + bp + bl);
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_offsets<const float>(params, o, &W1, &b1, &W2, &b2, &W3, &b3);
  float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
  mlp_offsets<float>(g, o, &gW1, &gb1, &gW2, &gb2, &gW3, &gb3);
  hipStream_t s = h->stream;
  HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), s));
  // forward
  launch_gemm(s, 0, B, LEARN_HID, LEARN_D_IN, X, LEARN_D_IN, W1, LEARN_D_IN, h1, LEARN_HID, b1,
              1, nullptr, 0);
  launch_gemm(s, 0, B, LEARN_HID, LEARN_HID, h1, LEARN_HID, W2, LEARN_HID, h2, LEARN_HID, b2, 1,
              nullptr, 0);
  launch_gemm(s, 0, B, (int)o, LEARN_HID, h2, LEARN_HID, W3, LEARN_HID, y, (int)o, b3, 0,
              nullptr, 0);
  // loss and its gradient with respect to the output
  launch_subspace_loss(s, (int)n, (int)r, B, y, T, 1.0, gy, lp, dflag);
  // backward
  launch_gemm(s, 2, (int)o, LEARN_HID, B, gy, (int)o, h2, LEARN_HID, gW3, LEARN_HID, nullptr, 0,
              nullptr, 0);
  launch_colsum(s, B, (int)o, gy, gb3);
  launch_gemm(s, 1, B, LEARN_HID, (int)o, gy, (int)o, W3, LEARN_HID, gh2, LEARN_HID, nullptr, 0,
              h2, LEARN_HID);
  launch_gemm(s, 2, LEARN_HID, LEARN_HID, B, gh2, LEARN_HID, h1, LEARN_HID, gW2, LEARN_HID,
              nullptr, 0, nullptr, 0);
  launch_colsum(s, B, LEARN_HID, gh2, gb2);
  launch_gemm(s, 1, B, LEARN_HID, LEARN_HID, gh2, LEARN_HID, W2, LEARN_HID, gh1, LEARN_HID,
              nullptr, 0, h1, LEARN_HID);
  launch_gemm(s, 2, LEARN_HID, LEARN_D_IN, B, gh1, LEARN_HID, X, LEARN_D_IN, gW1, LEARN_D_IN,
              nullptr, 0, nullptr, 0);
  launch_colsum(s, B, LEARN_HID, gh1, gb1);
  if (grad_out != nullptr)
    HIPCHK(hipMemcpyAsync(grad_out, g, (size_t)P * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (step > 0) {
    const double b1c = 1.0 - pow(0.9, step), b2c = 1.0 - pow(0.999, step);
    launch_adam(s, P, params, g, adam_m, adam_v, (float)lr, 0.9, 0.999, 1e-8f, (float)b1c,
                (float)b2c);
  }
  std::vector<double> lh((size_t)B);
  int fl = 0;
  HIPCHK(hipMemcpyAsync(lh.data(), lp, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&fl, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double tot = 0.0;
  for (double v : lh) tot += v;
  if (loss) *loss = tot / B;
  return (fl & DEV_LEARN_FAIL) ? WLRA_E_RANK : WLRA_OK;
}

int wlra_profile(wlra_handle h, int32_t max, wlra_kstat *out, int32_t reset) {
  if (h == nullptr || max < 0 || (max > 0 && out == nullptr)) return WLRA_E_ARG;
  if (!(h->flags & WLRA_FLAG_PROFILE)) return 0;
  int n = 0;
  for (int i = 0; i < KK_COUNT; ++i) {
    if (h->launches[i] == 0) continue;
    if (n < max) {
      memset(out[n].name, 0, sizeof(out[n].name));
      strncpy(out[n].name, kKernelNames[i], sizeof(out[n].name) - 1);
      out[n].launches = h->launches[i];
      out[n].ms = h->ms[i];
      out[n].bytes = h->bytes[i];
      out[n].flops = h->flops[i];
    }
    ++n;
  }
  if (reset)
    for (int i = 0; i < KK_COUNT; ++i) {
      h->launches[i] = 0;
      h->ms[i] = 0.0;
      h->bytes[i] = 0.0;
      h->flops[i] = 0.0;
    }
  return n;
}

int wlra_destroy(wlra_handle h) {
  if (h == nullptr) return WLRA_OK;
  for (hipStream_t st : h->bstreams)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t e : h->bjoin)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->bdone)
    if (e) (void)hipEventDestroy(e);
  if (h->bws) (void)hipFree(h->bws);
  if (h->bhost) (void)hipHostFree(h->bhost);
  for (auto &pe : h->pending) {
    h->pool.push_back(pe.e0);
    h->pool.push_back(pe.e1);
  }
  for (hipEvent_t e : h->pool)
    if (e) hipEventDestroy(e);
  if (h->ws) hipFree(h->ws);
  if (h->lws) hipFree(h->lws);
  if (h->st_host) hipHostFree(h->st_host);
  if (h->flags_host) hipHostFree(h->flags_host);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  if (h->tev0) hipEventDestroy(h->tev0);
  if (h->tev1) hipEventDestroy(h->tev1);
  if (h->owns_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return WLRA_OK;
}

}  // extern "C"
