"""ctypes binding of libwlra (the C ABI declared in include/wlra.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  Matrices
are column-major on the device; `colmajor(t)` gives a tensor whose storage is
column-major (stride (1, m)).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwlra.so")

OK, MAX_SWEEPS, INEXACT = 0, 1, 2
E_ARG, E_WEIGHT, E_NONFINITE, E_RANK, E_NOMEM, E_HIP, E_NODEVICE = -1, -2, -3, -4, -5, -6, -7
E_ROWSOLVE, E_EIG, E_SCRATCH = -8, -9, -10
NOALLOC_SCRATCH_BYTES = 32 << 20
OPT_EIG_MAXIT, OPT_EIG_ONE_WG, OPT_AUTOTUNE = 1, 2, 3
FP64, FP32, MIXED_BF16 = 0, 1, 2
INIT_RANDOM, INIT_GIVEN, INIT_A1, INIT_LEARNED = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED_BF16}
INITS = {"random": INIT_RANDOM, "given": INIT_GIVEN, "a1": INIT_A1, "learned": INIT_LEARNED}
SKETCH_DIM = 512


class Problem(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("r", ctypes.c_int64),
        ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
        ("W1", ctypes.c_void_p), ("ldw", ctypes.c_int64),
        ("w1_const", ctypes.c_double), ("tol", ctypes.c_double),
        ("max_sweeps", ctypes.c_int32), ("init", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("X1_init", ctypes.c_void_p), ("ldx0", ctypes.c_int64),
        ("X1_out", ctypes.c_void_p), ("ldx1", ctypes.c_int64),
        ("X2_out", ctypes.c_void_p), ("ldx2", ctypes.c_int64),
        ("trace", ctypes.POINTER(ctypes.c_double)),
        ("eig_tol", ctypes.c_double),
        ("model", ctypes.c_void_p),
        ("factors_out", ctypes.c_void_p),
        ("W2", ctypes.c_void_p),
        ("mask_out", ctypes.c_void_p), ("ldm", ctypes.c_int64), ("mask_tau", ctypes.c_double),
        ("V_init", ctypes.c_void_p), ("ldv0", ctypes.c_int64), ("v0_rows", ctypes.c_int64),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("sweeps", ctypes.c_int32),
        ("objective", ctypes.c_double), ("abs_change", ctypes.c_double),
        ("rel_change", ctypes.c_double), ("gap", ctypes.c_double),
        ("ms", ctypes.c_float), ("eig_iters", ctypes.c_int32), ("eig_matvecs", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


FLAG_PROFILE = 1

SYMBOLS = ("wlra_create", "wlra_reserve", "wlra_solve", "wlra_solve_noalloc",
           "wlra_solve_batched",
           "wlra_set_batch_lanes", "wlra_set_option", "wlra_destroy", "wlra_profile",
           "wlra_validate",
           "wlra_strerror", "wlra_version", "wlra_mlp_param_count", "wlra_mlp_init",
           "wlra_sketch", "wlra_mlp_forward", "wlra_mlp_train_step")

_lib = None


def load(path: str = LIB_PATH):
    """Load libwlra.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libwlra.so not found at {path}; run paper_1703_06303_amd/build.py")
    lib = ctypes.CDLL(path)
    lib.wlra_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_int, ctypes.c_uint32]
    lib.wlra_reserve.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * 4
    lib.wlra_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Result)]
    lib.wlra_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                       ctypes.POINTER(Result)]
    lib.wlra_solve_batched.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Problem),
                                       ctypes.POINTER(Result)]
    lib.wlra_set_batch_lanes.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.wlra_set_option.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]
    lib.wlra_destroy.argtypes = [ctypes.c_void_p]
    lib.wlra_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(KStat),
                                 ctypes.c_int32]
    lib.wlra_validate.argtypes = [ctypes.POINTER(Problem), ctypes.c_int]
    lib.wlra_strerror.argtypes = [ctypes.c_int]
    lib.wlra_strerror.restype = ctypes.c_char_p
    lib.wlra_version.argtypes = []
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.wlra_mlp_param_count.argtypes = [i64, i64]
    lib.wlra_mlp_param_count.restype = i64
    lib.wlra_mlp_init.argtypes = [vp, vp, i64, i64, ctypes.c_uint64]
    lib.wlra_sketch.argtypes = [vp, i64, i64, vp, i64, vp]
    lib.wlra_mlp_forward.argtypes = [vp, vp, i64, i64, i32, vp, vp]
    lib.wlra_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, i64, i64, i32, vp, vp,
                                        ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
    for name in ("wlra_mlp_init", "wlra_sketch", "wlra_mlp_forward", "wlra_mlp_train_step"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("wlra_create", "wlra_reserve", "wlra_solve", "wlra_solve_noalloc",
                 "wlra_solve_batched",
                 "wlra_set_batch_lanes", "wlra_set_option", "wlra_destroy", "wlra_profile",
                 "wlra_validate",
                 "wlra_version"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().wlra_strerror(code).decode()


class WlraError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"libwlra status {code}: {strerror(code)}")
        self.code = code


def colmajor(t):
    """Column-major copy of a 2-D tensor (stride (1, rows))."""
    return t.t().contiguous().t()


def empty_colmajor(rows, cols, dtype, device):
    """Uninitialised column-major rows x cols tensor (no copy kernel)."""
    import torch
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def mlp_param_count(n, r):
    """Number of parameters of the warm-start network for (n, r)."""
    c = load().wlra_mlp_param_count(int(n), int(r))
    if c < 0:
        raise WlraError(E_ARG)
    return int(c)


def factors_size(n, k, r):
    n2, l = n - k, r - k
    return k * k + k * n2 + n2 * l + l


def make_problem(A, k, r, W1=None, w1_const=0.0, tol=1e-7, max_sweeps=200, init="random",
                 seed=0, X1_init=None, X1_out=None, X2_out=None, trace=None, eig_tol=0.0,
                 model=None, factors_out=None, W2=None, mask_out=None, mask_tau=0.0,
                 V_init=None):
    """Fill a Problem from tensors (column-major device tensors or None).
    W2: n - k column weights (1-D); mask_out: m x n uint8; V_init: a
    v0_rows x (r - k) float64 start block of the eigen step."""
    m, n = A.shape
    p = Problem()
    p.m, p.n, p.k, p.r = m, n, k, r
    p.A, p.lda = _ptr(A), A.stride(1) if n > 1 else m
    p.W1 = _ptr(W1)
    p.ldw = W1.stride(1) if (W1 is not None and W1.shape[1] > 1) else m
    p.w1_const = float(w1_const)
    p.tol = float(tol)
    p.max_sweeps = int(max_sweeps)
    p.init = INITS[init] if isinstance(init, str) else int(init)
    p.seed = int(seed)
    p.X1_init = _ptr(X1_init)
    p.ldx0 = X1_init.stride(1) if (X1_init is not None and X1_init.shape[1] > 1) else m
    p.X1_out = _ptr(X1_out)
    p.ldx1 = X1_out.stride(1) if (X1_out is not None and X1_out.shape[1] > 1) else m
    p.X2_out = _ptr(X2_out)
    p.ldx2 = X2_out.stride(1) if (X2_out is not None and X2_out.shape[1] > 1) else m
    p.trace = trace if trace is not None else ctypes.POINTER(ctypes.c_double)()
    p.eig_tol = float(eig_tol)
    p.model = _ptr(model)
    p.factors_out = _ptr(factors_out)
    p.W2 = _ptr(W2)
    p.mask_out = _ptr(mask_out)
    p.ldm = mask_out.stride(1) if (mask_out is not None and n > 1) else m
    p.mask_tau = float(mask_tau)
    p.V_init = _ptr(V_init)
    if V_init is not None:
        p.v0_rows = V_init.shape[0]
        p.ldv0 = V_init.stride(1) if V_init.shape[1] > 1 else V_init.shape[0]
    return p


def validate(problem: Problem, precision: int) -> int:
    """Host-only argument check (no device access)."""
    return load().wlra_validate(ctypes.byref(problem), int(precision))


class Solver:
    """One libwlra handle bound to a device and a stream."""

    def __init__(self, precision="fp32", device=0, stream=None, profile=False):
        import torch
        lib = load()
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.wlra_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                             self.precision, FLAG_PROFILE if profile else 0)
        if rc != OK:
            raise WlraError(rc)
        self.h = h
        self.lib = lib

    def close(self):
        if getattr(self, "h", None):
            self.lib.wlra_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, reset=False, work=False):
        """Per-kernel totals {name: (launches, ms)} of a profiling handle;
        with work=True {name: (launches, ms, bytes, flops)} (algorithmic
        totals of those launches)."""
        buf = (KStat * 32)()
        n = self.lib.wlra_profile(self.h, 32, buf, 1 if reset else 0)
        if n < 0:
            raise WlraError(n)
        if work:
            return {buf[i].name.decode(): (buf[i].launches, buf[i].ms, buf[i].bytes, buf[i].flops)
                    for i in range(min(n, 32))}
        return {buf[i].name.decode(): (buf[i].launches, buf[i].ms) for i in range(min(n, 32))}

    def reserve(self, m, n, k, r):
        rc = self.lib.wlra_reserve(self.h, m, n, k, r)
        if rc != OK:
            raise WlraError(rc)

    def solve(self, A, k, r, W1=None, w1_const=0.0, tol=1e-7, max_sweeps=200, init="random",
              seed=0, X1_init=None, want_x2=False, want_trace=False, eig_tol=0.0, raise_on_error=True,
              model=None, want_factors=False, out=None, noalloc=False, W2=None, mask_tau=None,
              V_init=None):
        """Solve problem (5).  A, W1, X1_init: column-major device tensors of
        the handle's dtype; model: float32 device tensor of network parameters
        (init="learned").  Returns (X1, X2 or None, result dict); with
        want_factors the dict holds "factors" = (R, C, V, theta) as float64
        device tensors.  out = (X1, X2 or None) passes preallocated outputs.
        noalloc=True calls wlra_solve_noalloc (the library's fixed scratch
        instead of the handle's workspace).  W2: n - k column weights (device,
        handle dtype); mask_tau: also return info["mask"], the m x n uint8
        mask |A - X| > mask_tau; V_init: float64 device start block of the
        eigen step (rows x (r - k), column-major)."""
        import torch
        m, n = A.shape
        fac = (torch.empty(factors_size(n, k, r), dtype=torch.float64, device=A.device)
               if want_factors else None)
        if out is not None:
            X1, X2 = out
        else:
            X1 = empty_colmajor(m, k, self.dtype, A.device)
            X2 = empty_colmajor(m, n - k, self.dtype, A.device) if want_x2 else None
        tr = (ctypes.c_double * (2 * (max_sweeps + 1)))() if want_trace else None
        mask = (torch.empty((n, m), dtype=torch.uint8, device=A.device).t()
                if mask_tau is not None else None)
        if V_init is not None:
            V_init = colmajor(V_init.to(torch.float64))
        p = make_problem(A, k, r, W1=W1, w1_const=w1_const, tol=tol, max_sweeps=max_sweeps,
                         init=init, seed=seed, X1_init=X1_init, X1_out=X1, X2_out=X2,
                         trace=ctypes.cast(tr, ctypes.POINTER(ctypes.c_double)) if tr is not None else None,
                         eig_tol=eig_tol, model=model, factors_out=fac, W2=W2, mask_out=mask,
                         mask_tau=mask_tau if mask_tau is not None else 0.0, V_init=V_init)
        res = Result()
        entry = self.lib.wlra_solve_noalloc if noalloc else self.lib.wlra_solve
        rc = entry(self.h, ctypes.byref(p), ctypes.byref(res))
        if rc < 0 and raise_on_error:
            raise WlraError(rc)
        info = res.as_dict()
        info["rc"] = rc
        if tr is not None:
            info["trace_F"] = list(tr[:max_sweeps + 1])
            info["trace_err"] = list(tr[max_sweeps + 1:])
        if mask is not None:
            info["mask"] = mask
        if fac is not None:
            n2, l = n - k, r - k
            o1, o2, o3 = k * k, k * k + k * n2, k * k + k * n2 + n2 * l
            info["factors"] = (fac[:o1].view(k, k).t(), fac[o1:o2].view(n2, k).t(),
                               fac[o2:o3].view(l, n2).t(), fac[o3:])
        return X1, X2, info

    # -- learned warm start -------------------------------------------------
    def _chk(self, rc):
        if rc != OK:
            raise WlraError(rc)

    def mlp_init(self, params, n, r, seed):
        self._chk(self.lib.wlra_mlp_init(self.h, _ptr(params), n, r, seed))

    def sketch(self, A):
        """512-float sketch of a column-major device matrix A."""
        import torch
        m, n = A.shape
        out = torch.empty(SKETCH_DIM, dtype=torch.float32, device=A.device)
        lda = A.stride(1) if n > 1 else m
        self._chk(self.lib.wlra_sketch(self.h, m, n, _ptr(A), lda, _ptr(out)))
        return out

    def mlp_forward(self, params, n, r, X):
        import torch
        Y = torch.empty((X.shape[0], n * r), dtype=torch.float32, device=X.device)
        self._chk(self.lib.wlra_mlp_forward(self.h, _ptr(params), n, r, X.shape[0],
                                            _ptr(X.contiguous()), _ptr(Y)))
        return Y

    def mlp_train_step(self, params, adam_m, adam_v, step, n, r, X, T, lr, want_grad=False):
        """One training step (step <= 0: loss and gradient only).  X: B x 512,
        T: B x (n r) targets (each n x r column-major).  Returns (loss, grad)."""
        import torch
        loss = ctypes.c_double()
        g = torch.empty_like(params) if want_grad else None
        rc = self.lib.wlra_mlp_train_step(self.h, _ptr(params), _ptr(adam_m), _ptr(adam_v), step,
                                          n, r, X.shape[0], _ptr(X.contiguous()),
                                          _ptr(T.contiguous()), float(lr), ctypes.byref(loss),
                                          _ptr(g))
        self._chk(rc)
        return loss.value, g

    def solve_noalloc(self, A, k, r, **kw):
        """solve(..., noalloc=True): wlra_solve_noalloc."""
        return self.solve(A, k, r, noalloc=True, **kw)

    def set_option(self, option, value):
        rc = self.lib.wlra_set_option(self.h, int(option), int(value))
        if rc != OK:
            raise WlraError(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_batch_lanes(self, lanes):
        rc = self.lib.wlra_set_batch_lanes(self.h, int(lanes))
        if rc != OK:
            raise WlraError(rc)

    def solve_batched(self, problems):
        """Solve a list of Problem structs (already filled with pointers)."""
        cnt = len(problems)
        arr = (Problem * cnt)(*problems)
        res = (Result * cnt)()
        rc = self.lib.wlra_solve_batched(self.h, cnt, arr, res)
        if rc < 0:
            raise WlraError(rc)
        return [r.as_dict() for r in res]
