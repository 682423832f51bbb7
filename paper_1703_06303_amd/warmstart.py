"""Training data, training loop and evaluation of the learned warm start.

Everything numerical runs in libwlra through its C ABI (sketch, solve,
network forward/backward and Adam); this module only generates the seeded
synthetic clips on the host, moves them to the device, and assembles the
training targets from the solution factors:

    T = [[I_k, C], [0, V^T]]^T   (n x r, column-major),

whose column space is the row space of the solution X = [X1, X1 C + D].

Host generation runs in worker processes that must be started before the
calling process touches the GPU (`make_pool` first, then the solver).
"""
from __future__ import annotations

import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _gen_config2(seed):
    from gen import video
    inst = video.config2(seed=seed)
    return seed, inst.A.astype(np.float32), inst.W1.astype(np.float32)


def _noop(x):
    return x


def make_pool(workers=12):
    """Worker pool for instance generation; call before any GPU use so the
    workers are forked from a process without GPU state."""
    pool = ProcessPoolExecutor(max_workers=workers)
    list(pool.map(_noop, range(workers)))  # start every worker now
    return pool


def target_basis(C, V, k, r):
    """[[I_k, C], [0, V^T]]^T flattened column-major (n r floats, device)."""
    import torch
    n2 = V.shape[0] if V.numel() else C.shape[1]
    n = k + n2
    T = torch.zeros((r, n), dtype=torch.float32, device=C.device)  # T^T, row-major
    T[:k, :k] = torch.eye(k, dtype=torch.float32, device=C.device)
    if k > 0:
        T[:k, k:] = C.to(torch.float32)
    if r > k:
        T[k:, k:] = V.t().to(torch.float32)
    return T.reshape(-1)


def build_dataset(solver, pool, seeds, k=20, r=25, tol=1e-7, log=None):
    """Sketches X (N x 512) and targets T (N x n r) of config-2 clips, from
    GPU solves started at A1.  log(msg) is called every 500 clips."""
    import torch
    from . import wlra
    X, T, info = [], [], []
    t0 = time.perf_counter()
    for seed, A, W1 in pool.map(_gen_config2, seeds, chunksize=4):
        Ad = wlra.colmajor(torch.from_numpy(A).cuda())
        Wd = wlra.colmajor(torch.from_numpy(W1).cuda())
        X.append(solver.sketch(Ad))
        _, _, res = solver.solve(Ad, k, r, W1=Wd, tol=tol, init="a1", want_factors=True)
        R, C, V, th = res["factors"]
        T.append(target_basis(C, V, k, r))
        info.append((seed, res["status"], res["sweeps"], res["objective"]))
        if log and len(info) % 500 == 0:
            log(f"{len(info)} clips solved ({time.perf_counter() - t0:.0f} s)")
    return torch.stack(X), torch.stack(T), info, time.perf_counter() - t0


def train(solver, X, T, n, r, epochs=30, batch=128, lr=1e-3, seed=1, log=None):
    """Adam on the subspace loss; returns (params, per-epoch mean losses)."""
    import torch
    from . import wlra
    P = wlra.mlp_param_count(n, r)
    params = torch.empty(P, dtype=torch.float32, device="cuda")
    solver.mlp_init(params, n, r, seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    g = torch.Generator().manual_seed(seed)
    N = X.shape[0]
    step, hist = 0, []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, N - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            step += 1
            loss, _ = solver.mlp_train_step(params, m, v, step, n, r, X[idx], T[idx], lr)
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return params, hist


def evaluate(solver, pool, params, seeds, k=20, r=25, tol=1e-7, inits=("random", "a1", "learned"),
             log=None):
    """Solve each held-out clip from each start; returns {init: [(sweeps,
    ms, objective, status)]}."""
    import torch
    from . import wlra
    out = {i: [] for i in inits}
    for seed, A, W1 in pool.map(_gen_config2, seeds, chunksize=4):
        Ad = wlra.colmajor(torch.from_numpy(A).cuda())
        Wd = wlra.colmajor(torch.from_numpy(W1).cuda())
        for init in inits:
            _, _, res = solver.solve(Ad, k, r, W1=Wd, tol=tol, init=init, seed=seed,
                                     model=params if init == "learned" else None)
            out[init].append((res["sweeps"], res["ms"], res["objective"], res["status"]))
        if log and len(out[inits[0]]) % 250 == 0:
            log(f"{len(out[inits[0]])} held-out clips evaluated")
    return out


def summarize(ev):
    """Mean, p99 and maximum sweeps and solve times per start, and the
    largest relative objective difference to the random start's solves."""
    Fr = np.array([x[2] for x in ev["random"]]) if "random" in ev else None
    out = {}
    for init, v in ev.items():
        sw = np.array([x[0] for x in v])
        ms = np.array([x[1] for x in v])
        F = np.array([x[2] for x in v])
        out[init] = {"sweeps_mean": float(sw.mean()), "sweeps_p99": float(np.percentile(sw, 99)),
                     "sweeps_max": int(sw.max()), "solve_ms_mean": float(ms.mean()),
                     "solve_ms_p99": float(np.percentile(ms, 99)),
                     "converged": int(sum(x[3] == 0 for x in v))}
        if Fr is not None:
            out[init]["max_rel_objective_vs_random_start"] = float(np.max(np.abs(F - Fr) / Fr))
    return out
