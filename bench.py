#!/usr/bin/env python3
"""Throughput of the sWLR solve (Dutta & Li, arXiv 1703.06303) on one MI355X.

One step = one complete solve of problem (5) with Algorithm 1, on a seeded
synthetic video matrix resident in HBM (default workload: 120 x 160 frames,
m = 19200, n = 200, rank-3 background, 10% 8x8 blob foreground,
N(0, 0.02^2) noise, k = 20 background frames with W1 = 10**U(1, 4), r = 25,
FP32 storage).  Every solve's objective is checked against F*, the FP64
oracle's converged objective (or the closed form for a constant W1), at
relative 1e-6.

Schedules timed side by side (`variants` in the output):
  plain_tol<t>   FP32 from the library's random start, the Section 4.1 rule
                 with tol t for t in 1e-7 (the paper's threshold, also
                 reported as "plain"), 1e-6, 1e-5, 1e-4, 1e-3
  mixed          A2 staged in BF16 for the X1 update's product with A2 (every
                 other step exact), sweeps to max(tol, 1e-5), then one exact
                 sweep; tol 1e-7 (no suffix), 1e-4 and 1e-3 (mixed_tol<t>)
  a1+mixed       the same from X1_0 = A1
  learned+mixed  the same from the learned warm start: the network is trained
                 on GPU solves of --learn-train clips of the same generator
                 (disjoint seeds), or loaded from --learn-weights, and
                 compared with the random and A1 starts on --learn-heldout
                 held-out clips (`learned_start` in the output)
Every family is quoted at its fastest stopping rule whose every solve meets
1e-6 (`fastest_meeting_1e-6`).  `value` is that of the learned+mixed family
(mixed when no network is built); `vs_plain` divides it by the plain family's
(`vs_plain_schedule` names it): the comparison at equal final objective.  The
chosen rules are then run on the held-out clips against each clip's FP64
reference (`heldout_stopping_rules`), so that a rule fitted to the timed clip
shows whether it carries over.

The default run also times, as sub-objects of the same line:
  config3  240 x 320 frames, m = 76800, n = 600, k = 50, r = 60, W1 = 1e3
           (plain FP32, mixed, A1 + mixed), against the closed form
  config4  64 clips of uneven shape (m in {4800, 19200, 76800}, n in
           [100, 400], k in [5, 40], r = k + [2, 8], W1 log-uniform), one
           wlra_solve_batched call per step (FP32 and mixed, four streams):
           solves/s, p50/p99 per-solve latency (from the batch's start to
           each clip's result), and the HBM rate of the streaming kernels
           (working set above the 256 MB MALL)
  extensions  column weights of the unweighted block, the foreground mask
           and appended frames warm-started from the previous solve
Other workloads (`--workload`): config1, config3, config4 alone, frames
(solve time against the number of frames, GPU vs oracle).

Prints one JSON line.  `roofline` is for the kernel with the largest device
time, from HIP events bracketing each launch on the library's stream in a
profiled repeat of the timed steps (for the eigen step also its share of the
FP64 rate of the CUs it runs on: one, or one per 16 rows of M for the
cooperative kernel).  `cpu_baseline` is the FP64 oracle
(NumPy/LAPACK) on the host cores, on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "WLRA solves/s to rel. objective 1e-6 vs FP64 oracle; learned+mixed vs plain"
PLAIN_TOLS = (1e-7, 1e-6, 1e-5, 1e-4, 1e-3)
# the mixed schedules' stopping rules: below 1e-5 they all run the BF16 sweeps
# to 1e-5 and one exact sweep, so the grid starts there (named without suffix)
MIXED_TOLS = (1e-7, 1e-4, 1e-3)
STREAMING = ("update", "gram_X1", "change", "gram_A2", "validate")

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs, scaled by
# the same counters read for a plain copy of known size (reads x2.0, writes
# x1.0).  An entry holds only while the kernel's source files are
# byte-identical to the ones measured (SHA-256 of their concatenation, in the
# order listed); otherwise traffic is reported as null.
TRAFFIC = {
    ("eig", "config2", "mixed"): (736043, ("k_eig.hip", "eig_small.h", "launch.h", "common.h"),
                                  "8c6a99a2e026c654776e87310c58e1c1ad54d4ab71faede390810c925523f754"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload_name, precision):
    import hashlib
    ent = TRAFFIC.get((kernel, workload_name, precision))
    if ent is None:
        return None
    nbytes, srcs, sha = ent
    h = hashlib.sha256()
    try:
        for src in srcs:
            with open(os.path.join(ROOT, "paper_1703_06303_amd", "csrc", src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return nbytes if h.hexdigest() == sha else None


def workload(name):
    """(instance, storage precision of the plain solve)."""
    from gen import video
    if name == "config2":
        return video.config2(), "fp32"
    if name == "config1":
        return video.config1(), "fp64"
    if name == "config3":
        return video.config3(), "fp32"
    raise SystemExit(f"unknown workload {name}")


def reference_objective(inst):
    """F* of the workload: the closed form when W1 is constant
    (problem (5) with eq. (2): F* = sum of sigma_i(A S)^2, i > r,
    S = diag(w..w, 1..1)), else the FP64 oracle converged far below the
    paper's threshold."""
    import numpy as np
    from oracle import swlr as O
    if inst.W1 is None:
        _, f = O.closed_form_column_weights(inst.A, np.full(inst.k, inst.w1_const), inst.k, inst.r)
        return f, "closed form H_r(A S) S^-1"
    ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0)
    return ref.F[-1], f"FP64 oracle at tol 1e-13 ({ref.sweeps} sweeps)"


def variants(plain_prec, learned=False):
    v = {}
    for t in PLAIN_TOLS:
        v[f"plain_tol{t:.0e}"] = dict(precision=plain_prec, tol=t, init="random", plain=True)
    if plain_prec == "fp32":
        fams = [("mixed", "random"), ("a1+mixed", "a1")] + ([("learned+mixed", "learned")]
                                                           if learned else [])
        for fam, init in fams:
            for t in MIXED_TOLS:
                v[fam if t == MIXED_TOLS[0] else f"{fam}_tol{t:.0e}"] = dict(
                    precision="mixed", tol=t, init=init)
    return v


def train_learned(pool, args):
    """Train the warm-start network on GPU solves of config-2 clips (training
    seeds), or load trained weights, then compare the random, A1 and learned
    starts on held-out seeds."""
    import numpy as np
    import torch
    from gen import video
    from paper_1703_06303_amd import warmstart as WS
    from paper_1703_06303_amd import wlra
    report = {}
    with wlra.Solver("fp32") as s:
        if args.learn_weights and os.path.exists(args.learn_weights):
            w = np.fromfile(args.learn_weights, dtype=np.float32)
            if w.size != wlra.mlp_param_count(200, 25):
                raise SystemExit(f"{args.learn_weights}: {w.size} floats, expected "
                                 f"{wlra.mlp_param_count(200, 25)}")
            params = torch.from_numpy(w).cuda()
            meta = args.learn_weights + ".json"
            report["weights"] = os.path.relpath(args.learn_weights, ROOT)
            if os.path.exists(meta):
                with open(meta) as f:
                    report["training"] = json.load(f)
            log(f"# warm start: weights loaded from {args.learn_weights}")
        else:
            tr = [video.config5_seed(i) for i in range(args.learn_train)]
            X, T, info, t_data = WS.build_dataset(s, pool, tr, log=lambda m_: log("# warm start: " + m_))
            log(f"# warm start: {len(tr)} training solves in {t_data:.1f} s")
            t0 = time.perf_counter()
            params, hist = WS.train(s, X, T, 200, 25, epochs=args.learn_epochs, batch=128, lr=1e-3,
                                    log=(lambda m_: log("# warm start: " + m_)) if len(tr) > 4096 else None)
            t_train = time.perf_counter() - t0
            log(f"# warm start: {args.learn_epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3f} "
                f"-> {hist[-1]:.3f}")
            report.update({"train_instances": len(tr), "train_data_s": t_data,
                           "epochs": args.learn_epochs, "train_s": t_train,
                           "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
                           "training_solves_converged": int(sum(x[1] == 0 for x in info))})
            if args.save_weights:
                os.makedirs(os.path.dirname(os.path.abspath(args.save_weights)), exist_ok=True)
                params.detach().cpu().numpy().astype(np.float32).tofile(args.save_weights)
                with open(args.save_weights + ".json", "w") as f:
                    json.dump({k_: v for k_, v in report.items()}, f, indent=1)
                log(f"# warm start: weights written to {args.save_weights}")
        ho = [video.config5_seed(i, heldout=True) for i in range(args.learn_heldout)]
        ev = (WS.evaluate(s, pool, params, ho, log=lambda m_: log("# warm start: " + m_))
              if ho else None)
    report["heldout_instances"] = len(ho)
    report["heldout"] = WS.summarize(ev) if ev else None
    return params, report


def cpu_baseline(inst, sample_solves, tol):
    """The oracle (FP64 NumPy/LAPACK) on the host: `sample_solves` full solves
    with the BLAS threads it uses by default, and one solve on one thread."""
    from oracle import swlr as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    w = inst.W1 if inst.W1 is not None else inst.w1_const
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(sample_solves):
        res = O.swlr(inst.A, w, inst.k, inst.r, tol=tol, max_sweeps=200, X1_0=inst.X1_0)
        sweeps.append(res.sweeps)
    dt = time.perf_counter() - t0
    out = {"value": sample_solves / dt, "unit": "solves/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"{sample_solves} full solves of the same workload with the paper's "
                     f"schedule (tol {tol}, {sweeps} sweeps), FP64 NumPy/LAPACK, {dt:.1f} s",
           "os_cpu_count": os.cpu_count(), "blas_threads": int(threads)}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            O.swlr(inst.A, w, inst.k, inst.r, tol=tol, max_sweeps=200, X1_0=inst.X1_0)
            d1 = time.perf_counter() - t0
        out["one_thread"] = {"value": 1.0 / d1, "unit": "solves/s", "seconds_per_solve": d1}
    return out


def roofline_of(name, launches, ms, nbytes, flops, res_list, n2):
    """Roofline entry of one kernel kind from its profiled totals."""
    avg_s = ms / launches / 1e3
    if name == "eig":
        mv = sum(x["eig_matvecs"] for x in res_list)
        fl = 2.0 * n2 * n2 * mv / launches
        roof = {"bound": "alu", "achieved": fl / avg_s / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
        # the step runs in one workgroup for n - k < 256, else in one
        # workgroup per 16 rows of M (cooperative): the share of the chip's
        # FP64 rate that those CUs hold (of 256), for context
        cus = 1 if n2 < 256 else (n2 + 15) // 16
        roof["cus_used"] = cus
        roof["peak_cus_used"] = FP64_PEAK_TFLOPS * cus / 256
        roof["frac_cus_used"] = roof["achieved"] / roof["peak_cus_used"]
    elif nbytes > 0:
        roof = {"bound": "hbm", "achieved": nbytes / launches / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": 0.0, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    return roof


def time_schedules(inst, specs, fstar, steps, warmup, inputs, model=None, tag=""):
    """Time every schedule: `steps` solves after `warmup` untimed ones."""
    import numpy as np
    import torch
    from paper_1703_06303_amd import wlra
    out = {}
    for name, spec in specs.items():
        with wlra.Solver(spec["precision"]) as solver:
            solver.reserve(inst.m, inst.n, inst.k, inst.r)

            def run(step):
                A, W1 = inputs(spec["precision"])
                return solver.solve(A, inst.k, inst.r, W1=W1, w1_const=inst.w1_const or 1.0,
                                    tol=spec["tol"], max_sweeps=200, init=spec["init"],
                                    seed=1000 + step,
                                    model=model if spec["init"] == "learned" else None)[2]
            for i in range(warmup):
                run(i)
            torch.cuda.synchronize()
            results = []
            t0 = time.perf_counter()
            for i in range(steps):
                results.append(run(i))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        objs = np.array([r["objective"] for r in results])
        relF = np.abs(objs - fstar) / fstar
        ok = int(np.sum((relF <= 1e-6) & (np.array([r["status"] for r in results]) == 0)))
        sw = np.array([r["sweeps"] for r in results])
        out[name] = {"solves_per_s": steps / dt, "ms_per_solve": 1e3 * dt / steps,
                     "sweeps_per_solve": float(sw.mean()), "sweeps_per_s": float(sw.sum() / dt),
                     "solves_meeting_1e-6": f"{ok}/{steps}", "all_meet_1e-6": ok == steps,
                     "max_rel_objective_err": float(relF.max()), "precision": spec["precision"],
                     "tol": spec["tol"], "init": spec["init"]}
        log(f"# {tag}{name}: {out[name]['solves_per_s']:.1f} solves/s, "
            f"{out[name]['sweeps_per_solve']:.1f} sweeps, {ok}/{steps} meet 1e-6")
    return out


def best_plain(out):
    """Fastest plain FP32 schedule whose every solve meets 1e-6."""
    return best_of(out, "plain")


def best_of(out, family):
    """Fastest schedule of a family (its stopping rules: `family` and
    `family_tol...`) whose every solve meets 1e-6."""
    ok = [(v["solves_per_s"], k) for k, v in out.items()
          if (k == family or k.startswith(family + "_tol")) and v["all_meet_1e-6"]]
    return max(ok)[1] if ok else None


def heldout_stopping(pool, params, seeds, chosen):
    """The chosen schedules (stopping rules picked on the timed clip) on
    held-out clips of the same generator: each clip's reference objective is
    the FP64 GPU solve at tol 1e-12 from the A1 start (the FP64 path agrees
    with the oracle to 1e-10); a clip counts when the schedule ends within
    1e-6 of it with status 0."""
    import numpy as np
    import torch
    from paper_1703_06303_amd import wlra
    from paper_1703_06303_amd import warmstart as WS
    solvers = {p: wlra.Solver(p) for p in ("fp64", "fp32", "mixed")}
    ok = {name: 0 for name in chosen}
    worst = {name: 0.0 for name in chosen}
    sweeps = {name: [] for name in chosen}
    try:
        for seed, A, W1 in pool.map(WS._gen_config2, seeds, chunksize=4):
            A64 = wlra.colmajor(torch.from_numpy(A.astype(np.float64)).cuda())
            W64 = wlra.colmajor(torch.from_numpy(W1.astype(np.float64)).cuda())
            ref = solvers["fp64"].solve(A64, 20, 25, W1=W64, tol=1e-12, max_sweeps=500,
                                        init="a1")[2]["objective"]
            A32 = wlra.colmajor(torch.from_numpy(A).cuda())
            W32 = wlra.colmajor(torch.from_numpy(W1).cuda())
            for name, spec in chosen.items():
                res = solvers[spec["precision"]].solve(
                    A32, 20, 25, W1=W32, tol=spec["tol"], max_sweeps=200, init=spec["init"],
                    seed=seed, model=params if spec["init"] == "learned" else None)[2]
                rel = abs(res["objective"] - ref) / ref
                ok[name] += int(rel <= 1e-6 and res["status"] == 0)
                worst[name] = max(worst[name], rel)
                sweeps[name].append(res["sweeps"])
    finally:
        for sv in solvers.values():
            sv.close()
    return {name: {"meeting_1e-6": f"{ok[name]}/{len(seeds)}", "max_rel_objective_err": worst[name],
                   "sweeps_mean": float(np.mean(sweeps[name])), "tol": chosen[name]["tol"]}
            for name in chosen}


def device_inputs(inst):
    import torch
    from paper_1703_06303_amd import wlra
    dev = torch.device("cuda", 0)
    tensors = {}

    def inputs(prec):
        tdt = torch.float64 if prec == "fp64" else torch.float32
        if tdt not in tensors:
            A = wlra.colmajor(torch.tensor(inst.A, dtype=tdt, device=dev))
            W1 = (wlra.colmajor(torch.tensor(inst.W1, dtype=tdt, device=dev))
                  if inst.W1 is not None else None)
            tensors[tdt] = (A, W1)
        return tensors[tdt]
    return inputs


def run_config3(steps, warmup):
    """Sub-object: the mixed-precision workload (constant W1, closed-form F*)."""
    from gen import video
    t0 = time.perf_counter()
    inst = video.config3()
    fstar, fsrc = reference_objective(inst)
    log(f"# config3: instance and F* in {time.perf_counter() - t0:.1f} s")
    specs = {"plain_tol1e-07": dict(precision="fp32", tol=1e-7, init="random"),
             "plain_tol1e-05": dict(precision="fp32", tol=1e-5, init="random"),
             "mixed": dict(precision="mixed", tol=1e-7, init="random"),
             "a1+mixed": dict(precision="mixed", tol=1e-7, init="a1")}
    out = time_schedules(inst, specs, fstar, steps, warmup, device_inputs(inst), tag="config3 ")
    bp = best_plain(out)
    return {"workload": f"config3: m={inst.m} (240x320) n={inst.n} k={inst.k} r={inst.r}, "
                        "W1 = 1e3", "reference_objective": {"value": fstar, "source": fsrc},
            "variants": out, "vs_plain_schedule": bp,
            "mixed_vs_plain": (out["mixed"]["solves_per_s"] / out[bp]["solves_per_s"]
                               if bp else None)}


def _gen_c4(args_):
    from gen import video
    import numpy as np
    i, shape = args_
    inst = video.config4_instance(i, shape)
    return i, inst.A.astype(np.float32), inst.W1.astype(np.float32), inst.k, inst.r


def run_config4(pool, steps, warmup, lanes=4, precisions=("fp32", "mixed"), one_lane=False):
    """Sub-object: 64 clips per wlra_solve_batched call, inputs resident in
    HBM; F* per clip from tests/golden/config4_fstar.json (FP64 oracle)."""
    import numpy as np
    import torch
    from gen import video
    from paper_1703_06303_amd import wlra
    shapes = video.config4_shapes()
    with open(os.path.join(ROOT, "tests", "golden", "config4_fstar.json")) as f:
        fstar = {d["i"]: d["fstar"] for d in json.load(f)["instances"]}
    t0 = time.perf_counter()
    jobs = list(enumerate(shapes))
    gen = pool.map(_gen_c4, jobs, chunksize=2) if pool is not None else map(_gen_c4, jobs)
    dev = torch.device("cuda", 0)
    A, W, X1, KR = {}, {}, {}, {}
    for i, a, w, k, r in gen:
        A[i] = wlra.colmajor(torch.from_numpy(a).to(dev))
        W[i] = wlra.colmajor(torch.from_numpy(w).to(dev))
        X1[i] = wlra.colmajor(torch.empty((a.shape[0], k), dtype=torch.float32, device=dev))
        KR[i] = (k, r)
    idx = sorted(A)
    ws_bytes = sum(A[i].numel() * 4 + W[i].numel() * 4 for i in idx)
    log(f"# config4: {len(idx)} clips generated and moved in {time.perf_counter() - t0:.1f} s "
        f"({ws_bytes / 1e9:.2f} GB of A and W1)")

    def problems(step):
        return [wlra.make_problem(A[i], KR[i][0], KR[i][1], W1=W[i], tol=1e-7, max_sweeps=200,
                                  init="random", seed=1000 * step + i, X1_out=X1[i])
                for i in idx]

    runs = [(p, lanes) for p in precisions]
    if one_lane:
        runs = [("fp32", 1)] + runs
    out = {}
    for prec, nl in runs:
        name = f"{prec}_{nl}stream{'s' if nl > 1 else ''}"
        with wlra.Solver(prec) as solver:
            solver.set_batch_lanes(nl)
            for w in range(max(1, warmup)):
                solver.solve_batched(problems(100 + w))
            torch.cuda.synchronize()
            allres = []
            t0 = time.perf_counter()
            for st in range(steps):
                allres.append(solver.solve_batched(problems(st)))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        with wlra.Solver(prec, profile=True) as ps:
            ps.set_batch_lanes(nl)
            ps.solve_batched(problems(0))
            torch.cuda.synchronize()
            prof = ps.profile(work=True)
        ms = np.array([r["ms"] for rs in allres for r in rs])
        sweeps = np.array([r["sweeps"] for rs in allres for r in rs])
        ok, worst = 0, 0.0
        for rs in allres:
            for j, r in enumerate(rs):
                e = abs(r["objective"] - fstar[idx[j]]) / fstar[idx[j]]
                worst = max(worst, e)
                ok += int(e <= 1e-6 and r["status"] == 0)
        nsolve = len(idx) * steps
        hbm = {}
        for kname in STREAMING:
            if kname in prof and prof[kname][2] > 0:
                lc, kms, kb, kf = prof[kname]
                hbm[kname] = {"GB_per_s": kb / (kms / 1e3) / 1e9,
                              "frac_of_hbm_peak": kb / (kms / 1e3) / 1e9 / HBM_PEAK_GBS,
                              "ms_per_batch": kms, "launches": lc}
        tot = sum(v[1] for v in prof.values())
        out[name] = {"solves_per_s": nsolve / dt, "batch_ms": 1e3 * dt / steps,
                     "p50_solve_ms": float(np.percentile(ms, 50)),
                     "p99_solve_ms": float(np.percentile(ms, 99)),
                     "sweeps_per_solve": float(sweeps.mean()),
                     "sweeps_per_s": float(sweeps.sum() / dt),
                     "solves_meeting_1e-6": f"{ok}/{nsolve}", "max_rel_objective_err": worst,
                     "precision": prec, "streams": nl, "streaming_hbm": hbm,
                     "kernel_share": {k_: v[1] / tot for k_, v in
                                      sorted(prof.items(), key=lambda kv: -kv[1][1])[:6]}}
        log(f"# config4 {name}: {out[name]['solves_per_s']:.1f} solves/s, p50 "
            f"{out[name]['p50_solve_ms']:.1f} ms, p99 {out[name]['p99_solve_ms']:.1f} ms, "
            f"{ok}/{nsolve} meet 1e-6")
    return {"workload": "config4: 64 clips, m in {4800, 19200, 76800}, n in [100, 400], "
                        "k in [5, 40], r = k + [2, 8], W1 log-uniform; one wlra_solve_batched "
                        "call per step", "instances": len(idx),
            "working_set_bytes": ws_bytes, "variants": out}


def run_extensions(steps, warmup):
    """Sub-object: the solve's extensions on the 19200 x 200 workload (FP32).
      colweights  eq. (6) with one weight per column of the unweighted block
                  (w2 = 10**U(log10 0.5, log10 2)): solves/s and the objective
                  against the oracle's column-scaled Algorithm 1 converged
      foreground  the mask |A - X| > tau (tau 0.25) of the returned iterate,
                  written by the output pass: its cost per solve and its
                  counts against the generator's foreground support
      appended    frames arriving 20 at a time (n = 100, 120, .., 200): each
                  solve warm-started from the previous X1 and V, against
                  cold solves from the A1 start (ms and sweeps per append;
                  objective of the last against the oracle)"""
    import numpy as np
    import torch
    from gen import video
    from oracle import foreground as FG
    from oracle import swlr as O
    from paper_1703_06303_amd import wlra
    out = {}
    inst = video.config2()
    k, r = inst.k, inst.r
    inputs = device_inputs(inst)
    A, W1 = inputs("fp32")
    # column weights
    w2 = video.column_weights(inst.n - k, seed=6).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    fs = O.swlr_colweights(inst.A, inst.W1, w2, k, r, tol=1e-13, max_sweeps=500,
                           X1_0=inst.X1_0).F[-1]
    log(f"# extensions: column-weight F* in {time.perf_counter() - t0:.1f} s")
    W2 = torch.tensor(w2, dtype=torch.float32, device="cuda")
    with wlra.Solver("fp32") as s:
        def cw(i):
            return s.solve(A, k, r, W1=W1, tol=1e-7, init="random", seed=1000 + i, W2=W2)[2]
        for i in range(warmup):
            cw(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [cw(i) for i in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    relF = max(abs(x["objective"] - fs) / fs for x in res)
    out["colweights"] = {"solves_per_s": steps / dt, "ms_per_solve": 1e3 * dt / steps,
                         "sweeps_per_solve": float(np.mean([x["sweeps"] for x in res])),
                         "max_rel_objective_err": relF,
                         "solves_meeting_1e-6": f"{sum(abs(x['objective'] - fs) / fs <= 1e-6 for x in res)}/{steps}"}
    # foreground mask
    with wlra.Solver("fp32", profile=True) as s:
        for i in range(warmup + steps):
            if i == warmup:
                s.profile(reset=True)
            _, _, rs = s.solve(A, k, r, W1=W1, tol=1e-7, init="random", seed=2000 + i,
                               mask_tau=0.25)
        torch.cuda.synchronize()
        prof = s.profile()
    mask = rs["mask"].cpu().numpy()
    tp, fp, fn, tn = FG.mask_counts(mask, inst.fg)
    out["foreground"] = {"tau": 0.25, "output_pass_ms": prof.get("x2_out", (0, 0.0))[1] / steps,
                         "TP": tp, "FP": fp, "FN": fn, "TN": tn,
                         "precision": tp / max(tp + fp, 1), "recall": tp / max(tp + fn, 1)}
    # appended frames
    ns = list(range(100, inst.n + 1, 20))
    Af = torch.tensor(inst.A, dtype=torch.float32, device="cuda")
    W1d = W1
    warm, cold = [], []
    with wlra.Solver("fp32") as s:
        for rep in range(2):   # the first pass warms up
            X1p, Vp = None, None
            for n_t in ns:
                At = wlra.colmajor(Af[:, :n_t])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if X1p is None:
                    X1, _, rw = s.solve(At, k, r, W1=W1d, tol=1e-7, init="a1", want_factors=True)
                else:
                    X1, _, rw = s.solve(At, k, r, W1=W1d, tol=1e-7, init="given", X1_init=X1p,
                                        V_init=Vp, want_factors=True)
                torch.cuda.synchronize()
                tw = time.perf_counter() - t0
                t0 = time.perf_counter()
                _, _, rc = s.solve(At, k, r, W1=W1d, tol=1e-7, init="a1")
                torch.cuda.synchronize()
                tc = time.perf_counter() - t0
                X1p, Vp = X1, rw["factors"][2]
                if rep == 1:
                    warm.append((n_t, 1e3 * tw, rw["sweeps"], rw["objective"]))
                    cold.append((n_t, 1e3 * tc, rc["sweeps"], rc["objective"]))
    fl = O.swlr(inst.A, inst.W1, k, r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0).F[-1]
    out["appended"] = {
        "frames": ns,
        "warm_ms": [w[1] for w in warm], "warm_sweeps": [w[2] for w in warm],
        "cold_a1_ms": [c[1] for c in cold], "cold_a1_sweeps": [c[2] for c in cold],
        "warm_ms_per_append": float(np.mean([w[1] for w in warm[1:]])),
        "cold_ms_per_append": float(np.mean([c[1] for c in cold[1:]])),
        "last_rel_objective_err_warm": abs(warm[-1][3] - fl) / fl,
        "last_rel_objective_err_cold": abs(cold[-1][3] - fl) / fl}
    log(f"# extensions: colweights {out['colweights']['solves_per_s']:.1f} solves/s; mask "
        f"precision {out['foreground']['precision']:.3f} recall {out['foreground']['recall']:.3f}; "
        f"appended {out['appended']['warm_ms_per_append']:.2f} vs "
        f"{out['appended']['cold_ms_per_append']:.2f} ms")
    return out


def run_frames(args):
    """Solve time against the number of frames n at a fixed frame size
    (the analogue of the paper's Fig. 3(c)): GPU FP32 vs the FP64 oracle on
    the same clip and start, each point parity-checked (F within 1e-6 of the
    oracle's converged F)."""
    import numpy as np
    import torch
    from gen import video
    from oracle import swlr as O
    from paper_1703_06303_amd import wlra
    k, r = 15, 16
    rows = []
    for n in args.frames:
        inst = video.make_instance(120, 160, n, k, r, 3, fg="blobs", w1=("loguniform", 1.0, 4.0),
                                   seed=video.BASE_SEED + 7000 + n, dtype=np.float32)
        t0 = time.perf_counter()
        ref = O.swlr(inst.A, inst.W1, k, r, tol=1e-7, max_sweeps=200, X1_0=inst.X1_0)
        t_cpu = time.perf_counter() - t0
        fs = O.swlr(inst.A, inst.W1, k, r, tol=1e-12, max_sweeps=500, X1_0=ref.X1).F[-1]
        inputs = device_inputs(inst)
        A, W1 = inputs("fp32")
        X0 = wlra.colmajor(torch.tensor(inst.X1_0, dtype=torch.float32, device="cuda"))
        with wlra.Solver("fp32") as s:
            s.reserve(inst.m, inst.n, k, r)
            for _ in range(2):
                s.solve(A, k, r, W1=W1, tol=1e-7, init="given", X1_init=X0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, _, res = s.solve(A, k, r, W1=W1, tol=1e-7, init="given", X1_init=X0)
            torch.cuda.synchronize()
            t_gpu = (time.perf_counter() - t0) / args.steps
        e = abs(res["objective"] - fs) / fs
        rows.append({"n": n, "gpu_ms": 1e3 * t_gpu, "oracle_ms": 1e3 * t_cpu,
                     "gpu_sweeps": res["sweeps"], "oracle_sweeps": ref.sweeps,
                     "rel_objective_err": e, "meets_1e-6": bool(e <= 1e-6 and res["status"] == 0)})
        log(f"# frames n={n}: GPU {1e3 * t_gpu:.2f} ms ({res['sweeps']} sweeps), oracle "
            f"{1e3 * t_cpu:.0f} ms ({ref.sweeps} sweeps), relF {e:.1e}")
    ok = sum(r_["meets_1e-6"] for r_ in rows)
    line = {"metric": "sWLR solve time vs number of frames (GPU FP32 vs FP64 oracle)",
            "value": rows[-1]["gpu_ms"], "unit": "ms per solve at the largest n", "n_gpus": 1,
            "steps": args.steps, "warmup": 2, "ms_per_step": rows[-1]["gpu_ms"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"frames: 120x160 frames (m=19200), n in {list(args.frames)}, "
                                   f"k={k}, r={r}, W1 log-uniform; paper's rule tol 1e-7"},
            "points_meeting_1e-6": f"{ok}/{len(rows)}", "points": rows}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2",
                    choices=("config1", "config2", "config3", "config4", "frames", "learn"))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="config2 only: skip the config3 and config4 sub-objects")
    ap.add_argument("--cpu-solves", type=int, default=6)
    ap.add_argument("--learn-train", type=int, default=1024,
                    help="training clips for the warm-start network (0: no learned start)")
    ap.add_argument("--learn-epochs", type=int, default=200)
    ap.add_argument("--learn-heldout", type=int, default=48)
    ap.add_argument("--save-weights", default="",
                    help="write the trained network's parameters (raw float32) here")
    ap.add_argument("--learn-weights", default=None,
                    help="raw float32 network weights to load instead of training (default: "
                         "the committed weights trained on 20000 clips; the learn workload "
                         "trains unless this is given)")
    ap.add_argument("--frames", type=int, nargs="+", default=[50, 100, 200, 300, 400, 500, 600])
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.learn_weights is None:
        args.learn_weights = ("" if args.workload == "learn" else
                              os.path.join(ROOT, "paper_1703_06303_amd", "weights",
                                           "warmstart_config2.f32"))
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    # host generation (warm-start clips, batched clips) runs in worker
    # processes forked here, before this process touches the GPU
    pool = None
    wants_pool = (args.calib_copy == 0 and
                  ((args.workload == "config2" and (args.learn_train > 0 or not args.no_extra))
                   or args.workload in ("config4", "learn")))
    if wants_pool:
        from paper_1703_06303_amd import warmstart as WS
        pool = WS.make_pool(12)

    import numpy as np
    import torch
    if args.calib_copy > 0:
        # A plain device-to-device copy of known size: HBM counters read for
        # it give the scale between counter units and bytes moved.
        nbytes = args.calib_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": nbytes, "calib_copy_bytes_written": nbytes}))
        return
    from paper_1703_06303_amd import wlra

    if args.workload == "frames":
        run_frames(args)
        return
    if args.workload == "learn":
        # train (or load) the warm-start network and compare the random, A1
        # and learned starts on the held-out clips; no schedule timing
        _, rep = train_learned(pool, args)
        print(json.dumps({"metric": "learned warm start: held-out sweeps and solve time",
                          "learned_start": rep}), flush=True)
        return
    if args.workload == "config4":
        sub = run_config4(pool, args.steps, args.warmup, one_lane=True)
        head = sub["variants"]["mixed_4streams"]
        line = {"metric": METRIC, "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["batch_ms"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "bf16+f32", "data": "synthetic",
                "config": {"workload": sub["workload"], "instances": sub["instances"],
                           "variant": "mixed_4streams"},
                "vs_plain": head["solves_per_s"] / sub["variants"]["fp32_4streams"]["solves_per_s"],
                "variants": sub["variants"]}
        print(json.dumps(line), flush=True)
        return

    inst, plain_prec = workload(args.workload)
    t0 = time.perf_counter()
    fstar, fsrc = reference_objective(inst)
    log(f"# F* = {fstar!r} from {fsrc} ({time.perf_counter() - t0:.1f} s)")
    inputs = device_inputs(inst)

    learned_params, learned_report = None, None
    if args.workload == "config2" and (args.learn_train > 0 or args.learn_weights):
        learned_params, learned_report = train_learned(pool, args)

    specs = variants(plain_prec, learned_params is not None)
    out = time_schedules(inst, specs, fstar, args.steps, args.warmup, inputs,
                         model=learned_params)
    # the headline family is the metric's (learned start + mixed precision)
    # when it is built for the workload; like the plain schedule, it is
    # quoted at its fastest stopping rule whose every solve meets 1e-6
    fam = next(h for h in ("learned+mixed", "mixed", "plain") if h in out or h == "plain")
    head = best_of(out, fam) or (fam if fam in out else "plain_tol1e-07")
    hv = out[head]
    spec = specs[head]
    bp = best_plain(out)
    fam_best = {f: best_of(out, f) for f in ("plain", "mixed", "a1+mixed", "learned+mixed")
                if f == "plain" or f in out}
    held = None
    if learned_params is not None and args.learn_heldout > 0:
        from gen import video
        chosen = {b: specs[b] for b in fam_best.values() if b is not None}
        ho = [video.config5_seed(i, heldout=True) for i in range(args.learn_heldout)]
        t0 = time.perf_counter()
        held = heldout_stopping(pool, learned_params, ho, chosen)
        log(f"# held-out stopping rules ({time.perf_counter() - t0:.1f} s): " +
            ", ".join(f"{k_} {v['meeting_1e-6']}" for k_, v in held.items()))

    # profiled repeat of the headline steps: per-kernel device time from events
    with wlra.Solver(spec["precision"], profile=True) as psolver:
        psolver.reserve(inst.m, inst.n, inst.k, inst.r)

        def prun(step):
            A, W1 = inputs(spec["precision"])
            return psolver.solve(A, inst.k, inst.r, W1=W1, w1_const=inst.w1_const or 1.0,
                                 tol=spec["tol"], max_sweeps=200, init=spec["init"],
                                 seed=1000 + step, model=learned_params)[2]
        prun(0)
        psolver.profile(reset=True)
        presults = [prun(i) for i in range(args.steps)]
        torch.cuda.synchronize()
        prof = psolver.profile(work=True)
    total_ms = sum(v[1] for v in prof.values())
    dname, (dlaunch, dms, dbytes, dflops) = max(prof.items(), key=lambda kv: kv[1][1])
    roof = roofline_of(dname, dlaunch, dms, dbytes, dflops, presults, inst.n - inst.k)
    roof["traffic"] = measured_traffic(dname, args.workload, spec["precision"])
    roof["kernel"] = dname
    roof["launches"] = dlaunch
    roof["avg_launch_us"] = dms / dlaunch * 1e3
    roof["share_of_device_time"] = dms / total_ms if total_ms else None

    start = {"learned": "learned start", "a1": "A1 start", "random": "random start"}[spec["init"]]
    line = {
        "metric": METRIC,
        "value": hv["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hv["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "mixed": "bf16+f32"}[spec["precision"]],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: m={inst.m} ({inst.frame_hw[0]}x{inst.frame_hw[1]}) "
                               f"n={inst.n} k={inst.k} r={inst.r}, {head} schedule, {start}",
                   "m": inst.m, "n": inst.n, "k": inst.k, "r": inst.r, "variant": head},
        "vs_plain": hv["solves_per_s"] / out[bp]["solves_per_s"] if bp else None,
        "vs_plain_schedule": bp,
        "fastest_meeting_1e-6": fam_best,
        "heldout_stopping_rules": held,
        "solves_meeting_1e-6": hv["solves_meeting_1e-6"],
        "max_rel_objective_err": hv["max_rel_objective_err"],
        "reference_objective": {"value": fstar, "source": fsrc},
        "variants": out,
        "learned_start": learned_report,
        "roofline": roof,
        "kernel_ms_per_solve": {k_: v[1] / args.steps for k_, v in sorted(prof.items())},
    }
    if args.workload == "config2" and not args.no_extra:
        line["config3"] = run_config3(5, 1)
        line["config4"] = run_config4(pool, 2, 1)
        line["extensions"] = run_extensions(10, 2)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, args.cpu_solves, 1e-7)
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
