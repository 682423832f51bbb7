#!/usr/bin/env python3
"""Throughput of the sWLR solve (Dutta & Li, arXiv 1703.06303) on one MI355X.

One step = one complete solve of problem (5) with Algorithm 1 from a random
start, on a seeded synthetic video matrix resident in HBM (default: 120 x 160
frames, m = 19200, n = 200, rank-3 background, 10% 8x8 blob foreground,
N(0, 0.02^2) noise, k = 20 background frames with W1 = 10**U(1, 4), r = 25,
FP32 storage).  Every solve's objective is checked against F*, the FP64
oracle's converged objective (or the closed form for a constant W1), at
relative 1e-6.

Schedules timed side by side (`variants` in the output):
  plain          FP32 (FP64 for config1), the Section 4.1 rule with tol 1e-7
  plain_tol1e-5  the same with tol 1e-5 (where the mixed phase stops)
  mixed          A2 staged in BF16, sweeps to 1e-5, then one exact sweep
  a1+mixed       the same from X1_0 = A1
  learned+mixed  the same from the learned warm start (config2): the network
                 is first trained on GPU solves of --learn-train clips of the
                 same generator (disjoint seeds) and compared with the random
                 and A1 starts on --learn-heldout held-out clips
                 (`learned_start` in the output)
`value` is the headline schedule's solves/s (learned+mixed when built, else
mixed) and `vs_plain` its ratio to the plain schedule.
`--workload config4` times the batched workload instead (64 clips of uneven
shape per wlra_solve_batched call).

Prints one JSON line (see the keys below).  `roofline` is for the kernel with
the largest device time, from HIP events bracketing each launch on the
library's stream in a profiled repeat of the timed steps.  `cpu_baseline` is
the FP64 oracle (NumPy/LAPACK) on the host cores, on a bounded sample.
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

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs, scaled by
# the same counters read for a plain copy of known size (reads x2.0, writes
# x1.0).  An entry holds only while the kernel's source files are
# byte-identical to the ones measured (SHA-256 of their concatenation, in the
# order listed); otherwise traffic is reported as null.
TRAFFIC = {
    ("eig", "config2", "mixed"): (595867, ("k_eig.hip", "eig_small.h", "launch.h", "common.h"),
                                  "0f5ed553bd32245c669c0148bae03fe2a22dc347e8294e90cf1fc0834c713e3d"),
}


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
    """(instance, storage precision of the plain solve, F* source)."""
    from gen import video
    if name == "config2":
        return video.config2(), "fp32"
    if name == "config1":
        return video.config1(), "fp64"
    if name == "config3":
        return video.config3(), "fp32"
    raise SystemExit(f"unknown workload {name}")


def reference_objective(inst, name):
    """F* of the workload: the FP64 oracle converged far below the paper's
    threshold, or the closed form when W1 is constant (problem (5) with
    eq. (2): F* = sum of sigma_i(A S)^2, i > r, S = diag(w..w, 1..1))."""
    import numpy as np
    from oracle import swlr as O
    if inst.W1 is None and inst.m * inst.n > 5_000_000:
        s = np.ones(inst.n)
        s[:inst.k] = inst.w1_const
        sv = np.linalg.svd(inst.A * s, compute_uv=False)
        return float(np.sum(sv[inst.r:] ** 2)), "closed form H_r(A S) S^-1"
    w = inst.W1 if inst.W1 is not None else inst.w1_const
    ref = O.swlr(inst.A, w, inst.k, inst.r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0)
    return ref.F[-1], f"FP64 oracle at tol 1e-13 ({ref.sweeps} sweeps)"


# Schedules compared at equal final objective.  "plain" is Algorithm 1 with
# the paper's threshold; "plain_tol1e-5" stops where the mixed phase stops;
# "mixed" stages A2 in BF16 and ends with one exact sweep.
def variants(plain_prec, learned=False):
    v = {"plain": dict(precision=plain_prec, tol=1e-7, init="random"),
         "plain_tol1e-5": dict(precision=plain_prec, tol=1e-5, init="random")}
    if plain_prec == "fp32":
        v["mixed"] = dict(precision="mixed", tol=1e-7, init="random")
        v["a1+mixed"] = dict(precision="mixed", tol=1e-7, init="a1")
        if learned:
            v["learned+mixed"] = dict(precision="mixed", tol=1e-7, init="learned")
    return v


def train_learned(pool, args, log):
    """Train the warm-start network on GPU solves of config-2 clips (training
    seeds), then compare the random, A1 and learned starts on held-out seeds."""
    import numpy as np
    from gen import video
    from paper_1703_06303_amd import warmstart as WS
    from paper_1703_06303_amd import wlra
    s = wlra.Solver("fp32")
    tr = [video.config5_seed(i) for i in range(args.learn_train)]
    X, T, info, t_data = WS.build_dataset(s, pool, tr)
    log(f"# warm start: {len(tr)} training solves in {t_data:.1f} s")
    t0 = time.perf_counter()
    params, hist = WS.train(s, X, T, 200, 25, epochs=args.learn_epochs, batch=128, lr=1e-3)
    t_train = time.perf_counter() - t0
    log(f"# warm start: {args.learn_epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3f} -> "
        f"{hist[-1]:.3f}")
    ho = [video.config5_seed(i, heldout=True) for i in range(args.learn_heldout)]
    ev = WS.evaluate(s, pool, params, ho)
    Fr = np.array([x[2] for x in ev["random"]])
    held = {}
    for init, v in ev.items():
        sw = np.array([x[0] for x in v])
        ms = np.array([x[1] for x in v])
        F = np.array([x[2] for x in v])
        held[init] = {"sweeps_mean": float(sw.mean()), "sweeps_max": int(sw.max()),
                      "solve_ms_mean": float(ms.mean()),
                      "converged": int(sum(x[3] == 0 for x in v)),
                      "max_rel_objective_vs_random_start": float(np.max(np.abs(F - Fr) / Fr))}
    report = {"train_instances": len(tr), "train_data_s": t_data, "epochs": args.learn_epochs,
              "train_s": t_train, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
              "heldout_instances": len(ho), "heldout": held,
              "training_solves_converged": int(sum(x[1] == 0 for x in info))}
    return params, report


def kernel_work(name, inst, res_list, elt, elt_a2, launches):
    """Algorithmic bytes and flops of one launch of kernel `name` (`launches`
    of it ran over the solves in res_list)."""
    m, n, k, r = inst.m, inst.n, inst.k, inst.r
    n2, l = n - k, r - k
    if name == "update":
        bytes_ = m * k * elt + m * n2 * elt_a2 + 2 * m * k * elt
        flops = 2 * m * n * k + 2 * m * k * k
        return bytes_, flops, "hbm"
    if name == "gram_X1A2":
        return m * k * elt + m * n2 * elt_a2, 2 * m * k * n2, "hbm"
    if name == "gram_A2":
        return m * n2 * elt_a2, m * n2 * n2, "fp64"
    if name == "change":
        # a2 [V_p dV] per row, then the K x K form (K = 2l + 2k) per row
        return m * n2 * elt_a2 + 2 * m * k * elt, m * (4 * l * n2 + (2 * l + 2 * k) ** 2), "hbm"
    if name == "eig":
        mv = sum(x["eig_matvecs"] for x in res_list)
        return 0, 2.0 * n2 * n2 * mv / max(launches, 1), "fp64"
    return 0, 0, "latency"


def cpu_baseline(inst, sample_solves, tol):
    import numpy as np
    from oracle import swlr as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    w = inst.W1 if inst.W1 is not None else inst.w1_const
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(sample_solves):
        res = O.swlr(inst.A, w, inst.k, inst.r, tol=tol, max_sweeps=200, X1_0=inst.X1_0)
        sweeps.append(res.sweeps)
    dt = time.perf_counter() - t0
    return {"value": sample_solves / dt, "unit": "solves/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{sample_solves} full solves of the same workload with the paper's "
                      f"schedule (tol {tol}, {sweeps} sweeps), FP64 NumPy/LAPACK, {dt:.1f} s"}


def run_batched(args):
    """Batched workload: 64 seeded clips of uneven shape solved by one
    wlra_solve_batched call per step, all inputs resident in HBM.  Compared:
    one lane (instances one after another) vs four lanes, FP32 and mixed."""
    import numpy as np
    import torch
    from gen import video
    from paper_1703_06303_amd import wlra
    shapes = video.config4_shapes()
    gold_path = os.path.join(ROOT, "tests", "golden", "config4_fstar.json")
    fstar = {}
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            fstar = {d["i"]: d["fstar"] for d in json.load(f)["instances"]}
    t0 = time.perf_counter()
    insts = [video.config4_instance(i, sh) for i, sh in enumerate(shapes)]
    print(f"# generated {len(insts)} instances in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    A = [wlra.colmajor(torch.tensor(x.A, dtype=torch.float32, device=dev)) for x in insts]
    W = [wlra.colmajor(torch.tensor(x.W1, dtype=torch.float32, device=dev)) for x in insts]
    X1 = [wlra.colmajor(torch.empty((x.m, x.k), dtype=torch.float32, device=dev)) for x in insts]

    def problems(step):
        return [wlra.make_problem(A[i], x.k, x.r, W1=W[i], tol=1e-7, max_sweeps=200,
                                  init="random", seed=1000 * step + i, X1_out=X1[i])
                for i, x in enumerate(insts)]

    out = {}
    for name, prec, lanes in (("fp32_1lane", "fp32", 1), ("fp32_4lanes", "fp32", 4),
                              ("mixed_4lanes", "mixed", 4)):
        solver = wlra.Solver(prec)
        solver.set_batch_lanes(lanes)
        for w in range(max(1, args.warmup)):
            solver.solve_batched(problems(100 + w))
        torch.cuda.synchronize()
        allres = []
        t0 = time.perf_counter()
        for st in range(args.steps):
            allres.append(solver.solve_batched(problems(st)))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms = np.array([r["ms"] for rs in allres for r in rs])
        sweeps = np.array([r["sweeps"] for rs in allres for r in rs])
        ok = errs = 0
        worst = 0.0
        for rs in allres:
            for i, r in enumerate(rs):
                if i in fstar:
                    e = abs(r["objective"] - fstar[i]) / fstar[i]
                    worst = max(worst, e)
                    ok += int(e <= 1e-6 and r["status"] == 0)
                    errs += 1
        nsolve = len(insts) * args.steps
        out[name] = {"solves_per_s": nsolve / dt, "batch_ms": 1e3 * dt / args.steps,
                     "p50_solve_ms": float(np.percentile(ms, 50)),
                     "p99_solve_ms": float(np.percentile(ms, 99)),
                     "sweeps_per_solve": float(sweeps.mean()),
                     "sweeps_per_s": float(sweeps.sum() / dt),
                     "solves_meeting_1e-6": f"{ok}/{errs}" if errs else "no reference",
                     "max_rel_objective_err": worst if errs else None,
                     "precision": prec, "lanes": lanes}
        print(f"# {name}: {out[name]}", file=sys.stderr, flush=True)
        del solver
    head = out["mixed_4lanes"]
    line = {
        "metric": "WLRA solves/s to rel. objective 1e-6 vs FP64 oracle; learned+mixed vs plain",
        "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["batch_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": "config4: 64 clips, m in {4800, 19200, 76800}, n in [100, 400], "
                               "k in [5, 40], r = k + [2, 8], W1 log-uniform; one "
                               "wlra_solve_batched call per step",
                   "instances": len(insts), "variant": "mixed_4lanes"},
        "vs_plain": head["solves_per_s"] / out["fp32_1lane"]["solves_per_s"],
        "variants": out,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-solves", type=int, default=6)
    ap.add_argument("--learn-train", type=int, default=1024,
                    help="training clips for the warm-start network (0: no learned start)")
    ap.add_argument("--learn-epochs", type=int, default=200)
    ap.add_argument("--learn-heldout", type=int, default=48)
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    # instance generation for the warm-start network runs in worker processes
    # forked here, before this process touches the GPU
    pool = None
    if args.workload == "config2" and args.learn_train > 0 and args.calib_copy == 0:
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

    if args.workload == "config4":
        run_batched(args)
        return
    inst, plain_prec = workload(args.workload)
    t0 = time.perf_counter()
    fstar, fsrc = reference_objective(inst, args.workload)
    print(f"# F* = {fstar!r} from {fsrc} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)

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

    learned_params, learned_report = None, None
    if pool is not None:
        learned_params, learned_report = train_learned(
            pool, args, lambda msg: print(msg, file=sys.stderr, flush=True))

    def run(solver, spec, step):
        A, W1 = inputs(spec["precision"])
        return solver.solve(A, inst.k, inst.r, W1=W1, w1_const=inst.w1_const or 1.0,
                            tol=spec["tol"], max_sweeps=200, init=spec["init"], seed=1000 + step,
                            model=learned_params if spec["init"] == "learned" else None)

    out = {}
    specs = variants(plain_prec, learned_params is not None)
    for name, spec in specs.items():
        solver = wlra.Solver(spec["precision"])
        solver.reserve(inst.m, inst.n, inst.k, inst.r)
        for i in range(args.warmup):
            run(solver, spec, i)
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            results.append(run(solver, spec, i)[2])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        objs = np.array([r["objective"] for r in results])
        relF = np.abs(objs - fstar) / fstar
        ok = int(np.sum((relF <= 1e-6) & (np.array([r["status"] for r in results]) == 0)))
        sw = np.array([r["sweeps"] for r in results])
        out[name] = {"solves_per_s": args.steps / dt, "ms_per_solve": 1e3 * dt / args.steps,
                     "sweeps_per_solve": float(sw.mean()), "sweeps_per_s": float(sw.sum() / dt),
                     "solves_meeting_1e-6": f"{ok}/{args.steps}",
                     "max_rel_objective_err": float(relF.max()), "precision": spec["precision"],
                     "tol": spec["tol"], "init": spec["init"], "_dt": dt, "_ok": ok}
        print(f"# {name}: {out[name]['solves_per_s']:.1f} solves/s, "
              f"{out[name]['sweeps_per_solve']:.1f} sweeps, {ok}/{args.steps} meet 1e-6",
              file=sys.stderr, flush=True)

    # the headline schedule is the metric's (learned start + mixed precision)
    # when it is built for the workload; the plain paper schedule is the
    # comparison
    head = next(h for h in ("learned+mixed", "mixed", "plain") if h in out)
    hv = out[head]
    spec = specs[head]

    # profiled repeat of the headline steps: per-kernel device time from events
    psolver = wlra.Solver(spec["precision"], profile=True)
    psolver.reserve(inst.m, inst.n, inst.k, inst.r)
    run(psolver, spec, 0)
    psolver.profile(reset=True)
    presults = []
    for i in range(args.steps):
        r_ = run(psolver, spec, i)[2]
        presults.append(r_)
    torch.cuda.synchronize()
    prof = psolver.profile()
    total_ms = sum(v[1] for v in prof.values())
    dname, (dlaunch, dms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_s = dms / dlaunch / 1e3
    elt = 8 if spec["precision"] == "fp64" else 4
    elt_a2 = 2 if spec["precision"] == "mixed" else elt
    bytes_, flops, bound = kernel_work(dname, inst, presults, elt, elt_a2, dlaunch)
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    elif bound == "fp64":
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "alu", "achieved": 0.0, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dname, args.workload, spec["precision"])
    roof["kernel"] = dname
    roof["launches"] = dlaunch
    roof["avg_launch_us"] = avg_s * 1e6
    roof["share_of_device_time"] = dms / total_ms if total_ms else None

    line = {
        "metric": "WLRA solves/s to rel. objective 1e-6 vs FP64 oracle; learned+mixed vs plain",
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
                               f"n={inst.n} k={inst.k} r={inst.r}, {head} schedule, random start",
                   "m": inst.m, "n": inst.n, "k": inst.k, "r": inst.r, "variant": head},
        "vs_plain": hv["solves_per_s"] / out["plain"]["solves_per_s"],
        "solves_meeting_1e-6": hv["solves_meeting_1e-6"],
        "max_rel_objective_err": hv["max_rel_objective_err"],
        "reference_objective": {"value": fstar, "source": fsrc},
        "variants": {k_: {kk: vv for kk, vv in v.items() if not kk.startswith("_")}
                     for k_, v in out.items()},
        "learned_start": learned_report,
        "roofline": roof,
        "kernel_ms_per_solve": {k_: v[1] / args.steps for k_, v in sorted(prof.items())},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, args.cpu_solves, 1e-7)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
