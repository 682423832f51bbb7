"""Write config4_fstar.json: the converged objective F* of each instance of the
batched workload (64 synthetic clips of uneven shape), from the FP64 oracle
alone (Algorithm 1 to tol 1e-12 from the instance's seeded start).

Run from the repository root:  python tests/golden/make_config4_fstar.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import video  # noqa: E402
from oracle import swlr as O  # noqa: E402


def one(args):
    i, shape = args
    inst = video.config4_instance(i, shape)
    t0 = time.perf_counter()
    ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-12, max_sweeps=300, X1_0=inst.X1_0)
    return {"i": i, "shape": list(shape), "m": inst.m, "n": inst.n, "k": inst.k, "r": inst.r,
            "fstar": ref.F[-1], "sweeps": ref.sweeps, "status": ref.status,
            "seconds": round(time.perf_counter() - t0, 1)}


def main():
    shapes = video.config4_shapes()
    jobs = list(enumerate(shapes))
    workers = int(os.environ.get("WORKERS", "4"))
    with ProcessPoolExecutor(workers) as ex:
        out = list(ex.map(one, jobs))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_fstar.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle/swlr.py, Algorithm 1 at tol 1e-12, max 300 sweeps",
                   "instances": out}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
