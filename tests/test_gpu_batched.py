"""Batched solves (wlra_solve_batched) on the GPU through the C ABI.

A batch advances its instances in lockstep: the single-workgroup small steps
of all of them run as one launch each, their streaming passes on several
streams.  Each instance must come out exactly as a single solve of it would
(the kernels are deterministic and the batch runs the same ones), match the
FP64 oracle, and report its own status.
"""
import numpy as np
import pytest

from gen import video
from oracle import swlr as O

from .gpu_util import batch_problems, gpu_solve, host, rel

pytestmark = pytest.mark.gpu

# uneven (h, w, n, k, r, const W1): shapes differ in every dimension
BATCH = [
    (10, 10, 13, 3, 5, True), (257, 1, 40, 17, 20, False), (13, 10, 70, 33, 36, False),
    (8, 8, 9, 1, 2, True), (9, 10, 20, 5, 5, False), (15, 5, 12, 0, 4, False),
    (20, 30, 150, 20, 24, False), (30, 40, 60, 10, 12, True), (17, 23, 90, 7, 12, False),
    (12, 12, 33, 6, 9, False),
]


def _inst(i, h, w, n, k, r, const):
    wspec = ("const", 7.5) if const else ("loguniform", 0.0, 2.5)
    return video.make_instance(h, w, n, k, r, 2, fg="bernoulli", fg_p=0.1, fg_lo=0.5, fg_hi=1.0,
                               noise=0.05, w1=wspec, seed=5000 + 7 * i)


@pytest.fixture(scope="module")
def s64():
    from paper_1703_06303_amd.wlra import Solver
    s = Solver("fp64")
    yield s
    s.close()


@pytest.mark.parametrize("lanes", [1, 4, 7])
def test_batched_equals_single_and_oracle(s64, lanes):
    insts = [_inst(i, *sh) for i, sh in enumerate(BATCH)]
    probs, keep = batch_problems(s64, insts, 0.0, 4)
    s64.set_batch_lanes(lanes)
    res = s64.solve_batched(probs)
    for j, inst in enumerate(insts):
        X1b, X2b = host(keep["X1"][j]), host(keep["X2"][j])
        X1s, X2s, rs = gpu_solve(s64, inst, 0.0, 4)
        print("batched", lanes, BATCH[j], res[j], flush=True)
        # k = 0 is H_r(A) directly: converged with no X1 update
        want = (0, 0) if inst.k == 0 else (1, 4)
        assert (res[j]["status"], res[j]["sweeps"]) == (rs["status"], rs["sweeps"]) == want
        assert np.array_equal(X2b, X2s) and np.array_equal(X1b, X1s)
        assert res[j]["objective"] == rs["objective"]
        w = inst.W1 if inst.W1 is not None else inst.w1_const
        ref = O.swlr(inst.A, w, inst.k, inst.r, tol=0.0, max_sweeps=4, X1_0=inst.X1_0)
        X = np.hstack([X1b, X2b]) if inst.k > 0 else X2b
        assert rel(X, ref.X) <= 1e-10


def test_batched_converged_mixed_precision():
    """A batch in mixed precision: every instance converges and meets its own
    oracle objective."""
    from paper_1703_06303_amd.wlra import Solver
    insts = [video.make_instance(h, w, n, k, r, 3, fg="blobs", w1=("loguniform", 1.0, 4.0),
                                 seed=7000 + i, dtype=np.float32)
             for i, (h, w, n, k, r) in enumerate([(24, 32, 60, 8, 11), (40, 48, 100, 12, 17),
                                                   (16, 20, 45, 5, 9), (30, 40, 80, 20, 23)])]
    with Solver("mixed") as smx:
        probs, keep = batch_problems(smx, insts, 1e-7, 200)
        res = smx.solve_batched(probs)
    for j, inst in enumerate(insts):
        ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0)
        print("mixed batch", j, res[j], "F*", ref.F[-1], flush=True)
        assert res[j]["status"] == 0
        assert abs(res[j]["objective"] - ref.F[-1]) <= 1e-6 * ref.F[-1]


def test_batched_statuses(s64):
    import torch
    from paper_1703_06303_amd import wlra
    insts = [_inst(i, *sh) for i, sh in enumerate(BATCH[:4])]
    probs, keep = batch_problems(s64, insts, 0.0, 2)
    # instance 1: a zero weight -> its own status E_WEIGHT, the others run
    keep["W1"][1].zero_()
    s64.set_batch_lanes(3)
    res = s64.solve_batched(probs)
    assert [r["status"] for r in res] == [1, wlra.E_WEIGHT, 1, 1]
    # a malformed instance rejects the whole batch before anything runs
    bad = list(probs)
    bad[2] = wlra.make_problem(keep["A"][2], insts[2].k, insts[2].n + 1, X1_out=keep["X1"][2])
    with pytest.raises(wlra.WlraError) as e:
        s64.solve_batched(bad)
    assert e.value.code == wlra.E_ARG
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_batched_largest_config4_clips_meet_fstar(precision):
    """The six largest clips of the 64-clip batched workload (240 x 320
    frames, m = 76800, k >= 33, n - k >= 256: the LDS per-row solves and the
    cooperative eigen kernel) in one wlra_solve_batched call on four
    concurrent lanes, from the library's random starts.  Each objective must
    land within 1e-6 (relative) of the FP64 oracle's converged objective
    stored in tests/golden/config4_fstar.json."""
    import json
    import os
    from paper_1703_06303_amd.wlra import Solver
    with open(os.path.join(os.path.dirname(__file__), "golden", "config4_fstar.json")) as f:
        fstar = {d["i"]: d["fstar"] for d in json.load(f)["instances"]}
    shapes = video.config4_shapes()
    big = [i for i, (h, w, n, k, r) in enumerate(shapes)
           if h * w == 76800 and k >= 33 and n - k >= 256]
    assert len(big) >= 4
    insts = [video.config4_instance(i, shapes[i]) for i in big]
    with Solver(precision) as s:
        s.set_batch_lanes(4)
        probs, keep = batch_problems(s, insts, 1e-7, 200, init="random",
                                     seeds=[11 + i for i in big])
        res = s.solve_batched(probs)
    for j, i in enumerate(big):
        e = abs(res[j]["objective"] - fstar[i]) / fstar[i]
        print("config4 clip", i, shapes[i], precision, res[j], "relF", e, flush=True)
        assert res[j]["status"] == 0
        assert e <= 1e-6
