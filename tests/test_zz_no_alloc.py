"""wlra_solve_noalloc (the entry point for callers that cannot allocate)
against wlra_solve on the same handle and inputs: two calls in a row, the
second on a smaller problem, each compared with wlra_solve to the parity bar
of its precision; and the size check that rejects a problem whose workspace
exceeds the fixed scratch.  Runs through the C ABI."""
import numpy as np
import pytest

from gen import video
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-5}


def _run(s, inst, noalloc, tol, max_sweeps):
    import torch
    dt = s.dtype
    A = dev(inst.A, dt)
    W1 = dev(inst.W1_dense(), dt) if inst.W1 is not None else None
    X0 = dev(inst.X1_0, dt)
    X1, X2, res = s.solve(A, inst.k, inst.r, W1=W1, w1_const=inst.w1_const or 1.0, tol=tol,
                          max_sweeps=max_sweeps, init="given", X1_init=X0, want_x2=True,
                          raise_on_error=False, noalloc=noalloc)
    torch.cuda.synchronize()
    return host(X1), host(X2), res


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", ["fp32", "mixed", "fp64"])
def test_noalloc_matches_solve_on_two_calls(precision):
    from paper_1703_06303_amd import wlra
    big = video.config2() if precision != "fp64" else video.config1()
    small = video.small(m_hw=(30, 40), n=70, k=9, r=13, seed=11)
    with wlra.Solver(precision) as s:
        for inst, tol, ms in ((big, 1e-7, 60), (small, 0.0, 5)):
            X1a, X2a, ra = _run(s, inst, False, tol, ms)
            X1b, X2b, rb = _run(s, inst, True, tol, ms)
            same = bool(np.array_equal(X1a, X1b) and np.array_equal(X2a, X2b))
            print(precision, inst.m, inst.n, inst.k, inst.r, "status", ra["status"], rb["status"],
                  "sweeps", ra["sweeps"], rb["sweeps"], "relX1", _rel(X1b, X1a), "relX2",
                  _rel(X2b, X2a), "bit-identical", same, flush=True)
            assert ra["status"] >= 0 and rb["status"] == ra["status"]
            assert rb["sweeps"] == ra["sweeps"]
            assert _rel(X1b, X1a) <= TOL[precision] and _rel(X2b, X2a) <= TOL[precision]
            assert abs(rb["objective"] - ra["objective"]) <= 1e-12 * abs(ra["objective"]) + 1e-300


def test_noalloc_rejects_problem_beyond_scratch():
    import torch
    from paper_1703_06303_amd import wlra
    m, n, k, r = 76800, 600, 50, 60
    with wlra.Solver("fp32") as s:
        A = torch.zeros((n, m), dtype=torch.float32, device="cuda").t()
        X1 = torch.zeros((k, m), dtype=torch.float32, device="cuda").t()
        p = wlra.make_problem(A, k, r, w1_const=1e3, tol=1e-7, max_sweeps=5, init="a1", X1_out=X1)
        res = wlra.Result()
        rc = s.lib.wlra_solve_noalloc(s.h, p, res)
        assert rc == wlra.E_SCRATCH and res.status == wlra.E_SCRATCH
    with wlra.Solver("fp32", profile=True) as sp:
        inst = video.small(m_hw=(10, 12), n=20, k=3, r=5, seed=2)
        A = dev(inst.A, torch.float32)
        with pytest.raises(wlra.WlraError):
            sp.solve(A, inst.k, inst.r, W1=dev(inst.W1_dense(), torch.float32), noalloc=True)
