"""GPU parity of the mixed-precision mode (the X1 updates' A2 product on a
BF16 copy, then one exact refinement sweep), called through the C ABI.

Bars: at the same start and the same number of sweeps, X = [X1 X2] within
1e-5 (relative Frobenius) of the oracle's mixed schedule (`swlr_mixed`: the
same steps in float64 with step 7's A2 product on bf16(A2), then one exact
sweep); and the objective of a
converged mixed solve within 1e-6 (relative) of the converged FP64 optimum.
"""
import numpy as np
import pytest

from gen import video
from oracle import swlr as O

from .gpu_util import gpu_solve, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smx():
    from paper_1703_06303_amd.wlra import Solver
    s = Solver("mixed")
    yield s
    s.close()


@pytest.fixture(scope="module")
def s32():
    from paper_1703_06303_amd.wlra import Solver
    s = Solver("fp32")
    yield s
    s.close()


def _w(inst):
    return inst.W1 if inst.W1 is not None else inst.w1_const


def _blob_instance(seed=31, m_hw=(40, 48), n=80, k=10, r=14):
    return video.make_instance(m_hw[0], m_hw[1], n, k, r, 3, fg="blobs",
                               w1=("loguniform", 1.0, 4.0), seed=seed, dtype=np.float32)


@pytest.mark.parametrize("sweeps", [0, 1, 2, 4])
def test_mixed_same_sweeps(smx, sweeps):
    inst = _blob_instance()
    ref = O.swlr_mixed(inst.A, _w(inst), inst.k, inst.r, tol=0.0, max_sweeps=sweeps,
                       X1_0=inst.X1_0)
    X1, X2, res = gpu_solve(smx, inst, 0.0, sweeps)
    print("mixed sweeps", sweeps, res, flush=True)
    assert res["rc"] == 1 and res["sweeps"] == sweeps == ref.sweeps
    assert rel(np.hstack([X1, X2]), ref.X) <= 1e-5
    assert abs(res["objective"] - ref.F[-1]) <= 1e-6 * ref.F[-1]


@pytest.mark.parametrize("shape", [
    ((13, 11), 37, 0, 4),    # k = 0: exact H_r(A) after the BF16 pass
    ((13, 11), 37, 5, 5),    # r = k: D = 0
    ((17, 23), 90, 7, 12),   # ragged m = 391
])
def test_mixed_edge_shapes(smx, shape):
    m_hw, n, k, r = shape
    inst = _blob_instance(seed=41 + n + k, m_hw=m_hw, n=n, k=k, r=r)
    ref = O.swlr_mixed(inst.A, _w(inst), k, r, tol=0.0, max_sweeps=3, X1_0=inst.X1_0)
    X1, X2, res = gpu_solve(smx, inst, 0.0, 3)
    print("mixed shape", shape, res, flush=True)
    X = np.hstack([X1, X2]) if k > 0 else X2
    assert rel(X, ref.X) <= 1e-5
    assert abs(res["objective"] - ref.F[-1]) <= 1e-6 * ref.F[-1]


@pytest.fixture(scope="module")
def config2_fstar():
    inst = video.config2()
    ref = O.swlr(inst.A, inst.W1, inst.k, inst.r, tol=1e-13, max_sweeps=500, X1_0=inst.X1_0)
    return inst, ref.F[-1]


def test_mixed_config2_converged(smx, config2_fstar):
    inst, fstar = config2_fstar
    ref = O.swlr_mixed(inst.A, inst.W1, inst.k, inst.r, tol=1e-7, max_sweeps=200,
                       X1_0=inst.X1_0)
    X1, X2, res = gpu_solve(smx, inst, 1e-7, 200)
    print("mixed config2", res, "oracle mixed sweeps", ref.sweeps, flush=True)
    assert res["rc"] == 0
    assert abs(res["objective"] - fstar) <= 1e-6 * fstar
    assert abs(ref.F[-1] - fstar) <= 1e-6 * fstar
    if res["sweeps"] == ref.sweeps:
        assert rel(np.hstack([X1, X2]), ref.X) <= 1e-5


def test_mixed_config2_random_starts(smx, config2_fstar):
    """The library's own random starts: every solve meets the objective."""
    inst, fstar = config2_fstar
    for seed in (1, 2, 3):
        _, _, res = gpu_solve(smx, inst, 1e-7, 200, init="random", want_x2=False)
        print("mixed config2 random", seed, res, flush=True)
        assert res["rc"] == 0
        assert abs(res["objective"] - fstar) <= 1e-6 * fstar


def test_config3_mixed_and_fp32_meet_closed_form(smx, s32):
    """Config 3 has a constant W1, so the optimum is known in closed form:
    X* = H_r(A S) S^-1 with S = diag(w, .., w, 1, .., 1), and
    F* = sum of sigma_i(A S)^2 for i > r (problem (5) and eq. (2))."""
    inst = video.config3()
    s = np.ones(inst.n)
    s[:inst.k] = inst.w1_const
    sv = np.linalg.svd(inst.A * s, compute_uv=False)
    fstar = float(np.sum(sv[inst.r:] ** 2))
    for solver, name in ((smx, "mixed"), (s32, "fp32")):
        _, _, res = gpu_solve(solver, inst, 1e-7, 200, want_x2=False)
        print("config3", name, res, "F*", fstar, flush=True)
        assert res["rc"] == 0
        assert abs(res["objective"] - fstar) <= 1e-6 * fstar
