"""Mixed-precision path: Schur-update products in complex64 on FP32 MFMA, the
inverses, reduced system and residual check in FP64.  Bar: max relative
Frobenius error per block <= 1e-4 against the oracle, or the FP64 re-run
taken; the error estimate is reported for every result.
"""
import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import gen_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


def run(S, A, B, P=1, tol=1e-4):
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=P, precision=S.BT_MIXED, tol=tol)
    est, fb = sol.solve(dA, dB, XR, XL)
    sol.sync()
    out = XR.to_host(), XL.to_host(), est, fb
    sol.destroy()
    return out


@pytest.mark.parametrize("n,b,a,P,eta", [(12, 64, 0, 1, 1e-2), (12, 64, 0, 2, 1e-2),
                                         (10, 48, 32, 3, 1e-2), (16, 96, 0, 1, 1e-3)])
def test_mixed_within_tolerance_or_fallback(S, n, b, a, P, eta):
    A, B = gen_problem(n, b, a, E=0.3, eta=eta, seed=7 + n + b)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL, est, fb = run(S, A, B, P)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"n={n} b={b} a={a} P={P} eta={eta}: err R={eR:.2e} L={eL:.2e} est={est:.2e} fallback={fb}",
          flush=True)
    assert np.isfinite(est) and est > 0
    if fb:
        assert eR < 1e-11 and eL < 1e-11
    else:
        assert eR <= 1e-4 and eL <= 1e-4
        assert est <= 1e-4
        # the estimate does not understate the true error by much
        assert est >= 0.1 * max(eR, eL)


def test_forced_fallback_gives_fp64_accuracy(S):
    """tol below what FP64 reaches: the re-run happens, its results are written
    and FP64-accurate, and the call reports that the estimate is still above tol."""
    A, B = gen_problem(10, 40, 16, eta=1e-2, seed=3)
    R0, L0 = oracle.solve_dense(A, B)
    n, b, a = 10, 40, 16
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=2, precision=S.BT_MIXED, tol=1e-15)
    with pytest.raises(S.BTToleranceError) as ex:
        sol.solve(dA, dB, XR, XL)
    sol.sync()
    assert ex.value.fallback and ex.value.err > 1e-15
    assert rel_err(XR.to_host(), R0) < 1e-11 and rel_err(XL.to_host(), L0) < 1e-11
    sol.destroy()


def test_split_mixed_fallback_refactors(S):
    """factor() then selected_solve() on a mixed handle: the FP64 re-run that
    the estimate triggers repeats the factor too, so X^R and X^< both reach
    FP64 accuracy even though the factor's A-chain ran with FP32 products."""
    n, b, a = 12, 48, 0
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-2, seed=21)
    R0, L0 = oracle.solve_dense(A, B)
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=1, precision=S.BT_MIXED, tol=1e-9)
    sol.factor(dA, XR)
    sol.sync()
    eR_mixed = rel_err(XR.to_host(), R0)
    try:
        est, fb = sol.selected_solve(dB, XL)
    except S.BTToleranceError as ex:     # estimate still above 1e-9 after FP64: results written
        est, fb = ex.err, ex.fallback
    sol.sync()
    eR, eL = rel_err(XR.to_host(), R0), rel_err(XL.to_host(), L0)
    print(f"mixed factor X^R err {eR_mixed:.2e}; after selected_solve est={est:.2e} fb={fb} "
          f"X^R {eR:.2e} X^< {eL:.2e}", flush=True)
    assert eR_mixed > 1e-9          # the mixed factor alone is FP32-accurate
    assert fb
    assert eR < 1e-11 and eL < 1e-11
    sol.destroy()


def test_mixed_is_less_accurate_than_fp64_but_close(S):
    """Without fallback the mixed result differs from FP64 at the FP32 level, not more."""
    A, B = gen_problem(8, 64, 0, eta=5e-2, seed=5)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL, est, fb = run(S, A, B, 1, tol=1.0)
    assert not fb
    e = max(rel_err(XR, R0), rel_err(XL, L0))
    assert 1e-9 < e < 1e-4
