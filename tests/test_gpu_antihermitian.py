"""BT_SIGMA_ANTIHERMITIAN: for anti-Hermitian Sigma^< (as in NEGF) the solve
forms one block of each conjugate pair of B updates, and the k-row products
of the X^< sweep, from the other.  The result must match the oracle to the
FP64 bar and the general path on the same input; an ill-conditioned case
checks that the derived blocks do not amplify rounding beyond a small factor
of the general path.
"""
import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import gen_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


def run(S, A, B, P=1, bounds=None, flags=0, precision=None):
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    kw = {} if precision is None else {"precision": precision}
    sol = S.Solver(n, b, a, partitions=P, bounds=bounds, flags=flags, **kw)
    res = sol.solve(dA, dB, XR, XL)
    sol.sync()
    out = XR.to_host(), XL.to_host(), res
    sol.destroy()
    return out


CASES = [
    (1, 5, 0, 1, None),
    (2, 3, 0, 1, None),
    (16, 32, 0, 1, None),
    (16, 32, 0, 4, None),
    (9, 37, 0, 3, [0, 3, 6, 9]),
    (7, 40, 19, 1, None),
    (12, 24, 20, 3, None),
    (10, 33, 65, 4, [0, 2, 4, 6, 10]),
    (6, 70, 17, 2, [0, 1, 6]),
    (24, 64, 48, 6, None),
]


@pytest.mark.parametrize("n,b,a,P,bounds", CASES)
def test_antihermitian_parity(S, n, b, a, P, bounds):
    print(f"case n={n} b={b} a={a} P={P} bounds={bounds}", flush=True)
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-3, seed=100 + n + b + a + P)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL, _ = run(S, A, B, P, bounds, flags=S.BT_SIGMA_ANTIHERMITIAN)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"  err R={eR:.3e} L={eL:.3e}", flush=True)
    assert eR < TOL and eL < TOL
    # the general path on the same input agrees to rounding
    XR1, XL1, _ = run(S, A, B, P, bounds)
    assert rel_err(XR, XR1) < 1e-13 and rel_err(XL, XL1) < TOL


def test_antihermitian_mixed_within_tolerance_or_fallback(S):
    A, B = gen_problem(12, 64, 32, E=0.3, eta=1e-2, seed=5)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL, (est, fb) = run(S, A, B, 3, flags=S.BT_SIGMA_ANTIHERMITIAN, precision=S.BT_MIXED)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"mixed: err R={eR:.2e} L={eL:.2e} est={est:.2e} fallback={fb}", flush=True)
    if fb:
        assert eR < TOL and eL < TOL
    else:
        assert eR <= 1e-4 and eL <= 1e-4 and est <= 1e-4


def test_antihermitian_ill_conditioned_stays_near_general_path(S):
    """A BTA case whose middle partition is ill-conditioned (the general path
    itself is at 4e-11 here): the derived blocks stay within a small factor."""
    n, b, a, P = 24, 64, 48, 3
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-3, seed=100 + n + b + a + P)
    R0, L0 = oracle.solve_dense(A, B)
    for P in (1, 3):
        _, XL0, _ = run(S, A, B, P)
        _, XL1, _ = run(S, A, B, P, flags=S.BT_SIGMA_ANTIHERMITIAN)
        e0, e1 = rel_err(XL0, L0), rel_err(XL1, L0)
        print(f"P={P}: general {e0:.2e}, anti-Hermitian {e1:.2e}", flush=True)
        assert e1 < max(TOL, 4 * e0)


def test_antihermitian_fluctuation_dissipation(S):
    """B = c(A^H - A) (anti-Hermitian for real c) gives X^< = c(X^R - X^R^H)
    blockwise: a closed-form check of the flag's path against its own SI."""
    from paper_2601_04904_amd.synth import equilibrium_B
    n, b, a = 20, 64, 40
    A, _ = gen_problem(n, b, a, eta=1e-2, seed=8)
    c = 0.5
    B = equilibrium_B(A, c)
    for P in (1, 4):
        XR, XL, _ = run(S, A, B, P, flags=S.BT_SIGMA_ANTIHERMITIAN)
        worst = 0.0
        for i in range(n):
            ref = c * (XR.diag[i] - XR.diag[i].conj().T)
            worst = max(worst, np.linalg.norm(XL.diag[i] - ref) / np.linalg.norm(ref))
        for i in range(n - 1):
            ref = c * (XR.upper[i] - XR.lower[i].conj().T)
            worst = max(worst, np.linalg.norm(XL.upper[i] - ref) / np.linalg.norm(ref))
            ref = c * (XR.lower[i] - XR.upper[i].conj().T)
            worst = max(worst, np.linalg.norm(XL.lower[i] - ref) / np.linalg.norm(ref))
        for i in range(n):
            ref = c * (XR.arrow_right[i] - XR.arrow_bottom[i].conj().T)
            worst = max(worst, np.linalg.norm(XL.arrow_right[i] - ref) / np.linalg.norm(ref))
        ref = c * (XR.tip - XR.tip.conj().T)
        worst = max(worst, np.linalg.norm(XL.tip - ref) / np.linalg.norm(ref))
        print(f"P={P}: worst {worst:.2e}", flush=True)
        assert worst < TOL
