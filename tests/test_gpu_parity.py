"""End-to-end parity of the HIP path against the CPU oracle, through the C ABI.

FP64 bar: max relative Frobenius error per selected block <= 1e-11
(rel_err in tests/_util.py).  Sizes span several 64 x 32 product tiles,
several 16-column inverse panels and ragged tails; partitioned runs use
explicit and cost-model bounds.
"""
import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import gen_problem, equilibrium_B
from tests._util import rel_err, even_bounds

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


def run_solver(S, A, B, partitions=1, bounds=None, fused=True, with_xr=True):
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR = S.DeviceBlocks.empty(n, b, a) if with_xr else None
    XL = S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=partitions, bounds=bounds)
    if fused:
        sol.solve(dA, dB, XR, XL)
    else:
        sol.factor(dA, XR)
        sol.selected_solve(dB, XL)
    sol.sync()
    out = (XR.to_host() if with_xr else None), XL.to_host()
    sol.destroy()
    return out


CASES = [
    # n, b, a, partitions, bounds
    (1, 5, 0, 1, None),
    (2, 3, 0, 1, None),
    (16, 32, 0, 1, None),
    (16, 32, 0, 2, None),
    (16, 32, 0, 4, None),
    (9, 37, 0, 3, [0, 3, 6, 9]),
    (7, 40, 19, 1, None),
    (12, 24, 20, 3, None),
    (10, 33, 65, 4, [0, 2, 4, 6, 10]),
    (6, 70, 17, 2, [0, 1, 6]),
    # reduced systems of 16 to 30 blocks (long halves in the reduced solve)
    (24, 16, 0, 9, None),
    (18, 9, 5, 9, [0, 1, 3, 5, 7, 9, 11, 13, 15, 18]),
    (30, 12, 20, 12, None),
    (40, 8, 12, 16, None),
    # more than 16 partitions with an arrow: the tip sum of P + 1 inputs is chained
    (40, 8, 12, 17, None),
    (48, 6, 10, 24, None),
]


@pytest.mark.parametrize("n,b,a,P,bounds", CASES)
def test_parity_small(S, n, b, a, P, bounds):
    print(f"case n={n} b={b} a={a} P={P} bounds={bounds}", flush=True)
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-3, seed=n + b + a + P)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL = run_solver(S, A, B, P, bounds)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"  err R={eR:.3e} L={eL:.3e}", flush=True)
    assert eR < TOL and eL < TOL


def run_flags(S, A, B, partitions, flags):
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=partitions, flags=flags)
    sol.solve(dA, dB, XR, XL)
    sol.sync()
    out = XR.to_host(), XL.to_host()
    sol.destroy()
    return out


REDUCED_CASES = [
    # n, b, a, partitions, reduced_parts (reduced system of 2(P - 1) blocks)
    (24, 16, 0, 9, 1),
    (24, 16, 0, 9, 3),
    (24, 16, 0, 9, 4),
    (30, 12, 20, 12, 3),
    (40, 8, 12, 16, 4),
    (40, 8, 12, 16, 8),
    (48, 6, 10, 24, 1024),
    (18, 9, 5, 9, 5),
    # at the recursion's limits: reduced systems of 4 to 12 blocks, middle parts
    # of two blocks (nothing eliminated in them), a one-block first partition
    (6, 8, 0, 3, 3),
    (9, 10, 6, 4, 3),
    (10, 12, 0, 5, 4),
    (12, 9, 7, 5, 4),
    (14, 8, 5, 7, 3),
]


@pytest.mark.parametrize("n,b,a,P,Q", REDUCED_CASES)
def test_recursive_reduced_solve_parity(S, n, b, a, P, Q):
    """The reduced system solved by the partitioned scheme with Q parts,
    recursively (Sec. III-B), against the dense inverse and against the
    oracle's partitioned solve in the same order of elimination.

    Broadening 0.05: the partitioned orders eliminate without pivoting across
    blocks, and at 1e-3 the oracle's own partitioned solve of several of these
    small instances is 1e-9 to 3e-8 away from the dense inverse (rounding
    amplified by near-singular Schur complements of the middle parts), which
    is the method's conditioning, not the kernels'.  At 0.05 it is at most 2e-13."""
    print(f"case reduced_parts n={n} b={b} a={a} P={P} Q={Q}", flush=True)
    A, B = gen_problem(n, b, a, E=0.3, eta=0.05, seed=70 + n + b + a + P + Q)
    R0, L0 = oracle.solve_dense(A, B)
    bounds = S.partition_bounds(n, b, a, P)
    if Q == 1:
        R1, L1 = oracle.prgf(A, B, bounds)
    else:
        R1, L1 = oracle.prgf(A, B, bounds, reduced_split=True, reduced_parts=Q)
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=P, bounds=bounds, reduced_parts=Q)
    sol.solve(dA, dB, XR, XL)
    sol.sync()
    XR, XL = XR.to_host(), XL.to_host()
    sol.destroy()
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    oR, oL = rel_err(XR, R1), rel_err(XL, L1)
    print(f"  err vs dense R={eR:.3e} L={eL:.3e}; vs same-order oracle R={oR:.3e} L={oL:.3e}", flush=True)
    assert eR < TOL and eL < TOL
    assert oR < TOL and oL < TOL


@pytest.mark.parametrize("n,b,a,P", [(12, 40, 0, 1), (14, 33, 0, 3), (9, 36, 20, 1), (10, 28, 24, 2)])
def test_plain_schedule_parity(S, n, b, a, P):
    """BT_PLAIN, the one-launch-per-product reference schedule behind every
    "vs plain RGF" figure, against the oracle."""
    print(f"case BT_PLAIN n={n} b={b} a={a} P={P}", flush=True)
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-3, seed=40 + n + b + a + P)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL = run_flags(S, A, B, P, S.BT_PLAIN)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"  err R={eR:.3e} L={eL:.3e}", flush=True)
    assert eR < TOL and eL < TOL


@pytest.mark.parametrize("P", [1, 2])
def test_config_bt_n16_b32_seed0(S, P):
    """The small configuration as specified (n=16, b=32, E=0.3, eta=1e-3,
    seed 0), sequential RGF and two partitions, every selected block."""
    from paper_2601_04904_amd.synth import config_problem
    A, B = config_problem("bt_n16_b32")
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL = run_flags(S, A, B, P, 0)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"bt_n16_b32 P={P}: err R={eR:.3e} L={eL:.3e}", flush=True)
    assert eR < TOL and eL < TOL


def test_factor_then_selected_solve_matches_fused(S):
    A, B = gen_problem(10, 48, 16, seed=3)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL = run_solver(S, A, B, 2, None, fused=False)
    assert rel_err(XR, R0) < TOL and rel_err(XL, L0) < TOL


def test_without_xr_output(S):
    A, B = gen_problem(8, 40, 0, seed=4)
    _, L0 = oracle.solve_dense(A, B)
    _, XL = run_solver(S, A, B, 1, None, with_xr=False)
    assert rel_err(XL, L0) < TOL


def test_two_right_hand_sides_share_factors(S):
    """G^< and G^> style: one factor, two selected solves."""
    import torch
    n, b, a = 9, 32, 12
    A, B1 = gen_problem(n, b, a, seed=11)
    from paper_2601_04904_amd.synth import gen_B
    B2 = gen_B(np.random.Generator(np.random.PCG64(12)), n, b, a)
    dA = S.DeviceBlocks.from_host(A)
    XR, XL1, XL2 = (S.DeviceBlocks.empty(n, b, a) for _ in range(3))
    sol = S.Solver(n, b, a, partitions=2)
    sol.factor(dA, XR)
    sol.selected_solve(S.DeviceBlocks.from_host(B1), XL1)
    sol.selected_solve(S.DeviceBlocks.from_host(B2), XL2)
    sol.sync()
    R0, L1 = oracle.solve_dense(A, B1)
    _, L2 = oracle.solve_dense(A, B2)
    assert rel_err(XR.to_host(), R0) < TOL
    assert rel_err(XL1.to_host(), L1) < TOL
    assert rel_err(XL2.to_host(), L2) < TOL
    sol.destroy()
    torch.cuda.synchronize()


def test_repeat_calls_identical(S):
    """Same handle, same inputs: bitwise identical results (no races)."""
    n, b, a = 12, 64, 32
    A, B = gen_problem(n, b, a, seed=21)
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    sol = S.Solver(n, b, a, partitions=3)
    outs = []
    for _ in range(3):
        XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
        sol.solve(dA, dB, XR, XL)
        sol.sync()
        outs.append((XR.to_host(), XL.to_host()))
    for o in outs[1:]:
        for f in ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip"):
            assert np.array_equal(getattr(o[0], f), getattr(outs[0][0], f))
            assert np.array_equal(getattr(o[1], f), getattr(outs[0][1], f))
    sol.destroy()


def test_singular_block_reported(S):
    from paper_2601_04904_amd._lib import BTError, BT_ERR_SINGULAR
    n, b = 4, 16
    A, B = gen_problem(n, b, 0, seed=1)
    A.diag[0][:, 3] = 0.0
    A.upper[0][:, :] = 0.0      # keep block 0 decoupled so its Schur block stays singular
    A.lower[0][:, :] = 0.0
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, 0), S.DeviceBlocks.empty(n, b, 0)
    sol = S.Solver(n, b, 0)
    sol.solve(dA, dB, XR, XL)
    with pytest.raises(BTError) as ei:
        sol.sync()
    assert ei.value.status == BT_ERR_SINGULAR
    assert "block 0" in str(ei.value)
    sol.sync()   # the flag is cleared after being reported
    sol.destroy()


def test_state_and_argument_errors(S):
    from paper_2601_04904_amd._lib import BTError, BT_ERR_STATE, BT_ERR_INVALID
    sol = S.Solver(4, 8, 0)
    XL = S.DeviceBlocks.empty(4, 8, 0)
    A, B = gen_problem(4, 8, 0, seed=0)
    with pytest.raises(BTError) as ei:
        sol.selected_solve(S.DeviceBlocks.from_host(B), XL)
    assert ei.value.status == BT_ERR_STATE
    sol.destroy()
    sol = S.Solver(4, 8, 3)
    A, B = gen_problem(4, 8, 0, seed=0)   # no arrow blocks for an a = 3 handle
    with pytest.raises(BTError) as ei:
        sol.solve(S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B), None, XL)
    assert ei.value.status == BT_ERR_INVALID
    sol.destroy()


def test_fluctuation_dissipation_on_gpu(S):
    """B = c(A^H - A) gives X^< = c(X^R - X^R^H) blockwise, a check of SQ against SI."""
    n, b, a = 20, 64, 40
    A, _ = gen_problem(n, b, a, eta=1e-2, seed=8)
    c = 0.5
    B = equilibrium_B(A, c)
    XR, XL = run_solver(S, A, B, 4, None)
    worst = 0.0
    for i in range(n):
        ref = c * (XR.diag[i] - XR.diag[i].conj().T)
        worst = max(worst, np.linalg.norm(XL.diag[i] - ref) / np.linalg.norm(ref))
    for i in range(n - 1):
        ref = c * (XR.upper[i] - XR.lower[i].conj().T)
        worst = max(worst, np.linalg.norm(XL.upper[i] - ref) / np.linalg.norm(ref))
    ref = c * (XR.tip - XR.tip.conj().T)
    worst = max(worst, np.linalg.norm(XL.tip - ref) / np.linalg.norm(ref))
    assert worst < TOL


@pytest.mark.parametrize("n,b,a,P", [(3, 1024, 0, 1), (2, 1024, 1024, 1), (4, 1000, 24, 2)])
def test_parity_at_maximum_block_size(S, n, b, a, P):
    """Blocks at the largest supported size (1024: the inverse kernel's limit)
    and a ragged size just under it."""
    print(f"case n={n} b={b} a={a} P={P}", flush=True)
    A, B = gen_problem(n, b, a, E=0.3, eta=1e-2, seed=31 + n + b + a)
    R0, L0 = oracle.solve_dense(A, B)
    XR, XL = run_solver(S, A, B, P, None)
    eR, eL = rel_err(XR, R0), rel_err(XL, L0)
    print(f"  err R={eR:.3e} L={eL:.3e}", flush=True)
    assert eR < TOL and eL < TOL
