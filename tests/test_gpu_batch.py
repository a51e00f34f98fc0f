"""Batched uneven instances in one schedule: each result equals the oracle
(FP64 bar 1e-11, mixed bar 1e-4 or FP64 re-run) and equals the same
instance solved alone (bitwise for FP64: the products of an instance do not
depend on what else shares the launch)."""
import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import gen_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu
FIELDS = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


SPECS = [
    dict(n=9, b=64, a=0, partitions=1, E=0.2, seed=1),
    dict(n=14, b=32, a=16, partitions=2, E=-0.5, seed=2),
    dict(n=5, b=96, a=40, partitions=1, E=0.9, seed=3),
    dict(n=12, b=48, a=0, partitions=3, E=0.0, seed=4),
    dict(n=1, b=20, a=7, partitions=1, E=0.4, seed=5),
]


def _solve_batch(S, specs, problems):
    dA = [S.DeviceBlocks.from_host(A) for A, _ in problems]
    dB = [S.DeviceBlocks.from_host(B) for _, B in problems]
    XR = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
    XL = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
    bs = S.BatchSolver(specs)
    try:
        err, fb = bs.solve(dA, dB, XR, XL)
    except S.BTToleranceError as ex:     # a re-run instance still above its tol: results written
        err, fb = ex.err, ex.fallback
    bs.sync()
    out = [(x.to_host(), y.to_host()) for x, y in zip(XR, XL)]
    bs.destroy()
    return out, err, fb


def test_batch_fp64_matches_oracle_and_alone(S):
    problems = [gen_problem(sp["n"], sp["b"], sp["a"], E=sp["E"], eta=1e-3, seed=sp["seed"]) for sp in SPECS]
    out, err, fb = _solve_batch(S, SPECS, problems)
    for sp, (A, B), (XR, XL) in zip(SPECS, problems, out):
        R0, L0 = oracle.solve_dense(A, B)
        eR, eL = rel_err(XR, R0), rel_err(XL, L0)
        print(sp, f"R={eR:.2e} L={eL:.2e}", flush=True)
        assert eR < 1e-11 and eL < 1e-11
    # alone vs in the batch: identical bits
    for i in (0, 3):
        alone, _, _ = _solve_batch(S, [SPECS[i]], [problems[i]])
        for f in FIELDS:
            assert np.array_equal(getattr(alone[0][0], f), getattr(out[i][0], f)), f
            assert np.array_equal(getattr(alone[0][1], f), getattr(out[i][1], f)), f


def test_batch_mixed_and_fp64_instances(S):
    specs = [dict(SPECS[0], precision=S.BT_MIXED), dict(SPECS[1]), dict(SPECS[2], precision=S.BT_MIXED, tol=1e-15)]
    problems = [gen_problem(sp["n"], sp["b"], sp["a"], E=sp["E"], eta=1e-2, seed=sp["seed"]) for sp in specs]
    out, err, fb = _solve_batch(S, specs, problems)
    assert fb[2] is True            # tolerance 1e-15 forces the FP64 re-run
    assert err[2] > 1e-15           # ... whose estimate stays above it (BT_ERR_TOLERANCE)
    assert fb[1] is False and err[1] == 0.0
    for k, (sp, (A, B), (XR, XL)) in enumerate(zip(specs, problems, out)):
        R0, L0 = oracle.solve_dense(A, B)
        e = max(rel_err(XR, R0), rel_err(XL, L0))
        print(k, sp.get("precision", 0), e, err[k], fb[k], flush=True)
        if sp.get("precision", 0) == S.BT_MIXED and not fb[k]:
            assert e <= 1e-4
        else:
            assert e < 1e-11


def test_batch_with_caller_workspace_matches_library_allocation(S):
    """bt_si_sq_batch_create_in: the handle works in a torch-allocated
    workspace and gives the same bits as a handle that allocates its own;
    the workspace block is reused by a second handle after destroy."""
    import torch
    specs = [dict(n=10, b=40, a=12, partitions=2), dict(n=7, b=24, a=0, partitions=1),
             dict(n=12, b=33, a=0, partitions=3)]
    probs = [gen_problem(sp["n"], sp["b"], sp["a"], E=0.2, eta=1e-3, seed=200 + i) for i, sp in enumerate(specs)]
    dA = [S.DeviceBlocks.from_host(A) for A, _ in probs]
    dB = [S.DeviceBlocks.from_host(B) for _, B in probs]
    outs = []
    ws = torch.empty(S.batch_workspace_bytes(specs), dtype=torch.uint8, device="cuda")
    for workspace in (None, ws, ws):
        XR = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
        XL = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
        bs = S.BatchSolver(specs, workspace=workspace)
        bs.solve(dA, dB, XR, XL)
        bs.sync()
        bs.destroy()
        outs.append([(x.to_host(), y.to_host()) for x, y in zip(XR, XL)])
    for run in outs[1:]:
        for (xr0, xl0), (xr, xl) in zip(outs[0], run):
            for f in S.FIELDS:
                assert np.array_equal(getattr(xr, f), getattr(xr0, f))
                assert np.array_equal(getattr(xl, f), getattr(xl0, f))
    for (A, B), (xr, xl) in zip(probs, outs[0]):
        R0, L0 = oracle.solve_dense(A, B)
        assert rel_err(xr, R0) < 1e-11 and rel_err(xl, L0) < 1e-11


def test_batch_instance_with_recursive_reduced_solve(S):
    """An instance whose reduced system is split into three parts recursively
    (Sec. III-B) in a batch with others: against the oracle's partitioned solve
    in the same order, and bitwise equal to the same instance solved alone."""
    specs = [dict(n=24, b=16, a=0, partitions=9, reduced_parts=3),
             dict(n=10, b=40, a=12, partitions=2), dict(n=30, b=12, a=20, partitions=12, reduced_parts=4)]
    problems = [gen_problem(sp["n"], sp["b"], sp["a"], E=0.3, eta=0.05, seed=200 + i)
                for i, sp in enumerate(specs)]
    out, err, fb = _solve_batch(S, specs, problems)
    for sp, (A, B), (XR, XL) in zip(specs, problems, out):
        bounds = S.partition_bounds(sp["n"], sp["b"], sp["a"], sp["partitions"])
        q = sp.get("reduced_parts", 0)
        R1, L1 = oracle.prgf(A, B, bounds, reduced_split=True, reduced_parts=q if q else 2)
        eR, eL = rel_err(XR, R1), rel_err(XL, L1)
        print(sp, f"R={eR:.2e} L={eL:.2e}", flush=True)
        assert eR < 1e-11 and eL < 1e-11
    alone, _, _ = _solve_batch(S, [specs[2]], [problems[2]])
    for f in FIELDS:
        assert np.array_equal(getattr(alone[0][0], f), getattr(out[2][0], f)), f
        assert np.array_equal(getattr(alone[0][1], f), getattr(out[2][1], f)), f
