"""The SD-style workload at full size (n = 32 blocks of b = 1024, Sec. IV's
single-GPU sweep shape): the two-partition form the bench reports and the
sequential sweep, on every selected block, against the oracle's partitioned
solve with the library's bounds (Sec. III-B).

Tolerance 1e-11 per block (rel_err).  Oracle-only evaluations of this input
fix the rounding spread: the sequential sweep on the block-reversed matrix is
within 1.8e-12 of the sequential sweep, and the two-partition order within
1.7e-12 of it.
"""
import pytest

import oracle
from paper_2601_04904_amd.synth import config_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11


def test_sd_workload_full_size():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver as S
    n, b = 32, 1024
    print("generating sd_n32_b1024", flush=True)
    A, B = config_problem("sd_n32_b1024")
    bounds = S.partition_bounds(n, b, 0, 2)
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    out = {}
    for P in (2, 1):
        XR, XL = S.DeviceBlocks.empty(n, b, 0), S.DeviceBlocks.empty(n, b, 0)
        sol = S.Solver(n, b, 0, partitions=P, bounds=bounds if P == 2 else None, flags=S.BT_GRAPH)
        sol.solve(dA, dB, XR, XL)
        sol.sync()
        out[P] = XR.to_host(), XL.to_host()
        sol.destroy()
        print(f"GPU P={P} done", flush=True)
    del dA, dB
    print(f"oracle partitioned solve, bounds {bounds}", flush=True)
    R0, L0 = oracle.prgf(A, B, bounds)
    for P, (XR, XL) in out.items():
        eR, eL = rel_err(XR, R0), rel_err(XL, L0)
        print(f"P={P}: err R={eR:.2e} L={eL:.2e}", flush=True)
        assert eR < TOL and eL < TOL
