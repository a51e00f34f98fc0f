"""The uneven-batch workload at its real sizes: the first wave of eight
instances of the 512-instance sweep (`batch_specs`: n 16..96, b 64..384,
a 0..256, E drawn in [-1, 1], broadening 1e-3), solved as one FP64 batch
with HIP-graph replay as the batch bench runs it, against the oracle's
sequential sweep (Alg. 1/2 and the arrowhead extension of Sec. III-A) on
every selected block.

Inputs come from the host generator with the same recipe and seeds (the
bench draws them on the device; the values differ, the shapes and
distributions do not).  Tolerance 1e-11 per block (rel_err): the oracle's
own sweep on the block-reversed matrix, an independent evaluation, agrees
with it to at most 3.4e-12 on these eight instances (X^<; 1.4e-12 for X^R).
"""
import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import batch_specs, gen_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-11
FIELDS = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


def test_first_wave_of_batch_workload(S):
    specs = batch_specs(512)[:8]
    problems = [gen_problem(sp["n"], sp["b"], sp["a"], E=sp["E"], eta=sp["eta"], seed=sp["seed"])
                for sp in specs]
    wspecs = [dict(n=sp["n"], b=sp["b"], a=sp["a"], flags=S.BT_GRAPH) for sp in specs]
    dA = [S.DeviceBlocks.from_host(A) for A, _ in problems]
    dB = [S.DeviceBlocks.from_host(B) for _, B in problems]
    XR = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
    XL = [S.DeviceBlocks.empty(sp["n"], sp["b"], sp["a"]) for sp in specs]
    bs = S.BatchSolver(wspecs)
    print("batch of 8 uneven instances: capture", flush=True)
    bs.solve(dA, dB, XR, XL)
    bs.sync()
    first = [(x.to_host(), y.to_host()) for x, y in zip(XR, XL)]
    print("replay", flush=True)
    bs.solve(dA, dB, XR, XL)
    bs.sync()
    out = [(x.to_host(), y.to_host()) for x, y in zip(XR, XL)]
    bs.destroy()
    for (r0, l0), (r1, l1) in zip(first, out):
        for f in FIELDS:
            assert np.array_equal(getattr(r0, f), getattr(r1, f)), f
            assert np.array_equal(getattr(l0, f), getattr(l1, f)), f
    for sp, (A, B), (R, L) in zip(specs, problems, out):
        solve = oracle.rgf_bta if sp["a"] else oracle.rgf_bt
        R0, L0 = solve(A, B)
        eR, eL = rel_err(R, R0), rel_err(L, L0)
        print(f"n={sp['n']} b={sp['b']} a={sp['a']} E={sp['E']:.3f}: err R={eR:.2e} L={eL:.2e}", flush=True)
        assert eR < TOL and eL < TOL
