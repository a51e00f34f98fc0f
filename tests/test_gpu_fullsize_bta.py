"""Parity at the full bta_n128_b384_a512 size (n=128 blocks of b=384 plus an
arrow tip of a=512, N=49664, E=0.3, eta=1e-3) in the launch configuration the
benchmark times (16 concurrent partitions, default bounds).

The same two checks as the BT full-size test: the block-row identities
sum_j A_ij X^R_ji = I and sum_j A_ij X^<_ji = sum_j B_ij (X^R_ij)^H on every
block row, the arrow tip row included (j over i-1, i, i+1 and the tip; every
block for the tip row), held to 4x the residual the oracle's own 16-partition
sweep leaves; and the element-wise comparison with the oracle's result of the
same form (oracle.prgf, same bounds, reduced system split in two), held to
max(1e-11, 4 x that form's FP64 floor: the spread between two oracle
evaluations whose rounding differs).  Both references are stored in
tests/golden/fullsize_floors_bta_n128_b384_a512.json, written by
tests/golden/make_fullsize_floors.py from the oracle alone.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2601_04904_amd.synth import config_problem
from tests._util import rel_err

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps
DEFAULT_BOUNDS_P16 = list(range(0, 129, 8))   # library default for n=128, b=384, a=512, P=16


def blk(M, i, j, n):
    """Block (i, j) of a BTA block set; index n is the arrow tip."""
    if i == n and j == n:
        return M.tip
    if j == n:
        return M.arrow_right[i]
    if i == n:
        return M.arrow_bottom[j]
    if i == j:
        return M.diag[i]
    if j == i + 1:
        return M.upper[i]
    return M.lower[j]          # j == i - 1


def residuals_bta(A, B, XR, XL):
    n = A.diag.shape[0]
    wr = wl = 0.0
    for i in range(n + 1):
        js = list(range(n + 1)) if i == n else [j for j in (i - 1, i, i + 1) if 0 <= j < n] + [n]
        d = blk(A, i, i, n).shape[0]
        R = sum(blk(A, i, j, n) @ blk(XR, j, i, n) for j in js) - np.eye(d)
        sR = sum(np.linalg.norm(blk(A, i, j, n)) * np.linalg.norm(blk(XR, j, i, n)) for j in js)
        L = sum(blk(A, i, j, n) @ blk(XL, j, i, n) for j in js) \
            - sum(blk(B, i, j, n) @ blk(XR, i, j, n).conj().T for j in js)
        sL = sum(np.linalg.norm(blk(A, i, j, n)) * np.linalg.norm(blk(XL, j, i, n)) for j in js) \
            + sum(np.linalg.norm(blk(B, i, j, n)) * np.linalg.norm(blk(XR, i, j, n)) for j in js)
        wr = max(wr, float(np.linalg.norm(R) / sR))
        wl = max(wl, float(np.linalg.norm(L) / sL))
    return wr, wl


def floors():
    with open(os.path.join(HERE, "golden", "fullsize_floors_bta_n128_b384_a512.json")) as f:
        rec = json.load(f)
    assert rec["workload"] == "bta_n128_b384_a512"
    return rec["forms"]


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


@pytest.fixture(scope="module")
def result(S):
    A, B = config_problem("bta_n128_b384_a512")
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    print(f"[fullsize-bta] GPU solve n={n} b={b} a={a} partitions=16", flush=True)
    dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
    XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
    sol = S.Solver(n, b, a, partitions=16, bounds=DEFAULT_BOUNDS_P16)
    sol.solve(dA, dB, XR, XL)
    sol.sync()
    out = (A, B, XR.to_host(), XL.to_host())
    sol.destroy()
    return out


def test_fullsize_bta_default_bounds(S):
    assert S.partition_bounds(128, 384, 512, 16) == DEFAULT_BOUNDS_P16


def test_fullsize_bta_identities(result):
    A, B, XR, XL = result
    wr, wl = residuals_bta(A, B, XR, XL)
    ref = floors()["P16"]["residuals"]
    base = 16 * EPS * A.tip.shape[0]
    br, bl = max(base, 4 * ref["XR"]), max(base, 4 * ref["XL"])
    print(f"[fullsize-bta] residuals X^R {wr:.2e} X^< {wl:.2e} (bounds {br:.2e} / {bl:.2e})", flush=True)
    assert wr < br and wl < bl, (wr, wl)


def test_fullsize_bta_against_oracle_same_form(result):
    A, B, XR, XL = result
    fl = floors()["P16"]["floor"]
    print("[fullsize-bta] oracle, same form as the GPU: P=16", flush=True)
    XRo, XLo = oracle.prgf(A, B, DEFAULT_BOUNDS_P16, reduced_split=True)
    eR, eL = rel_err(XR, XRo), rel_err(XL, XLo)
    bR, bL = max(1e-11, 4 * fl["XR"]), max(1e-11, 4 * fl["XL"])
    print(f"[fullsize-bta] vs oracle (same form): X^R {eR:.2e} X^< {eL:.2e} "
          f"(floor {fl['XR']:.2e} / {fl['XL']:.2e}, bounds {bR:.2e} / {bL:.2e})", flush=True)
    assert eR <= bR, eR
    assert eL <= bL, eL
