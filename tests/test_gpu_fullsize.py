"""Parity at the full bt_n64_b512 size (n=64, b=512, N=32768, E=0.3,
eta=1e-4) in the launch configurations the benchmark times: the sequential
sweep, 2 partitions and 8 partitions (the library's default bounds).

Each form is compared element by element with the oracle's result of the
SAME form (oracle.rgf_bt for the sequential sweep, oracle.prgf with the same
bounds and the reduced system split in two for the partitioned ones), held to
max(1e-11, 4 x that form's FP64 floor).  The floors come from the oracle
alone (tests/golden/make_fullsize_floors.py): the spread between two
evaluations of the form whose rounding differs (inputs perturbed by one unit
roundoff; for the sequential sweep also the block-reversed sweep).  On this
input the middle partitions of the 8-partition form eliminate chains cut off
from both leads; their pivot blocks are close to singular at eta = 1e-4, so
that form's floor (and its distance from the sequential result, also stored)
is far above 1e-11 in the oracle itself.  The test shows that the GPU adds no
error beyond what the form's own arithmetic leaves.

The block-row identities sum_j A_ij X^R_ji = I and
sum_j A_ij X^<_ji = sum_j B_ij (X^R_ij)^H (from A X^< = B X^A, Sec. II) are
checked too: the sequential and 2-partition forms to 16 eps b (normalised by
sum_j ||A_ij|| ||X_ji|| plus the B terms), the 8-partition form to 4x the
residual the oracle's own 8-partition sweep leaves.
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
DEFAULT_BOUNDS_P8 = [0, 14, 20, 26, 32, 38, 44, 50, 64]   # library default for n=64, P=8
BOUNDS = {1: [0, 64], 2: [0, 32, 64], 8: DEFAULT_BOUNDS_P8}


def floors():
    with open(os.path.join(HERE, "golden", "fullsize_floors_bt_n64_b512.json")) as f:
        rec = json.load(f)
    assert rec["workload"] == "bt_n64_b512"
    return rec["forms"]


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


@pytest.fixture(scope="module")
def problem():
    return config_problem("bt_n64_b512")


_results = {}
_oracle = {}


def gpu_result(S, A, B, P):
    if P not in _results:
        n, b = A.diag.shape[0], A.diag.shape[1]
        print(f"[fullsize] GPU solve n={n} b={b} partitions={P}", flush=True)
        dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
        XR, XL = S.DeviceBlocks.empty(n, b, 0), S.DeviceBlocks.empty(n, b, 0)
        sol = S.Solver(n, b, 0, partitions=P, bounds=BOUNDS[P] if P > 1 else None)
        sol.solve(dA, dB, XR, XL)
        sol.sync()
        _results[P] = (XR.to_host(), XL.to_host())
        sol.destroy()
    return _results[P]


def oracle_result(A, B, P):
    if P not in _oracle:
        print(f"[fullsize] oracle, same form as the GPU: P={P}", flush=True)
        if P == 1:
            _oracle[P] = oracle.rgf_bt(A, B)
        else:
            _oracle[P] = oracle.prgf(A, B, BOUNDS[P], reduced_split=True)
    return _oracle[P]


def block(M, i, j):
    if i == j:
        return M.diag[i]
    if j == i + 1:
        return M.upper[i]
    return M.lower[j]          # j == i - 1


def residuals(A, B, XR, XL):
    n, b = A.diag.shape[0], A.diag.shape[1]
    eye = np.eye(b)
    wr = wl = 0.0
    for i in range(n):
        js = [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        R = sum(block(A, i, j) @ block(XR, j, i) for j in js) - eye
        sR = sum(np.linalg.norm(block(A, i, j)) * np.linalg.norm(block(XR, j, i)) for j in js)
        L = sum(block(A, i, j) @ block(XL, j, i) for j in js) \
            - sum(block(B, i, j) @ block(XR, i, j).conj().T for j in js)
        sL = sum(np.linalg.norm(block(A, i, j)) * np.linalg.norm(block(XL, j, i)) for j in js) \
            + sum(np.linalg.norm(block(B, i, j)) * np.linalg.norm(block(XR, i, j)) for j in js)
        wr = max(wr, float(np.linalg.norm(R) / sR))
        wl = max(wl, float(np.linalg.norm(L) / sL))
    return wr, wl


def test_fullsize_default_bounds(S):
    assert S.partition_bounds(64, 512, 0, 8) == DEFAULT_BOUNDS_P8
    assert S.partition_bounds(64, 512, 0, 2) == BOUNDS[2]


@pytest.mark.parametrize("P", [1, 2, 8])
def test_fullsize_identities(S, problem, P):
    A, B = problem
    XR, XL = gpu_result(S, A, B, P)
    wr, wl = residuals(A, B, XR, XL)
    base = 16 * EPS * A.diag.shape[1]
    if P in (1, 2):
        br = bl = base
    else:
        ref = floors()[f"P{P}"]["residuals"]
        br, bl = max(base, 4 * ref["XR"]), max(base, 4 * ref["XL"])
    print(f"[fullsize] P={P} residuals X^R {wr:.2e} X^< {wl:.2e} (bounds {br:.2e} / {bl:.2e})", flush=True)
    assert wr < br and wl < bl, (wr, wl)


@pytest.mark.parametrize("P", [1, 2, 8])
def test_fullsize_against_oracle_same_form(S, problem, P):
    A, B = problem
    fl = floors()[f"P{P}"]["floor"]
    XRo, XLo = oracle_result(A, B, P)
    XR, XL = gpu_result(S, A, B, P)
    eR, eL = rel_err(XR, XRo), rel_err(XL, XLo)
    bR, bL = max(1e-11, 4 * fl["XR"]), max(1e-11, 4 * fl["XL"])
    print(f"[fullsize] P={P} vs oracle (same form): X^R {eR:.2e} X^< {eL:.2e} "
          f"(floor {fl['XR']:.2e} / {fl['XL']:.2e}, bounds {bR:.2e} / {bL:.2e})", flush=True)
    assert eR <= bR, eR
    assert eL <= bL, eL
