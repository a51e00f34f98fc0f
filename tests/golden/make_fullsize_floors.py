"""Writes fullsize_floors_<workload>.json: the FP64 floor of every form the
full-size GPU tests check, from the oracle alone.

For each form (sequential sweep P=1, and the partitioned sweeps with the
library's default bounds, reduced system split in two) the floor is how far
two evaluations of that same form land apart when only their rounding
differs:
  * perturbed: the form run on the input and on a copy whose entries are
    perturbed by one unit roundoff (seeded, synth.perturb), so the two runs
    make independent rounding errors in the same elimination order;
  * reversed (P=1 only): the sequential sweep run on the block-reversed
    matrix J A J (and J B J), i.e. the bottom-up sweep, mapped back.
The GPU result of a form is held to max(1e-11, 4 x the floor of that form)
against the oracle's result of the same form, element by element.

It also records the block-row identity residuals each form leaves, each
partitioned form's distance from the sequential result, and the reason the
middle partitions lose accuracy: the block-diagonal-dominance ratio
||A_ii^-1||_2 (||A_i,i-1||_2 + ||A_i,i+1||_2) of the input (Sec. II-A assumes
it below one) and the largest ||S_k||_2 = ||Atil_kk^-1||_2 met in the
sequential sweep, in the end partitions and in the middle partitions.
Calls only the oracle and the seeded input generators.

    python tests/golden/make_fullsize_floors.py bt_n64_b512          (about 5 min on 8 cores)
    python tests/golden/make_fullsize_floors.py bta_n128_b384_a512   (about 10 min)
    python tests/golden/make_fullsize_floors.py vb_n48_b256to512     (about 2 min; blocks of
    python tests/golden/make_fullsize_floors.py vbta_n48_b256to512_a256   different sizes)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.partitioned import _forward_partitions  # noqa: E402
from paper_2601_04904_amd.synth import BTA, CONFIGS, VAR_CONFIGS, VBTA, config_problem, perturb  # noqa: E402
from tests._util import rel_err  # noqa: E402

# the library's default partition bounds for these sizes (pinned by the ABI tests)
FORMS = {
    "bt_n64_b512": {2: [0, 32, 64], 8: [0, 14, 20, 26, 32, 38, 44, 50, 64]},
    "bta_n128_b384_a512": {2: [0, 64, 128], 16: list(range(0, 129, 8))},
    "vb_n48_b256to512": {4: [0, 17, 24, 31, 48]},
    "vbta_n48_b256to512_a256": {4: [0, 16, 24, 32, 48]},
}
REL = 2.0 ** -53        # perturbation: one unit roundoff


def reverse(M):
    """J M J for a block matrix: block i -> n-1-i (upper and lower swap)."""
    if isinstance(M.diag, list):
        return VBTA(M.diag[::-1], M.lower[::-1], M.upper[::-1], M.arrow_right[::-1],
                    M.arrow_bottom[::-1], np.array(M.tip))
    return BTA(M.diag[::-1].copy(), M.lower[::-1].copy(), M.upper[::-1].copy(),
               M.arrow_right[::-1].copy(), M.arrow_bottom[::-1].copy(), np.array(M.tip))


def blk(M, i, j, n):
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
    return M.lower[j]


def residuals(A, B, XR, XL):
    """Max over block rows of ||sum_j A_ij X^R_ji - I|| / sum_j ||A_ij|| ||X^R_ji|| and of
    ||sum_j A_ij X^<_ji - sum_j B_ij (X^R_ij)^H|| / (the matching sum of norms)."""
    n, a = len(A.diag), A.tip.shape[0]
    rows = n + (1 if a > 0 else 0)
    wr = wl = 0.0
    for i in range(rows):
        if i == n:
            js = list(range(n + 1))
        else:
            js = [j for j in (i - 1, i, i + 1) if 0 <= j < n] + ([n] if a > 0 else [])
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


def sequential(A, B):
    return oracle.rgf_bta(A, B) if A.tip.shape[0] else oracle.rgf_bt(A, B)


def conditioning(A, B, bounds_by_P):
    n = len(A.diag)
    dom = []
    for i in range(n):
        off = (np.linalg.norm(A.lower[i - 1], 2) if i > 0 else 0.0) + \
              (np.linalg.norm(A.upper[i], 2) if i < n - 1 else 0.0)
        dom.append(float(np.linalg.norm(np.linalg.inv(A.diag[i]), 2) * off))
    out = {"block_dominance_ratio": {"min": min(dom), "median": float(np.median(dom)), "max": max(dom)}}
    smax = {}
    for P, bounds in [(1, [0, n])] + sorted(bounds_by_P.items()):
        _, _, recs, _, _ = _forward_partitions(A, None, bounds)
        for p, part in enumerate(recs):
            kind = "sequential" if P == 1 else ("end partitions" if p in (0, P - 1) else "middle partitions")
            key = f"P{P} {kind}"
            for r in part:
                smax[key] = max(smax.get(key, 0.0), float(np.linalg.norm(r.S, 2)))
        print(f"conditioning P={P} done", flush=True)
    out["max_S_norm_2"] = smax
    return out


def main():
    name = sys.argv[1]
    if name in VAR_CONFIGS:
        E, eta = VAR_CONFIGS[name]["E"], VAR_CONFIGS[name]["eta"]
    else:
        E, eta = CONFIGS[name].E, CONFIGS[name].eta
    A, B = config_problem(name)
    Ap, Bp = perturb(A, REL, 1), perturb(B, REL, 2)
    t0 = time.perf_counter()
    out = {"workload": name, "E": E, "eta": eta,
           "metric": "max over selected blocks of ||X1 - X2||_F / max(||X2||_F, 1e-6 max_j ||X2_j||_F)",
           "perturbation": "entries x (1 + 2^-53 u), u uniform in [-1,1] + i[-1,1], seeds 1 (A) and 2 (B)",
           "forms": {}}
    XR1, XL1 = sequential(A, B)
    res = residuals(A, B, XR1, XL1)
    XRp, XLp = sequential(Ap, Bp)
    pert = (rel_err(XRp, XR1), rel_err(XLp, XL1))
    del XRp, XLp
    XRf, XLf = sequential(reverse(A), reverse(B))
    XRf, XLf = reverse(XRf), reverse(XLf)
    flip = (rel_err(XRf, XR1), rel_err(XLf, XL1))
    del XRf, XLf
    out["forms"]["P1"] = {
        "ordering": "sequential sweep",
        "floor_perturbed": {"XR": pert[0], "XL": pert[1]},
        "floor_reversed": {"XR": flip[0], "XL": flip[1]},
        "floor": {"XR": max(pert[0], flip[0]), "XL": max(pert[1], flip[1])},
        "residuals": {"XR": res[0], "XL": res[1]},
    }
    print(f"P=1 done {time.perf_counter() - t0:.0f} s: {out['forms']['P1']}", flush=True)
    for P, bounds in sorted(FORMS[name].items()):
        XR2, XL2 = oracle.prgf(A, B, bounds, reduced_split=True)
        res = residuals(A, B, XR2, XL2)
        vs_seq = (rel_err(XR2, XR1), rel_err(XL2, XL1))
        XRp, XLp = oracle.prgf(Ap, Bp, bounds, reduced_split=True)
        pert = (rel_err(XRp, XR2), rel_err(XLp, XL2))
        del XR2, XL2, XRp, XLp
        out["forms"][f"P{P}"] = {
            "ordering": f"partitioned, bounds {bounds}, reduced system split in two",
            "bounds": bounds,
            "floor_perturbed": {"XR": pert[0], "XL": pert[1]},
            "floor": {"XR": pert[0], "XL": pert[1]},
            "residuals": {"XR": res[0], "XL": res[1]},
            "vs_sequential": {"XR": vs_seq[0], "XL": vs_seq[1]},
        }
        print(f"P={P} done {time.perf_counter() - t0:.0f} s: {out['forms'][f'P{P}']}", flush=True)
    del XR1, XL1
    out["conditioning"] = conditioning(A, B, FORMS[name])
    out["seconds"] = round(time.perf_counter() - t0, 1)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fullsize_floors_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
