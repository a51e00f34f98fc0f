"""Writes fullsize_spread.json: how far two orderings of the oracle's own
complex128 arithmetic land apart on the bt_n64_b512 input (n=64, b=512,
E=0.3, eta=1e-4, seed 0), and the block-row residuals each ordering leaves.

The sequential RGF sweep and the partitioned sweep with 8 partitions compute
the same selected blocks of A^-1 and A^-1 B A^-H in exact arithmetic (Sec.
III); in FP64 their per-block relative difference measures how strongly this
input amplifies rounding (eta = 1e-4 leaves A close to singular).  The
partitioned ordering (middle partitions eliminated without pivoting across
blocks, then the reduced system) is also less backward stable here, which its
residuals show.  The partition bounds are the library's default ones for n=64,
P=8 (pinned by the ABI tests).  The GPU full-size parity test takes its
tolerances from these figures.  Calls only the oracle and the seeded input
generator.

    python tests/golden/make_fullsize_spread.py   (about a minute on 8 cores)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_04904_amd.synth import CONFIGS, config_problem  # noqa: E402
from tests._util import rel_err  # noqa: E402
from tests.test_gpu_fullsize import DEFAULT_BOUNDS_P8, residuals  # noqa: E402


def main():
    cfg = CONFIGS["bt_n64_b512"]
    A, B = config_problem("bt_n64_b512")
    t0 = time.perf_counter()
    XR1, XL1 = oracle.rgf_bt(A, B)
    P = 8
    bounds = DEFAULT_BOUNDS_P8
    XR2, XL2 = oracle.prgf(A, B, bounds, reduced_split=True)
    r1, r2 = residuals(A, B, XR1, XL1), residuals(A, B, XR2, XL2)
    out = {
        "workload": cfg.name,
        "orderings": ["sequential", f"partitioned P={P}, bounds {bounds}, reduced system split in two"],
        "metric": "max over selected blocks of ||X1 - X2||_F / max(||X1||_F, 1e-6 max ||X1||_F)",
        "XR_spread": rel_err(XR2, XR1),
        "XL_spread": rel_err(XL2, XL1),
        "residual_metric": "max over block rows of the identity residuals, normalised as in test_gpu_fullsize",
        "sequential_residuals": {"XR": r1[0], "XL": r1[1]},
        "partitioned_residuals": {"XR": r2[0], "XL": r2[1]},
        "seconds": round(time.perf_counter() - t0, 1),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_spread.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
