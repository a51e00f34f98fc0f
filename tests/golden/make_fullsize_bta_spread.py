"""Writes fullsize_bta_spread.json: how far two orderings of the oracle's own
complex128 arithmetic land apart on the bta_n128_b384_a512 input (n=128,
b=384, arrow tip a=512, E=0.3, eta=1e-3, seed 0), and the block-row residuals
each ordering leaves (the BTA counterpart of make_fullsize_spread.py).

The sequential BTA sweep (Sec. III-A) and the partitioned sweep with 16
partitions (Sec. III-B; the library's default bounds for this size, reduced
system split in two) compute the same selected blocks in exact arithmetic;
their per-block FP64 difference measures how strongly the input amplifies
rounding.  The GPU full-size BTA test takes its tolerances from these figures.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_fullsize_bta_spread.py   (a few minutes on 8 cores)
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
from tests.test_gpu_fullsize_bta import DEFAULT_BOUNDS_P16, residuals_bta  # noqa: E402


def main():
    cfg = CONFIGS["bta_n128_b384_a512"]
    A, B = config_problem(cfg.name)
    t0 = time.perf_counter()
    XR1, XL1 = oracle.rgf_bta(A, B)
    print(f"sequential sweep {time.perf_counter() - t0:.0f} s", flush=True)
    XR2, XL2 = oracle.prgf(A, B, DEFAULT_BOUNDS_P16, reduced_split=True)
    print(f"partitioned sweep {time.perf_counter() - t0:.0f} s", flush=True)
    r1, r2 = residuals_bta(A, B, XR1, XL1), residuals_bta(A, B, XR2, XL2)
    out = {
        "workload": cfg.name,
        "orderings": ["sequential", f"partitioned P=16, bounds {DEFAULT_BOUNDS_P16}, reduced system split in two"],
        "metric": "max over selected blocks of ||X1 - X2||_F / max(||X1||_F, 1e-6 max ||X1||_F)",
        "XR_spread": rel_err(XR2, XR1),
        "XL_spread": rel_err(XL2, XL1),
        "residual_metric": "max over block rows (arrow tip row included) of the identity residuals, "
                           "normalised as in test_gpu_fullsize_bta",
        "sequential_residuals": {"XR": r1[0], "XL": r1[1]},
        "partitioned_residuals": {"XR": r2[0], "XL": r2[1]},
        "seconds": round(time.perf_counter() - t0, 1),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_bta_spread.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
