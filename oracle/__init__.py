"""CPU oracle for selected inversion (SI) and the selected quadratic solve (SQ).

TEST INFRASTRUCTURE ONLY.  Plain, slow, complex128 NumPy code written from
the paper (arXiv 2601.04904).  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never does, and
this package imports nothing from the library (it accepts any object with the
block fields diag/upper/lower/arrow_right/arrow_bottom/tip).

  dense.solve_dense      the plain definition: X^R = A^-1, X^< = A^-1 B A^-H,
                         restricted to the BT/BTA pattern (Sec. II-A; the
                         dense solve of Alg. 4).
  rgf.rgf_bt             Alg. 1 (forward Schur complement) + Alg. 2 (backward
                         SI and SQ) for BT matrices, as printed.
  rgf.rgf_bta            the BTA extension of RGF (Sec. III-A): block k is
                         eliminated against its neighbours {k+1, t}.
  partitioned.prgf       the partitioned scheme (Sec. III-B): concurrent
                         partition eliminations with fill-in, reduced system
                         solved by the sequential BTA RGF, partition backward
                         sweeps.

Every function here is pinned by the non-GPU tests against closed forms,
invariants and brute force (see tests/test_oracle_*.py).
"""
from .blocks import Sel
from .dense import assemble, extract, solve_dense
from .rgf import rgf_bt, rgf_bta
from .partitioned import prgf, reduced_system

__all__ = ["Sel", "assemble", "extract", "solve_dense", "rgf_bt", "rgf_bta",
           "prgf", "reduced_system"]
