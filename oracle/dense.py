"""Plain definition of SI and SQ (test infrastructure only).

Sec. II-A states the two problems: A X = I and A X A^H = B, with A and B
sharing one BT/BTA pattern and only the entries of X on that pattern wanted.
The dense approach of Sec. II-C (Alg. 4) computes X in full and then keeps the
pattern; that is what this module does, with LAPACK's inverse as the one
library step.  Cost O(N^3), memory O(N^2): tiny and small inputs only.
Blocks may differ in size (Sec. II-A: RGF applies unchanged to diagonal blocks
of different sizes); then every block field is a list of blocks.
"""
from __future__ import annotations

import numpy as np

from .blocks import Sel, block_sizes, tip_size, uniform


def _offsets(sizes):
    off = [0]
    for sz in sizes:
        off.append(off[-1] + sz)
    return off


def assemble(M) -> np.ndarray:
    """Dense N x N matrix (N = sum of the block sizes + a) from block storage;
    tip rows/cols last.  Blocks may differ in size (lists of blocks)."""
    sizes = block_sizes(M)
    n = len(sizes)
    a = tip_size(M)
    off = _offsets(sizes)
    nb = off[-1]
    N = nb + a
    D = np.zeros((N, N), dtype=np.complex128)
    for i in range(n):
        r = slice(off[i], off[i + 1])
        D[r, r] = M.diag[i]
        if i < n - 1:
            r1 = slice(off[i + 1], off[i + 2])
            D[r, r1] = M.upper[i]
            D[r1, r] = M.lower[i]
        if a > 0:
            t = slice(nb, N)
            D[r, t] = M.arrow_right[i]
            D[t, r] = M.arrow_bottom[i]
    if a > 0:
        D[nb:, nb:] = M.tip
    return D


def extract(X: np.ndarray, n, b, a: int) -> Sel:
    """The entries of a dense X on the BT/BTA pattern.  b is the block size,
    or the list of the n block sizes (then every field is a list)."""
    sizes = list(b) if np.ndim(b) > 0 else [int(b)] * n
    out = Sel.zeros(n, sizes[0] if n else 0, a) if np.ndim(b) == 0 else Sel.zeros_var(sizes, a)
    off = _offsets(sizes)
    nb = off[-1]
    for i in range(n):
        r = slice(off[i], off[i + 1])
        out.diag[i] = X[r, r]
        if i < n - 1:
            r1 = slice(off[i + 1], off[i + 2])
            out.upper[i] = X[r, r1]
            out.lower[i] = X[r1, r]
        if a > 0:
            t = slice(nb, nb + a)
            out.arrow_right[i] = X[r, t]
            out.arrow_bottom[i] = X[t, r]
    if a > 0:
        out.tip[:] = X[nb:, nb:]
    return out


def solve_dense(A, B=None):
    """(X^R, X^<) on the pattern: X^R = A^-1, X^< = A^-1 B A^-H.

    With B None only X^R is returned (as (X^R, None)).
    """
    sizes = block_sizes(A)
    n, a = len(sizes), tip_size(A)
    b = sizes[0] if uniform(sizes) and n > 0 else sizes
    G = np.linalg.inv(assemble(A))
    XR = extract(G, n, b, a)
    if B is None:
        return XR, None
    XL = extract(G @ assemble(B) @ G.conj().T, n, b, a)
    return XR, XL
