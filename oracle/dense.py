"""Plain definition of SI and SQ (test infrastructure only).

Sec. II-A states the two problems: A X = I and A X A^H = B, with A and B
sharing one BT/BTA pattern and only the entries of X on that pattern wanted.
The dense approach of Sec. II-C (Alg. 4) computes X in full and then keeps the
pattern; that is what this module does, with LAPACK's inverse as the one
library step.  Cost O(N^3), memory O(N^2): tiny and small inputs only.
"""
from __future__ import annotations

import numpy as np

from .blocks import Sel


def assemble(M) -> np.ndarray:
    """Dense N x N matrix (N = n b + a) from block storage; tip rows/cols last."""
    n, b = M.diag.shape[0], M.diag.shape[1]
    a = M.tip.shape[0]
    N = n * b + a
    D = np.zeros((N, N), dtype=np.complex128)
    for i in range(n):
        r = slice(i * b, (i + 1) * b)
        D[r, r] = M.diag[i]
        if i < n - 1:
            r1 = slice((i + 1) * b, (i + 2) * b)
            D[r, r1] = M.upper[i]
            D[r1, r] = M.lower[i]
        if a > 0:
            t = slice(n * b, N)
            D[r, t] = M.arrow_right[i]
            D[t, r] = M.arrow_bottom[i]
    if a > 0:
        D[n * b:, n * b:] = M.tip
    return D


def extract(X: np.ndarray, n: int, b: int, a: int) -> Sel:
    """The entries of a dense X on the BT/BTA pattern."""
    out = Sel.zeros(n, b, a)
    for i in range(n):
        r = slice(i * b, (i + 1) * b)
        out.diag[i] = X[r, r]
        if i < n - 1:
            r1 = slice((i + 1) * b, (i + 2) * b)
            out.upper[i] = X[r, r1]
            out.lower[i] = X[r1, r]
        if a > 0:
            t = slice(n * b, n * b + a)
            out.arrow_right[i] = X[r, t]
            out.arrow_bottom[i] = X[t, r]
    if a > 0:
        out.tip[:] = X[n * b:, n * b:]
    return out


def solve_dense(A, B=None):
    """(X^R, X^<) on the pattern: X^R = A^-1, X^< = A^-1 B A^-H.

    With B None only X^R is returned (as (X^R, None)).
    """
    n, b = A.diag.shape[0], A.diag.shape[1]
    a = A.tip.shape[0]
    G = np.linalg.inv(assemble(A))
    XR = extract(G, n, b, a)
    if B is None:
        return XR, None
    XL = extract(G @ assemble(B) @ G.conj().T, n, b, a)
    return XR, XL
