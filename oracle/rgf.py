"""Recursive Green's function (RGF) oracle (test infrastructure only).

rgf_bt follows Alg. 1 (forward Schur complement) and Alg. 2 (backward
selected inversion and selected quadratic solve) of the paper for a BT
matrix, with the inverse-instead-of-trsm formulation of Sec. II-B: every
diagonal block is inverted explicitly (LAPACK) and the updates are products.

rgf_bta is the BTA extension of Sec. III-A.  The paper gives it through the
block slicing of Figs. 4-5 (not reproduced in the text); here it is written
as the block Schur-complement step that slicing describes.  Eliminating
block k whose remaining neighbours are N(k) (for BTA: {k+1, t}) with
Atil/Btil the current (updated) blocks:

  forward   S   = Atil_kk^-1,  S_B = S Btil_kk S^H,  T_u = Atil_uk S,
            Atil_uv -= T_u Atil_kv,
            Btil_uv += T_u Btil_kk T_v^H - T_u Btil_kv - Btil_uk T_v^H
  backward  tau_v = S Atil_kv,  rho_u = sum_w X_uw Atil_wk,
            X_uk = -rho_u S,  X_kv = -sum_w tau_w X_wv,
            X_kk = S - sum_w tau_w X_wk,
            Y21_u = (sum_w X_uw Btil_wk) S^H - rho_u S_B,
            Y12_v = S (sum_w Btil_kw X_vw^H) - S_B rho_v^H,
            L_kv = Y12_v - sum_w tau_w L_wv,  L_uk = Y21_u - sum_w L_uw tau_w^H,
            L_kk = S_B - sum_w L_kw tau_w^H - sum_w tau_w Y21_w
  (u, v, w over N(k); X = X^R, L = X^<).  For N(k) = {k+1} this is exactly
  Alg. 1 / Alg. 2 (the five-term X_B,ii of Alg. 2 expands to L_kk above).
The same step, with other neighbour sets, drives the partitioned oracle.
"""
from __future__ import annotations

import numpy as np

from .blocks import Sel, block_sizes, tip_size, uniform


def _H(M: np.ndarray) -> np.ndarray:
    return M.conj().T


def _sel_zeros(sizes, a):
    """Uniform blocks as 3-D arrays, blocks of different sizes as lists."""
    if uniform(sizes):
        return Sel.zeros(len(sizes), sizes[0] if sizes else 0, a)
    return Sel.zeros_var(sizes, a)


def rgf_bt(A, B=None):
    """Alg. 1 + Alg. 2 for a BT matrix (the arrowhead, if any, is ignored).
    Blocks may differ in size (Sec. II-A).

    Returns (X^R, X^<) as Sel; X^< is None when B is None.
    """
    sizes = block_sizes(A)
    n = len(sizes)
    quad = B is not None
    Ad = [np.array(A.diag[i], dtype=np.complex128) for i in range(n)]
    Bd = [np.array(B.diag[i], dtype=np.complex128) for i in range(n)] if quad else None
    SA = [None] * n
    SB = [None] * n
    # Alg. 1: forward pass.
    for i in range(n - 1):
        SA[i] = np.linalg.inv(Ad[i])
        if quad:
            SB[i] = SA[i] @ Bd[i] @ _H(SA[i])
        T1 = A.lower[i] @ SA[i]
        Ad[i + 1] = Ad[i + 1] - T1 @ A.upper[i]
        if quad:
            Bd[i + 1] = (Bd[i + 1] + A.lower[i] @ SB[i] @ _H(A.lower[i])
                         - B.lower[i] @ _H(T1) - T1 @ B.upper[i])
    SA[n - 1] = np.linalg.inv(Ad[n - 1])
    if quad:
        SB[n - 1] = SA[n - 1] @ Bd[n - 1] @ _H(SA[n - 1])

    # Alg. 2: backward pass.
    XR = _sel_zeros(sizes, 0)
    XL = _sel_zeros(sizes, 0) if quad else None
    XR.diag[n - 1] = SA[n - 1]
    if quad:
        XL.diag[n - 1] = SB[n - 1]
    for i in range(n - 2, -1, -1):
        T1A = SA[i] @ A.upper[i]
        T2A = XR.diag[i + 1] @ A.lower[i]
        XR.lower[i] = -T2A @ SA[i]
        XR.upper[i] = -T1A @ XR.diag[i + 1]
        XR.diag[i] = SA[i] - T1A @ XR.lower[i]
        if quad:
            T1B = XL.diag[i + 1] @ _H(T1A)
            T2B = SB[i] @ _H(T2A)
            T3B = T2A @ SB[i]
            T4B = SA[i] @ B.upper[i] @ _H(XR.diag[i + 1])
            T5B = XR.diag[i + 1] @ B.lower[i] @ _H(SA[i])
            XL.upper[i] = -T1A @ XL.diag[i + 1] - T2B + T4B
            XL.lower[i] = -T1B - T3B + T5B
            XL.diag[i] = (SB[i] + T1A @ T1B + T1A @ T3B + T2B @ _H(T1A)
                          - T1A @ T5B - T4B @ _H(T1A))
    return XR, XL


# --------------------------------------------------------------------------
# Neighbour-set elimination on a block graph (BTA and partitioned schemes).
# Blocks are held in dicts keyed by (row node, column node); a missing key is
# an a-priori zero block.  Nodes are block indices 0..n-1 and the tip 't'.
# --------------------------------------------------------------------------

class Record:
    """What the forward step keeps for the backward step of block k."""

    def __init__(self, k, N, S, SB, A_kv, A_uk, B_kv, B_uk):
        self.k, self.N, self.S, self.SB = k, list(N), S, SB
        self.A_kv, self.A_uk, self.B_kv, self.B_uk = A_kv, A_uk, B_kv, B_uk


def _zero(dim, r, c):
    return np.zeros((dim[r], dim[c]), dtype=np.complex128)


def _get(D, key, dim):
    return D[key] if key in D else _zero(dim, *key)


def forward_step(k, N, At, Bt, dim, quad=True) -> Record:
    """Eliminate block k against its neighbours N (forward Schur complement)."""
    S = np.linalg.inv(At[(k, k)])
    A_kv = {v: _get(At, (k, v), dim) for v in N}
    A_uk = {u: _get(At, (u, k), dim) for u in N}
    T = {u: A_uk[u] @ S for u in N}
    if quad:
        SB = S @ Bt[(k, k)] @ _H(S)
        B_kk = Bt[(k, k)]
        B_kv = {v: _get(Bt, (k, v), dim) for v in N}
        B_uk = {u: _get(Bt, (u, k), dim) for u in N}
    else:
        SB, B_kv, B_uk = None, None, None
    for u in N:
        for v in N:
            At[(u, v)] = _get(At, (u, v), dim) - T[u] @ A_kv[v]
            if quad:
                Bt[(u, v)] = (_get(Bt, (u, v), dim) + T[u] @ B_kk @ _H(T[v])
                              - T[u] @ B_kv[v] - B_uk[u] @ _H(T[v]))
    return Record(k, N, S, SB, A_kv, A_uk, B_kv, B_uk)


def backward_step(rec: Record, XR, XL, quad=True):
    """Selected inversion / quadratic solve of block k, given X on N x N."""
    k, N, S, SB = rec.k, rec.N, rec.S, rec.SB
    tau = {v: S @ rec.A_kv[v] for v in N}
    rho = {u: sum((XR[(u, w)] @ rec.A_uk[w] for w in N), 0 * rec.A_uk[u])
           for u in N}
    for u in N:
        XR[(u, k)] = -rho[u] @ S
    for v in N:
        XR[(k, v)] = -sum((tau[w] @ XR[(w, v)] for w in N), 0 * rec.A_kv[v])
    XR[(k, k)] = S - sum((tau[w] @ XR[(w, k)] for w in N), 0 * S)
    if not quad:
        return
    Y21 = {}
    for u in N:
        GB = sum((XR[(u, w)] @ rec.B_uk[w] for w in N), 0 * rec.A_uk[u])
        Y21[u] = GB @ _H(S) - rho[u] @ SB
    Y12 = {}
    for v in N:
        BG = sum((rec.B_kv[w] @ _H(XR[(v, w)]) for w in N), 0 * rec.A_kv[v])
        Y12[v] = S @ BG - SB @ _H(rho[v])
    for v in N:
        XL[(k, v)] = Y12[v] - sum((tau[w] @ XL[(w, v)] for w in N), 0 * Y12[v])
    for u in N:
        XL[(u, k)] = Y21[u] - sum((XL[(u, w)] @ _H(tau[w]) for w in N), 0 * Y21[u])
    XL[(k, k)] = (SB - sum((XL[(k, w)] @ _H(tau[w]) for w in N), 0 * SB)
                  - sum((tau[w] @ Y21[w] for w in N), 0 * SB))


def to_dicts(M, n, a):
    """Block dict {(u, v): block} of a BT/BTA matrix (tip node 't')."""
    D = {}
    for i in range(n):
        D[(i, i)] = np.array(M.diag[i], dtype=np.complex128)
        if i < n - 1:
            D[(i, i + 1)] = np.array(M.upper[i], dtype=np.complex128)
            D[(i + 1, i)] = np.array(M.lower[i], dtype=np.complex128)
        if a > 0:
            D[(i, "t")] = np.array(M.arrow_right[i], dtype=np.complex128)
            D[("t", i)] = np.array(M.arrow_bottom[i], dtype=np.complex128)
    if a > 0:
        D[("t", "t")] = np.array(M.tip, dtype=np.complex128)
    return D


def from_dicts(X, n, b, a) -> Sel:
    """Sel of the pattern blocks of a block dict; b is the block size or the
    list of block sizes."""
    sizes = list(b) if np.ndim(b) > 0 else [int(b)] * n
    out = _sel_zeros(sizes, a)
    for i in range(n):
        out.diag[i] = X[(i, i)]
        if i < n - 1:
            out.upper[i] = X[(i, i + 1)]
            out.lower[i] = X[(i + 1, i)]
        if a > 0:
            out.arrow_right[i] = X[(i, "t")]
            out.arrow_bottom[i] = X[("t", i)]
    if a > 0:
        out.tip[:] = X[("t", "t")]
    return out


def rgf_bta(A, B=None):
    """Sequential RGF for BT (a == 0) or BTA: eliminate 0, 1, ..., n-1, then t.

    Block i is eliminated against N(i) = {i+1, t} (i+1 absent for the last
    block, t absent when a == 0).  Returns (X^R, X^<) as Sel.
    """
    sizes = block_sizes(A)
    n, a = len(sizes), tip_size(A)
    quad = B is not None
    dim = {i: sizes[i] for i in range(n)}
    dim["t"] = a
    At = to_dicts(A, n, a)
    Bt = to_dicts(B, n, a) if quad else {}
    order = list(range(n)) + (["t"] if a > 0 else [])
    recs = []
    for pos, k in enumerate(order):
        N = []
        if k != "t" and k + 1 < n:
            N.append(k + 1)
        if k != "t" and a > 0:
            N.append("t")
        recs.append(forward_step(k, N, At, Bt, dim, quad))
    XR, XL = {}, {}
    for rec in reversed(recs):
        backward_step(rec, XR, XL, quad)
    return from_dicts(XR, n, sizes, a), (from_dicts(XL, n, sizes, a) if quad else None)
