"""Which block products of the sequential BT(A) sweep can run in complex64
and keep the result within 1e-4 of the all-FP64 sweep?  (Writes the numbers
DESIGN quotes for the mixed path; CPU only, about two minutes.)

The sweep is the oracle's neighbour-set step (Sec. III-A; Alg. 1/2 for BT)
with every block product routed through mm(): products of the groups named in
a policy are rounded to complex64 and multiplied with complex64 operands
(NumPy's complex64 product accumulates in FP32, as the mixed path's FP32
MFMA does); the diagonal-block inverses stay FP64 in every policy, as in the
library.  Groups: T (T_u = Atil_uk S), schurA (Atil_uv -= T_u Atil_kv),
SB (S Btil_kk S^H), B (the other B-chain products), si (backward selected
inversion), sq (backward quadratic solve).  Inputs: the batch recipe
(eta = 1e-3), sizes small enough for the CPU.

    python tests/golden/mixed_split_study.py > tests/golden/mixed_split_study.txt
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle
from paper_2601_04904_amd.synth import gen_problem
from tests._util import rel_err

H = lambda M: M.conj().T

def mm(X, Y, grp, low):
    if grp in low:
        return (X.astype(np.complex64) @ Y.astype(np.complex64)).astype(np.complex128)
    return X @ Y

def sweep(A, B, low):
    n, b = A.diag.shape[0], A.diag.shape[1]
    a = A.tip.shape[0]
    dim = {i: b for i in range(n)}; dim['t'] = a
    from oracle.rgf import to_dicts, from_dicts, _get
    At, Bt = to_dicts(A, n, a), to_dicts(B, n, a)
    order = list(range(n)) + (['t'] if a else [])
    recs = []
    for k in order:
        N = []
        if k != 't' and k + 1 < n: N.append(k + 1)
        if k != 't' and a: N.append('t')
        S = np.linalg.inv(At[(k, k)])
        Akv = {v: _get(At, (k, v), dim) for v in N}; Auk = {u: _get(At, (u, k), dim) for u in N}
        T = {u: mm(Auk[u], S, 'T', low) for u in N}
        Bkk = Bt[(k, k)]
        SB = mm(mm(S, Bkk, 'SB', low), H(S), 'SB', low)
        Bkv = {v: _get(Bt, (k, v), dim) for v in N}; Buk = {u: _get(Bt, (u, k), dim) for u in N}
        W = {u: mm(T[u], Bkk, 'B', low) for u in N}
        for u in N:
            for v in N:
                At[(u, v)] = _get(At, (u, v), dim) - mm(T[u], Akv[v], 'schurA', low)
                Bt[(u, v)] = (_get(Bt, (u, v), dim) + mm(W[u], H(T[v]), 'B', low)
                              - mm(T[u], Bkv[v], 'B', low) - mm(Buk[u], H(T[v]), 'B', low))
        recs.append((k, N, S, SB, Akv, Auk, Bkv, Buk))
    XR, XL = {}, {}
    for k, N, S, SB, Akv, Auk, Bkv, Buk in reversed(recs):
        tau = {v: mm(S, Akv[v], 'si', low) for v in N}
        rho = {u: sum((mm(XR[(u, w)], Auk[w], 'si', low) for w in N), 0 * Auk[u]) for u in N}
        for u in N: XR[(u, k)] = -mm(rho[u], S, 'si', low)
        for v in N: XR[(k, v)] = -sum((mm(tau[w], XR[(w, v)], 'si', low) for w in N), 0 * Akv[v])
        XR[(k, k)] = S - sum((mm(tau[w], XR[(w, k)], 'si', low) for w in N), 0 * S)
        Y21 = {u: mm(sum((mm(XR[(u, w)], Buk[w], 'sq', low) for w in N), 0 * Auk[u]), H(S), 'sq', low) - mm(rho[u], SB, 'sq', low) for u in N}
        Y12 = {v: mm(S, sum((mm(Bkv[w], H(XR[(v, w)]), 'sq', low) for w in N), 0 * Akv[v]), 'sq', low) - mm(SB, H(rho[v]), 'sq', low) for v in N}
        for v in N: XL[(k, v)] = Y12[v] - sum((mm(tau[w], XL[(w, v)], 'sq', low) for w in N), 0 * Y12[v])
        for u in N: XL[(u, k)] = Y21[u] - sum((mm(XL[(u, w)], H(tau[w]), 'sq', low) for w in N), 0 * Y21[u])
        XL[(k, k)] = SB - sum((mm(XL[(k, w)], H(tau[w]), 'sq', low) for w in N), 0 * SB) - sum((mm(tau[w], Y21[w], 'sq', low) for w in N), 0 * SB)
    return from_dicts(XR, n, b, a), from_dicts(XL, n, b, a)

groups = ['T', 'schurA', 'SB', 'B', 'si', 'sq']
cases = [(24, 64, 0, 0.3), (24, 128, 0, -0.5), (16, 128, 64, 0.7), (32, 96, 0, 0.1)]
policies = {
    'all c64': set(groups),
    'B-chain+backward (A-chain FP64)': {'SB', 'B', 'si', 'sq'},
    'B-chain + SQ backward': {'SB', 'B', 'sq'},
    'SQ backward only': {'sq'},
    'B-chain only': {'B', 'SB'},
    'SI backward only': {'si'},
    'A-chain only': {'T', 'schurA'},
}
for (n, b, a, E) in cases:
    A, B = gen_problem(n, b, a, E=E, eta=1e-3, seed=n + b + a)
    R0, L0 = sweep(A, B, set())
    line = f"n={n} b={b} a={a} E={E}:"
    for name, low in policies.items():
        R, L = sweep(A, B, low)
        line += f"\n   {name:34s} XR {rel_err(R, R0):.1e} XL {rel_err(L, L0):.1e}"
    print(line, flush=True)
