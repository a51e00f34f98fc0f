"""Partitioned (distributed) RGF oracle, Sec. III-B (test infrastructure only).

The block rows are split into P contiguous partitions [s_p, e_p].  The
permutation of Sec. III-B-2 is implicit: only the elimination order changes.

  * first partition (p = 0):   eliminates s..e-1 top-down, N(k) = {k+1, t}
  * middle partitions:         eliminate s+1..e-1 top-down against their top
                               block s, N(k) = {s, k+1, t}; this creates the
                               fill-in coupling s to k+1
  * last partition (p = P-1):  eliminates e..s+1 bottom-up, N(k) = {k-1, t}

The partitions are independent except for the tip, to which each adds its
own contribution (the paper's AllReduce); the kept blocks e_0, s_1, e_1, ...,
s_{P-1} with their original and fill couplings form the reduced system, a
BTA matrix of 2(P-1) blocks plus the tip (the paper's AllGather).  It is
solved with the sequential BTA RGF, after which every partition runs its
backward sweep (selected inversion and quadratic solve) in reverse
elimination order.  The per-block step is the Schur-complement step of
rgf.forward_step / rgf.backward_step.

With reduced_split=True a reduced system of at least four blocks is itself
solved by this partitioned elimination (the recursive call of Sec. III-B):
with reduced_parts = 2 (the default) by two partitions, its first half
top-down and its second half bottom-up, each with its own tip contribution,
then its two middle blocks and the tip; with reduced_parts = Q > 2 by
q = min(Q, m // 2) partitions of an m-block reduced system, first, middle and
last as above, whose own reduced system is solved the same way in turn.
Every order gives the same selected blocks in exact arithmetic.
"""
from __future__ import annotations

import numpy as np

from .blocks import Sel
from .blocks import block_sizes, tip_size, uniform
from .rgf import backward_step, forward_step, from_dicts, rgf_bta, to_dicts


def _check_bounds(bounds, n):
    P = len(bounds) - 1
    if P < 1 or bounds[0] != 0 or bounds[-1] != n:
        raise ValueError("bounds must start at 0 and end at n")
    sizes = [bounds[p + 1] - bounds[p] for p in range(P)]
    if P == 1:
        if sizes[0] < 1:
            raise ValueError("empty partition")
        return P
    for p, sz in enumerate(sizes):
        need = 1 if p in (0, P - 1) else 2
        if sz < need:
            raise ValueError(f"partition {p} has {sz} blocks, needs >= {need}")
    return P


def elimination_plan(bounds, n, a):
    """[(k, N(k)), ...] for each partition, and the reduced-system nodes."""
    P = _check_bounds(bounds, n)
    tip = ["t"] if a > 0 else []
    plans = []
    if P == 1:
        plans.append([(k, ([k + 1] if k + 1 < n else []) + tip) for k in range(n)])
        return plans, []
    reduced = []
    for p in range(P):
        s, e = bounds[p], bounds[p + 1] - 1
        if p == 0:
            plans.append([(k, [k + 1] + tip) for k in range(s, e)])
            reduced.append(e)
        elif p == P - 1:
            plans.append([(k, [k - 1] + tip) for k in range(e, s, -1)])
            reduced.append(s)
        else:
            plans.append([(k, [s, k + 1] + tip) for k in range(s + 1, e)])
            reduced.extend([s, e])
    return plans, reduced


class _Reduced:
    """BTA block storage of the reduced system (same fields as the input)."""

    def __init__(self, M, nodes, a):
        m = len(nodes)
        dims = [M[(r, r)].shape[0] for r in nodes]
        pack = np.array if uniform(dims) else list

        def z(r, c):
            return np.zeros((r, c), np.complex128)
        self.diag = pack([M[(r, r)] for r in nodes])
        self.upper = pack([M.get((nodes[j], nodes[j + 1]), z(dims[j], dims[j + 1]))
                           for j in range(m - 1)])
        self.lower = pack([M.get((nodes[j + 1], nodes[j]), z(dims[j + 1], dims[j]))
                           for j in range(m - 1)])
        if a > 0:
            self.arrow_right = pack([M[(r, "t")] for r in nodes])
            self.arrow_bottom = pack([M[("t", r)] for r in nodes])
            self.tip = np.array(M[("t", "t")])
        else:
            self.arrow_right = pack([z(dims[j], 0) for j in range(m)])
            self.arrow_bottom = pack([z(0, dims[j]) for j in range(m)])
            self.tip = np.zeros((0, 0), np.complex128)


def _forward_partitions(A, B, bounds):
    sizes = block_sizes(A)
    n, a = len(sizes), tip_size(A)
    quad = B is not None
    dim = {i: sizes[i] for i in range(n)}
    dim["t"] = a
    At = to_dicts(A, n, a)
    Bt = to_dicts(B, n, a) if quad else {}
    plans, reduced = elimination_plan(bounds, n, a)
    recs = []
    if len(plans) == 1:
        recs.append([forward_step(k, N, At, Bt, dim, quad) for k, N in plans[0]])
        return At, Bt, recs, reduced, dim
    tip_A = At.pop(("t", "t"), None)
    tip_B = Bt.pop(("t", "t"), None) if quad else None
    dA, dB = [], []
    for plan in plans:
        if a > 0:
            At[("t", "t")] = np.zeros((a, a), np.complex128)
            if quad:
                Bt[("t", "t")] = np.zeros((a, a), np.complex128)
        recs.append([forward_step(k, N, At, Bt, dim, quad) for k, N in plan])
        if a > 0:
            dA.append(At.pop(("t", "t")))
            if quad:
                dB.append(Bt.pop(("t", "t")))
    if a > 0:
        At[("t", "t")] = tip_A + sum(dA)
        if quad:
            Bt[("t", "t")] = tip_B + sum(dB)
    return At, Bt, recs, reduced, dim


def reduced_system(A, B, bounds):
    """(reduced A, reduced B, nodes) after the partition eliminations."""
    a = tip_size(A)
    At, Bt, _, reduced, _ = _forward_partitions(A, B, bounds)
    Ar = _Reduced(At, reduced, a)
    Br = _Reduced(Bt, reduced, a) if B is not None else None
    return Ar, Br, reduced


def reduced_bounds(m, parts):
    """Partition bounds of an m-block reduced system split into
    q = min(parts, m // 2) contiguous parts of near-equal length."""
    q = max(2, min(parts, m // 2))
    return [i * m // q for i in range(q + 1)]


def prgf(A, B, bounds, reduced_split=False, reduced_parts=2):
    """Partitioned SI (+ SQ when B is given).  Returns (X^R, X^<) as Sel.
    Blocks may differ in size (Sec. II-A)."""
    sizes = block_sizes(A)
    n, a = len(sizes), tip_size(A)
    b = sizes
    quad = B is not None
    At, Bt, recs, reduced, dim = _forward_partitions(A, B, bounds)
    XR, XL = {}, {}
    if len(recs) == 1:
        if a > 0:
            recs[0].append(forward_step("t", [], At, Bt, dim, quad))
        for rec in reversed(recs[0]):
            backward_step(rec, XR, XL, quad)
        return from_dicts(XR, n, b, a), (from_dicts(XL, n, b, a) if quad else None)
    Ar = _Reduced(At, reduced, a)
    Br = _Reduced(Bt, reduced, a) if quad else None
    m = len(reduced)
    if reduced_split and m >= 4:
        YR, YL = prgf(Ar, Br, reduced_bounds(m, reduced_parts), reduced_split=reduced_parts > 2,
                      reduced_parts=reduced_parts)
    else:
        YR, YL = rgf_bta(Ar, Br)
    for Y, X in ((YR, XR), (YL, XL)) if quad else ((YR, XR),):
        for j, r in enumerate(reduced):
            X[(r, r)] = Y.diag[j]
            if j < m - 1:
                X[(r, reduced[j + 1])] = Y.upper[j]
                X[(reduced[j + 1], r)] = Y.lower[j]
            if a > 0:
                X[(r, "t")] = Y.arrow_right[j]
                X[("t", r)] = Y.arrow_bottom[j]
        if a > 0:
            X[("t", "t")] = Y.tip
    for part in recs:
        for rec in reversed(part):
            backward_step(rec, XR, XL, quad)
    return from_dicts(XR, n, b, a), (from_dicts(XL, n, b, a) if quad else None)
