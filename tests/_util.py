"""Shared test helpers: error metric and closed-form test matrices.

Nothing here is part of the method: the metric compares results, and the
chain builder constructs inputs whose exact solution is known.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")


def blocks_of(X):
    """List of (name, index, block) over the selected blocks of X."""
    out = []
    for f in FIELDS:
        val = getattr(X, f)
        if isinstance(val, (list, tuple)):       # blocks of different sizes
            for i, blk in enumerate(val):
                if np.size(blk):
                    out.append((f, i, np.asarray(blk)))
            continue
        arr = np.asarray(val)
        if arr.size == 0:
            continue
        if f == "tip":
            out.append((f, 0, arr))
        else:
            for i in range(arr.shape[0]):
                out.append((f, i, arr[i]))
    return out


def rel_err(X, Ref, floor: float = 1e-6):
    """max_k ||X_k - Ref_k||_F / max(||Ref_k||_F, floor * max_j ||Ref_j||_F).

    The per-block relative Frobenius error over the selected blocks; the
    floor keeps blocks that are (near) zero from dividing by zero.
    """
    xb = blocks_of(X)
    rb = blocks_of(Ref)
    assert [(f, i) for f, i, _ in xb] == [(f, i) for f, i, _ in rb]
    big = max((np.linalg.norm(r) for _, _, r in rb), default=0.0)
    worst = 0.0
    for (_, _, x), (_, _, r) in zip(xb, rb):
        den = max(np.linalg.norm(r), floor * big, 1e-300)
        worst = max(worst, float(np.linalg.norm(np.asarray(x) - r) / den))
    return worst


class Blocks:
    """Minimal block container for hand-built test matrices."""

    def __init__(self, diag, upper, lower, arrow_right=None, arrow_bottom=None, tip=None):
        n, b = diag.shape[0], diag.shape[1]
        self.diag, self.upper, self.lower = diag, upper, lower
        self.arrow_right = arrow_right if arrow_right is not None else np.zeros((n, b, 0), complex)
        self.arrow_bottom = arrow_bottom if arrow_bottom is not None else np.zeros((n, 0, b), complex)
        self.tip = tip if tip is not None else np.zeros((0, 0), complex)


def random_unitary(rng, m):
    Z = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def chain_problem(n, b, E, eta, t, f, seed, gauge=True):
    """Multi-band uniform chain with matched leads, and its exact solution.

    Textbook tight-binding result (not from the paper): every block row has
    onsite H0 (Hermitian b x b, eigen-decomposition V diag(eps) V^H) and
    hopping t I.  Per mode m, with z = E + i eta, s_m = sqrt((z-eps_m)^2 -
    4t^2) on the branch where lambda_m = (z - eps_m - s_m)/(2t) has
    |lambda_m| < 1, the semi-infinite lead self-energy is Sigma = V diag(t
    lambda_m) V^H.  Subtracting it from the end blocks makes the finite
    chain's Green's function equal to the infinite chain's:
        G_{jk} = V diag(lambda^|j-k| / s) V^H.
    With B_00 = i f Gamma, Gamma = i (Sigma - Sigma^H) (zero elsewhere):
        G^<_{jk} = G_{j0} B_00 G_{k0}^H.
    A block-diagonal unitary gauge U = diag(U_j) maps A -> U A U^H, B -> U B
    U^H and X_{jk} -> U_j X_{jk} U_k^H, so the blocks are dense and differ
    from block to block.
    Returns (A, B, XR, XL) as Blocks.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.normal(size=(b, b)) + 1j * rng.normal(size=(b, b))
    H0 = (M + M.conj().T) / (2 * np.sqrt(b))
    eps, V = np.linalg.eigh(H0)
    z = E + 1j * eta
    s = np.sqrt((z - eps) ** 2 - 4 * t * t + 0j)
    lam = (z - eps - s) / (2 * t)
    flip = np.abs(lam) >= 1
    s = np.where(flip, -s, s)
    lam = (z - eps - s) / (2 * t)
    assert np.all(np.abs(lam) < 1)
    Sig = V @ np.diag(t * lam) @ V.conj().T
    Gam = 1j * (Sig - Sig.conj().T)
    I = np.eye(b)
    diag = np.array([z * I - H0 for _ in range(n)], dtype=complex)
    diag[0] -= Sig
    diag[n - 1] -= Sig
    upper = np.array([-t * I for _ in range(n - 1)], dtype=complex).reshape(n - 1, b, b)
    lower = upper.copy()
    Bd = np.zeros((n, b, b), complex)
    Bd[0] = 1j * f * Gam
    Bu = np.zeros((n - 1, b, b), complex)
    Bl = np.zeros((n - 1, b, b), complex)

    def G(j, k):
        return V @ np.diag(lam ** abs(j - k) / s) @ V.conj().T

    XRd = np.array([G(j, j) for j in range(n)])
    XRu = np.array([G(j, j + 1) for j in range(n - 1)]).reshape(n - 1, b, b)
    XRl = np.array([G(j + 1, j) for j in range(n - 1)]).reshape(n - 1, b, b)
    Bfull = 1j * f * Gam
    XLd = np.array([G(j, 0) @ Bfull @ G(j, 0).conj().T for j in range(n)])
    XLu = np.array([G(j, 0) @ Bfull @ G(j + 1, 0).conj().T for j in range(n - 1)]).reshape(n - 1, b, b)
    XLl = np.array([G(j + 1, 0) @ Bfull @ G(j, 0).conj().T for j in range(n - 1)]).reshape(n - 1, b, b)
    if gauge:
        U = [random_unitary(rng, b) for _ in range(n)]

        def g(arr, off_r, off_c):
            return np.array([U[i + off_r] @ arr[i] @ U[i + off_c].conj().T
                             for i in range(arr.shape[0])]).reshape(arr.shape)

        diag, upper, lower = g(diag, 0, 0), g(upper, 0, 1), g(lower, 1, 0)
        Bd, Bu, Bl = g(Bd, 0, 0), g(Bu, 0, 1), g(Bl, 1, 0)
        XRd, XRu, XRl = g(XRd, 0, 0), g(XRu, 0, 1), g(XRl, 1, 0)
        XLd, XLu, XLl = g(XLd, 0, 0), g(XLu, 0, 1), g(XLl, 1, 0)
    return (Blocks(diag, upper, lower), Blocks(Bd, Bu, Bl),
            Blocks(XRd, XRu, XRl), Blocks(XLd, XLu, XLl))


def even_bounds(n, P):
    """Simple partition bounds for tests: ends get the remainder."""
    if P == 1:
        return [0, n]
    sz = [1] + [2] * (P - 2) + [1]
    rest = n - sum(sz)
    assert rest >= 0
    share = rest // P
    sz = [s + share for s in sz]
    rest -= share * P
    sz[0] += rest // 2
    sz[-1] += rest - rest // 2
    return list(np.cumsum([0] + sz))
