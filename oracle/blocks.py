"""Selected-block container used by the oracle (test infrastructure only)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Sel:
    """Blocks of a matrix on the BT/BTA pattern (Sec. II-A).

    diag[i] = X_{i,i}, upper[i] = X_{i,i+1}, lower[i] = X_{i+1,i},
    arrow_right[i] = X_{i,t}, arrow_bottom[i] = X_{t,i}, tip = X_{t,t}.
    """
    diag: np.ndarray
    upper: np.ndarray
    lower: np.ndarray
    arrow_right: np.ndarray
    arrow_bottom: np.ndarray
    tip: np.ndarray

    @staticmethod
    def zeros(n: int, b: int, a: int) -> "Sel":
        z = np.complex128
        m = max(n - 1, 0)
        return Sel(np.zeros((n, b, b), z), np.zeros((m, b, b), z),
                   np.zeros((m, b, b), z), np.zeros((n, b, a), z),
                   np.zeros((n, a, b), z), np.zeros((a, a), z))

    @staticmethod
    def zeros_var(sizes, a: int) -> "Sel":
        """Zero blocks for diagonal blocks of different sizes (Sec. II-A notes
        that RGF applies unchanged when the blocks of A differ in size): every
        field is a list of 2-D arrays, block i of size sizes[i]."""
        z = np.complex128
        n = len(sizes)
        return Sel([np.zeros((sizes[i], sizes[i]), z) for i in range(n)],
                   [np.zeros((sizes[i], sizes[i + 1]), z) for i in range(n - 1)],
                   [np.zeros((sizes[i + 1], sizes[i]), z) for i in range(n - 1)],
                   [np.zeros((sizes[i], a), z) for i in range(n)],
                   [np.zeros((a, sizes[i]), z) for i in range(n)],
                   np.zeros((a, a), z))

    @staticmethod
    def of(M) -> "Sel":
        """Copy the six block fields of any object that has them (lists of
        blocks stay lists)."""
        def cp(x):
            if isinstance(x, (list, tuple)):
                return [np.array(y, dtype=np.complex128, copy=True) for y in x]
            return np.array(x, dtype=np.complex128, copy=True)
        return Sel(*(cp(getattr(M, f)) for f in ("diag", "upper", "lower", "arrow_right",
                                                  "arrow_bottom", "tip")))

    @property
    def sizes(self):
        return block_sizes(self)

    def named(self):
        return {"diag": self.diag, "upper": self.upper, "lower": self.lower,
                "arrow_right": self.arrow_right, "arrow_bottom": self.arrow_bottom,
                "tip": self.tip}


def block_sizes(M):
    """Sizes of the diagonal blocks of M (a 3-D array or a list of blocks)."""
    return [int(np.shape(M.diag[i])[0]) for i in range(len(M.diag))]


def uniform(sizes):
    """True when every diagonal block has the same size."""
    return len(set(sizes)) <= 1


def tip_size(M) -> int:
    return int(np.shape(M.tip)[0])
