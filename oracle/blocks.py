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
    def of(M) -> "Sel":
        """Copy the six block fields of any object that has them."""
        return Sel(*(np.array(getattr(M, f), dtype=np.complex128, copy=True)
                     for f in ("diag", "upper", "lower", "arrow_right",
                               "arrow_bottom", "tip")))

    def named(self):
        return {"diag": self.diag, "upper": self.upper, "lower": self.lower,
                "arrow_right": self.arrow_right, "arrow_bottom": self.arrow_bottom,
                "tip": self.tip}
