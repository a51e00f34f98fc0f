"""Seeded synthetic inputs: nanoribbon-shaped block-tridiagonal (BT) and
BT-with-arrowhead (BTA) matrices A and right-hand sides B = Sigma^<.

This module builds the *inputs* of the problem stated in Sec. II-A of the
paper (A X = I and A X A^H = B on a BT/BTA pattern with n diagonal blocks of
size b and an arrow tip of size a).  It holds none of the method's
arithmetic: the oracle and the HIP path both take what it returns.

Recipe (a stand-in for the paper's NR-FET dataset, which is not available):
  * H_ii = (M + M^H)/sqrt(2b) + diag(U(-1, 1)),  M complex N(0, 1)
    (so the off-diagonal entries of H_ii are N(0, 1/b)).
  * A_ii = (E + i eta) I - H_ii; blocks 0 and n-1 get the boundary
    self-energy Sigma^R = -0.5i I, i.e. A_00 and A_{n-1,n-1} gain +0.5i I.
  * A_{i,i+1} = -T_i, A_{i+1,i} = -T_i^H,  T_i complex N(0, 0.5/b).
  * Arrowhead (a > 0): A_{i,t} = -K_i, A_{t,i} = -K_i^H, K_i complex
    N(0, 0.1/b) (b x a); A_tt = (E + i eta) I - H_t + 0.5i I with H_t built
    like H_ii at size a.
  * B = Sigma^< (anti-Hermitian): B_ii = i C_i C_i^H / b, B_{i,i+1} = 0.1i D_i,
    B_{i+1,i} = 0.1i D_i^H, B_{i,t} = 0.1i F_i, B_{t,i} = 0.1i F_i^H,
    B_tt = i C_t C_t^H / a, with C, D, F complex N(0, 1).
  Im(A) = (A - A^H)/(2i) is eta I plus non-negative boundary terms, so A and
  every Schur complement taken from it are nonsingular.

Complex N(0, s2) means (N(0, s2/2) + i N(0, s2/2)).  Draw order with
numpy.random.Generator(PCG64(seed)): for i = 0..n-1: M_i, onsite_i, then
(i < n-1) T_i; then for i = 0..n-1: C_i, then (i < n-1) D_i; then, if a > 0:
K_0..K_{n-1}, M_t, onsite_t, F_0..F_{n-1}, C_t.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BTA", "VBTA", "gen_A", "gen_B", "gen_problem", "gen_problem_var", "ramp_sizes",
    "CONFIGS", "VAR_CONFIGS", "config_problem", "batch_specs", "serving_trace",
    "equilibrium_B", "perturb",
]


@dataclass
class BTA:
    """Block storage of a BT (a == 0) or BTA matrix, complex128, row-major blocks.

    diag[i] = M_{i,i} (b x b), upper[i] = M_{i,i+1}, lower[i] = M_{i+1,i},
    arrow_right[i] = M_{i,t} (b x a), arrow_bottom[i] = M_{t,i} (a x b),
    tip = M_{t,t} (a x a).
    """
    diag: np.ndarray
    upper: np.ndarray
    lower: np.ndarray
    arrow_right: np.ndarray
    arrow_bottom: np.ndarray
    tip: np.ndarray

    @property
    def n(self) -> int:
        return self.diag.shape[0]

    @property
    def b(self) -> int:
        return self.diag.shape[1]

    @property
    def a(self) -> int:
        return self.tip.shape[0]

    def fields(self):
        return (self.diag, self.upper, self.lower, self.arrow_right,
                self.arrow_bottom, self.tip)

    def copy(self) -> "BTA":
        return BTA(*(np.array(f, copy=True) for f in self.fields()))

    @staticmethod
    def zeros(n: int, b: int, a: int, dtype=np.complex128) -> "BTA":
        return BTA(np.zeros((n, b, b), dtype), np.zeros((max(n - 1, 0), b, b), dtype),
                   np.zeros((max(n - 1, 0), b, b), dtype), np.zeros((n, b, a), dtype),
                   np.zeros((n, a, b), dtype), np.zeros((a, a), dtype))


@dataclass
class VBTA:
    """Block storage with diagonal blocks of different sizes (Sec. II-A: RGF
    applies unchanged when the blocks differ in size, e.g. a device whose
    cross-section varies between source and drain).  Every field is a list of
    2-D complex128 blocks: diag[i] is sizes[i] x sizes[i], upper[i] is
    sizes[i] x sizes[i+1], lower[i] is sizes[i+1] x sizes[i], arrow_right[i]
    is sizes[i] x a, arrow_bottom[i] is a x sizes[i], tip is a x a."""
    diag: list
    upper: list
    lower: list
    arrow_right: list
    arrow_bottom: list
    tip: np.ndarray

    @property
    def sizes(self):
        return [int(d.shape[0]) for d in self.diag]

    @property
    def n(self) -> int:
        return len(self.diag)

    @property
    def a(self) -> int:
        return self.tip.shape[0]

    def fields(self):
        return (self.diag, self.upper, self.lower, self.arrow_right,
                self.arrow_bottom, self.tip)

    @staticmethod
    def zeros(sizes, a: int, dtype=np.complex128) -> "VBTA":
        n = len(sizes)
        return VBTA([np.zeros((sizes[i], sizes[i]), dtype) for i in range(n)],
                    [np.zeros((sizes[i], sizes[i + 1]), dtype) for i in range(n - 1)],
                    [np.zeros((sizes[i + 1], sizes[i]), dtype) for i in range(n - 1)],
                    [np.zeros((sizes[i], a), dtype) for i in range(n)],
                    [np.zeros((a, sizes[i]), dtype) for i in range(n)],
                    np.zeros((a, a), dtype))


def _cn(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    s = np.sqrt(var / 2.0)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


def _hermitian(rng: np.random.Generator, m: int) -> np.ndarray:
    M = _cn(rng, (m, m), 1.0)
    H = (M + M.conj().T) / np.sqrt(2.0 * m)
    onsite = rng.uniform(-1.0, 1.0, m)
    return H + np.diag(onsite)


def gen_A(rng: np.random.Generator, n: int, b: int, a: int, E: float, eta: float,
          boundary: float = 0.5) -> BTA:
    A = BTA.zeros(n, b, a)
    z = E + 1j * eta
    for i in range(n):
        H = _hermitian(rng, b)
        A.diag[i] = z * np.eye(b) - H
        if i < n - 1:
            T = _cn(rng, (b, b), 0.5 / b)
            A.upper[i] = -T
            A.lower[i] = -T.conj().T
    A.diag[0] += 1j * boundary * np.eye(b)
    if n > 1:
        A.diag[n - 1] += 1j * boundary * np.eye(b)
    if a > 0:
        for i in range(n):
            K = _cn(rng, (b, a), 0.1 / b)
            A.arrow_right[i] = -K
            A.arrow_bottom[i] = -K.conj().T
        Ht = _hermitian(rng, a)
        A.tip[:] = z * np.eye(a) - Ht + 1j * boundary * np.eye(a)
    return A


def gen_B(rng: np.random.Generator, n: int, b: int, a: int) -> BTA:
    B = BTA.zeros(n, b, a)
    for i in range(n):
        C = _cn(rng, (b, b), 1.0)
        B.diag[i] = 1j * (C @ C.conj().T) / b
        if i < n - 1:
            D = _cn(rng, (b, b), 1.0)
            B.upper[i] = 0.1j * D
            B.lower[i] = 0.1j * D.conj().T
    if a > 0:
        for i in range(n):
            F = _cn(rng, (b, a), 1.0)
            B.arrow_right[i] = 0.1j * F
            B.arrow_bottom[i] = 0.1j * F.conj().T
        Ct = _cn(rng, (a, a), 1.0)
        B.tip[:] = 1j * (Ct @ Ct.conj().T) / a
    return B


def gen_problem(n: int, b: int, a: int = 0, E: float = 0.3, eta: float = 1e-3,
                seed: int = 0):
    """(A, B) for one instance, drawn from one PCG64 stream: A first, then B."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = gen_A(rng, n, b, a, E, eta)
    B = gen_B(rng, n, b, a)
    return A, B


def gen_problem_var(sizes, a: int = 0, E: float = 0.3, eta: float = 1e-3, seed: int = 0):
    """(A, B) with diagonal blocks of the given sizes: the recipe above with b
    replaced by the size of the block at hand, and the couplings scaled by
    the geometric mean of the two sizes they join (T_i complex
    N(0, 0.5/sqrt(b_i b_{i+1})), b_i x b_{i+1}).  Same draw order as
    gen_problem; with equal sizes the values equal gen_problem's."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(sizes)
    z = E + 1j * eta
    A = VBTA.zeros(sizes, a)
    for i in range(n):
        b = sizes[i]
        A.diag[i] = z * np.eye(b) - _hermitian(rng, b)
        if i < n - 1:
            T = _cn(rng, (b, sizes[i + 1]), 0.5 / np.sqrt(b * sizes[i + 1]))
            A.upper[i] = -T
            A.lower[i] = -T.conj().T
    A.diag[0] += 0.5j * np.eye(sizes[0])
    if n > 1:
        A.diag[n - 1] += 0.5j * np.eye(sizes[n - 1])
    if a > 0:
        for i in range(n):
            K = _cn(rng, (sizes[i], a), 0.1 / sizes[i])
            A.arrow_right[i] = -K
            A.arrow_bottom[i] = -K.conj().T
        A.tip[:] = z * np.eye(a) - _hermitian(rng, a) + 0.5j * np.eye(a)
    B = VBTA.zeros(sizes, a)
    for i in range(n):
        C = _cn(rng, (sizes[i], sizes[i]), 1.0)
        B.diag[i] = 1j * (C @ C.conj().T) / sizes[i]
        if i < n - 1:
            D = _cn(rng, (sizes[i], sizes[i + 1]), 1.0)
            B.upper[i] = 0.1j * D
            B.lower[i] = 0.1j * D.conj().T
    if a > 0:
        for i in range(n):
            F = _cn(rng, (sizes[i], a), 1.0)
            B.arrow_right[i] = 0.1j * F
            B.arrow_bottom[i] = 0.1j * F.conj().T
        Ct = _cn(rng, (a, a), 1.0)
        B.tip[:] = 1j * (Ct @ Ct.conj().T) / a
    return A, B


def ramp_sizes(n: int, lo: int, hi: int, steps: int):
    """Block sizes of a device whose cross-section widens from the contacts
    (size lo) to the channel (size hi) over `steps` blocks at each end."""
    out = []
    for i in range(n):
        j = min(i, n - 1 - i, steps)
        out.append(int(lo + (hi - lo) * j // steps))
    return out


def equilibrium_B(A: BTA, c: complex = 1.0) -> BTA:
    """B = c (A^H - A) restricted to the pattern (anti-Hermitian for real c).

    For this right-hand side the exact solution is X^< = c (G^R - G^A), a
    property the tests use at any size.  Pure input construction.
    """
    n, b, a = A.diag.shape[0], A.diag.shape[1], A.tip.shape[0]
    B = BTA.zeros(n, b, a)
    for i in range(n):
        B.diag[i] = c * (A.diag[i].conj().T - A.diag[i])
    for i in range(n - 1):
        B.upper[i] = c * (A.lower[i].conj().T - A.upper[i])
        B.lower[i] = c * (A.upper[i].conj().T - A.lower[i])
    if a > 0:
        for i in range(n):
            B.arrow_right[i] = c * (A.arrow_bottom[i].conj().T - A.arrow_right[i])
            B.arrow_bottom[i] = c * (A.arrow_right[i].conj().T - A.arrow_bottom[i])
        B.tip[:] = c * (A.tip.conj().T - A.tip)
    return B


def perturb(M: BTA, rel: float, seed: int) -> BTA:
    """Copy of M with every entry x replaced by x (1 + rel u), u uniform in the
    complex square [-1, 1] + i[-1, 1] (seeded).  With rel near the unit
    roundoff, solving the copy with the same algorithm gives a second result
    whose rounding errors are independent of the first: the spread of the two
    measures how much that algorithm and input amplify rounding.  Pure input
    construction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if isinstance(M, VBTA):
        out = VBTA(*([np.array(x, copy=True) for x in f] if isinstance(f, list) else np.array(f, copy=True)
                     for f in M.fields()))
        pieces = [x for f in out.fields() for x in (f if isinstance(f, list) else [f])]
    else:
        out = M.copy()
        pieces = list(out.fields())
    for f in pieces:
        if f.size:
            u = rng.uniform(-1.0, 1.0, f.shape) + 1j * rng.uniform(-1.0, 1.0, f.shape)
            f *= 1.0 + rel * u
    return out


@dataclass
class ProblemConfig:
    name: str
    n: int
    b: int
    a: int = 0
    E: float = 0.3
    eta: float = 1e-3
    seed: int = 0
    partitions: tuple = field(default_factory=lambda: (1,))


# Workloads: single-instance configurations (sequential and partitioned).
CONFIGS = {
    "bt_n16_b32": ProblemConfig("bt_n16_b32", 16, 32, 0, 0.3, 1e-3, 0, (1, 2, 4)),
    "bt_n64_b512": ProblemConfig("bt_n64_b512", 64, 512, 0, 0.3, 1e-4, 0, (1, 8)),
    "bta_n128_b384_a512": ProblemConfig("bta_n128_b384_a512", 128, 384, 512, 0.3, 1e-3, 0, (16,)),
    # the synthetic-device (SD) weak-scaling series of Sec. IV at its one-GPU
    # size: n = 32 diagonal blocks of b = 1024 (same input recipe)
    "sd_n32_b1024": ProblemConfig("sd_n32_b1024", 32, 1024, 0, 0.3, 1e-3, 0, (1, 2, 4)),
}

# Diagonal blocks of different sizes (Sec. II-A): a device whose cross-section
# widens from 256 at the contacts to 512 in the channel over 4 blocks at each
# end (n = 48), without and with an arrowhead of 256.
VAR_CONFIGS = {
    "vb_n48_b256to512": dict(sizes=ramp_sizes(48, 256, 512, 4), a=0, E=0.3, eta=1e-3, seed=0,
                             partitions=(1, 4)),
    "vbta_n48_b256to512_a256": dict(sizes=ramp_sizes(48, 256, 512, 4), a=256, E=0.3, eta=1e-3,
                                    seed=0, partitions=(1, 4)),
}


def config_problem(name: str):
    if name in VAR_CONFIGS:
        c = VAR_CONFIGS[name]
        return gen_problem_var(c["sizes"], c["a"], c["E"], c["eta"], c["seed"])
    c = CONFIGS[name]
    return gen_problem(c.n, c.b, c.a, c.E, c.eta, c.seed)


def batch_specs(count: int = 512, master_seed: int = 0):
    """Uneven batched energy sweep: per instance (n, b, a, E, eta, seed).

    n ~ U{16..96}, b ~ U{64,128,192,256,384}, a ~ U{0,128,256}, E ~ U[-1,1],
    eta = 1e-3, instance seed = 1000 + index.
    """
    rng = np.random.Generator(np.random.PCG64(master_seed))
    bs = (64, 128, 192, 256, 384)
    as_ = (0, 128, 256)
    out = []
    for idx in range(count):
        n = int(rng.integers(16, 97))
        b = int(bs[rng.integers(0, len(bs))])
        a = int(as_[rng.integers(0, len(as_))])
        E = float(rng.uniform(-1.0, 1.0))
        out.append(dict(n=n, b=b, a=a, E=E, eta=1e-3, seed=1000 + idx))
    return out


def serving_trace(count: int = 256, rate: float = 200.0, seed: int = 0,
                  n_range=(16, 256), b_choices=None, a_choices=(0, 256, 512),
                  fp64_fraction: float = 0.3):
    """Poisson arrival trace of SI+SQ requests.

    Each request: arrival time (s), n ~ U{n_range}, b ~ U{b_choices}
    (default multiples of 64 in 128..1024), a ~ U{a_choices}, precision
    ('fp64' with probability fp64_fraction, else 'mixed'), E ~ U[-1, 1],
    eta = 1e-3, seed, and k in {1, 2} right-hand sides (50/50; the second
    right-hand side is generated with seed + 1).
    """
    if b_choices is None:
        b_choices = tuple(range(128, 1025, 64))
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for idx in range(count):
        t += float(rng.exponential(1.0 / rate))
        out.append(dict(
            arrival=t,
            n=int(rng.integers(n_range[0], n_range[1] + 1)),
            b=int(b_choices[rng.integers(0, len(b_choices))]),
            a=int(a_choices[rng.integers(0, len(a_choices))]),
            precision="fp64" if rng.uniform() < fp64_fraction else "mixed",
            E=float(rng.uniform(-1.0, 1.0)),
            eta=1e-3,
            seed=100000 + 2 * idx,
            nrhs=int(rng.integers(1, 3)),
        ))
    return out
