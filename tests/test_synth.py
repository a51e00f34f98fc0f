"""Seeded input generator: determinism and the structure the recipe promises."""
import numpy as np

from paper_2601_04904_amd.synth import (gen_problem, batch_specs, serving_trace,
                                        equilibrium_B, CONFIGS, config_problem)


def test_deterministic_per_seed():
    A1, B1 = gen_problem(4, 5, 3, seed=7)
    A2, B2 = gen_problem(4, 5, 3, seed=7)
    A3, _ = gen_problem(4, 5, 3, seed=8)
    for f1, f2 in zip(A1.fields() + B1.fields(), A2.fields() + B2.fields()):
        assert np.array_equal(f1, f2)
    assert not np.array_equal(A1.diag, A3.diag)


def test_structure():
    n, b, a, E, eta = 5, 6, 4, 0.3, 1e-3
    A, B = gen_problem(n, b, a, E=E, eta=eta, seed=1)
    for i in range(n):
        H = (E + 1j * eta) * np.eye(b) - A.diag[i]
        if i in (0, n - 1):
            H = H + 0.5j * np.eye(b)
        assert np.allclose(H, H.conj().T, atol=1e-15)          # Hermitian H_ii
        assert np.allclose(B.diag[i], -B.diag[i].conj().T)      # anti-Hermitian B_ii
    for i in range(n - 1):
        assert np.allclose(A.lower[i], A.upper[i].conj().T)
        assert np.allclose(B.lower[i], -B.upper[i].conj().T)
    for i in range(n):
        assert np.allclose(A.arrow_bottom[i], A.arrow_right[i].conj().T)
        assert np.allclose(B.arrow_bottom[i], -B.arrow_right[i].conj().T)
    assert np.allclose(B.tip, -B.tip.conj().T)


def test_imaginary_part_positive_definite():
    """Im(A) = (A - A^H)/(2i) has smallest eigenvalue eta (boundary terms add 0.5)."""
    import oracle
    A, _ = gen_problem(6, 4, 3, E=0.1, eta=1e-3, seed=3)
    D = oracle.assemble(A)
    ImA = (D - D.conj().T) / 2j
    w = np.linalg.eigvalsh(ImA)
    assert abs(w.min() - 1e-3) < 1e-12


def test_equilibrium_B_is_antihermitian():
    A, _ = gen_problem(4, 3, 2, seed=0)
    B = equilibrium_B(A, 2.0)
    for i in range(4):
        assert np.allclose(B.diag[i], -B.diag[i].conj().T)
        assert np.allclose(B.arrow_bottom[i], -B.arrow_right[i].conj().T)


def test_config_shapes():
    A, B = config_problem("bt_n16_b32")
    assert A.diag.shape == (16, 32, 32) and A.tip.shape == (0, 0)
    assert CONFIGS["bt_n64_b512"].eta == 1e-4
    c = CONFIGS["bta_n128_b384_a512"]
    assert (c.n, c.b, c.a) == (128, 384, 512)


def test_batch_and_trace_specs():
    specs = batch_specs(512)
    assert len(specs) == 512
    assert all(16 <= s["n"] <= 96 and s["b"] in (64, 128, 192, 256, 384) and s["a"] in (0, 128, 256)
               for s in specs)
    assert specs == batch_specs(512)
    tr = serving_trace(64)
    t = [r["arrival"] for r in tr]
    assert all(x < y for x, y in zip(t, t[1:]))
    assert all(r["b"] % 64 == 0 and 128 <= r["b"] <= 1024 for r in tr)
