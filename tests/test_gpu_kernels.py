"""Kernel-level GPU checks through the diagnostic C entry points:
the grouped complex product (every op(A)/op(B) combination, ragged shapes,
alpha/beta, in-place C == D, FP64 and mixed) against NumPy complex128, and
the batched diagonal-block inverse against numpy.linalg.inv, including
matrices that need pivoting and singular ones.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def crand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


SHAPES = [(1, 1, 1), (64, 32, 16), (100, 37, 53), (128, 64, 200), (5, 300, 7), (65, 33, 17),
          (512, 512, 512)]


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_fp64(torch, m, n, k, opA, opB, shape):
    from paper_2601_04904_amd.solver import diag_gemm
    rng = np.random.default_rng(m * 7 + n * 3 + k + 10 * opA + 20 * opB)
    A = crand(rng, *((k, m) if opA else (m, k)))
    B = crand(rng, *((n, k) if opB else (k, n)))
    C = crand(rng, m, n)
    alpha, beta = 0.7 - 0.3j, -1.1 + 0.4j
    ref = beta * C + alpha * ((A.conj().T if opA else A) @ (B.conj().T if opB else B))
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C))
    out = diag_gemm(alpha, dA, opA, dB, opB, beta=beta, Cin=dC, shape=shape)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-13 * max(1, np.sqrt(k)), err


def test_gemm_in_place_and_no_c(torch):
    from paper_2601_04904_amd.solver import diag_gemm
    rng = np.random.default_rng(1)
    A, B, C = crand(rng, 70, 90), crand(rng, 90, 45), crand(rng, 70, 45)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C))
    diag_gemm(-1.0, dA, 0, dB, 0, beta=1.0, Cin=dC, D=dC)        # C -= A B in place
    out0 = diag_gemm(2.0j, dA, 0, dB, 0)                            # no C
    torch.cuda.synchronize()
    assert np.allclose(dC.cpu().numpy(), C - A @ B, rtol=0, atol=1e-12)
    assert np.allclose(out0.cpu().numpy(), 2j * (A @ B), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(64, 32, 16), (200, 100, 300), (384, 384, 384)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 1), (0, 1)])
def test_gemm_mixed(torch, m, n, k, opA, opB, shape):
    from paper_2601_04904_amd.solver import diag_gemm
    rng = np.random.default_rng(5)
    A = crand(rng, *((k, m) if opA else (m, k)))
    B = crand(rng, *((n, k) if opB else (k, n)))
    ref = (A.conj().T if opA else A) @ (B.conj().T if opB else B)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    out = diag_gemm(1.0, dA, opA, dB, opB, mixed=True, shape=shape)
    torch.cuda.synchronize()
    err = np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 2e-6, err     # complex64 products with FP32 accumulation


@pytest.mark.parametrize("d", [1, 2, 15, 16, 17, 32, 33, 100, 384, 512, 513, 1024])
def test_inverse_random(torch, d):
    from paper_2601_04904_amd.solver import diag_inverse
    rng = np.random.default_rng(d)
    M = crand(rng, 3, d, d) + 0.5 * np.eye(d)
    dst, bad = diag_inverse(torch.from_numpy(M).cuda())
    torch.cuda.synchronize()
    assert bad == -1
    got = dst.cpu().numpy()
    for i in range(3):
        ref = np.linalg.inv(M[i])
        err = np.linalg.norm(got[i] - ref) / np.linalg.norm(ref)
        assert err < 1e-14 * np.linalg.cond(M[i]) * np.sqrt(d) + 1e-14, (i, err)


def test_inverse_needs_pivoting(torch):
    from paper_2601_04904_amd.solver import diag_inverse
    rng = np.random.default_rng(3)
    d = 40
    P = np.eye(d)[rng.permutation(d)].astype(complex)          # zero leading entries
    Z = crand(rng, d, d)
    Z[0, 0] = 0.0                                                # exact zero pivot candidate
    Z[:, 5] *= 1e-9                                              # badly scaled column
    M = np.stack([P, Z, P @ crand(rng, d, d)])
    dst, bad = diag_inverse(torch.from_numpy(M).cuda())
    torch.cuda.synchronize()
    assert bad == -1
    got = dst.cpu().numpy()
    for i in range(3):
        ref = np.linalg.inv(M[i])
        assert np.linalg.norm(got[i] - ref) / np.linalg.norm(ref) < 1e-11


def test_inverse_mixed_sizes_in_batch_via_solver(torch):
    """A BTA tip of a different size is inverted in the same batch as b x b blocks."""
    from paper_2601_04904_amd.solver import diag_inverse
    rng = np.random.default_rng(9)
    for d in (48, 600):
        M = crand(rng, 2, d, d)
        dst, bad = diag_inverse(torch.from_numpy(M).cuda())
        torch.cuda.synchronize()
        ref = np.linalg.inv(M)
        assert np.linalg.norm(dst.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-11


def test_inverse_singular_is_flagged(torch):
    from paper_2601_04904_amd.solver import diag_inverse
    rng = np.random.default_rng(4)
    d = 20
    M = crand(rng, 3, d, d)
    M[1, :, 7] = 0.0             # singular second matrix
    _, bad = diag_inverse(torch.from_numpy(M).cuda())
    torch.cuda.synchronize()
    assert bad == 1
    M[1, :, 7] = np.nan          # non-finite
    _, bad = diag_inverse(torch.from_numpy(M).cuda())
    torch.cuda.synchronize()
    assert bad == 1


def test_inverse_pivot_choice_matters(torch):
    """Each column has one large entry (1e3) in a random row and small ones (1e-3)
    elsewhere: any pivot other than the largest entry costs about six digits,
    so this checks the pivot search picks the maximum."""
    from paper_2601_04904_amd.solver import diag_inverse
    rng = np.random.default_rng(11)
    for d in (64, 300, 512):
        M = 1e-3 * crand(rng, d, d)
        perm = rng.permutation(d)
        M[perm, np.arange(d)] = 1e3 * (1.0 + rng.uniform(size=d)) * np.exp(2j * np.pi * rng.uniform(size=d))
        dst, bad = diag_inverse(torch.from_numpy(M[None]).cuda())
        torch.cuda.synchronize()
        assert bad == -1
        ref = np.linalg.inv(M)
        err = np.linalg.norm(dst.cpu().numpy()[0] - ref) / np.linalg.norm(ref)
        assert err < 1e-14 * np.sqrt(d) * 10, (d, err)


def test_autotune_fills_table_and_solves_still_match(torch):
    """The autotuner times every shape, stores a shape for each class it
    reaches, and a solve compiled with the tuned table matches the oracle."""
    from paper_2601_04904_amd import solver as S
    import oracle
    from paper_2601_04904_amd.synth import gen_problem
    saved = S.tune_table()
    try:
        report = S.autotune()
        assert report, "no classes timed"
        table = S.tune_table()
        for line in report:
            prec, mc, tc, shape = (int(v) for v in line.split()[:4])
            assert table[(prec * 6 + mc) * 14 + tc] == shape
            assert all(float(v) > 0 for v in line.split()[4:])
        A, B = gen_problem(12, 96, 40, 0.3, 1e-2, 3)
        n, b, a = 12, 96, 40
        dA, dB = S.DeviceBlocks.from_host(A), S.DeviceBlocks.from_host(B)
        XR, XL = S.DeviceBlocks.empty(n, b, a), S.DeviceBlocks.empty(n, b, a)
        sol = S.Solver(n, b, a, partitions=2)
        sol.solve(dA, dB, XR, XL)
        sol.sync()
        sol.destroy()
        from tests._util import rel_err
        ref = oracle.solve_dense(A, B)
        assert rel_err(XR.to_host(), ref[0]) < 1e-11
        assert rel_err(XL.to_host(), ref[1]) < 1e-11
    finally:
        S.set_tune_table(saved)
