"""The allocation-free batched inverse (bt_si_sq_diag_inverse_noalloc) against
the allocating one (bt_si_sq_diag_inverse), through the C ABI: same kernels,
so the same result to the FP64 bar, on two calls in a row (the second
smaller, so it runs on what the first left in the fixed scratch array), and
the same singular-block report."""
import numpy as np
import pytest

from tests._util import random_unitary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import solver
    return solver


def batch(count, d, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        # U diag(sigma) V^H with singular values in [0.5, 4]: well conditioned, dense
        s = rng.uniform(0.5, 4.0, d)
        out.append(random_unitary(rng, d) @ np.diag(s) @ random_unitary(rng, d).conj().T)
    return np.array(out)


def rel(x, y):
    return max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(x, y))


@pytest.mark.parametrize("calls", [[(6, 200), (3, 120)], [(2, 1024), (5, 33)]])
def test_noalloc_matches_allocating_inverse(S, calls):
    import torch
    for count, d in calls:
        print(f"[noalloc] count={count} d={d}", flush=True)
        M = batch(count, d, seed=count * 1000 + d)
        src = torch.from_numpy(M).cuda()
        dst = torch.empty_like(src)
        ref, bad_ref = S.diag_inverse(src)
        out, bad = S.diag_inverse_noalloc(src, dst)
        torch.cuda.synchronize()
        assert bad == -1 and bad_ref == -1
        o, r = out.cpu().numpy(), ref.cpu().numpy()
        assert rel(o, r) <= 1e-11
        assert rel(o, np.linalg.inv(M)) <= 1e-11


def test_noalloc_reports_singular_block(S):
    import torch
    M = batch(4, 64, seed=7)
    M[2, :, 5] = 0.0                      # block 2 has a zero column
    src = torch.from_numpy(M).cuda()
    _, bad_ref = S.diag_inverse(src)
    _, bad = S.diag_inverse_noalloc(src)
    assert bad == bad_ref == 2
    # the next call starts from a clean status word
    M2 = batch(2, 40, seed=8)
    out, bad2 = S.diag_inverse_noalloc(torch.from_numpy(M2).cuda())
    assert bad2 == -1
    assert rel(out.cpu().numpy(), np.linalg.inv(M2)) <= 1e-11
