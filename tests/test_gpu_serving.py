"""Serving loop: continuous batching over the batch ABI.  Every request
completes; admission never exceeds the device-memory budget; each result is
the same solved alone and inside the mix (bitwise: an instance's products do
not depend on what shares the launches); results match the oracle."""
import numpy as np
import pytest

import oracle
from tests._util import rel_err

pytestmark = pytest.mark.gpu
FIELDS = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2601_04904_amd import serving, solver
    return serving, solver


def make_requests(serving, count=10, seed=3):
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for k in range(count):
        t += float(rng.exponential(0.002))
        reqs.append(serving.Request(rid=k, n=int(rng.integers(4, 16)), b=int(rng.choice([32, 64, 96])),
                                    a=int(rng.choice([0, 16, 40])),
                                    precision=str(rng.choice(["fp64", "mixed"])), E=float(rng.uniform(-1, 1)),
                                    eta=1e-2, seed=1000 + 17 * k, nrhs=int(rng.integers(1, 3)), arrival=t,
                                    keep_outputs=True))
    return reqs


def test_serving_mix_equals_alone_and_oracle(mods):
    serving, S = mods
    check_mix(serving, S, make_requests(serving))


def test_serving_mix_with_antihermitian_requests(mods):
    """Requests that assert an anti-Hermitian Sigma^< (every other one) share
    waves with general ones; each is still the same alone and in the mix."""
    serving, S = mods
    reqs = make_requests(serving, count=8, seed=9)
    for r in reqs:
        if r.rid % 2:
            r.flags |= S.BT_SIGMA_ANTIHERMITIAN
    check_mix(serving, S, reqs)


def check_mix(serving, S, reqs):
    eng = serving.ServingEngine(budget_bytes=int(64e9), max_inflight=2, max_wave=4)
    stats = eng.replay(reqs)
    print(stats, "waves", eng.waves, flush=True)
    assert not eng.errors, eng.errors
    assert stats["requests"] == len(reqs)
    assert eng.waves >= 2
    for r in reqs:
        assert r.t_done >= r.arrival
        A, B, B2 = serving.ServingEngine._device_inputs(r)
        XR, XL = S.DeviceBlocks.empty(r.n, r.b, r.a), S.DeviceBlocks.empty(r.n, r.b, r.a)
        bs = S.BatchSolver([r.spec()])
        bs.solve([A], [B], [XR], [XL])
        XL2 = None
        if r.nrhs > 1:
            XL2 = S.DeviceBlocks.empty(r.n, r.b, r.a)
            bs.selected_solve([B2], [XL2])
        bs.sync()
        bs.destroy()
        mixR, mixL, mixL2 = r.outputs
        for f in FIELDS:
            assert np.array_equal(getattr(XR, f).cpu().numpy(), getattr(mixR, f).cpu().numpy()), (r.rid, f)
            assert np.array_equal(getattr(XL, f).cpu().numpy(), getattr(mixL, f).cpu().numpy()), (r.rid, f)
            if XL2 is not None:
                assert np.array_equal(getattr(XL2, f).cpu().numpy(), getattr(mixL2, f).cpu().numpy())
        # against the oracle (inputs copied from the device)
        if r.rid % 3 == 0:
            Ah, Bh = A.to_host(), B.to_host()
            R0, L0 = oracle.solve_dense(Ah, Bh)
            e = max(rel_err(mixR.to_host(), R0), rel_err(mixL.to_host(), L0))
            tol = 1e-4 if (r.precision == "mixed" and not any(r.fallback)) else 1e-11
            print(r.rid, r.precision, r.n, r.b, r.a, f"err={e:.2e}", r.err, r.fallback, flush=True)
            assert e <= tol


def test_admission_respects_budget(mods):
    serving, S = mods
    reqs = make_requests(serving, count=8, seed=5)
    for r in reqs:
        r.keep_outputs = False
    biggest = max(serving.request_footprint(r) for r in reqs)
    eng = serving.ServingEngine(budget_bytes=int(biggest * 1.5), max_inflight=3, max_wave=8)
    stats = eng.replay(reqs)
    assert not eng.errors, eng.errors
    assert stats["requests"] == len(reqs)
    assert eng.max_used <= eng.budget
