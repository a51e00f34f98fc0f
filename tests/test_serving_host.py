"""Host-side logic of the serving layer (no GPU): precision routing and
footprint accounting."""
from paper_2601_04904_amd import serving
from paper_2601_04904_amd import solver as S


def test_router_probes_then_routes_and_reprobes():
    r = serving.PrecisionRouter(threshold=0.5, probe=2, reprobe=4)
    # first requests of a class try the mixed path, no more at once than needed
    assert r.choose(1e-3, 0) == S.BT_MIXED
    assert r.choose(2e-3, 0) == S.BT_MIXED          # same decade, same class
    assert r.choose(1e-3, 0) == S.BT_FP64           # two probes already in flight
    r.record(1e-3, 0, True)
    r.record(2e-3, 0, True)
    r.routed = 0
    picks = [r.choose(1e-3, 0) for _ in range(8)]
    # every 4th request still probes; the others go to FP64
    assert picks.count(S.BT_MIXED) == 2 and picks.count(S.BT_FP64) == 6
    assert r.routed == 6
    # other classes are independent
    assert r.choose(1e-1, 0) == S.BT_MIXED
    assert r.choose(1e-3, 64) == S.BT_MIXED


def test_router_recovers_when_mixed_succeeds():
    r = serving.PrecisionRouter(threshold=0.5, probe=1, reprobe=2, decay=0.5)
    r.choose(1e-2, 0)
    r.record(1e-2, 0, True)
    for _ in range(6):
        r.record(1e-2, 0, False)        # successful mixed runs bring the rate down
    assert r.rate[(-2, False)] < 0.5
    assert all(r.choose(1e-2, 0) == S.BT_MIXED for _ in range(5))


def test_request_footprint_counts_workspace_io_and_generator():
    req = serving.Request(rid=0, n=8, b=64, a=0, nrhs=2)
    ws = S.batch_workspace_bytes([req.spec()])
    fp = serving.request_footprint(req)
    assert fp == ws + 16 * req.pattern_elems() * 6 + 16 * 3 * 8 * 64 * 64


def test_requests_from_trace_keep_order_and_fields():
    from paper_2601_04904_amd.synth import serving_trace
    tr = serving_trace(5, rate=100.0, seed=1, n_range=(4, 8), b_choices=(64, 128))
    reqs = serving.requests_from_trace(tr)
    assert [r.rid for r in reqs] == list(range(5))
    assert all(4 <= r.n <= 8 and r.b in (64, 128) for r in reqs)
    assert all(reqs[i].arrival <= reqs[i + 1].arrival for i in range(4))


def test_router_probes_only_cheap_requests():
    r = serving.PrecisionRouter(probe=1, probe_max_flops=1e9)
    assert r.choose(1e-3, 0, flops=5e9) == S.BT_FP64     # expensive, nothing known: FP64
    assert r.routed == 1
    assert r.choose(1e-3, 0, flops=1e8) == S.BT_MIXED    # cheap: probe
    r.record(1e-3, 0, False)                             # mixed passed
    assert r.choose(1e-3, 0, flops=5e9) == S.BT_MIXED    # now known to pass


def test_wave_stops_at_very_different_request():
    eng = serving.ServingEngine.__new__(serving.ServingEngine)
    eng.pending = serving.deque()
    eng.used, eng.budget, eng.max_wave, eng.max_used = 0, 1 << 60, 8, 0
    eng.size_ratio = 8.0
    eng.t0 = 0.0
    eng.now = lambda: 0.0
    small = [serving.Request(rid=i, n=8, b=64, a=0) for i in range(3)]
    big = serving.Request(rid=9, n=64, b=512, a=0)
    for r in small[:2] + [big] + small[2:]:
        r.footprint = 1
        eng.pending.append(r)
    wave = eng._take_wave()
    assert [r.rid for r in wave] == [0, 1]
    assert eng.pending[0].rid == 9
