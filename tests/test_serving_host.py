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
    # six matrices of blocks (A, B, XR, XL, B2, XL2), each field 256-aligned;
    # the generator's temporaries for CHUNK blocks at a time
    assert serving.blocks_bytes(8, 64, 0) == 16 * req.pattern_elems()
    assert fp == ws + 16 * req.pattern_elems() * 6 + 16 * 4 * 8 * 64 * 64


def test_device_arena_first_fit_and_merge():
    arena = serving.DeviceArena.__new__(serving.DeviceArena)
    arena.size = 4096
    arena.free = [(0, 4096)]
    a = arena.alloc(1000)          # rounded to 1024
    b = arena.alloc(256)
    c = arena.alloc(2048)
    assert (a, b, c) == (0, 1024, 1280)
    assert arena.alloc(1024) is None          # only 768 left
    arena.release(b, 256)
    assert arena.alloc(800) is None            # a 256 hole and 768 at the end
    arena.release(a, 1000)                     # merges with the hole: [0, 1280)
    assert arena.free[0] == (0, 1280)
    assert arena.alloc(1280) == 0
    arena.release(0, 1280)
    arena.release(c, 2048)
    assert arena.free == [(0, 4096)]


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


def _bare_engine():
    eng = serving.ServingEngine.__new__(serving.ServingEngine)
    eng.pending = serving.deque()
    eng.used, eng.budget, eng.max_wave, eng.max_used = 0, 1 << 60, 8, 0
    eng.size_ratio, eng.chain_ratio = 4.0, 1.5
    eng.t0 = 0.0
    eng.now = lambda: 0.0
    return eng


def test_wave_groups_compatible_requests_and_keeps_the_rest_in_order():
    eng = _bare_engine()
    small = [serving.Request(rid=i, n=8, b=64, a=0) for i in range(3)]
    big = serving.Request(rid=9, n=64, b=512, a=0)
    long_chain = serving.Request(rid=7, n=16, b=48, a=0)    # similar work, twice the chain
    for r in small[:2] + [big, long_chain] + small[2:]:
        r.footprint = 1
        eng.pending.append(r)
    wave = eng._take_wave()
    assert [r.rid for r in wave] == [0, 1, 2]
    assert [r.rid for r in eng.pending] == [9, 7]
    # the oldest remaining request heads the next wave
    assert [r.rid for r in eng._take_wave()] == [9]
    assert [r.rid for r in eng._take_wave()] == [7]


def test_wave_respects_memory_budget_and_size():
    eng = _bare_engine()
    eng.budget, eng.max_wave = 10, 2
    reqs = [serving.Request(rid=i, n=8, b=64, a=0) for i in range(4)]
    for r, fp in zip(reqs, (4, 7, 3, 2)):
        r.footprint = fp
        eng.pending.append(r)
    wave = eng._take_wave()
    assert [r.rid for r in wave] == [0, 2] and eng.used == 7
    assert [r.rid for r in eng.pending] == [1, 3]
    assert eng._take_wave() == []          # the head (7 units) does not fit beside 7 in use


def _arena(size):
    arena = serving.DeviceArena.__new__(serving.DeviceArena)
    arena.size = size
    arena.free = [(0, size)]
    return arena


def test_reserve_sends_joiners_back_when_the_arena_is_fragmented():
    eng = _bare_engine()
    eng.arena_waits = 0
    reqs = [serving.Request(rid=i, n=8, b=64, a=0, arrival=0.1 * i) for i in range(4)]
    one = eng._wave_bytes(reqs[:1])
    two = eng._wave_bytes(reqs[:2])
    assert two > one
    for r in reqs:
        r.footprint = 1
        eng.pending.append(r)
    wave = eng._take_wave()
    assert [r.rid for r in wave] == [0, 1, 2, 3] and eng.used == 4
    # room for the first two requests' range only
    eng.arena = _arena(serving._al(two))
    wave, (off, total) = eng._reserve(wave)
    assert [r.rid for r in wave] == [0, 1] and (off, total) == (0, two)
    assert [r.rid for r in eng.pending] == [2, 3] and eng.used == 2
    # nothing left: the head waits in the queue, in arrival order
    eng.pending.append(serving.Request(rid=5, n=8, b=64, a=0, arrival=0.45))
    eng.pending[-1].footprint = 1
    head = eng._take_wave()
    assert [r.rid for r in head] == [2, 3, 5]
    assert eng._reserve(head) == ([], None)
    assert [r.rid for r in eng.pending] == [2, 3, 5] and eng.used == 2 and eng.arena_waits == 1
    eng.arena.release(off, total)
    wave, res = eng._reserve(eng._take_wave())
    assert [r.rid for r in wave] == [2, 3] and res == (0, two)


def test_mixed_request_footprint_covers_either_precision():
    req = serving.Request(rid=0, n=8, b=64, a=32, precision="mixed")
    fp64 = serving.Request(rid=1, n=8, b=64, a=32)
    ws = max(S.batch_workspace_bytes([req.spec()]), S.batch_workspace_bytes([fp64.spec()]))
    assert serving.request_footprint(req) - serving.request_io_bytes(req) - 16 * 4 * 8 * 64 * 64 == ws
