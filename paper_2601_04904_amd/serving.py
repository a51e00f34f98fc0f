"""Continuous-batching serving loop for SI+SQ requests (energy points of an
NEGF sweep arriving over time).

Requests of different (n, b, a, precision) arrive on a clock.  The engine
keeps a device-memory budget: a request is admitted when its footprint (the
library's workspace for it plus its input and output blocks) fits beside the
requests already admitted.  The memory itself is one device allocation made
when the replay starts (an arena the size of the budget): each wave takes one
range of it for its requests' blocks and its batch handle's workspace
(bt_si_sq_batch_create_in) and returns it when done, so no device memory is
allocated or released while waves run (either would wait for the whole
device).  Admitted requests are grouped into waves; each
wave is one batch handle (all its instances in one schedule) run by a worker
thread on its own HIP stream, so up to `max_inflight` waves overlap on the
device and requests that arrive while a wave runs are admitted as soon as a
worker and memory are free.  Factors stay resident inside the wave: a
request with a second right-hand side gets it by a selected solve on the
same factors.  Per request the engine records arrival, start and completion
times, the error estimate and whether the FP64 re-run was taken.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

from . import solver as S
from .synth_device import CHUNK, gen_problem_device, gen_rhs_device


@dataclass
class Request:
    rid: int
    n: int
    b: int
    a: int
    precision: str = "fp64"        # "fp64" or "mixed"
    E: float = 0.3
    eta: float = 1e-3
    seed: int = 0
    nrhs: int = 1
    arrival: float = 0.0
    partitions: int = 1
    flags: int = 0
    # filled in by the engine
    footprint: int = 0
    t_admit: float = -1.0
    t_start: float = -1.0
    t_done: float = -1.0
    err: list = field(default_factory=list)
    fallback: list = field(default_factory=list)
    keep_outputs: bool = False
    outputs: object = None
    run_precision: int = -1            # precision actually run (set by the router), -1: as asked

    def spec(self):
        prec = S.BT_MIXED if self.precision == "mixed" else S.BT_FP64
        if self.run_precision >= 0:
            prec = self.run_precision
        return dict(n=self.n, b=self.b, a=self.a, partitions=self.partitions,
                    precision=prec, tol=1e-4, flags=self.flags)

    def pattern_elems(self):
        n, b, a = self.n, self.b, self.a
        return n * b * b + 2 * max(n - 1, 0) * b * b + 2 * n * a * b + a * a

    def flops(self):
        """Executed real flops of this request's solves (fused solve + extra right-hand sides)."""
        ex, _ = S.flops(self.n, self.b, self.a, self.partitions)
        return ex * (1.0 + 0.6 * (self.nrhs - 1))


ALIGN = 256


def _al(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


def field_bytes(n: int, b: int, a: int):
    """Bytes of the six fields of one matrix's blocks (complex128)."""
    m = max(n - 1, 0)
    return [16 * n * b * b, 16 * m * b * b, 16 * m * b * b, 16 * n * b * a, 16 * n * a * b, 16 * a * a]


def blocks_bytes(n: int, b: int, a: int) -> int:
    return sum(_al(x) for x in field_bytes(n, b, a))


def request_io_bytes(req: Request) -> int:
    """A, B, XR, XL (+ B2, XL2 for a second right-hand side)."""
    return (4 + 2 * (req.nrhs - 1)) * blocks_bytes(req.n, req.b, req.a)


def request_footprint(req: Request) -> int:
    """Device bytes a request may hold: the workspace of either precision it
    may be routed to, its blocks, and the generator's transient blocks."""
    spec = req.spec()
    ws = S.batch_workspace_bytes([spec])
    if req.precision == "mixed":
        ws = max(ws, S.batch_workspace_bytes([dict(spec, precision=S.BT_FP64)]))
    gen = 16 * 4 * min(req.n, CHUNK) * req.b * req.b             # transient blocks of the input generator
    return ws + request_io_bytes(req) + gen


class DeviceArena:
    """One device allocation handed out in ranges: first fit, and a released
    range is merged with free neighbours.  Offsets and sizes are multiples
    of 256 bytes.  Not thread-safe (the engine calls it under its lock)."""

    def __init__(self, torch, nbytes: int):
        self.buf = torch.empty(_al(nbytes), dtype=torch.uint8, device="cuda")
        self.size = self.buf.numel()
        self.free = [(0, self.size)]          # sorted (offset, size)

    def alloc(self, nbytes: int):
        n = _al(nbytes)
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, sz - n)
                return o
        return None

    def release(self, off: int, nbytes: int):
        n = _al(nbytes)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, sz in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((o, sz))
        self.free = merged


def carve_blocks(buf, off: int, n: int, b: int, a: int):
    """DeviceBlocks viewing buf[off:], fields one after another (256-aligned);
    returns the blocks and the offset after them."""
    import torch
    shapes = [(n, b, b), (max(n - 1, 0), b, b), (max(n - 1, 0), b, b), (n, b, a), (n, a, b), (a, a)]
    views = []
    for shp, nb in zip(shapes, field_bytes(n, b, a)):
        views.append(buf[off:off + nb].view(torch.complex128).view(shp))
        off += _al(nb)
    return S.DeviceBlocks(*views), off


class PrecisionRouter:
    """Routes requests that ask for the mixed path.

    The mixed path runs its bulk products in complex64 and re-runs an instance
    in FP64 when its error estimate exceeds the tolerance, so on inputs whose
    conditioning amplifies FP32 rounding past the tolerance it costs a mixed
    run plus an FP64 run.  The conditioning of A = (E + i eta) I - H - Sigma is
    governed mostly by the broadening eta (||A^-1|| <= 1/eta when the
    self-energies are absorbing), so requests are classed by the decade of
    eta and by whether there is an arrowhead.  The router keeps, per class, a
    running fallback rate of the mixed runs it has seen; once that rate is
    above `threshold` (after `probe` runs), further mixed requests of the class
    go straight to FP64, except every `reprobe`-th one, which still tries the
    mixed path so the rate can recover.
    """

    def __init__(self, threshold: float = 0.5, probe: int = 2, reprobe: int = 16, decay: float = 0.8,
                 probe_max_flops: float = float("inf")):
        self.threshold, self.probe, self.reprobe, self.decay = threshold, probe, reprobe, decay
        self.probe_max_flops = probe_max_flops
        self.rate = {}
        self.seen = {}
        self.outcomes = {}
        self.pending = {}
        self.routed = 0
        self.lock = threading.Lock()

    @staticmethod
    def key(eta: float, a: int):
        decade = int(math.floor(math.log10(eta))) if eta > 0 else -99
        return (decade, a > 0)

    def choose(self, eta: float, a: int, flops: float = 0.0) -> int:
        """Precision to run a mixed request with.  Probes (runs whose only use
        is to learn the class's fallback rate) are spent on requests of at most
        probe_max_flops; a costlier request of a class without enough outcomes
        runs in FP64."""
        k = self.key(eta, a)
        with self.lock:
            n = self.seen.get(k, 0)
            known = self.outcomes.get(k, 0)
            pending = self.pending.get(k, 0)
            cheap = flops <= self.probe_max_flops
            if known < self.probe:
                # no more probes in flight than still needed
                if not cheap or known + pending >= self.probe:
                    self.routed += 1
                    return S.BT_FP64
                self.pending[k] = pending + 1
                self.seen[k] = n + 1
                return S.BT_MIXED
            self.seen[k] = n + 1
            if self.rate.get(k, 0.0) <= self.threshold or (cheap and n % self.reprobe == 0):
                return S.BT_MIXED
            self.routed += 1
            return S.BT_FP64

    def record(self, eta: float, a: int, fell_back: bool):
        k = self.key(eta, a)
        with self.lock:
            self.outcomes[k] = self.outcomes.get(k, 0) + 1
            self.pending[k] = max(0, self.pending.get(k, 0) - 1)
            r = self.rate.get(k, float(fell_back))
            self.rate[k] = self.decay * r + (1.0 - self.decay) * float(fell_back)


class ServingEngine:
    def __init__(self, budget_bytes: int, max_inflight: int = 2, max_wave: int = 16,
                 input_fn=None, router: PrecisionRouter | None = None, log=None, use_arena: bool = True):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.used = 0
        self.max_inflight = max_inflight
        self.max_wave = max_wave
        self.pending = deque()
        self.done = []
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.busy = 0
        self.errors = []
        self.t0 = None
        self.input_fn = input_fn or self._device_inputs
        self.waves = 0
        self.max_used = 0
        self.router = router
        self.oom_retries = 0
        self.size_ratio = 4.0             # largest work ratio between requests of one wave
        self.chain_ratio = 1.5            # largest ratio of block counts in one wave
        self.threads = []
        self.log = log                    # callable taking a progress line (one per finished wave)
        self.use_arena = use_arena
        self.arena = None                 # DeviceArena of the budget, made when the replay starts
        self.arena_waits = 0              # times the queue head waited for an arena range

    def now(self) -> float:
        return time.perf_counter() - self.t0

    @staticmethod
    def _device_inputs(req: Request, out=None):
        """(A, B, B2) of a request, into out = (A, B, B2) if given."""
        oA, oB, oB2 = out if out is not None else (None, None, None)
        A, B = gen_problem_device(req.n, req.b, req.a, req.E, req.eta, req.seed, out=(oA, oB))
        B2 = gen_rhs_device(req.n, req.b, req.a, req.seed + 1, out=oB2) if req.nrhs > 1 else None
        return A, B, B2

    def submit(self, req: Request):
        req.footprint = request_footprint(req)
        if req.footprint > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint / 1e9:.1f} GB, above the "
                             f"budget of {self.budget / 1e9:.1f} GB")
        with self.lock:
            self.pending.append(req)

    def _compatible(self, head, r) -> bool:
        """Requests that share a wave well: similar work (within size_ratio)
        and similar chains of block inverses (block counts within
        chain_ratio), so that the instances' inverses and products share the
        schedule's launches level by level and none waits long for the
        slowest."""
        ratio = r.flops() / max(head.flops(), 1.0)
        if ratio > self.size_ratio or ratio < 1.0 / self.size_ratio:
            return False
        chain = r.n / max(head.n, 1)
        return 1.0 / self.chain_ratio <= chain <= self.chain_ratio

    def _take_wave(self):
        """The oldest pending request heads the wave (so no request is passed
        over for good); every later pending request compatible with it joins,
        in arrival order, while the wave has room and the memory budget
        allows.  The others keep their places for the next waves."""
        wave = []
        if not self.pending:
            return wave
        head = self.pending[0]
        if self.used + head.footprint > self.budget:
            return wave
        keep = deque()
        while self.pending:
            r = self.pending.popleft()
            fits = len(wave) < self.max_wave and self.used + r.footprint <= self.budget
            if fits and (not wave or self._compatible(head, r)):
                self.used += r.footprint
                self.max_used = max(self.max_used, self.used)
                r.t_admit = self.now()
                wave.append(r)
            else:
                keep.append(r)
        self.pending = keep
        return wave

    def _wave_bytes(self, wave) -> int:
        """Bytes of the wave's one range: every request's blocks, then the
        batch handle's workspace."""
        specs = [r.spec() for r in wave]
        return sum(request_io_bytes(r) for r in wave) + _al(S.batch_workspace_bytes(specs))

    def _reserve(self, wave):
        """Called under the lock.  Takes the wave's range from the arena; when
        the arena (fragmented by the waves in flight) has no such range, the
        latest joiners go back to the queue one by one until the rest fits.
        Returns (wave, (offset, bytes)), or ([], None) with every request
        back in the queue when not even the head fits: the wave then waits
        for a range to be released instead of allocating outside the arena."""
        back = []
        while wave:
            total = self._wave_bytes(wave)
            off = self.arena.alloc(total)
            if off is not None:
                break
            back.append(wave.pop())
        if back:
            for r in back:
                self.used -= r.footprint
            self.pending = deque(sorted(list(self.pending) + back, key=lambda r: (r.arrival, r.rid)))
        if not wave:
            self.arena_waits += 1
            return [], None
        return wave, (off, total)

    def _wave_memory(self, wave, reservation):
        """(buffer, release) of the wave: its arena range, or with no arena an
        allocation of its own."""
        if reservation is not None:
            off, total = reservation

            def release():
                with self.lock:
                    self.arena.release(off, total)
            return self.arena.buf[off:off + _al(total)], release
        buf = self.torch.empty(_al(self._wave_bytes(wave)), dtype=self.torch.uint8, device="cuda")
        return buf, (lambda: None)

    def _run_wave(self, wave, reservation=None):
        torch = self.torch
        stream = torch.cuda.Stream()
        bs = None
        phases = None
        release = None
        try:
            with torch.cuda.stream(stream):
                t_start = self.now()
                for r in wave:
                    r.t_start = t_start
                specs = [r.spec() for r in wave]
                buf, release = self._wave_memory(wave, reservation)
                off = 0
                inputs, XR, XL, XL2s = [], [], [], []
                for r in wave:
                    A, off = carve_blocks(buf, off, r.n, r.b, r.a)
                    B, off = carve_blocks(buf, off, r.n, r.b, r.a)
                    xr, off = carve_blocks(buf, off, r.n, r.b, r.a)
                    xl, off = carve_blocks(buf, off, r.n, r.b, r.a)
                    B2 = xl2 = None
                    if r.nrhs > 1:
                        B2, off = carve_blocks(buf, off, r.n, r.b, r.a)
                        xl2, off = carve_blocks(buf, off, r.n, r.b, r.a)
                    inputs.append(self.input_fn(r, (A, B, B2)))
                    XR.append(xr)
                    XL.append(xl)
                    XL2s.append(xl2)
                ws = buf[off:]
                stream.synchronize()
                t_inputs = self.now()
                bs = S.BatchSolver(specs, stream=stream, workspace=ws)
                t_created = self.now()
                err, fb = bs.solve([x[0] for x in inputs], [x[1] for x in inputs], XR, XL)
                errs = [[e] for e in err]
                fbs = [[f] for f in fb]
                XL2 = None
                if any(r.nrhs > 1 for r in wave):
                    XL2 = XL2s
                    e2, f2 = bs.selected_solve([x[2] for x in inputs], XL2)
                    for i, r in enumerate(wave):
                        if r.nrhs > 1:
                            errs[i].append(e2[i])
                            fbs[i].append(f2[i])
                bs.sync()
                t_done = self.now()
                bs.destroy()
                bs = None
                phases = (t_inputs - t_start, t_created - t_inputs, t_done - t_created, self.now() - t_done)
                if self.router is not None:
                    with self.lock:
                        for i, r in enumerate(wave):
                            if r.spec()["precision"] == S.BT_MIXED:
                                self.router.record(r.eta, r.a, bool(fbs[i][0]))
                for i, r in enumerate(wave):
                    r.t_done = t_done
                    r.err = errs[i]
                    r.fallback = fbs[i]
                    if r.keep_outputs:        # copies: the wave's range is reused afterwards
                        r.outputs = tuple(_copy_blocks(x) for x in (XR[i], XL[i], XL2[i] if XL2 else None))
                stream.synchronize()
                del inputs
        except Exception as ex:  # keep the loop alive; report at the end
            self.errors.append(repr(ex))
            for r in wave:
                r.failed = True
        finally:
            if bs is not None:
                try:
                    bs.destroy()
                except Exception as ex:
                    self.errors.append(repr(ex))
            if release is not None:
                stream.synchronize()      # nothing of the wave may still use its range
                release()
            with self.cv:
                for r in wave:
                    self.used -= r.footprint
                    self.done.append(r)
                self.busy -= 1
                ndone = len(self.done)
                self.cv.notify_all()
            if self.log is not None:
                ph = phases
                detail = (f": inputs {ph[0]:.3f} s, create {ph[1]:.3f} s, solves {ph[2]:.3f} s, "
                          f"destroy {ph[3]:.3f} s, {sum(r.flops() for r in wave) / 1e12:.1f} TFLOP"
                          if ph else "")
                self.log(f"[serve] wave of {len(wave)} finished at {self.now():.2f} s "
                         f"({ndone} requests done){detail}")

    def dispatch(self) -> bool:
        """Start a wave if a worker is free and requests fit; returns True if one started."""
        with self.lock:
            if self.busy >= self.max_inflight or not self.pending:
                return False
            wave = self._take_wave()
            if not wave:
                return False
            if self.router is not None:     # the precision fixes the workspace size
                for r in wave:
                    if r.precision == "mixed":
                        r.run_precision = self.router.choose(r.eta, r.a, r.flops())
            reservation = None
            if self.arena is not None:
                wave, reservation = self._reserve(wave)
                if not wave:
                    return False
            self.busy += 1
            self.waves += 1
        th = threading.Thread(target=self._run_wave, args=(wave, reservation))
        self.threads.append(th)
        th.start()
        return True

    def replay(self, requests, poll: float = 0.0005):
        """Play requests at their arrival times (seconds from start); returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = request_footprint(r)
        if self.use_arena and self.arena is None:
            self.arena = DeviceArena(self.torch, self.budget)
        self.t0 = time.perf_counter()
        i = 0
        total = len(reqs)
        while True:
            t = self.now()
            while i < total and reqs[i].arrival <= t:
                self.submit(reqs[i])
                i += 1
            while self.dispatch():
                pass
            with self.cv:
                if len(self.done) == total:
                    break
                self.cv.wait(timeout=poll)
        wall = self.now()
        for th in self.threads:          # no worker outlives the replay
            th.join()
        self.threads = []
        self.arena = None                # back to torch's cache for the next engine
        return summarize(self.done, wall)


def _copy_blocks(X):
    if X is None:
        return None
    return S.DeviceBlocks(*(getattr(X, f).clone() for f in S.FIELDS))


def summarize(done, wall):
    lat = sorted(r.t_done - r.arrival for r in done if r.t_done >= 0 and not getattr(r, "failed", False))

    def pct(q):
        if not lat:
            return None
        k = min(len(lat) - 1, max(0, int(round(q / 100.0 * (len(lat) - 1)))))
        return lat[k]

    ok = [r for r in done if not getattr(r, "failed", False)]
    solves = sum(r.nrhs for r in ok)
    return dict(requests=len(done), failed=len(done) - len(ok), solves=solves, wall_s=wall,
                solves_per_s=solves / wall if wall > 0 else 0.0,
                requests_per_s=len(done) / wall if wall > 0 else 0.0,
                p50_s=pct(50), p99_s=pct(99),
                max_err=max((max(r.err) for r in done if r.err), default=0.0),
                fallbacks=sum(any(r.fallback) for r in done))


def auto_partitions(n: int) -> int:
    """Partitions for a served request: two (the first half eliminated
    top-down, the second bottom-up, Sec. III-B with P = 2) halve the
    sequential chain of block inverses at almost no extra work (no middle
    partitions, no fill-in); very short chains stay sequential."""
    return 2 if n >= 8 else 1


def requests_from_trace(trace, partitions=1):
    """Requests of a trace; partitions is a count or a function of n."""
    out = []
    for k, t in enumerate(trace):
        P = partitions(t["n"]) if callable(partitions) else partitions
        out.append(Request(rid=k, n=t["n"], b=t["b"], a=t["a"], precision=t["precision"], E=t["E"],
                           eta=t["eta"], seed=t["seed"], nrhs=t["nrhs"], arrival=t["arrival"],
                           partitions=P))
    return out
