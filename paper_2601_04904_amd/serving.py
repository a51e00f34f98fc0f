"""Continuous-batching serving loop for SI+SQ requests (energy points of an
NEGF sweep arriving over time).

Requests of different (n, b, a, precision) arrive on a clock.  The engine
keeps a device-memory budget: a request is admitted when its footprint (the
library's workspace for it plus its input and output blocks) fits beside the
requests already admitted.  Admitted requests are grouped into waves; each
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
from .synth_device import gen_problem_device, gen_rhs_device


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


def request_footprint(req: Request) -> int:
    ws = S.batch_workspace_bytes([req.spec()])
    io = 16 * req.pattern_elems() * (4 + 2 * (req.nrhs - 1))   # A, B, XR, XL (+ B2, XL2)
    gen = 16 * 3 * req.n * req.b * req.b                         # transient blocks of the input generator
    return ws + io + gen


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
                 input_fn=None, router: PrecisionRouter | None = None, log=None):
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
        self.release_above = 8 << 30      # cached-but-unused torch memory released before a wave
        self.size_ratio = 8.0             # largest work ratio between requests of one wave
        self.threads = []
        self.log = log                    # callable taking a progress line (one per finished wave)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    @staticmethod
    def _device_inputs(req: Request):
        A, B = gen_problem_device(req.n, req.b, req.a, req.E, req.eta, req.seed)
        B2 = gen_rhs_device(req.n, req.b, req.a, req.seed + 1) if req.nrhs > 1 else None
        return A, B, B2

    def submit(self, req: Request):
        req.footprint = request_footprint(req)
        if req.footprint > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint / 1e9:.1f} GB, above the "
                             f"budget of {self.budget / 1e9:.1f} GB")
        with self.lock:
            self.pending.append(req)

    def _take_wave(self):
        """FIFO requests that fit the memory budget (head-of-line order kept).
        A wave finishes with its slowest request, so it stops at the first
        request whose work differs from the wave's first one by more than
        `size_ratio` either way; that request heads the next wave."""
        wave = []
        while self.pending and len(wave) < self.max_wave:
            r = self.pending[0]
            if self.used + r.footprint > self.budget:
                break
            if wave:
                ratio = r.flops() / max(wave[0].flops(), 1.0)
                if ratio > self.size_ratio or ratio < 1.0 / self.size_ratio:
                    break
            self.pending.popleft()
            self.used += r.footprint
            self.max_used = max(self.max_used, self.used)
            r.t_admit = self.now()
            wave.append(r)
        return wave

    def _run_wave(self, wave):
        torch = self.torch
        stream = torch.cuda.Stream()
        bs = None
        try:
            with torch.cuda.stream(stream):
                t_start = self.now()
                for r in wave:
                    r.t_start = t_start
                inputs = [self.input_fn(r) for r in wave]
                XR = [S.DeviceBlocks.empty(r.n, r.b, r.a) for r in wave]
                XL = [S.DeviceBlocks.empty(r.n, r.b, r.a) for r in wave]
                if self.router is not None:
                    for r in wave:
                        if r.precision == "mixed":
                            r.run_precision = self.router.choose(r.eta, r.a, r.flops())
                bs = self._batch_solver([r.spec() for r in wave], stream)
                err, fb = bs.solve([x[0] for x in inputs], [x[1] for x in inputs], XR, XL)
                errs = [[e] for e in err]
                fbs = [[f] for f in fb]
                XL2 = None
                if any(r.nrhs > 1 for r in wave):
                    XL2 = [S.DeviceBlocks.empty(r.n, r.b, r.a) if r.nrhs > 1 else None for r in wave]
                    e2, f2 = bs.selected_solve([x[2] for x in inputs], XL2)
                    for i, r in enumerate(wave):
                        if r.nrhs > 1:
                            errs[i].append(e2[i])
                            fbs[i].append(f2[i])
                bs.sync()
                t_done = self.now()
                bs.destroy()
                bs = None
                if self.router is not None:
                    for i, r in enumerate(wave):
                        if r.spec()["precision"] == S.BT_MIXED:
                            self.router.record(r.eta, r.a, bool(fbs[i][0]))
                for i, r in enumerate(wave):
                    r.t_done = t_done
                    r.err = errs[i]
                    r.fallback = fbs[i]
                    if r.keep_outputs:
                        r.outputs = (XR[i], XL[i], XL2[i] if XL2 else None)
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
            with self.cv:
                for r in wave:
                    self.used -= r.footprint
                    self.done.append(r)
                self.busy -= 1
                ndone = len(self.done)
                self.cv.notify_all()
            if self.log is not None:
                self.log(f"[serve] wave of {len(wave)} finished at {self.now():.2f} s "
                         f"({ndone} requests done)")

    def _batch_solver(self, specs, stream):
        """The library allocates its workspace outside torch's caching allocator,
        so blocks that torch has cached (the input generator's temporaries) are
        released first; an allocation failure is retried once after that."""
        torch = self.torch
        if torch.cuda.memory_reserved() - torch.cuda.memory_allocated() > self.release_above:
            torch.cuda.empty_cache()
        try:
            return S.BatchSolver(specs, stream=stream)
        except S.BTError as ex:
            if "OOM" not in str(ex):
                raise
            self.oom_retries += 1
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            return S.BatchSolver(specs, stream=stream)

    def dispatch(self) -> bool:
        """Start a wave if a worker is free and requests fit; returns True if one started."""
        with self.lock:
            if self.busy >= self.max_inflight or not self.pending:
                return False
            wave = self._take_wave()
            if not wave:
                return False
            self.busy += 1
            self.waves += 1
        th = threading.Thread(target=self._run_wave, args=(wave,))
        self.threads.append(th)
        th.start()
        return True

    def replay(self, requests, poll: float = 0.0005):
        """Play requests at their arrival times (seconds from start); returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = request_footprint(r)
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
        return summarize(self.done, wall)


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
