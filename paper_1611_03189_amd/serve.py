"""Request loop: a stream of SPD systems A x = b solved on one GPU with continuous batching.

Requests (a matrix with 1..8 right-hand sides and an arrival time) are analysed as they
arrive (host symbolic analysis, which also bounds the device memory the request can need).
A fixed set of slots, each a host thread with its own HIP stream, take the oldest analysed
request whose bound fits the free budget, run the factorization and one batched solve of
all its right-hand sides through the C ABI in the slot's arena (the factors stay resident
for all of them), then destroy the plan. A slot keeps one arena for a run and grows it when
a request's bound exceeds it. Work of different slots overlaps on the device; the library
calls release the interpreter lock, so the slot and analysis threads run concurrently.

Admission: a request is admitted when its arena bound (hsolve_analyze) fits in the budget
left by the running ones, or when nothing runs; the budget is charged with exactly that
bound while the request runs, and the same amount is returned when it ends. (Idle slots
keep their arenas; these are at most the largest bound each slot has served.)

Every result depends only on its own request: the kernels are deterministic and a plan
shares no device state with another, so a request gives the same bits alone and in the
mix.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hsolve as H

# device memory kept free for the HIP runtime's own allocations (queue scratch, internal buffers)
RUNTIME_HEADROOM = 4 << 30


@dataclass
class Request:
    rid: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    coords: np.ndarray | None
    b: np.ndarray                 # n x nrhs (host)
    leaf: int = 16
    eps: float = 1e-2
    variant: str = "gc"
    arrival: float = 0.0          # seconds after the start of the run

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1


@dataclass
class Result:
    rid: int
    x: np.ndarray
    iterations: int
    converged: bool
    rel_residual: float
    device_bytes: int
    t_arrival: float
    t_start: float
    t_done: float
    slot: int

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class RunSummary:
    results: list[Result] = field(default_factory=list)
    makespan: float = 0.0

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.results]) * 1e3
        nrhs = sum(r.x.shape[1] for r in self.results)
        return {
            "requests": len(self.results),
            "rhs": int(nrhs),
            "makespan_s": round(self.makespan, 4),
            "requests_per_s": round(len(self.results) / self.makespan, 3) if self.makespan > 0 else None,
            "solves_per_s": round(nrhs / self.makespan, 3) if self.makespan > 0 else None,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
            "all_converged": all(r.converged for r in self.results),
        }


class RequestLoop:
    """Continuous-batching request loop over `slots` concurrent HIP streams. The plans factor
    their pivot blocks and both compression chains in order on their slot's stream
    (overlap_pivots=False): with several requests in flight the GPU is already shared, and more
    streams per plan only add queue contention (measured on the 512-request stream with the
    pivot and compression streams: 26-30% fewer solves/s). `analysers` host threads run the
    symbolic analyses as requests arrive."""

    def __init__(self, slots: int = 4, memory_budget: int | None = None, overlap_pivots: bool = False,
                 analysers: int = 2, solver_factory=None, mixed: bool = False):
        self.slots = slots
        self.mixed = mixed          # FP32 factorization inside FP64 flexible PCG
        self.overlap_pivots = overlap_pivots
        self.analysers = max(1, analysers)
        self._factory = solver_factory
        if memory_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            memory_budget = int(0.8 * free)
        self.budget = memory_budget
        self.streams = None
        self._arenas = {}           # per slot stream, for the duration of a run

    def _solver(self, r: Request):
        if self._factory is not None:
            return self._factory(r)
        kw = dict(factor_prec=32, krylov="fpcg") if self.mixed else {}
        return H.HSolver(r.row_ptr, r.col_idx, coords=r.coords, leaf=r.leaf, eps=r.eps, variant=r.variant,
                         tol=1e-10, overlap_pivots=self.overlap_pivots, max_nrhs=max(1, r.b.shape[1]), **kw)

    def _execute(self, S, r: Request, stream):
        """Factor and solve one admitted request on `stream`; returns (x, stats, device bytes)."""
        import torch
        with torch.cuda.stream(stream):
            S.set_stream(stream)
            need = max(S.arena_bound, 256)
            # One arena per slot, grown when a request needs more: a slot's requests run one
            # after another on its stream, so its arena is free again when the next one starts.
            # (An arena per request filled PyTorch's cache with arenas of every size; releasing
            # that cache synchronises the device.) Unless a new arena fits with
            # RUNTIME_HEADROOM left free, the unused cache is released first: a full device
            # leaves the HIP runtime unable to allocate a queue's scratch memory.
            arena = self._arenas.get(stream)
            if arena is None or arena.numel() < need:
                self._arenas.pop(stream, None)
                arena = None
                free, _ = torch.cuda.mem_get_info()
                if free < need + RUNTIME_HEADROOM:
                    torch.cuda.empty_cache()
                arena = torch.empty(need, dtype=torch.uint8, device="cuda")
                self._arenas[stream] = arena
            B = torch.from_numpy(np.ascontiguousarray(r.b)).to("cuda")
            stream.synchronize()
            S.factor(r.values, arena=arena)          # host values: copied into the arena
            X, st = S.solve(B)
            x = X.cpu().numpy()
            dev = int(S.stats()["device_bytes"])
        return x, st, dev

    def run(self, requests: list[Request], realtime: bool = True) -> RunSummary:
        """Serve `requests`; with realtime, a request becomes visible at its arrival time."""
        if self.streams is None and self._factory is None:
            import torch
            self.streams = [torch.cuda.Stream() for _ in range(self.slots)]
        order = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: list = []                 # analysed: (request, solver, bound)
        lock = threading.Condition()
        state = {"used": 0, "running": 0, "analysed": 0, "error": None, "peak_used": 0}
        summary = RunSummary()
        total = len(requests)
        t0 = time.perf_counter()

        def now() -> float:
            return time.perf_counter() - t0

        def fail(e):
            with lock:
                if state["error"] is None:
                    state["error"] = e
                lock.notify_all()

        def analyser():
            while True:
                with lock:
                    if state["error"] is not None or not order:
                        return
                    r = order.popleft()
                if realtime:
                    delay = r.arrival - now()
                    if delay > 0:
                        time.sleep(delay)
                try:
                    S = self._solver(r)
                except Exception as e:           # surfaced to the caller after the run
                    fail(e)
                    return
                with lock:
                    waiting.append((r, S, int(S.arena_bound)))
                    waiting.sort(key=lambda w: (w[0].arrival, w[0].rid))
                    state["analysed"] += 1
                    lock.notify_all()

        def take():
            """The oldest analysed request whose arena bound fits the free budget (or any, when
            nothing runs), with the amount charged for it."""
            with lock:
                while True:
                    if state["error"] is not None:
                        return None
                    for i, (r, S, need) in enumerate(waiting):
                        if state["used"] + need <= self.budget or state["running"] == 0:
                            del waiting[i]
                            state["used"] += need
                            state["peak_used"] = max(state["peak_used"], state["used"])
                            state["running"] += 1
                            return r, S, need
                    if state["analysed"] == total and not waiting:
                        return None
                    lock.wait(timeout=0.05)

        def worker(slot: int):
            if self.streams is not None:
                import torch
                torch.cuda.set_device(0)
            stream = self.streams[slot] if self.streams is not None else None
            while True:
                got = take()
                if got is None:
                    return
                r, S, charged = got
                t_start = now()
                try:
                    x, st, dev = self._execute(S, r, stream)
                    t_done = now()
                except Exception as e:           # surfaced to the caller after the run
                    with lock:
                        state["used"] -= charged
                        state["running"] -= 1
                    fail(e)
                    return
                finally:
                    S.close()
                with lock:
                    state["used"] -= charged
                    state["running"] -= 1
                    summary.results.append(Result(r.rid, x.reshape(r.n, -1), st["iterations"], st["converged"],
                                                  st["rel_residual"], dev, r.arrival, t_start, t_done, slot))
                    lock.notify_all()

        threads = [threading.Thread(target=analyser, daemon=True) for _ in range(self.analysers)]
        threads += [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(self.slots)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        for _, S, _ in waiting:
            S.close()
        self._arenas = {}
        if state["error"] is not None:
            raise state["error"]
        summary.makespan = now()
        summary.results.sort(key=lambda r: r.rid)
        self.last_peak_used = state["peak_used"]
        self.last_final_used = state["used"]
        return summary


def requests_from_stream(specs: list[dict]) -> list[Request]:
    """Materialise the seeded synthetic systems of a serving stream."""
    from . import problems as pb
    out = []
    for s in specs:
        p, b = pb.serving_problem(s)
        out.append(Request(s["rid"], p.row_ptr, p.col_idx, p.values, p.coords, b, leaf=s["leaf"],
                           eps=s["eps"], arrival=s["arrival"]))
    return out
