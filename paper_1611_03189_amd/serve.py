"""Request loop: a stream of SPD systems A x = b solved on one GPU with continuous batching.

Requests (a matrix with 1..8 right-hand sides and an arrival time) enter a queue as they
arrive. A fixed set of slots, each a host thread with its own HIP stream, take the oldest
waiting request whose device-memory estimate fits the free budget, run the symbolic
analysis, the factorization and one batched PCG solve of all its right-hand sides through
the C ABI (the factors stay resident for all of them), then destroy the plan and return
its memory. Work of different slots overlaps on the device; the library calls release the
interpreter lock, so the slot threads run concurrently.

Admission: a request's device footprint is estimated as bytes_per_unknown * n, with the
ratio taken from the requests already finished (the largest ratio seen, times a margin;
an initial guess before any has finished). A request is admitted when its estimate fits
in the budget left by the running ones; the budget is charged with the measured footprint
once the factorization is done.

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
    their pivot blocks in order on their slot's stream (overlap_pivots=False): with several
    requests in flight the GPU is already shared, and a second stream per plan only adds
    queue contention (measured: about 10% fewer solves/s with it)."""

    def __init__(self, slots: int = 4, memory_budget: int | None = None,
                 bytes_per_unknown: float = 16e3, margin: float = 1.25, overlap_pivots: bool = False):
        import torch
        self.slots = slots
        self.overlap_pivots = overlap_pivots
        if memory_budget is None:
            free, _ = torch.cuda.mem_get_info()
            memory_budget = int(0.8 * free)
        self.budget = memory_budget
        self.bpu = bytes_per_unknown
        self.margin = margin
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def _estimate(self, req: Request) -> int:
        return int(self.bpu * self.margin * req.n)

    def run(self, requests: list[Request], realtime: bool = True) -> RunSummary:
        """Serve `requests`; with realtime, a request becomes visible at its arrival time."""
        import torch
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: deque[Request] = deque()
        lock = threading.Condition()
        state = {"used": 0, "running": 0, "error": None}
        summary = RunSummary()
        t0 = time.perf_counter()

        def now() -> float:
            return time.perf_counter() - t0

        def take(slot: int) -> Request | None:
            with lock:
                while True:
                    if state["error"] is not None:
                        return None
                    while pending and (not realtime or pending[0].arrival <= now()):
                        waiting.append(pending.popleft())
                    for i, r in enumerate(waiting):
                        need = self._estimate(r)
                        if state["used"] + need <= self.budget or state["running"] == 0:
                            del waiting[i]
                            state["used"] += need
                            state["running"] += 1
                            return r
                    if not pending and not waiting:
                        return None
                    timeout = None
                    if pending and realtime:
                        timeout = max(0.0, pending[0].arrival - now())
                    lock.wait(timeout=timeout if timeout is not None else 0.05)

        def worker(slot: int):
            torch.cuda.set_device(0)
            stream = self.streams[slot]
            while True:
                r = take(slot)
                if r is None:
                    return
                est = self._estimate(r)
                t_start = now()
                try:
                    with torch.cuda.stream(stream):
                        S = H.HSolver(r.row_ptr, r.col_idx, coords=r.coords, leaf=r.leaf, eps=r.eps,
                                      variant=r.variant, tol=1e-10, stream=stream,
                                      overlap_pivots=self.overlap_pivots)
                        vals = torch.from_numpy(r.values).to("cuda", non_blocking=False)
                        B = torch.from_numpy(np.ascontiguousarray(r.b)).to("cuda")
                        stream.synchronize()
                        S.factor(vals)
                        X, st = S.solve(B)
                        x = X.cpu().numpy()
                        dev = int(S.stats()["device_bytes"])
                        S.close()
                    t_done = now()
                except Exception as e:          # surfaced to the caller after the run
                    with lock:
                        state["error"] = e
                        state["used"] -= est
                        state["running"] -= 1
                        lock.notify_all()
                    return
                with lock:
                    state["used"] -= est
                    state["running"] -= 1
                    self.bpu = max(self.bpu, dev / max(1, r.n))
                    summary.results.append(Result(r.rid, x.reshape(r.n, -1), st["iterations"], st["converged"],
                                                  st["rel_residual"], dev, r.arrival, t_start, t_done, slot))
                    lock.notify_all()

        threads = [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(self.slots)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        if state["error"] is not None:
            raise state["error"]
        summary.makespan = now()
        summary.results.sort(key=lambda r: r.rid)
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
