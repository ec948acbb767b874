"""Continuous batching of independent transport problems on one GPU.

Requests arrive over time.  A request is admitted as soon as a slot is free
and its HBM reservation fits in what the running requests leave of the budget
(first waiting request that fits, in arrival order).  The reservation starts
as a bound from the request's size (points, ordinates) and is replaced by the
exact bytes -- the problem's device inputs plus its four stage workspaces,
from the library's workspace queries -- as soon as they are known (after the
assembly, before the solve's workspace is taken), which usually returns part
of the bound to the pool.  Every admitted request runs the library's four
stage calls (geometry, integration, assembly, one steady solve) on its own HIP
stream from its own host thread, so that the kernels of several problems
overlap on the device while each problem's Krylov state stays resident until
it completes.  All device memory comes from torch's caching allocator (the
workspaces are torch tensors), so a finished request's memory is reused by
the next without a device-wide free.

Control flow only: every numerical step runs in libmlpg.so.  Latency is
measured from arrival to the result being ready on the host.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from typing import Callable, List, Optional

import numpy as np
import torch

from . import mlpg as api
from .problem import GpuProblem


def hbm_estimate(n: int, n_ord: int, precision: int, nnz_per_row: float = 52.0, restart: int = 30) -> int:
    """Bytes a 2D linear-RK problem holds on the device (blocks, streams,
    pattern, Krylov bases and vectors, state), with a quarter to spare."""
    nnz = nnz_per_row * n
    per_nnz = 8 * 10 + 8 * 12 + 4 * 3 + (4 * 6 if precision == api.MLPG_MIXED else 0)
    nm = float(n) * n_ord
    krylov = (restart + 6) * 8 * nm
    if precision == api.MLPG_MIXED:
        krylov += (restart + 6) * 4 * nm + 4 * 8 * nm
    state = 8 * 8 * nm
    return int(1.25 * (nnz * per_nnz + krylov + state) + (64 << 20))


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    phi: Optional[np.ndarray] = None
    point: Optional[np.ndarray] = None
    info: Optional[dict] = None
    error: Optional[str] = None
    reserved: int = 0          # bytes reserved at admission (the bound)
    exact_bytes: int = 0       # device bytes the problem holds, from the workspace queries

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Admits requests by HBM budget into at most ``slots`` concurrent problems."""

    def __init__(self, slots: int = 4, budget_bytes: Optional[int] = None,
                 precision: int = api.MLPG_MIXED, opts=None):
        api.lib()
        self.slots = slots
        if budget_bytes is None:
            free, _total = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.precision = precision
        self.opts = opts

    def _stream(self):
        """The HIP stream of one slot."""
        return torch.cuda.Stream()

    def _solve(self, build: Callable, spec, stream: torch.cuda.Stream, true_up: Optional[Callable] = None):
        x, R, dx, om, w, sig_t, sig_s, q = build(spec)
        with torch.cuda.stream(stream):
            P = GpuProblem(x, R, (0.0, 0.0), (1.0, 1.0))
            try:
                P.integrate(1)
                P.assemble(om, w, [sig_t], [sig_s], 0.0, dx, precision=self.precision)
                if true_up is not None:
                    true_up(P.device_bytes(self.opts))
                qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda", non_blocking=False)
                phi, pv, _, info = P.step(qd, None, self.opts, want_psi=False)
                phi_h, pv_h = phi.cpu().numpy(), pv.cpu().numpy()
                stream.synchronize()
            finally:
                P.close()
        return phi_h, pv_h, info

    def run(self, specs: List, build: Callable, realtime: bool = True, keep_fields: bool = True,
            on_done: Optional[Callable] = None) -> List[Result]:
        """Serve ``specs`` (objects with rid, arrival, side and n_ord); ``build(spec)``
        returns (x, R, dx, omega, w, sigma_t, sigma_s, q).  With ``realtime``, requests
        become visible at their arrival times; otherwise all are waiting at once.
        ``on_done(result, n_done)`` is called (under the server's lock, from the worker
        thread) as each request completes."""
        lock = threading.Condition()
        waiting: list = []
        state = {"bytes": 0, "running": 0}
        results: List[Result] = []
        order = sorted(specs, key=lambda s: s.arrival)
        streams = [self._stream() for _ in range(self.slots)]
        free_streams = list(range(self.slots))
        threads = []
        t0 = time.perf_counter()

        def worker(spec, sidx, need, t_adm):
            res = Result(spec.rid, spec.arrival, t_adm, 0.0, reserved=need)
            held = [need]

            def true_up(exact):
                # the exact footprint replaces the bound in the budget
                with lock:
                    state["bytes"] += int(exact) - held[0]
                    held[0] = int(exact)
                    res.exact_bytes = int(exact)
                    lock.notify_all()

            try:
                phi, pv, info = self._solve(build, spec, streams[sidx], true_up)
                if keep_fields:
                    res.phi, res.point = phi, pv
                res.info = info
            except Exception as e:   # reported per request; the stream goes on
                res.error = f"{type(e).__name__}: {e}"
            res.done = time.perf_counter() - t0
            with lock:
                results.append(res)
                if on_done is not None:
                    on_done(res, len(results))
                state["bytes"] -= held[0]
                state["running"] -= 1
                free_streams.append(sidx)
                lock.notify_all()

        k = 0
        with lock:
            while k < len(order) or waiting or state["running"]:
                now = time.perf_counter() - t0
                while k < len(order) and (not realtime or order[k].arrival <= now):
                    waiting.append(order[k])
                    k += 1
                # admit, in arrival order, every waiting request that fits
                i = 0
                while i < len(waiting) and state["running"] < self.slots:
                    s = waiting[i]
                    need = hbm_estimate(s.side * s.side, s.n_ord, self.precision)
                    if state["bytes"] + need <= self.budget or state["running"] == 0:
                        waiting.pop(i)
                        state["bytes"] += need
                        state["running"] += 1
                        sidx = free_streams.pop()
                        th = threading.Thread(target=worker, args=(s, sidx, need, time.perf_counter() - t0),
                                              daemon=True)
                        threads.append(th)
                        th.start()
                    else:
                        i += 1
                if k < len(order) and realtime:
                    lock.wait(timeout=max(order[k].arrival - (time.perf_counter() - t0), 0.0005))
                elif waiting or state["running"]:
                    lock.wait(timeout=0.5)
        for th in threads:
            th.join()
        return sorted(results, key=lambda r: r.rid)


def latency_summary(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results if r.error is None])
    span = max(r.done for r in results) - min(r.arrival for r in results)
    exact = [r for r in results if r.exact_bytes > 0]
    return {"requests": len(results), "failed": sum(r.error is not None for r in results),
            "exact_over_reserved": (float(np.mean([r.exact_bytes / r.reserved for r in exact]))
                                    if exact else None),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "throughput_req_s": len(results) / span if span > 0 else None}
