"""Serving loop for least-squares requests on one GPU (continuous batching).

Requests (A, B) arrive over time, each asking for min ||A X - B|| with FP64
answers.  The loop admits an arrived request as soon as a slot (a HIP stream)
is free and the device memory it needs fits in the HBM budget, so the work of
requests that arrive while others run overlaps on the GPU; every admitted
request runs on its own stream with a worker count sized to the problem,
either the mixed-precision solve ``tqr_solve_ls_mixed`` (FP32-update factor,
then FP64 CGLS with the factor's R as preconditioner until the backward-error
estimate converges; the default) or the FP64 ``tqr_solve_ls_ex`` (factor,
Q^T B, back substitution).  Latency is completion time minus arrival time on
the host's monotonic clock, queueing included.

The admission and bookkeeping core (``Scheduler``) does not touch the GPU;
``GpuExecutor`` is the HIP side.  The factorisation is bitwise independent of
the schedule, so a request's answer is the same alone and in the mix.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable

import numpy as np


# ---------------------------------------------------------------------------
# Problem-size rules
# ---------------------------------------------------------------------------

def tiling_for(m: int, n: int) -> tuple[int, int]:
    """Tile size and inner block for an m x n solve: the largest tile whose
    grid still has enough tiles for the device (a size-bucket table)."""
    if n >= 2048:
        return 256, 16
    if n >= 512:
        return 128, 16
    if n >= 64:
        return 64, 16
    return 32, 16


def workers_for(m: int, n: int, tile_b: int, device_slots: int) -> int:
    """Persistent workgroups for one solve: about one per tile-column strip
    of the trailing matrix (more would only wait), at most the device."""
    p, q = -(-m // tile_b), -(-n // tile_b)
    strips = max(1, tile_b // 64)
    return int(max(4, min(device_slots, p * q * strips)))


def footprint_bytes(m: int, n: int, nrhs: int, tile_b: int, inner_ib: int, work_bytes: int, t_elems: int) -> int:
    """Device bytes one request holds while in flight: A, B, X, T, the
    workspace and the info, status and statistics words."""
    return 8 * (m * n + m * nrhs + n * nrhs + t_elems) + work_bytes + 256 + 16 * nrhs


# a mixed solve's answer is accepted when its backward-error estimate is at
# most this (the FP64 solver's own level on these problems)
MIXED_ETA_ACCEPT = 1e-14


# ---------------------------------------------------------------------------
# Admission core (no GPU)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    t_arrive: float          # seconds after the start of the run
    m: int
    n: int
    nrhs: int
    footprint: int = 0       # device bytes, set by the executor
    payload: object = None   # executor data (host buffers)


@dataclasses.dataclass
class Completion:
    rid: int
    t_arrive: float
    t_admit: float
    t_done: float
    result: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class Scheduler:
    """FIFO admission by slots and HBM footprint.

    ``launch(req, slot)`` starts a request and returns a handle;
    ``poll(handle)`` returns None while it runs, else its result.  A request
    larger than the whole budget is still admitted when nothing else is in
    flight (it could never run otherwise)."""

    def __init__(self, slots: int, hbm_budget: int, launch: Callable, poll: Callable,
                 clock: Callable[[], float] = time.perf_counter, idle: Callable[[float], None] | None = None):
        self.slots, self.budget = slots, hbm_budget
        self.launch, self.poll, self.clock = launch, poll, clock
        self.idle = idle or (lambda dt: time.sleep(min(dt, 2e-4)))
        self.peak_bytes = 0
        self.peak_inflight = 0

    def run(self, requests: list[Request]) -> list[Completion]:
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrive))
        waiting: collections.deque[Request] = collections.deque()
        inflight: dict[int, tuple[Request, object, float]] = {}
        free_slots = list(range(self.slots))[::-1]
        used = 0
        done: list[Completion] = []
        t0 = self.clock()
        while pending or waiting or inflight:
            now = self.clock() - t0
            while pending and pending[0].t_arrive <= now:
                waiting.append(pending.popleft())
            progressed = False
            for slot in list(inflight):
                req, handle, t_admit = inflight[slot]
                res = self.poll(handle)
                if res is not None:
                    done.append(Completion(req.rid, req.t_arrive, t_admit, self.clock() - t0, res))
                    del inflight[slot]
                    free_slots.append(slot)
                    used -= req.footprint
                    progressed = True
            while waiting and free_slots and (used + waiting[0].footprint <= self.budget or not inflight):
                req = waiting.popleft()
                slot = free_slots.pop()
                handle = self.launch(req, slot)
                used += req.footprint
                inflight[slot] = (req, handle, self.clock() - t0)
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_inflight = max(self.peak_inflight, len(inflight))
                progressed = True
            if not progressed:
                nxt = pending[0].t_arrive - (self.clock() - t0) if (pending and not waiting and not inflight) else 0.0
                self.idle(max(nxt, 0.0))
        return done


def latency_stats(done: list[Completion], t_span: float | None = None) -> dict:
    lat = np.array(sorted(c.latency for c in done))
    if lat.size == 0:
        return {}
    span = t_span if t_span is not None else max(c.t_done for c in done) - min(c.t_arrive for c in done)
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat[-1] * 1e3),
            "solves_per_s": float(lat.size / span) if span > 0 else math.inf}


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Runs requests on HIP streams with the tqr library.  Host data live in
    pinned buffers, so the copies in and out are asynchronous on the
    request's stream.  ``solver`` is "mixed" (FP32-update factor + FP64
    CGLS, at most ``iterations`` iterations) or "fp64"."""

    def __init__(self, slots: int, device: str = "cuda", solver: str = "mixed", iterations: int = 10):
        import torch
        from . import tqr
        if solver not in ("mixed", "fp64"):
            raise ValueError("solver must be 'mixed' or 'fp64'")
        self.torch, self.tqr = torch, tqr
        self.device = device
        self.solver = solver
        self.iterations = iterations
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        props = torch.cuda.get_device_properties(device)
        self.device_slots = int(props.multi_processor_count)

    def tiling(self, m: int, n: int) -> tuple[int, int]:
        b, ib = tiling_for(m, n)
        # the mixed solver runs tiles of 64, 128 or 256
        return (max(b, 64), 16) if self.solver == "mixed" else (b, ib)

    def prepare(self, req: Request, A: np.ndarray, B: np.ndarray) -> Request:
        """Pins the request's host data and sets its footprint."""
        torch, tqr = self.torch, self.tqr
        m, n = A.shape
        nrhs = B.shape[1]
        b, ib = self.tiling(m, n)
        # column-major pinned host copies (a transposed row-major tensor)
        Ah = torch.empty((n, m), dtype=torch.float64, pin_memory=True)
        Ah.copy_(torch.from_numpy(np.ascontiguousarray(A.T)))
        Bh = torch.empty((nrhs, m), dtype=torch.float64, pin_memory=True)
        Bh.copy_(torch.from_numpy(np.ascontiguousarray(B.T)))
        Xh = torch.empty((nrhs, n), dtype=torch.float64, pin_memory=True)
        info_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
        status_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
        stats_h = torch.empty(2 * nrhs, dtype=torch.float64, pin_memory=True)
        if self.solver == "mixed":
            wb = int(tqr.lib().tqr_ls_mixed_workspace_bytes(m, n, nrhs, b))
        else:
            wb = tqr.workspace_bytes(m, n, nrhs, b, ib)
        te = tqr.t_elems(m, n, b, ib)
        req.footprint = footprint_bytes(m, n, nrhs, b, ib, wb, te)
        req.payload = {"A": Ah, "B": Bh, "X": Xh, "info": info_h, "status": status_h, "stats": stats_h,
                       "tile": (b, ib), "work_bytes": wb}
        return req

    def payload_copy(self, payload: dict) -> dict:
        """A payload for another request with the same pinned inputs: its
        own pinned result buffers, the input buffers shared (they are only
        read)."""
        torch = self.torch
        out = dict(payload)
        for key in ("X", "info", "status", "stats"):
            out[key] = torch.empty(payload[key].shape, dtype=payload[key].dtype, pin_memory=True)
        return out

    def launch(self, req: Request, slot: int):
        torch, tqr = self.torch, self.tqr
        pl = req.payload
        b, ib = pl["tile"]
        s = self.streams[slot]
        with torch.cuda.stream(s):
            dA = pl["A"].to(self.device, non_blocking=True).t()       # m x n column-major
            dB = pl["B"].to(self.device, non_blocking=True).t()       # m x nrhs column-major
            info = torch.zeros(1, dtype=torch.int32, device=self.device)
            status = torch.full((1,), -1, dtype=torch.int32, device=self.device)
            w = workers_for(req.m, req.n, b, self.device_slots)
            if self.solver == "mixed":
                work = torch.empty(pl["work_bytes"], dtype=torch.uint8, device=self.device)
                X, T, _, stats = tqr.solve_ls_mixed(dA, dB, b, self.iterations, workgroups=w, work=work, info=info,
                                                    status=status, policy=tqr.POLICY_COLUMN)
                pl["X"].copy_(X.t(), non_blocking=True)
                pl["stats"].copy_(stats, non_blocking=True)
                keep = (dA, dB, work, X, T, stats, info, status)
            else:
                ws = tqr.Workspace(req.m, req.n, req.nrhs, b, ib, self.device)
                tqr.solve_ls(dA, dB, b, ib, ws, workgroups=w, info=info, status=status, policy=tqr.POLICY_COLUMN)
                pl["X"].copy_(dB[: req.n].t(), non_blocking=True)
                keep = (dA, dB, ws, info, status)
            pl["info"].copy_(info, non_blocking=True)
            pl["status"].copy_(status, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # keep the device tensors alive until the event has passed
        return {"event": ev, "keep": keep, "payload": pl}

    def poll(self, handle):
        """None while the request runs; then {"X": nrhs x n pinned host
        tensor, "info": the dgels-style info word, "status": the scheduler's
        status word (0, or TQR_EABORTED when a wait bound or the abort flag
        ended the solve), "refine": the mixed solve's per-column statistics
        (None for the FP64 solver), "ok": info and status zero and, for the
        mixed solver, every column converged or stagnated at a backward-error
        estimate of at most MIXED_ETA_ACCEPT}."""
        if not handle["event"].query():
            return None
        handle["keep"] = None
        pl = handle["payload"]
        ok = int(pl["info"][0]) == 0 and int(pl["status"][0]) == 0
        refine = None
        if self.solver == "mixed":
            refine = self.tqr.refine_stats(pl["stats"])
            ok = ok and all(r["stop"] in (self.tqr.REFINE_CONVERGED, self.tqr.REFINE_STAGNATED)
                            and 0.0 <= r["eta"] <= MIXED_ETA_ACCEPT for r in refine)
        return {"X": pl["X"], "info": pl["info"], "status": pl["status"], "refine": refine, "ok": ok}
