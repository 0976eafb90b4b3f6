"""Serving spectrum requests on one GPU with continuous batching.

A request is one electron spectrum: a particle (lattice mask and dipole size),
a host index, the electron speed and trajectory, and n_E energies.  Each
distinct lattice gets one context with an open slot-pool engine (libdda's
dda_engine_*) on a stream of its own, driven by a worker thread.  Every
energy of a request is one system; systems of any request on that lattice,
whatever its host index, share the engine's slots and its kernel launches,
joining while others are halfway through their iterations.  Interaction
spectra stay resident in the context's cache (keyed by the host wavenumber),
so requests at the same wavenumbers reuse them.

Lattices are admitted by HBM footprint: opening an engine reserves
dda_workspace_bytes(slots) against the server's budget; a request whose
lattice does not fit waits until an idle engine is retired.  Workers on
different lattices overlap on the device through their own streams (the
ctypes calls release the GIL).

This module only orchestrates: every step of a solve (electron field,
material terms, FFT matvecs, Krylov iterations, loss sums) runs in libdda's
HIP kernels.
"""

from __future__ import annotations

import hashlib
import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import _lib as L
from .solver import DDASolver


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    mask: np.ndarray        # uint8 [nz][ny][nx]
    d: float                # dipole size, nm
    m_h: complex            # host index
    beta: float             # electron speed / c
    energies: np.ndarray    # [n_E] eV
    eps: np.ndarray         # absolute permittivity: [n_E] (homogeneous) or [n_E][n_occ]
    r0: np.ndarray          # [3] trajectory point, nm

    def lattice_key(self) -> str:
        m = np.ascontiguousarray(self.mask, dtype=np.uint8)
        h = hashlib.sha1(m.tobytes()).hexdigest()[:16]
        return f"{m.shape}-{self.d!r}-{h}"


@dataclass
class Completion:
    rid: int
    P: np.ndarray           # [n_E][4]: P_EELS, P_ext, P_abs, P_CL (1/eV)
    info: List[tuple]       # per energy (iters, matvecs, rel_residual, status)
    t_submit: float         # perf_counter seconds
    t_done: float
    lattice: str


@dataclass
class _Live:
    req: Request
    einc: torch.Tensor
    p: torch.Tensor
    eps: np.ndarray                     # [n_E][n_occ]
    left: int
    info: Dict[int, tuple] = field(default_factory=dict)
    t_submit: float = 0.0


class LatticeWorker:
    """One lattice: a context with an open engine and the thread that polls it."""

    def __init__(self, mask: np.ndarray, d: float, key: str, slots: int, precision: str,
                 tol: float, maxit: int, check_every: int, on_done: Callable,
                 poll_intervals: int = 4):
        self.key = key
        self.slots = slots
        self.solver = DDASolver(mask, d, 1.0, precision=precision, tol=tol, maxit=maxit,
                                solver="cocg", check_every=check_every)
        self.ctx = self.solver.ctx
        self.footprint = L.dda_workspace_bytes(self.ctx, slots)
        L.dda_engine_open(self.ctx, slots)
        self.on_done = on_done
        self.poll_intervals = poll_intervals
        self.inbox: deque = deque()
        self.live: Dict[int, _Live] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.last_busy = time.perf_counter()
        self.error: Optional[BaseException] = None
        self.thread = threading.Thread(target=self._run, name=f"lattice-{key}", daemon=True)
        self.thread.start()

    # -- called from other threads
    def submit(self, req: Request, t_submit: float) -> None:
        with self.cv:
            self.inbox.append((req, t_submit))
            self.cv.notify()

    def idle(self) -> bool:
        with self.cv:
            return not self.inbox and not self.live

    def close(self) -> None:
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()
        L.dda_engine_close(self.ctx)
        self.solver.close()

    # -- worker thread
    def _start(self, req: Request, t_submit: float) -> None:
        s = self.solver
        n = s.n_occ
        E = np.asarray(req.energies, dtype=np.float64)
        eps = np.asarray(req.eps, dtype=np.complex128)
        eps = np.repeat(eps[:, None], n, axis=1) if eps.ndim == 1 else eps.reshape(E.size, n)
        L.dda_set_host(self.ctx, req.m_h.real, req.m_h.imag)
        einc = s.einc(E, req.beta, np.asarray(req.r0, dtype=np.float64).reshape(1, 3))
        p = torch.empty_like(einc)
        live = _Live(req, einc, p, np.ascontiguousarray(eps), E.size, t_submit=t_submit)
        self.live[req.rid] = live
        stride = 3 * n
        for ie in range(E.size):
            tag = req.rid * 4096 + ie
            L.dda_engine_submit(self.ctx, tag, float(E[ie]), live.eps[ie],
                                einc.data_ptr() + 16 * stride * ie,
                                p.data_ptr() + 16 * stride * ie)

    def _finish(self, live: _Live) -> None:
        req = live.req
        L.dda_set_host(self.ctx, req.m_h.real, req.m_h.imag)
        P = self.solver.losses(req.energies, req.beta, live.eps,
                               np.asarray(req.r0, dtype=np.float64).reshape(1, 3),
                               live.einc, live.p)
        info = [live.info[i] for i in range(len(req.energies))]
        self.on_done(Completion(req.rid, P, info, live.t_submit, time.perf_counter(), self.key))

    def _run(self) -> None:
        try:
            while True:
                with self.cv:
                    while not self.stop and not self.inbox and not self.live:
                        self.cv.wait()
                    if self.stop and not self.inbox and not self.live:
                        return
                    todo = list(self.inbox)
                    self.inbox.clear()
                for req, t in todo:
                    self._start(req, t)
                done = L.dda_engine_poll(self.ctx, self.poll_intervals, capacity=1024)
                for tag, inf in done:
                    rid, ie = divmod(tag, 4096)
                    live = self.live[rid]
                    live.info[ie] = inf
                    live.left -= 1
                    if live.left == 0:
                        self._finish(live)  # stays live (not idle) until reported
                        with self.cv:
                            del self.live[rid]
                self.last_busy = time.perf_counter()
        except BaseException as e:  # surfaced by Server.drain
            self.error = e
            with self.cv:
                self.live.clear()


class Server:
    """Admits requests by lattice footprint and collects completions."""

    def __init__(self, hbm_budget_bytes: float, slots: int = 64, precision: str = "mixed",
                 tol: float = 1e-8, maxit: int = 50000, check_every: int = 8,
                 poll_intervals: int = 4, worker_factory: Optional[Callable] = None,
                 footprint_fn: Optional[Callable] = None):
        self.budget = float(hbm_budget_bytes)
        self.slots = slots
        self.opts = dict(precision=precision, tol=tol, maxit=maxit, check_every=check_every,
                         poll_intervals=poll_intervals)
        self.worker_factory = worker_factory or LatticeWorker
        self.footprint_fn = footprint_fn or self._probe_footprint
        self.peak_reserved = 0.0
        self.workers: Dict[str, LatticeWorker] = {}
        self.reserved = 0.0
        self.waiting: deque = deque()
        self.completions: List[Completion] = []
        self.lock = threading.RLock()
        self.done_cv = threading.Condition(self.lock)
        self.n_submitted = 0
        self.device = None

    def _on_done(self, c: Completion) -> None:
        with self.done_cv:
            self.completions.append(c)
            self.done_cv.notify_all()
        self._pump()

    def _slots_for(self, req: Request) -> int:
        return self.slots

    def _probe_footprint(self, req: Request, slots: int) -> int:
        if self.device is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        torch.cuda.set_device(self.device)
        probe = DDASolver(req.mask, req.d, 1.0, solver="cocg", precision=self.opts["precision"])
        try:
            return L.dda_workspace_bytes(probe.ctx, slots)
        finally:
            probe.close()

    def _pump(self) -> None:
        """Hands waiting requests to their lattice's worker, opening engines
        while the budget allows and retiring idle ones when it does not."""
        with self.lock:
            keep = deque()
            while self.waiting:
                req, t = self.waiting.popleft()
                key = req.lattice_key()
                w = self.workers.get(key)
                if w is None:
                    w = self._open(req, key)
                if w is None:
                    keep.append((req, t))
                else:
                    w.submit(req, t)
            self.waiting = keep

    def _open(self, req: Request, key: str) -> Optional[LatticeWorker]:
        need = self.footprint_fn(req, self._slots_for(req))
        while self.reserved + need > self.budget and self.workers:
            me = threading.current_thread()
            idle = [w for w in self.workers.values()
                    if w.idle() and getattr(w, "thread", None) is not me]
            if not idle:
                return None  # waits until a lattice goes idle
            victim = min(idle, key=lambda w: w.last_busy)
            del self.workers[victim.key]
            self.reserved -= victim.footprint
            victim.close()
        # a lattice larger than the whole budget still runs, alone
        w = self.worker_factory(req.mask, req.d, key, self._slots_for(req),
                                on_done=self._on_done, **self.opts)
        self.workers[key] = w
        self.reserved += w.footprint
        self.peak_reserved = max(self.peak_reserved, self.reserved)
        return w

    def submit(self, req: Request) -> None:
        with self.lock:
            self.n_submitted += 1
            self.waiting.append((req, time.perf_counter()))
        self._pump()

    def drain(self, timeout_s: float = 600.0) -> List[Completion]:
        t_end = time.perf_counter() + timeout_s
        with self.done_cv:
            while len(self.completions) < self.n_submitted:
                for w in self.workers.values():
                    if w.error is not None:
                        raise RuntimeError(f"worker {w.key} failed") from w.error
                left = t_end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError(f"{len(self.completions)} of {self.n_submitted} done")
                self.done_cv.wait(timeout=min(left, 0.5))
                self._pump()
        return list(self.completions)

    def close(self) -> None:
        with self.lock:
            for w in self.workers.values():
                w.close()
            self.workers.clear()
            self.reserved = 0.0


def replay(server: Server, requests: List[Request], time_scale: float = 1.0,
           timeout_s: float = 600.0):
    """Submits each request at its arrival time (scaled) and waits for all.
    Returns (completions sorted by rid, latency per request in s, makespan s);
    a latency runs from the request's arrival to its last loss probability."""
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    arrive = {}
    for r in order:
        t_arr = t0 + r.arrival * time_scale
        dt = t_arr - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        arrive[r.rid] = t_arr
        server.submit(r)
    comps = server.drain(timeout_s)
    t1 = max(c.t_done for c in comps)
    lat = {c.rid: c.t_done - arrive[c.rid] for c in comps}
    return sorted(comps, key=lambda c: c.rid), lat, t1 - t0


def requests_from_stream(stream, eps_fn=None) -> List[Request]:
    """Requests from (arrival, Workload) pairs (workloads.c5_request_stream)."""
    out = []
    for i, (t, w) in enumerate(stream):
        out.append(Request(rid=i, arrival=float(t), mask=w.mask, d=w.d, m_h=complex(w.m_h),
                           beta=float(w.beta), energies=np.asarray(w.energies, np.float64),
                           eps=w.eps_table(), r0=np.asarray(w.r0, np.float64).reshape(3)))
    return out
