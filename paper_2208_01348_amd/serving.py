"""Serving spectrum requests on one GPU with continuous batching.

A request is one electron spectrum: a particle (lattice mask and dipole size),
a host index, the electron speed and trajectory, and n_E energies.  Each
box of lattice cells (shape and dipole size) gets one context with an open
slot-pool engine (libdda's dda_engine_*) on a stream of its own, driven by a
worker thread; every lattice in the box has a small context of its own for
its electron field, loss sums and index map.  Every energy of a request is one
system; systems of any request in that box, whatever its particle shape or
host index, share the engine's slots and its kernel launches, joining while
others are halfway through their iterations (each slot reads its lattice's
index map).  Interaction
spectra stay resident in the context's cache (keyed by the host wavenumber,
about one per slot, evicted least recently used into buffers the next
wavenumber reuses), so requests at the same wavenumbers share them.

Engines are admitted by HBM footprint: opening one reserves
dda_workspace_bytes(slots) against the server's budget; a request whose
engine does not fit waits until an idle engine is retired.  Workers on
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
from collections import OrderedDict, deque
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

    def box_key(self) -> str:
        """Lattices with one box of cells and one dipole size share D(k)."""
        return f"{np.shape(self.mask)}-{self.d!r}"


@dataclass
class Completion:
    rid: int
    P: np.ndarray           # [n_E][4]: P_EELS, P_ext, P_abs, P_CL (1/eV)
    info: List[tuple]       # per energy (iters, matvecs, rel_residual, status)
    t_submit: float         # perf_counter seconds
    t_done: float
    lattice: str            # the request's lattice key
    engine: str = ""        # the engine that served it (a box or a lattice key)


@dataclass
class _Live:
    req: Request
    einc: torch.Tensor
    p: torch.Tensor
    eps: np.ndarray                     # [n_E][n_occ]
    left: int
    info: Dict[int, tuple] = field(default_factory=dict)
    t_submit: float = 0.0


def engine_mask(mask: np.ndarray, share_box: bool) -> np.ndarray:
    """The engine context's lattice: the request's, or the full box."""
    return np.ones(np.shape(mask), np.uint8) if share_box else mask


class LatticeWorker:
    """One engine and the thread that polls it.

    share_box=False: the engine's context is the request's lattice.
    share_box=True: the engine's context fills the box (every cell occupied),
    and each lattice in that box has a context of its own for its electron
    field, loss sums and index map; its systems take engine slots through
    dda_engine_submit_lattice, beside systems of any other lattice in the
    box."""

    def __init__(self, mask: np.ndarray, d: float, key: str, slots: int, precision: str,
                 tol: float, maxit: int, check_every: int, on_done: Callable,
                 poll_intervals: int = 4, solver: Optional[DDASolver] = None,
                 share_box: bool = False, max_lattices: int = 64):
        self.key = key
        self.slots = slots
        self.share_box = share_box
        self.opts = dict(precision=precision, tol=tol, maxit=maxit, solver="cocg",
                         check_every=check_every)
        # the context may come from the server's footprint probe
        self.solver = solver or DDASolver(engine_mask(mask, share_box), d, 1.0, **self.opts)
        # share_box: a context per lattice key, least recently used first; at
        # most max_lattices are kept (closing one waits for the whole device,
        # so it is done only when a new lattice would exceed the bound)
        self.lattices: "OrderedDict[str, DDASolver]" = OrderedDict()
        self.max_lattices = max_lattices
        self.ctx = self.solver.ctx
        self.footprint = L.dda_workspace_bytes(self.ctx, slots)
        L.dda_engine_open(self.ctx, slots)
        self.on_done = on_done
        self.poll_intervals = poll_intervals
        self.inbox: deque = deque()
        self.live: Dict[int, _Live] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.abandon = False
        self.last_busy = time.perf_counter()
        self.systems_done = 0   # energies solved, finished requests or not
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

    def request_stop(self, abandon: bool = False) -> None:
        """Asks the thread to end once its requests are done, or at its next
        poll with abandon=True (systems still queued or in slots are dropped)."""
        with self.cv:
            self.stop = True
            self.abandon = self.abandon or abandon
            self.cv.notify()

    def close(self, abandon: bool = False) -> None:
        """request_stop, then joins the thread and frees the engine and the
        context (the engine waits for the work already on its stream)."""
        self.request_stop(abandon)
        self.thread.join()
        L.dda_engine_close(self.ctx)
        self.solver.close()
        for lat in self.lattices.values():
            lat.close()
        self.lattices.clear()

    def counts(self):
        """(requests waiting in the inbox, requests being solved, systems queued
        in the engine, systems in its slots)."""
        with self.cv:
            inbox, live = len(self.inbox), len(self.live)
        q, r, _ = L.dda_engine_status(self.ctx) if not self.stop else (0, 0, 0)
        return inbox, live, q, r

    # -- worker thread
    def _lattice(self, req: Request) -> DDASolver:
        if not self.share_box:
            return self.solver
        key = req.lattice_key()
        lat = self.lattices.get(key)
        if lat is not None:
            self.lattices.move_to_end(key)
            return lat
        if len(self.lattices) >= self.max_lattices:
            busy = {lv.req.lattice_key() for lv in self.live.values()}
            for k in list(self.lattices):
                if k not in busy:
                    self.lattices.pop(k).close()
                    break
        lat = DDASolver(req.mask, req.d, 1.0, **self.opts)
        self.lattices[key] = lat
        return lat

    def _start(self, req: Request, t_submit: float) -> None:
        s = self._lattice(req)
        n = s.n_occ
        E = np.asarray(req.energies, dtype=np.float64)
        eps = np.asarray(req.eps, dtype=np.complex128)
        eps = np.repeat(eps[:, None], n, axis=1) if eps.ndim == 1 else eps.reshape(E.size, n)
        L.dda_set_host(s.ctx, req.m_h.real, req.m_h.imag)
        einc = s.einc(E, req.beta, np.asarray(req.r0, dtype=np.float64).reshape(1, 3))
        p = torch.empty_like(einc)
        live = _Live(req, einc, p, np.ascontiguousarray(eps), E.size, t_submit=t_submit)
        self.live[req.rid] = live
        stride = 3 * n
        for ie in range(E.size):
            tag = req.rid * 4096 + ie
            L.dda_engine_submit_lattice(self.ctx, s.ctx, tag, float(E[ie]), live.eps[ie],
                                        einc.data_ptr() + 16 * stride * ie,
                                        p.data_ptr() + 16 * stride * ie)

    def _finish(self, live: _Live) -> None:
        req = live.req
        s = self._lattice(req)
        L.dda_set_host(s.ctx, req.m_h.real, req.m_h.imag)
        P = s.losses(req.energies, req.beta, live.eps,
                     np.asarray(req.r0, dtype=np.float64).reshape(1, 3), live.einc, live.p)
        info = [live.info[i] for i in range(len(req.energies))]
        self.on_done(Completion(req.rid, P, info, live.t_submit, time.perf_counter(),
                                req.lattice_key(), self.key))

    def _run(self) -> None:
        try:
            while True:
                with self.cv:
                    while not self.stop and not self.inbox and not self.live:
                        self.cv.wait()
                    if self.stop and (self.abandon or (not self.inbox and not self.live)):
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
                    self.systems_done += 1
                    if live.left == 0:
                        with self.cv:
                            del self.live[rid]
                        self.last_busy = time.perf_counter()
                        self._finish(live)
                self.last_busy = time.perf_counter()
        except BaseException as e:  # surfaced by Server.drain
            self.error = e
            with self.cv:
                self.live.clear()


class Server:
    """Admits requests by lattice footprint and collects completions.

    submit() only queues a request; an admission thread hands queued requests
    to their lattice's worker, opening engines while the budget allows and
    retiring idle ones when it does not.  New lattices are admitted in arrival
    order (a large lattice waiting for room is not overtaken by later new
    lattices), while requests whose lattice already has an engine join it at
    once.  Slow steps (creating a context, opening or closing an engine) run
    without the server lock, so workers report completions meanwhile."""

    def __init__(self, hbm_budget_bytes: float, slots: int = 64, precision: str = "mixed",
                 tol: float = 1e-8, maxit: int = 50000, check_every: int = 8,
                 poll_intervals: int = 4, worker_factory: Optional[Callable] = None,
                 footprint_fn: Optional[Callable] = None,
                 max_inflight: Optional[int] = None, share_box: bool = True,
                 max_lattices: int = 64):
        self.budget = float(hbm_budget_bytes)
        self.share_box = share_box
        # requests handed to engines and not yet completed; beyond this many
        # the rest wait in arrival order, so that a backlog is served first
        # come first served instead of every request sharing the device
        self.max_inflight = max_inflight
        self._inflight = 0
        self.slots = slots
        self.opts = dict(precision=precision, tol=tol, maxit=maxit, check_every=check_every,
                         poll_intervals=poll_intervals)
        if share_box:
            self.opts["share_box"] = True
            self.opts["max_lattices"] = max_lattices  # lattice contexts kept per engine
        self.worker_factory = worker_factory or LatticeWorker
        self.footprint_fn = footprint_fn or self._probe_footprint
        self.footprints: Dict[str, int] = {}   # per lattice key, probed once
        self._parked: Dict[str, DDASolver] = {}  # probe contexts kept for the lattice's engine
        self.peak_reserved = 0.0
        self.workers: Dict[str, LatticeWorker] = {}
        self.reserved = 0.0
        self.waiting: deque = deque()
        self.completions: List[Completion] = []
        self.lock = threading.RLock()
        self.done_cv = threading.Condition(self.lock)
        self.n_submitted = 0
        self.device = None
        self.error: Optional[BaseException] = None
        self._dirty = False      # an arrival or a completion since the last admission pass
        self._closing = False
        self._in_admission = 0   # requests taken off the queue by the current admission pass
        self._systems_retired = 0  # systems solved by engines since retired
        self._admitter: Optional[threading.Thread] = None

    # -- any thread
    def submit(self, req: Request) -> None:
        with self.lock:
            if self._admitter is None:
                self._admitter = threading.Thread(target=self._admit_loop, name="admission",
                                                  daemon=True)
                self._admitter.start()
            self.n_submitted += 1
            self.waiting.append((req, time.perf_counter()))
            self._dirty = True
            self.done_cv.notify_all()

    def _on_done(self, c: Completion) -> None:
        with self.done_cv:
            self.completions.append(c)
            self._inflight -= 1
            self._dirty = True
            self.done_cv.notify_all()

    def _slots_for(self, req: Request) -> int:
        return self.slots

    def _probe_footprint(self, req: Request, slots: int) -> int:
        if self.device is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        torch.cuda.set_device(self.device)
        o = self.opts
        probe = DDASolver(engine_mask(req.mask, self.share_box), req.d, 1.0, solver="cocg",
                          precision=o["precision"], tol=o["tol"], maxit=o["maxit"],
                          check_every=o["check_every"])
        # kept (a context without an engine holds little device memory) and
        # handed to the engine's worker: destroying it would wait for the
        # whole device
        self._parked[self._key(req)] = probe
        return L.dda_workspace_bytes(probe.ctx, slots)

    def _key(self, req: Request) -> str:
        return req.box_key() if self.share_box else req.lattice_key()

    def _footprint(self, req: Request, key: str) -> int:
        need = self.footprints.get(key)
        if need is None:
            need = int(self.footprint_fn(req, self._slots_for(req)))
            self.footprints[key] = need
        return need

    # -- admission thread
    def _admit_loop(self) -> None:
        if self.device is not None:
            torch.cuda.set_device(self.device)
        try:
            while True:
                with self.lock:
                    while not self._closing and not (self._dirty and self.waiting):
                        self.done_cv.wait(timeout=0.5)
                    if self._closing:
                        return
                    self._dirty = False
                    pending = list(self.waiting)
                    self.waiting.clear()
                    self._in_admission = len(pending)
                keep = self._admit(pending)
                with self.lock:
                    self.waiting.extendleft(reversed(keep))  # ahead of later arrivals
                    self._in_admission = 0
        except BaseException as e:  # surfaced by drain and replay_window
            with self.lock:
                self.error = e
                self.done_cv.notify_all()

    def _admit(self, pending: List[tuple]) -> List[tuple]:
        keep = []
        blocked = False  # a new lattice is waiting for room: later new lattices queue behind it
        for req, t in pending:
            key = self._key(req)
            with self.lock:
                w = self.workers.get(key)
                closing = self._closing
                full = self.max_inflight is not None and self._inflight >= self.max_inflight
            if full:
                keep.append((req, t))
                continue
            if w is None and not blocked and not closing:
                w = self._open(req, key)
                blocked = w is None
            if w is None:
                keep.append((req, t))
                continue
            with self.lock:
                self._in_admission -= 1
                self._inflight += 1
            w.submit(req, t)
        return keep

    def _open(self, req: Request, key: str) -> Optional[LatticeWorker]:
        need = self._footprint(req, key)
        while True:
            with self.lock:
                if self._closing:
                    return None
                if self.reserved + need <= self.budget or not self.workers:
                    break  # a lattice larger than the whole budget still runs, alone
                idle = [w for w in self.workers.values() if w.idle()]
                if not idle:
                    return None  # waits until a lattice goes idle
                victim = min(idle, key=lambda w: w.last_busy)
                del self.workers[victim.key]
                self.reserved -= victim.footprint
                self._systems_retired += getattr(victim, "systems_done", 0)
            victim.close()
        extra = {"solver": self._parked.pop(key)} if key in self._parked else {}
        w = self.worker_factory(req.mask, req.d, key, self._slots_for(req),
                                on_done=self._on_done, **self.opts, **extra)
        with self.lock:
            self.workers[key] = w
            self.reserved += w.footprint
            self.peak_reserved = max(self.peak_reserved, self.reserved)
        return w

    def _raise_if_failed(self) -> None:
        if self.error is not None:
            raise RuntimeError("admission failed") from self.error
        for w in list(self.workers.values()):
            if w.error is not None:
                raise RuntimeError(f"worker {w.key} failed") from w.error

    def drain(self, timeout_s: float = 600.0) -> List[Completion]:
        t_end = time.perf_counter() + timeout_s
        with self.done_cv:
            while len(self.completions) < self.n_submitted:
                self._raise_if_failed()
                left = t_end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError(f"{len(self.completions)} of {self.n_submitted} done")
                self.done_cv.wait(timeout=min(left, 0.5))
        return list(self.completions)

    def close(self, abandon: bool = False) -> None:
        """Stops admission, then each worker (abandon=True drops what is
        queued or in the slots).  Workers are joined without the server lock:
        one that is just reporting a completion needs it to finish."""
        with self.lock:
            self._closing = True
            self.done_cv.notify_all()
            admitter = self._admitter
        if admitter is not None:
            admitter.join()
        with self.lock:
            workers = list(self.workers.values())
            self.workers.clear()
            self.reserved = 0.0
            self.waiting.clear()
            parked = list(self._parked.values())
            self._parked.clear()
        # every worker stops launching before any frees memory (a free waits
        # for the whole device, including the streams of running workers)
        for w in workers:
            if hasattr(w, "request_stop"):
                w.request_stop(abandon)
        for w in workers:
            w.close(abandon)
        for s in parked:
            s.close()

    def snapshot(self) -> dict:
        """Queue depth now: requests waiting for an engine, requests in the
        engines' inboxes or being solved, and the systems (energies) queued in
        the engines and in their slots."""
        with self.lock:
            waiting = len(self.waiting) + self._in_admission
            workers = list(self.workers.values())
            done = len(self.completions)
            solved = self._systems_retired
        inbox = live = q = r = 0
        for w in workers:
            a, b, c, d = w.counts()
            inbox += a
            live += b
            q += c
            r += d
            solved += getattr(w, "systems_done", 0)
        return {"waiting_requests": waiting + inbox, "requests_in_engines": live,
                "systems_queued": q, "systems_in_slots": r, "completed": done,
                "systems_solved": solved, "engines": len(workers)}


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


@dataclass
class WindowReport:
    completions: List[Completion]   # finished within the window, by rid
    latency: Dict[int, float]       # arrival -> last probability, finished requests
    waited: Dict[int, float]        # arrival -> end of window, unfinished requests
    samples: List[dict]             # queue depth over time (snapshot() plus "t")
    window_s: float
    points_done: int                # energies of the finished requests
    systems_solved: int             # energies solved in the window, finished requests or not


def replay_window(server: Server, requests: List[Request], window_s: float,
                  sample_every_s: float = 0.5,
                  progress: Optional[Callable[[dict], None]] = None,
                  progress_every_s: float = 15.0) -> WindowReport:
    """Submits each request at its arrival time and serves for window_s
    seconds from the first arrival (or until every request is done), sampling
    the queue depth; then abandons what is unfinished.  For streams that
    arrive faster than the GPU serves them, this measures the sustained rate
    and the growth of the backlog instead of waiting for the last request."""
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    arrive: Dict[int, float] = {}
    samples: List[dict] = []
    next_sample = t0
    next_progress = t0 + progress_every_s
    i = 0
    while True:
        now = time.perf_counter()
        while i < len(order) and t0 + order[i].arrival <= now:
            arrive[order[i].rid] = t0 + order[i].arrival
            server.submit(order[i])
            i += 1
        if now >= next_sample:
            snap = server.snapshot()
            snap["t"] = round(now - t0, 3)
            snap["arrived"] = i
            samples.append(snap)
            next_sample += sample_every_s
            if progress is not None and now >= next_progress:
                progress(snap)
                next_progress += progress_every_s
        with server.lock:
            n_done = len(server.completions)
        server._raise_if_failed()
        if (i == len(order) and n_done == len(order)) or now - t0 >= window_s:
            break
        wake = min(next_sample, t0 + order[i].arrival if i < len(order) else next_sample)
        time.sleep(max(0.0, min(0.05, wake - time.perf_counter())))
    t_end = time.perf_counter()
    solved = server.snapshot()["systems_solved"]
    with server.lock:
        comps = sorted(server.completions, key=lambda c: c.rid)
    done = {c.rid for c in comps}
    lat = {c.rid: c.t_done - arrive[c.rid] for c in comps}
    waited = {rid: t_end - ta for rid, ta in arrive.items() if rid not in done}
    for r in order[i:]:
        waited[r.rid] = 0.0  # never arrived inside the window
    server.close(abandon=True)
    pts = sum(len(c.info) for c in comps)
    return WindowReport(comps, lat, waited, samples, t_end - t0, pts, solved)


def requests_from_stream(stream, eps_fn=None) -> List[Request]:
    """Requests from (arrival, Workload) pairs (workloads.c5_request_stream)."""
    out = []
    for i, (t, w) in enumerate(stream):
        out.append(Request(rid=i, arrival=float(t), mask=w.mask, d=w.d, m_h=complex(w.m_h),
                           beta=float(w.beta), energies=np.asarray(w.energies, np.float64),
                           eps=w.eps_table(), r0=np.asarray(w.r0, np.float64).reshape(3)))
    return out
