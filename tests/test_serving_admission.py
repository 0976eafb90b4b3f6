"""Host logic of the serving layer (no GPU): lattices are admitted by HBM
footprint, idle engines are retired least-recently-used first when a new
lattice does not fit, requests wait while every open engine is busy, and
every submitted request completes exactly once."""

import threading
import time

import numpy as np

from paper_2208_01348_amd.serving import Completion, Request, Server, replay, replay_window


class FakeWorker:
    """Stands in for a lattice engine: completes each request after a delay
    on its own thread; records how many requests it held at once."""

    opened = []
    lock = threading.Lock()

    def __init__(self, mask, d, key, slots, on_done, delay=0.02, **_):
        self.key = key
        self.footprint = int(mask.sum()) * 1000
        self.on_done = on_done
        self.busy = 0
        self.closed = False
        self.last_busy = time.perf_counter()
        self.delay = delay
        self.error = None
        with FakeWorker.lock:
            FakeWorker.opened.append(self)

    def submit(self, req, t_submit):
        assert not self.closed
        self.busy += 1

        def done():
            time.sleep(self.delay)
            self.busy -= 1
            self.last_busy = time.perf_counter()
            n = len(req.energies)
            self.on_done(Completion(req.rid, np.full((n, 4), float(req.rid)), [], t_submit,
                                    time.perf_counter(), self.key))
        threading.Thread(target=done, daemon=True).start()

    def idle(self):
        return self.busy == 0

    def close(self, abandon=False):
        assert abandon or self.busy == 0, "a busy engine was retired"
        self.closed = True

    def counts(self):
        return 0, self.busy, 0, self.busy


def _req(rid, side, arrival=0.0):
    mask = np.zeros((side, side, side), np.uint8)
    mask[: side // 2] = 1
    return Request(rid=rid, arrival=arrival, mask=mask, d=1.0, m_h=1.45 + 0j, beta=0.55,
                   energies=np.linspace(1.0, 3.0, 4), eps=np.full(4, -10 + 1j),
                   r0=np.array([20.0, 0.0, 0.0]))


def test_admission_by_footprint_and_lru_retirement():
    FakeWorker.opened = []
    fp = lambda req, slots: int(req.mask.sum()) * 1000  # noqa: E731
    # lattices of 4^3/2, 6^3/2, 8^3/2 cells: footprints 32k, 108k, 256k bytes
    srv = Server(hbm_budget_bytes=300_000, worker_factory=FakeWorker, footprint_fn=fp)
    reqs = [_req(i, side, arrival=0.01 * i) for i, side in enumerate([4, 6, 4, 8, 6, 4, 8, 8])]
    comps, lat, span = replay(srv, reqs, timeout_s=30)
    assert sorted(c.rid for c in comps) == list(range(len(reqs)))
    for c in comps:
        assert np.all(c.P == c.rid)
    assert srv.peak_reserved <= 300_000 + 256_000  # one over-budget lattice may run alone
    # the 8^3 lattice cannot sit beside both others: some engine was retired
    assert any(w.closed for w in FakeWorker.opened)
    assert all(v >= 0 for v in lat.values())
    srv.close()


def test_one_engine_per_lattice_while_it_stays_open():
    FakeWorker.opened = []
    fp = lambda req, slots: 1  # noqa: E731
    srv = Server(hbm_budget_bytes=1e12, worker_factory=FakeWorker, footprint_fn=fp)
    reqs = [_req(i, 4 + 2 * (i % 2)) for i in range(10)]
    for r in reqs:
        srv.submit(r)
    comps = srv.drain(timeout_s=30)
    assert len(comps) == 10
    assert len(FakeWorker.opened) == 2
    srv.close()


def test_new_lattices_are_admitted_in_arrival_order():
    """A lattice waiting for room is not overtaken by a later new lattice
    that would fit; the footprint of each lattice is probed once."""
    FakeWorker.opened = []
    calls = []
    size = {4: 100, 6: 250, 8: 100}

    def fp(req, slots):
        calls.append(req.mask.shape[0])
        return size[req.mask.shape[0]]

    def factory(mask, d, key, slots, on_done, **kw):
        w = FakeWorker(mask, d, key, slots, on_done, delay=0.15)
        w.footprint = size[mask.shape[0]]
        return w

    srv = Server(hbm_budget_bytes=300, worker_factory=factory, footprint_fn=fp)
    reqs = [_req(0, 4, 0.0), _req(1, 6, 0.02), _req(2, 8, 0.04), _req(3, 4, 0.05),
            _req(4, 6, 0.06)]
    comps, lat, span = replay(srv, reqs, timeout_s=30)
    assert sorted(c.rid for c in comps) == list(range(len(reqs)))
    sides = [int(w.footprint) for w in FakeWorker.opened]
    # 4^3 first; the 6^3 lattice (250) waits for it to go idle; the 8^3 one,
    # which would have fitted beside the 4^3 engine, waits behind the 6^3 one
    assert sides.index(250) < sides.index(100, 1), sides
    assert sorted(calls) == [4, 6, 8]
    assert srv.peak_reserved <= 300
    srv.close()


def test_window_ends_on_time_with_a_backlog():
    """A stream that arrives faster than it is served: the window closes on
    time, the unfinished requests are reported with their waits, and the
    queue depth samples account for every arrived request."""
    FakeWorker.opened = []
    fp = lambda req, slots: 1  # noqa: E731

    class SerialFake(FakeWorker):  # one request at a time per lattice
        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.one = threading.Lock()

        def submit(self, req, t_submit):
            self.busy += 1

            def done():
                with self.one:
                    time.sleep(self.delay)
                self.busy -= 1
                self.on_done(Completion(req.rid, np.zeros((len(req.energies), 4)), [], t_submit,
                                        time.perf_counter(), self.key))
            threading.Thread(target=done, daemon=True).start()

    def factory(mask, d, key, slots, on_done, **kw):
        return SerialFake(mask, d, key, slots, on_done, delay=0.05)

    srv = Server(hbm_budget_bytes=1e12, worker_factory=factory, footprint_fn=fp)
    reqs = [_req(i, 4 + 2 * (i % 3), arrival=0.002 * i) for i in range(60)]
    t = time.perf_counter()
    rep = replay_window(srv, reqs, window_s=0.5, sample_every_s=0.05)
    assert time.perf_counter() - t < 5.0
    assert 0 < len(rep.completions) < len(reqs)
    assert len(rep.completions) + len(rep.waited) == len(reqs)
    for smp in rep.samples[1:]:  # a request being handed over may be missed, once per engine
        seen = smp["waiting_requests"] + smp["requests_in_engines"] + smp["completed"]
        assert smp["arrived"] - smp["engines"] <= seen <= smp["arrived"], smp


def test_inflight_cap_serves_a_backlog_in_arrival_order():
    """With max_inflight = 2, at most two requests are in the engines at any
    time and they are handed over in arrival order."""
    FakeWorker.opened = []
    fp = lambda req, slots: 1  # noqa: E731
    handed = []
    peak = [0]
    live = [0]
    guard = threading.Lock()

    class Counting(FakeWorker):
        def submit(self, req, t_submit):
            with guard:
                handed.append(req.rid)
                live[0] += 1
                peak[0] = max(peak[0], live[0])
            super().submit(req, t_submit)

    def factory(mask, d, key, slots, on_done, **kw):
        def done_cb(c):
            with guard:
                live[0] -= 1
            on_done(c)
        return Counting(mask, d, key, slots, done_cb, delay=0.03)

    srv = Server(hbm_budget_bytes=1e12, worker_factory=factory, footprint_fn=fp, max_inflight=2)
    reqs = [_req(i, 4 + 2 * (i % 3)) for i in range(12)]
    for r in reqs:
        srv.submit(r)
    comps = srv.drain(timeout_s=30)
    assert len(comps) == 12
    assert handed == list(range(12))
    assert peak[0] <= 2
    srv.close()


def test_lattices_of_one_box_share_an_engine_by_default():
    """Two particle shapes in the same box of cells (and dipole size) go to one
    engine; with share_box=False each lattice gets its own."""
    def two_shapes():
        a = _req(0, 6)
        b = _req(1, 6)
        b.mask = b.mask.copy()
        b.mask[:, :, :2] = 0  # another particle in the same 6^3 box
        assert a.lattice_key() != b.lattice_key() and a.box_key() == b.box_key()
        return [a, b]

    fp = lambda req, slots: 1  # noqa: E731
    for share, engines in [(True, 1), (False, 2)]:
        FakeWorker.opened = []
        srv = Server(hbm_budget_bytes=1e12, worker_factory=FakeWorker, footprint_fn=fp,
                     share_box=share)
        for r in two_shapes():
            srv.submit(r)
        comps = srv.drain(timeout_s=30)
        assert sorted(c.rid for c in comps) == [0, 1]
        assert len(FakeWorker.opened) == engines
        srv.close()
