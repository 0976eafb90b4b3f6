"""Host logic of the serving layer (no GPU): lattices are admitted by HBM
footprint, idle engines are retired least-recently-used first when a new
lattice does not fit, requests wait while every open engine is busy, and
every submitted request completes exactly once."""

import threading
import time

import numpy as np

from paper_2208_01348_amd.serving import Completion, Request, Server, replay


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

    def close(self):
        assert self.busy == 0, "a busy engine was retired"
        self.closed = True


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
