"""Host logic of the server's admission, with fake solves (no device work):
the memory budget and slot limit hold with the builder threads and without,
in both scheduling modes; arrivals gate admission; a failed build is raised
by the scheduler loop; a request cancelled while queued, being built or
active is withdrawn and its memory freed."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2501_16122_amd import serve, synth  # noqa: E402


class _Tracker:
    def __init__(self):
        self.lock = threading.Lock()
        self.live = 0
        self.peak_live = 0
        self.bytes = 0
        self.peak_bytes = 0


class _FakeSolver:
    """Done after a number of steps and a minimum wall time (ten times a
    build's, so that solves overlap); each step is 'in flight' until polled."""

    def __init__(self, n_steps, n_pix, seconds):
        self.left = n_steps
        self.in_flight = False
        self.n_pix = n_pix
        self.until = time.perf_counter() + seconds

    def step(self, k):
        self.left -= 1
        self.in_flight = True

    def poll(self):
        done = self.left <= 0 and time.perf_counter() >= self.until
        flight = self.in_flight
        self.in_flight = False
        return done, flight

    def finish(self):
        return {"maps": [torch.zeros(3 * self.n_pix, dtype=torch.float64)], "info": [{"converged": 1}]}


def _install(monkeypatch, build_s=0.002, fail_rid=None, on_build=None, forever=()):
    tr = _Tracker()
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: object())
    # the footprint of a request: its sample count
    monkeypatch.setattr(serve, "footprint_bytes", lambda w, opts, weights: w.n_samples)

    class FakeSlot:
        def __init__(self, req, dev, stream, opts, use_weights, now):
            if req.rid == fail_rid:
                raise RuntimeError(f"build of request {req.rid} failed")
            time.sleep(build_s)
            if on_build:
                on_build(req.rid)
            self.req = req
            self.admitted = now
            # a request in ``forever`` never finishes unless cancelled
            self.solver = _FakeSolver(10 ** 9 if req.rid in forever else 1 + req.rid % 3, req.workload.n_pix,
                                      10 * build_s)
            with tr.lock:
                tr.live += 1
                tr.peak_live = max(tr.peak_live, tr.live)
                tr.bytes += req.workload.n_samples
                tr.peak_bytes = max(tr.peak_bytes, tr.bytes)

        def release(self):
            with tr.lock:
                tr.live -= 1
                tr.bytes -= self.req.workload.n_samples

    monkeypatch.setattr(serve, "_Slot", FakeSlot)
    monkeypatch.setattr(serve.b, "batch_step", lambda solvers, k: [s.step(k) for s in solvers])
    return tr


def _requests(n=12, spread=0.0):
    rng = np.random.default_rng(5)
    out = []
    for i in range(n):
        n_samp = int(rng.integers(1000, 5000))
        w = synth.Workload(f"fake{i}", 990, 8, 8, 1, n_samp)
        out.append(serve.Request(i, float(rng.uniform(0.0, spread)), w))
    return out


@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("prefetch", [True, False])
def test_admission_respects_budget_and_slots(monkeypatch, prefetch, batched):
    tr = _install(monkeypatch)
    reqs = _requests()
    budget = int(2.5 * max(r.workload.n_samples for r in reqs))
    srv = serve.Server("cpu", hbm_budget=budget, max_slots=3, k_chunk=8, batched=batched, prefetch=prefetch)
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    assert all(r.info["converged"] == 1 for r in res)
    assert tr.live == 0 and tr.bytes == 0 and srv.in_use == 0
    assert tr.peak_live <= 3 and srv.peak_slots <= 3
    assert tr.peak_bytes <= budget and srv.peak_bytes <= budget
    assert tr.peak_live >= 2, "requests must overlap"


@pytest.mark.parametrize("prefetch", [True, False])
def test_arrivals_gate_admission(monkeypatch, prefetch):
    _install(monkeypatch)
    reqs = _requests(n=8, spread=0.05)
    srv = serve.Server("cpu", hbm_budget=10 ** 9, max_slots=4, k_chunk=8, prefetch=prefetch)
    res = srv.run(reqs, realtime=True)
    assert len(res) == 8
    for r in res:
        assert r.admitted >= r.arrival - 1e-9 and r.finished >= r.admitted


def test_failed_build_is_raised(monkeypatch):
    _install(monkeypatch, fail_rid=2)
    srv = serve.Server("cpu", hbm_budget=10 ** 9, max_slots=4, k_chunk=8, prefetch=True)
    n0 = threading.active_count()
    with pytest.raises(RuntimeError, match="request 2"):
        srv.run(_requests(), realtime=False)
    # the scheduler joined its builder threads before raising
    assert threading.active_count() == n0


def test_request_larger_than_budget_is_refused(monkeypatch):
    _install(monkeypatch)
    reqs = _requests(n=3)
    srv = serve.Server("cpu", hbm_budget=10, max_slots=2, k_chunk=8, prefetch=True)
    with pytest.raises(MemoryError):
        srv.run(reqs, realtime=False)


@pytest.mark.timeout(60)
@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("prefetch", [True, False])
def test_cancel_at_every_stage(monkeypatch, prefetch, batched):
    srv_box = []
    # request 5 is cancelled from inside its own build; request 7 never
    # finishes and is cancelled once it is active
    tr = _install(monkeypatch, on_build=lambda rid: srv_box[0].cancel(rid) if rid == 5 else None, forever=(7,))
    reqs = _requests(n=12)
    srv = serve.Server("cpu", hbm_budget=10 ** 9, max_slots=3, k_chunk=8, batched=batched, prefetch=prefetch)
    srv_box.append(srv)
    srv.cancel(0)  # still queued when the run starts

    def on_result(res):
        if any(sl.req.rid == 7 for sl in list(srv.active)):
            srv.cancel(7)

    res = srv.run(reqs, realtime=False, on_result=on_result)
    stages = {rid: stage for rid, stage, _ in srv.cancelled}
    assert stages == {0: "queued", 5: stages[5], 7: "active"}
    assert stages[5] in ("built", "active")
    assert sorted(r.rid for r in res) == sorted(set(range(12)) - {0, 5, 7})
    assert all(r.info["converged"] == 1 for r in res)
    # every slot released, cancelled ones included; no cancel left pending
    assert tr.live == 0 and tr.bytes == 0 and srv.in_use == 0
    assert not srv._cancel
