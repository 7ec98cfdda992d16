"""Host logic of the continuous-batching loop (admission, per-stream order,
grouping, at most one request per stream per step, completion), exercised
with a fake executor on the CPU.  The fake keeps per-slot windows in numpy
and returns a value that depends on the exact window contents, so any
reordering or lost update changes the results."""
import numpy as np
import pytest

from paper_2108_12430_amd.serve import Server


class FakeExecutor:
    def __init__(self, capacity, lag=1):
        self.capacity = capacity
        self.windows = {}
        self.lag = lag
        self.launches = []
        self.next_slot = 0

    def open(self, model, C, W):
        if len(self.windows) >= self.capacity:
            return None
        s = self.next_slot
        self.next_slot += 1
        self.windows[s] = np.zeros((C, W))
        return s

    def close(self, slot):
        del self.windows[slot]

    def launch(self, model, C, W, items):
        slots = [s for s, _ in items]
        assert len(set(slots)) == len(slots), "a stream appears twice in one step"
        self.launches.append((model, C, W, [r.stream for _, r in items]))
        res = []
        for slot, r in items:
            w = self.windows[slot]
            s = r.samples.shape[1]
            w = np.concatenate([w, r.samples], axis=1)[:, -W:]
            self.windows[slot] = w
            if model == "dc":
                res.append(r.strain - w.sum(axis=0)[-s:])
            else:
                res.append(float(w.sum()))
        return {"left": self.lag, "res": res}

    def poll(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def finish(self, h):
        return h["res"]


def window_after(stream_blocks, W):
    x = np.concatenate([np.zeros((stream_blocks[0].shape[0], W))] + stream_blocks, axis=1)
    return x[:, -W:]


def test_admission_queue_fifo():
    ex = FakeExecutor(capacity=3)
    srv = Server(ex)
    sids = [srv.open_stream("dc", 2, 16) for _ in range(5)]
    assert [srv.admitted(s) for s in sids] == [True, True, True, False, False]
    srv.close_stream(sids[1])
    assert srv.admitted(sids[3]) and not srv.admitted(sids[4])
    srv.close_stream(sids[0])
    assert srv.admitted(sids[4])


def test_order_and_one_request_per_step():
    ex = FakeExecutor(capacity=8)
    srv = Server(ex)
    rng = np.random.default_rng(0)
    a = srv.open_stream("dc", 2, 16)
    b = srv.open_stream("dc", 2, 16)
    c = srv.open_stream("bbh", 1, 8)
    blocks = {a: [], b: [], c: []}
    reqs = []
    for k in range(5):
        for sid, C, s in ((a, 2, 4), (b, 2, 3), (c, 1, 2)):
            if sid == b and k >= 2:
                continue
            x = rng.standard_normal((C, s)).astype(np.float32)
            blocks[sid].append(x)
            reqs.append((sid, len(blocks[sid]), srv.submit(sid, x, rng.standard_normal(s).astype(np.float32) if sid != c else None)))
    n1 = srv.step()
    assert n1 == 3                                  # one per stream
    assert len(ex.launches) == 2                    # grouped by (model, C, W)
    srv.drain()
    for sid, k, r in reqs:
        w = window_after(blocks[sid][:k], 16 if sid != c else 8)
        if sid == c:
            assert r.result == pytest.approx(w.sum())
        else:
            np.testing.assert_allclose(r.result, r.strain - w.sum(axis=0)[-r.samples.shape[1]:])
        assert r.latency is not None and r.latency >= 0
    # per-stream completion order follows submission order
    for sid in (a, b, c):
        seqs = [r.seq for r in srv.completed if r.stream == sid]
        assert seqs == sorted(seqs)


def test_continuous_admission_while_inflight():
    ex = FakeExecutor(capacity=8, lag=3)
    srv = Server(ex, max_inflight=8)
    a = srv.open_stream("dc", 1, 8)
    srv.submit(a, np.ones((1, 2)), np.zeros(2))
    srv.step()
    assert len(srv.inflight) == 1
    b = srv.open_stream("dc", 1, 8)                 # arrives while step 1 is on the device
    srv.submit(b, np.ones((1, 2)), np.zeros(2))
    srv.submit(a, np.ones((1, 2)), np.zeros(2))
    assert srv.step() == 2                          # joins the next step without waiting
    srv.drain()
    assert len(srv.completed) == 3


def test_bad_requests_rejected_without_side_effects():
    ex = FakeExecutor(capacity=4)
    srv = Server(ex)
    a = srv.open_stream("dc", 2, 16)
    b = srv.open_stream("dc", 2, 16)
    with pytest.raises(ValueError):
        srv.submit(a, np.ones((3, 4)), np.zeros(4))      # wrong channel count
    with pytest.raises(ValueError):
        srv.submit(a, np.ones((2, 17)), np.zeros(17))    # stride > W
    with pytest.raises(ValueError):
        srv.submit(a, np.ones((2, 4)), np.zeros(3))      # strain length mismatch
    r = srv.submit(b, np.ones((2, 4)), np.zeros(4))
    srv.drain()
    assert r.result is not None and srv.pending() == 0
    assert [x.stream for x in srv.completed] == [b]


def test_close_waits_for_queued_requests():
    ex = FakeExecutor(capacity=1)
    srv = Server(ex)
    a = srv.open_stream("dc", 1, 8)
    b = srv.open_stream("dc", 1, 8)                 # queued behind a
    r1 = srv.submit(a, np.ones((1, 2)), np.zeros(2))
    srv.close_stream(a)                              # deferred until r1 completes
    assert not srv.admitted(b)
    srv.drain()
    assert r1.result is not None
    assert srv.admitted(b)
