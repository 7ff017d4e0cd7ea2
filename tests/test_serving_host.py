"""Host logic of the request loop (serving.serve_engine) on the CPU: a fake
engine stands in for the device one, so the admission queue, the choice
between single steps and multi-step calls, and the latency bookkeeping are
checked without a GPU."""
import pytest

from paper_2106_15319_amd import serving


class FakeEngine:
    """Admits up to `slots` requests; request j needs need[j] steps; poll
    reports those whose steps are done (one call late, as the device
    engine reports the previous call's completions)."""

    def __init__(self, need, slots):
        self.need, self.slots = need, slots
        self.left, self.owner, self.calls = {}, {}, []
        self.done_prev, self.done_now = [], []
        self.next_ticket = 0
        self.closed = False

    def admit(self, signal, dims, out, n_imfs, D, K, S):
        if len(self.left) >= self.slots:
            return None
        t = self.next_ticket
        self.next_ticket += 1
        self.left[t] = self.need[signal]
        return t

    def _advance(self, n):
        self.done_prev, self.done_now = self.done_now, []
        for t in list(self.left):
            self.left[t] -= n
            if self.left[t] <= 0:
                self.done_now.append(t)

    def step(self, stream=None):
        self.calls.append(("step", 1, len(self.left)))
        self._advance(1)

    def step_n(self, n, stream=None):
        self.calls.append(("step_n", n, len(self.left)))
        self._advance(n)

    def poll(self):
        out = [t for t in self.done_prev if t in self.left]
        for t in out:
            del self.left[t]
        return out

    def resident(self):
        return len(self.left)

    def close(self):
        self.closed = True


def _serve(monkeypatch, need, arrivals, slots):
    eng = {}

    def make(budget, max_requests):
        eng["e"] = FakeEngine(need, slots)
        return eng["e"]

    monkeypatch.setattr(serving, "Engine", make)
    monkeypatch.setattr(serving.torch.cuda, "synchronize", lambda: None)
    reqs = [serving.Request(signal=j, dims=(1, 1), out=None, n_imfs=None, D=0, K=1, S=1)
            for j in range(len(need))]
    res = serving.serve_engine(reqs, arrivals, budget=1, max_requests=slots)
    return res, eng["e"]


def test_lone_request_takes_multi_step_calls(monkeypatch):
    res, e = _serve(monkeypatch, need=[20], arrivals=[0.0], slots=4)
    assert e.closed
    assert all(kind == "step_n" and n == serving.BURST_STEPS for kind, n, _ in e.calls)
    assert res["steps"] == serving.BURST_STEPS * len(e.calls)
    assert res["latency"][0] >= 0.0


def test_queued_requests_take_single_steps(monkeypatch):
    # one slot and three requests at once: while two wait for admission the
    # loop steps one at a time; the last one alone bursts
    need = [3, 3, 3]
    res, e = _serve(monkeypatch, need=need, arrivals=[0.0, 0.0, 0.0], slots=1)
    kinds = [k for k, _, _ in e.calls]
    first_burst = kinds.index("step_n")
    assert first_burst > 0 and set(kinds[:first_burst]) == {"step"}
    assert len(res["latency"]) == 3 and all(x >= 0.0 for x in res["latency"])
    assert res["max_resident"] == 1


def test_many_resident_take_single_steps(monkeypatch):
    n = serving.BURST_MAX_RESIDENT + 2
    res, e = _serve(monkeypatch, need=[5] * n, arrivals=[0.0] * n, slots=n)
    for kind, steps, resident in e.calls:
        if resident > serving.BURST_MAX_RESIDENT:
            assert kind == "step"
    assert res["max_resident"] == n


@pytest.mark.parametrize("need", [[1], [1, 40, 2, 9]])
def test_every_request_completes_once(monkeypatch, need):
    arrivals = [0.001 * j for j in range(len(need))]
    res, e = _serve(monkeypatch, need=need, arrivals=arrivals, slots=2)
    assert len(res["latency"]) == len(need)
    assert e.resident() == 0
