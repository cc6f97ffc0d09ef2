"""Host logic of the serving loop (serve.serve) on the CPU, against a stand-in
batch with lbm.Batch's interface: a group advances every admitted jet by k
steps (up to its target) and completes when the next group is queued or the
batch is waited on.  Checks admission by budget and slots, routing of long
FP16 requests, retirement of every jet exactly once after the group it
finished in, and that the pipelined and the synchronous loop serve the same
requests with the same results."""
import numpy as np
import pytest

from paper_1002_3028_amd import lbm, serve


class FakeBatch:
    instances = []

    def __init__(self, budget, max_slots, precision, layout="two", stream=None):
        self.budget, self.max_slots, self.precision = budget, max_slots, precision
        self.slots = {}  # slot -> dict(steps, target, bytes, prec, params)
        self.groups = []  # per group: {slot: steps after the group}
        self.done_groups = 0
        self.retired = []
        self.max_in_flight = 0
        FakeBatch.instances.append(self)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        pass

    def set_launch(self, *a):
        pass

    def set_streams(self, n):
        pass

    def set_cohort_bytes(self, n):
        pass

    @staticmethod
    def _bytes(p, prec):
        return p["nx"] * p["nr"] * 13 * (4 if prec == "fp32" else 2) * 2

    def try_admit(self, p, inlet, steps, precision=None):
        prec = precision or self.precision
        used = sum(s["bytes"] for s in self.slots.values())
        if len(self.slots) >= self.max_slots or used + self._bytes(p, prec) > self.budget:
            return lbm.ENOMEM, -1
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = {"steps": 0, "target": steps, "bytes": self._bytes(p, prec),
                            "prec": prec, "nx": p["nx"], "done_group": None}
        return lbm.OK, slot

    def active(self):
        return len(self.slots), sum(s["bytes"] for s in self.slots.values())

    def run(self, k):
        g = len(self.groups)
        for slot, s in self.slots.items():
            if s["steps"] < s["target"]:
                s["steps"] = min(s["steps"] + k, s["target"])
                if s["steps"] == s["target"]:
                    s["done_group"] = g
        self.groups.append(dict((slot, s["steps"]) for slot, s in self.slots.items()))
        self.max_in_flight = max(self.max_in_flight, len(self.groups) - self.done_groups)

    def wait(self, in_flight=0):
        self.done_groups = max(self.done_groups, len(self.groups) - in_flight)

    def poll(self, slot):
        return self.slots[slot]["steps"]

    def sync(self):
        self.done_groups = len(self.groups)

    def device_time(self):
        return 0.5 * len(self.groups), len(self.groups)  # 0.5 ms per group

    def profiles(self, slot):
        s = self.slots[slot]
        # the extraction waits for the group in which the jet finished
        assert s["done_group"] is not None
        self.done_groups = max(self.done_groups, s["done_group"] + 1)
        return {"ux_axis": np.full(s["nx"], float(s["target"])), "prec": s["prec"]}

    def retire(self, slot):
        s = self.slots.pop(slot)
        assert s["done_group"] is not None and self.done_groups > s["done_group"]
        self.retired.append((slot, s["target"]))


def _trace(n=40, seed=1):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for q in range(n):
        t += float(rng.exponential(0.0005))
        nx = int(rng.choice([64, 128, 256]))
        out.append((t, {"nx": nx, "nr": nx // 4}, None, int(rng.integers(50, 700))))
    return out


@pytest.fixture
def fake(monkeypatch):
    FakeBatch.instances = []
    monkeypatch.setattr(serve.lbm, "Batch", FakeBatch)
    return FakeBatch


@pytest.mark.parametrize("pipeline", [True, False])
def test_every_request_served_once(fake, pipeline):
    trace = _trace()
    summary, rec = serve.serve(trace, "fp16", budget_bytes=2 << 20, max_slots=5, k_steps=20,
                               realtime=False, keep_profiles=True, long_after=400,
                               pipeline=pipeline)
    b = fake.instances[-1]
    assert summary["requests"] == len(trace) and len(b.retired) == len(trace)
    assert summary["peak_slots"] <= 5 and summary["peak_bytes"] <= 2 << 20
    for q, (arr, p, _, steps) in enumerate(trace):
        r = rec[q]
        assert r["storage"] == ("fp16sr" if steps > 400 else "fp16")
        assert r["profiles"]["prec"] == r["storage"]
        assert r["profiles"]["ux_axis"][0] == steps and r["completed"] >= r["admitted"]
    assert sorted(t for _, t in b.retired) == sorted(s for *_, s in trace)
    assert summary["timed_groups"] == len(b.groups) and summary["device_ms_per_group"] == 0.5
    # the pipelined loop keeps one group queued ahead, the synchronous none
    assert b.max_in_flight == (2 if pipeline else 1)


def test_pipelined_and_synchronous_serve_the_same(fake):
    trace = _trace(30, seed=2)
    out = {}
    for pipeline in (True, False):
        summary, rec = serve.serve(trace, "fp32", budget_bytes=4 << 20, max_slots=3,
                                   k_steps=50, realtime=False, keep_profiles=True,
                                   pipeline=pipeline)
        out[pipeline] = [r["profiles"]["ux_axis"][0] for r in rec]
        assert summary["storage_counts"] == {"fp32": 30}
    assert out[True] == out[False]


def test_budget_smaller_than_one_jet_waits_for_room(fake):
    """Admission stops at the first request that does not fit and resumes as
    jets retire; requests keep their arrival order."""
    trace = _trace(12, seed=3)
    summary, rec = serve.serve(trace, "fp16", budget_bytes=1 << 20, max_slots=2, k_steps=100,
                               realtime=False, long_after=-1)
    admitted = [r["admitted"] for r in rec]
    assert admitted == sorted(admitted)
    assert summary["peak_slots"] <= 2


def test_request_that_never_fits_is_an_error(fake):
    """A request larger than the whole budget is reported, not waited for."""
    trace = [(0.0, {"nx": 512, "nr": 128}, None, 100)]
    with pytest.raises(lbm.LbmError, match="does not fit"):
        serve.serve(trace, "fp32", budget_bytes=1 << 20, max_slots=4, realtime=False)
