"""Serving: continuous batching of jet-solve requests.  Each request's
profiles are the same alone and in the mix (bitwise: same kernel, no
cross-jet arithmetic), admission respects the HBM budget, and the latency
bookkeeping is consistent."""
import numpy as np
import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _small_trace(n=14, rate=200.0):
    from paper_1002_3028_amd import inputs
    tr = inputs.arrival_trace(n, seed=3, rate=rate)
    out = []
    for arr, p, inlet, steps in tr:
        # same structure, smaller: keep the test to seconds
        nx, nr = max(64, p["nx"] // 8), max(16, p["nr"] // 8)
        q = dict(p, nx=nx, nr=nr)
        ux, ur, T = inputs.inlet_rows(nr, nr / 4.0, float(inlet[0].max()), float(inlet[2].max()))
        out.append((arr, q, (ux, ur, T), steps // 20))
    return out


@pytest.mark.parametrize("precision", ["fp16", "fp32"])
def test_result_alone_equals_in_mix(precision):
    from paper_1002_3028_amd import lbm, serve
    trace = _small_trace()
    summary, rec = serve.serve(trace, precision, budget_bytes=64 << 20, max_slots=6,
                               k_steps=20, realtime=True, keep_profiles=True)
    assert summary["requests"] == len(trace)
    assert summary["peak_slots"] <= 6 and summary["peak_bytes"] <= 64 << 20
    for q, (arr, p, inlet, steps) in enumerate(trace):
        r = rec[q]
        assert r["completed"] >= r["admitted"] >= 0.0 and r["latency"] > 0.0
        # by default FP16 requests are stored with stochastic rounding
        assert r["storage"] == serve.route(precision, steps) == \
            ("fp16sr" if precision == "fp16" else precision)
        with lbm.Batch(1 << 26, 1, r["storage"]) as alone:
            s = alone.admit(p, inlet, steps)
            alone.run(steps)
            prof = alone.profiles(s)
        for key in prof:
            assert np.array_equal(prof[key], r["profiles"][key]), (q, key)


def test_budget_limits_concurrency():
    """A budget that holds two of these jets never has more than two resident."""
    from paper_1002_3028_amd import lbm, serve
    trace = _small_trace(8)
    nx, nr = 64, 16
    big = [(a, dict(p, nx=nx, nr=nr), None, s) for a, p, _, s in trace]
    with lbm.Batch(1 << 24, 2, "fp16") as b:
        per_jet = b.jet_bytes(big[0][1])
    summary, rec = serve.serve(big, "fp16", budget_bytes=2 * per_jet + 128, max_slots=8,
                               k_steps=10, realtime=False)
    assert summary["peak_slots"] == 2
    assert all(r["latency"] > 0 for r in rec)


def test_long_requests_route_to_stochastic_rounding():
    """With FP16 storage, requests longer than the step limit run in FP16SR
    cohorts of the same batch; every result equals its alone run in the
    storage it was routed to, within the one budget and slot count."""
    from paper_1002_3028_amd import lbm, serve
    trace = _small_trace()
    limit = int(np.median([t[3] for t in trace]))
    summary, rec = serve.serve(trace, "fp16", budget_bytes=64 << 20, max_slots=6,
                               k_steps=20, realtime=True, keep_profiles=True, long_after=limit)
    counts = summary["storage_counts"]
    assert counts.get("fp16sr", 0) > 0 and counts.get("fp16", 0) > 0, counts
    assert summary["peak_slots"] <= 6 and summary["peak_bytes"] <= 64 << 20
    for q, (arr, p, inlet, steps) in enumerate(trace):
        want = "fp16sr" if steps > limit else "fp16"
        assert rec[q]["storage"] == want
        with lbm.Batch(1 << 26, 1, want) as alone:
            s = alone.admit(p, inlet, steps)
            alone.run(steps)
            prof = alone.profiles(s)
        for key in prof:
            assert np.array_equal(prof[key], rec[q]["profiles"][key]), (q, key)
