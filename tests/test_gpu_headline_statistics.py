"""Time-averaged profiles over steps [10 000, 20 000] of a 20 000-step run,
sampled every 50 steps (centreline u_x(x), T(x) and radial u_x(r), T(r) at
i = nx/2 and nx-1; profile error ||d||_2 / ||ref||_2 per quantity), for the
2048 x 512 jet (the benchmark's workload) and the 1024 x 256 twin of the
4096 x 1024 jet, against the FP64 oracle.

A chaotic LES jet makes such averages noisy: the same FP32 run with its inlet
rows perturbed by 1e-6 (relative) differs from itself by the realization
floor.  A storage form passes if each error is within max(1 %, 1.5 x floor).
FP16 storage rounds the temperature
populations with a bias that moves T far past the floor (an expected
failure that reports its numbers); stochastic rounding (fp16sr) removes it.

The oracle needs about four minutes of 16 host cores for the 26 G node
updates, so the tests run only when LBM_LONG_TESTS=1 is set."""
import json
import os
import time

import numpy as np
import pytest

from gpu_common import host_threads, require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("LBM_LONG_TESTS") != "1",
                                 reason="about 4 minutes of FP64 oracle; set LBM_LONG_TESTS=1")]

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


def _err(a, b):
    return {k: float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in b}


def _gpu_run(p, inlet, precision, perturb=0.0):
    """perturb > 0 scales the inlet rows of u_x and T by 1 + perturb N(0, 1).
    The perturbation enters at every step, so rounding cannot erase it before
    the jet forms, as it can erase one of the initial rest state."""
    from paper_1002_3028_amd import lbm
    if perturb:
        rng = np.random.default_rng(7)
        ux, ur, T = (np.asarray(a, dtype=np.float64) for a in inlet)
        inlet = (ux * (1.0 + perturb * rng.standard_normal(ux.shape)), ur,
                 T * (1.0 + perturb * rng.standard_normal(T.shape)))
    with lbm.Solver(p, precision, graph_steps=EVERY) as s:
        s.set_inlet(*inlet)
        return _averaged(s, precision + (" perturbed" if perturb else ""))


def _reference(p, inlet, name):
    require_gpu()
    import oracle
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        ref = _averaged(r, f"oracle {name}")
    floor = _err(_gpu_run(p, inlet, "fp32", 1e-6), _gpu_run(p, inlet, "fp32"))
    print(json.dumps({"grid": name, "realization_floor": floor}), flush=True)
    return p, inlet, ref, floor


@pytest.fixture(scope="module")
def headline():
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_single(n_t=N_STEPS)
    return _reference(p, inlet, "2048x512")


@pytest.fixture(scope="module")
def twin():
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_large(nx=1024, nr=256, n_t=N_STEPS)
    return _reference(p, inlet, "1024x256")


def _check(case, precision):
    p, inlet, ref, floor = case
    err = _err(_gpu_run(p, inlet, precision), ref)
    print(json.dumps({"grid": f"{p['nx']}x{p['nr']}", "steps": N_STEPS, "precision": precision,
                      "profile_error": err, "floor": floor}), flush=True)
    for k in err:
        assert err[k] < max(1e-2, 1.5 * floor[k]), (k, err[k], floor[k])


FP16_BIAS = pytest.mark.xfail(
    reason="FP16 storage biases T over 20 000 steps (2.8e-2 / 3.5e-2 measured, floor ~3e-3)",
    strict=False)
BF16_BIAS = pytest.mark.xfail(reason="BF16 storage: 6.2e-2 u_x / 0.21 T measured", strict=False)


@pytest.mark.parametrize("precision", ["fp32", pytest.param("fp16", marks=FP16_BIAS), "fp16sr"])
def test_headline_jet_time_averaged_profiles(headline, precision):
    _check(headline, precision)


@pytest.mark.parametrize("precision", ["fp32", pytest.param("fp16", marks=FP16_BIAS),
                                       pytest.param("bf16", marks=BF16_BIAS), "fp16sr"])
def test_twin_time_averaged_profiles(twin, precision):
    _check(twin, precision)
