"""Second tier of GPU-vs-oracle parity: after the first few hundred steps
FP32 (or 16-bit) and FP64 trajectories of a noisy LES jet separate slowly, so
they are compared through time-averaged profiles -- centreline u_x(x), T(x)
and radial u_x(r), T(r) at i = nx/2 and i = nx-1 -- averaged over steps
[N/2, N] every 50 steps, within 1 % (profile error as in the precision
tests: ||d||_2 / ||ref||_2 per quantity over all sampled points)."""
import json

import numpy as np
import pytest

from gpu_common import host_threads, require_gpu

pytestmark = pytest.mark.gpu

N_STEPS, EVERY = 4000, 50


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _sample(m):
    nx = m["ux"].shape[1]
    return {"ux": np.concatenate([m["ux"][0], m["ux"][:, nx // 2], m["ux"][:, -1]]),
            "T": np.concatenate([m["T"][0], m["T"][:, nx // 2], m["T"][:, -1]])}


def _averaged(solver):
    acc = {"ux": 0.0, "T": 0.0}
    n = 0
    solver.step(N_STEPS // 2)
    for q in range(N_STEPS // 2 // EVERY + 1):
        s = _sample(solver.moments())
        acc = {k: acc[k] + s[k] for k in acc}
        n += 1
        if q < N_STEPS // 2 // EVERY:
            solver.step(EVERY)
    return {k: v / n for k, v in acc.items()}


@pytest.fixture(scope="module")
def twin():
    import oracle
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_large(nx=1024, nr=256, n_t=N_STEPS)
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        ref = _averaged(r)
    return p, inlet, ref


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_time_averaged_profiles(twin, precision):
    from paper_1002_3028_amd import lbm
    p, inlet, ref = twin
    with lbm.Solver(p, precision, graph_steps=EVERY) as s:
        s.set_inlet(*inlet)
        got = _averaged(s)
    err = {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ref}
    print(json.dumps({"precision": precision, "profile_error": err}))
    assert err["ux"] < 1e-2 and err["T"] < 1e-2
