"""16-bit population storage (FP16 / BF16 deviations from the lattice
weights, FP32 arithmetic) against the FP64 oracle and against FP32 storage.

Errors are stated per field.  Profile error, per quantity (u_x and T):
||d||_2 / ||ref||_2 over all sampled profile points together -- the
centreline (j = 0) and the radial profiles at i = nx/2 and i = nx-1 -- and
the larger of the two is reported.  (A separate norm per profile is not
meaningful: far from the nozzle this diffusive jet's temperature decays to
zero.)  The FP16 bound (1e-3) is the one the method's target sets for 16-bit
storage; BF16 (8-bit significand) is reported with its own, looser bound.
The FP32 instantaneous bound of 1e-4 holds over the first 200 steps; longer
runs compare at 1e-3 (FP32 and FP64 trajectories drift apart slowly).
"""
import json
import os

import numpy as np
import pytest

from gpu_common import host_threads, rel_err, require_gpu, speed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def profiles_of(m):
    nx = m["ux"].shape[1]
    return {
        "ux_axis": m["ux"][0], "T_axis": m["T"][0],
        "ux_mid": m["ux"][:, nx // 2], "T_mid": m["T"][:, nx // 2],
        "ux_exit": m["ux"][:, -1], "T_exit": m["T"][:, -1],
    }


def profile_error(a, b):
    pa, pb = profiles_of(a), profiles_of(b)
    out = 0.0
    for q in ("ux", "T"):
        keys = [k for k in pa if k.startswith(q + "_")]
        da = np.concatenate([pa[k] - pb[k] for k in keys])
        rb = np.concatenate([pb[k] for k in keys])
        out = max(out, float(np.linalg.norm(da) / np.linalg.norm(rb)))
    return out


def field_errors(a, b):
    return {"u": rel_err(speed(a), speed(b)), "T": rel_err(a["T"], b["T"]),
            "rho-1": rel_err(a["rho"] - 1.0, b["rho"] - 1.0), "profile": profile_error(a, b)}


def _run_gpu(p, inlet, steps, precision, g_ref=0.0):
    from paper_1002_3028_amd import lbm
    with lbm.Solver(p, precision, g_ref=g_ref, graph_steps=50) as s:
        s.set_inlet(*inlet)
        s.step(steps)
        return s.moments()


def _run_ref(p, inlet, steps):
    import oracle
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        r.step(steps)
        return r.moments()


def _record(name, data):
    """Print the measured errors (visible with pytest -s); with
    LBM_PRECISION_LOG set, also append them to that file as JSON lines."""
    line = json.dumps({"case": name, **data})
    print(line)
    path = os.environ.get("LBM_PRECISION_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(line + "\n")


def test_small_jet_16bit_storage():
    """128 x 32 jet, 500 steps: per-field errors of each storage format."""
    from paper_1002_3028_amd import inputs
    p, inlet, steps = inputs.workload_small()
    ref = _run_ref(p, inlet, steps)
    errs = {}
    for prec, g_ref in (("fp32", 0.0), ("fp16", 0.0), ("fp16", 0.5), ("bf16", 0.0),
                        ("fp16sr", 0.0)):
        errs[f"{prec}/g_ref={g_ref}"] = field_errors(_run_gpu(p, inlet, steps, prec, g_ref), ref)
    print(json.dumps(errs, indent=1))
    _record("128x32x500", errs)
    assert errs["fp32/g_ref=0.0"]["u"] < 1e-4 and errs["fp32/g_ref=0.0"]["T"] < 1e-4
    assert errs["fp32/g_ref=0.0"]["profile"] < 2e-4
    assert errs["fp16/g_ref=0.0"]["profile"] < 1e-3
    # an offset of g_ref/4 moves the mostly cold (g ~ 0) populations away from
    # where binary16 is densest: worse for a jet into cold ambient
    assert errs["fp16/g_ref=0.5"]["profile"] < 5e-3
    assert errs["bf16/g_ref=0.0"]["profile"] < 2e-2
    assert errs["fp16sr/g_ref=0.0"]["profile"] < 1e-3


def test_downscaled_twin_16bit_storage():
    """1024 x 256 jet (the downscaled twin of the 4096 x 1024 jet, inlet
    radius 16, noisy inlet), 1000 steps: FP16 storage within 1e-3 of the FP64
    oracle on the profiles; also against FP32 storage."""
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_large(nx=1024, nr=256, n_t=1000)
    steps = 1000
    ref = _run_ref(p, inlet, steps)
    m32 = _run_gpu(p, inlet, steps, "fp32")
    m16 = _run_gpu(p, inlet, steps, "fp16")
    mbf = _run_gpu(p, inlet, steps, "bf16")
    msr = _run_gpu(p, inlet, steps, "fp16sr")
    errs = {"fp32": field_errors(m32, ref), "fp16": field_errors(m16, ref),
            "bf16": field_errors(mbf, ref), "fp16sr": field_errors(msr, ref),
            "fp16_vs_fp32": field_errors(m16, m32)}
    print(json.dumps(errs, indent=1))
    _record("1024x256x1000", errs)
    assert errs["fp32"]["u"] < 1e-3 and errs["fp32"]["T"] < 1e-3
    assert errs["fp32"]["profile"] < 5e-4
    assert errs["fp16"]["profile"] < 1e-3
    assert errs["fp16sr"]["profile"] < 1e-3
    assert errs["bf16"]["profile"] < 2e-2


def test_16bit_rest_state_exact():
    """The stored deviation of the rest state is exactly representable: a
    uniform state at rest stays exactly at rest in every storage format."""
    from paper_1002_3028_amd import lbm
    from gpu_common import tiny_params
    p = tiny_params(64, 16, "closed", 1)
    p["body_force_x"] = 0.0
    p["T0"] = 0.5
    for prec in ("fp16", "bf16", "fp16sr"):
        with lbm.Solver(p, prec, g_ref=0.5) as s:
            s.step(100)
            m = s.moments()
        assert np.abs(m["ux"]).max() == 0.0 and np.abs(m["ur"]).max() == 0.0
        assert np.abs(m["rho"] - 1.0).max() < 1e-6
        assert np.abs(m["T"] - 0.5).max() < 1e-6
