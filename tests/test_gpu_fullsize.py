"""The 4096 x 1024 jet at full size, launched as the benchmark launches it
(two steps per launch, graphs of 50 steps), against the FP64 oracle after the
first 200 steps: FP32 storage within 1e-4 of the field scale on u and T (the
method's bound for this comparison), 16-bit storage within the profile bounds
of the precision tests (FP16 1e-3, BF16 2e-2).  The two-step variants the
autotuner picks between on this grid (with and without non-temporal stores)
give the same bits.
"""
import json

import numpy as np
import pytest

from gpu_common import host_threads, rel_err, require_gpu, speed
from test_gpu_precision import field_errors

pytestmark = pytest.mark.gpu

STEPS = 200


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def reference():
    import oracle
    from paper_1002_3028_amd import inputs
    p, inlet, _ = inputs.workload_large(n_t=2 * STEPS)
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        r.step(STEPS)
        return p, inlet, r.moments()


def _pair_variants():
    """Default two-step shape and the same tile with non-temporal stores."""
    from paper_1002_3028_amd import lbm
    infos = lbm.tile_shape_infos()
    base = [q for q, i in enumerate(infos)
            if i["steps"] == 2 and i["by"] * i["ny"] == 8 and i["cache"] == 8]
    nt = [q for q, i in enumerate(infos)
          if i["steps"] == 2 and i["by"] * i["ny"] == 8 and i["cache"] == 9]
    return base + nt


def _run(p, inlet, precision, **kw):
    from paper_1002_3028_amd import lbm
    with lbm.Solver(p, precision, graph_steps=50, **kw) as s:
        s.set_inlet(*inlet)
        s.step(STEPS)
        return s.moments()


def test_fp32_full_size_first_200_steps(reference):
    p, inlet, mr = reference
    runs = [_run(p, inlet, "fp32", tile_shape=q) for q in _pair_variants()]
    assert len(runs) == 2
    mg = runs[0]
    eu, eT = rel_err(speed(mg), speed(mr)), rel_err(mg["T"], mr["T"])
    print(f"4096x1024, {STEPS} steps: |u| {eu:.2e}  T {eT:.2e}")
    assert eu < 1e-4 and eT < 1e-4
    for key in mg:
        assert np.array_equal(runs[1][key], mg[key]), key


@pytest.mark.parametrize("precision,bound", [("fp16", 1e-3), ("bf16", 2e-2)])
def test_16bit_full_size_first_200_steps(reference, precision, bound):
    p, inlet, mr = reference
    errs = field_errors(_run(p, inlet, precision), mr)
    print(json.dumps({"grid": "4096x1024", "steps": STEPS, "precision": precision, **errs}))
    assert errs["profile"] < bound
