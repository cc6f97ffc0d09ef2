"""Profile error of each storage form as a function of run length, on four
jets of the serving workload (the first request of the seed-3 trace in each
size octave, 240 x 60 to 1280 x 320), against the FP64 oracle's end-of-run
profiles stored in tests/golden/serving_profiles.txt (written by
tests/golden/make_serving_profiles.py, oracle only).

A serving request returns the centreline (j = 0) and exit-column (i = nx-1)
profiles of u_x and T after 1 000 to 10 000 steps; the profile error is
||d||_2 / ||ref||_2 per quantity over both profiles.

What the runs show, and what is checked:

* These jets are unsteady.  Past about 1 000 steps even FP32 storage drifts
  from the FP64 trajectory (FP32 arithmetic seeds the divergence): its u_x
  error grows to about 1e-2 by 10 000 steps, and the smallest jet (nozzle
  radius 3.75 nodes) diverges first.  16-bit storage, whose rounding noise
  is larger, diverges sooner: its u_x error reaches 1-2.5 % by 10 000 steps.
  So the instantaneous u_x is compared only before the trajectories
  separate: within 1e-3 at 1 000 steps for FP32, 2e-3 for 16-bit storage;
  later it is held to 3 % (the scale of the divergence, not a parity bound).
* The temperature is the smooth field, and the one that 16-bit storage
  endangers: rounding to nearest biases it (its error grows linearly in
  time), so FP16 keeps T within 1e-3 (1.5e-3 allowed) at 1 000 steps and
  within 1 % only up to 4 000 steps -- the step limit that serving applies
  to it.  FP16SR (stochastic rounding) keeps T within 1e-3 at 1 000 steps
  and within 1 % over all 10 000 steps, as FP32 does.
* BF16 (8 significant bits) is reported with loose bounds.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

# storage -> (u_x bound at 1000 steps, T bound at 1000 steps, longest run with
# T within 1 %, u_x bound at every length)
CLAIMS = {"fp32": (1e-3, 1e-3, 10000, 3e-2),
          "fp16sr": (2e-3, 1e-3, 10000, 3e-2),
          "fp16": (2e-3, 1.5e-3, 4000, 3e-2),
          "bf16": (1e-2, 5e-2, 0, 0.1)}


def _golden():
    spec = importlib.util.spec_from_file_location(
        "make_serving_profiles", os.path.join(HERE, "golden", "make_serving_profiles.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _err(got, ref):
    out = {}
    for q in ("ux", "T"):
        a = np.concatenate([got[f"{q}_axis"], got[f"{q}_exit"]])
        b = np.concatenate([ref[f"{q}_axis"], ref[f"{q}_exit"]])
        out[q] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return out


def _errors(mod, ref, precision):
    from paper_1002_3028_amd import lbm
    out = {}
    for q, p, inlet in mod.jets():
        with lbm.Solver(p, precision, graph_steps=50) as s:
            s.set_inlet(*inlet)
            done = 0
            for c in mod.CHECKPOINTS:
                s.step(c - done)
                done = c
                out[(q, c)] = _err(s.profiles(), ref[(q, c)])
                print(json.dumps({"request": q, "grid": f"{p['nx']}x{p['nr']}",
                                  "precision": precision, "steps": c,
                                  "profile_error": out[(q, c)]}), flush=True)
    return out


@pytest.fixture(scope="module")
def gold():
    require_gpu()
    mod = _golden()
    ref = mod.read(os.path.join(HERE, "golden", "serving_profiles.txt"))
    return mod, ref, _errors(mod, ref, "fp32")


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp16sr", "bf16"])
def test_profile_error_by_run_length(gold, precision):
    mod, ref, e32 = gold
    e = e32 if precision == "fp32" else _errors(mod, ref, precision)
    ux1k, T1k, t_steps, ux_all = CLAIMS[precision]
    bad = []
    for (q, c), v in e.items():
        if c == 1000 and (v["ux"] > ux1k or v["T"] > T1k):
            bad.append(("at 1000 steps", q, c, v))
        if c <= t_steps and v["T"] > 1e-2:
            bad.append(("T within 1 %", q, c, v))
        if v["ux"] > ux_all:
            bad.append(("u_x divergence", q, c, v))
        if precision == "bf16" and v["T"] > 0.3:
            bad.append(("bf16 T", q, c, v))
    assert not bad, bad
