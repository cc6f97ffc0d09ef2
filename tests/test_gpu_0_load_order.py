"""The library used before anything imports torch.  In a fresh interpreter
the first call of the binding is one that loads the library
(tile_shape_infos); a solver is then built, stepped and read, and a batch
runs one group.  Regression test: loading the library before torch used to
put two HIP runtimes in one process (the system's, linked by the library,
and the one that the torch wheel carries), and solver creation failed on
memory that torch had allocated.

The check runs in a child interpreter, started before this process has
touched the GPU (the module sorts first among the GPU tests); in a process
that already has, it is skipped."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
assert "torch" not in sys.modules
from paper_1002_3028_amd import inputs, lbm
infos = lbm.tile_shape_infos()
p, inlet, _ = inputs.workload_single(n_t=50)
small = dict(p, nx=300, nr=70)
rows = inputs.inlet_rows(70, 70 / 16.0, 0.08, 1.0)
for prec in ("fp32", "fp16"):
    with lbm.Solver(small, prec, graph_steps=10, tile_shape=0) as s:
        s.set_inlet(*rows)
        s.step(37)
        f, g = s.get_populations()
        assert f.shape == (9, 70, 300)
with lbm.Batch(1 << 26, 2, "fp32") as b:
    slot = b.admit(small, rows, 20)
    b.run(20)
    b.sync()
print("load order ok", len(infos))
"""


def test_library_loaded_before_torch():
    import torch
    if torch.cuda.device_count() == 0:  # (counting does not initialise the device)
        pytest.skip("no HIP device")
    if torch.cuda.is_initialized():
        pytest.skip("this process already uses the GPU: run the module first")
    code = SCRIPT.replace("ROOT", repr(ROOT))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and "load order ok" in r.stdout, (r.returncode, r.stdout[-2000:],
                                                               r.stderr[-2000:])
