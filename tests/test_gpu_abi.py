"""One test body, two libraries: the five calls of the C-ABI (lbm_create,
lbm_set_inlet, lbm_step, lbm_moments, lbm_destroy, after lbm_set_state) run
through the same ctypes signatures on the HIP library (FP32 populations) and
on the FP64 oracle library, and the moments after 23 steps agree within the
FP32 tolerance of the population parity tests (each stored population
rounded at ~1e-7 per step; fields compared relative to their scale)."""
import pytest

import abi
from gpu_common import noisy_inlet, rel_err, require_gpu, speed, tiny_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def libs():
    require_gpu()
    import oracle
    from paper_1002_3028_amd import lbm
    oracle.load()
    return {"hip": abi.load(lbm.LIB_PATH), "ref": abi.load(oracle.oracle.LIB_PATH)}


@pytest.mark.parametrize("case", ["jet", "substrate", "eq", "annulus"])
@pytest.mark.parametrize("nx,nr", [(40, 12), (131, 37)])
def test_same_calls_both_libraries(libs, case, nx, nr):
    from paper_1002_3028_amd import inputs
    p = tiny_params(nx, nr, case, hoop=1)
    inlet = noisy_inlet(nr, 7, 5)
    st = inputs.perturbed_state(nx, nr, 3, r0=p["r0"])
    out = {}
    for name, prec in (("hip", "fp32"), ("ref", "fp64")):
        codes, m = abi.run_jet(libs[name], p, prec, inlet, 23, state=st)
        assert all(v == 0 for k, v in codes.items() if k != "lbm_step_count"), (name, codes)
        assert codes["lbm_step_count"] == 23
        out[name] = m
    g, r = out["hip"], out["ref"]
    assert rel_err(speed(g), speed(r)) < 3e-5
    assert rel_err(g["T"], r["T"]) < 3e-5
    assert rel_err(g["rho"] - 1.0, r["rho"] - 1.0) < 3e-5


def test_fp64_is_the_checkers_only(libs):
    """The GPU library refuses FP64 populations; the oracle refuses anything
    else."""
    import ctypes
    p = tiny_params(40, 12, "jet", hoop=1)
    for name, prec in (("hip", "fp64"), ("ref", "fp32")):
        cfg, keep = abi.config(p, prec)
        h = ctypes.c_void_p(1)
        assert libs[name].lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
        assert not h.value
