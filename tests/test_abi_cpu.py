"""Host-side checks of the HIP library that need no GPU: it loads, exports
every entry point include/lbm.h declares, and rejects invalid configurations
before touching the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1002_3028_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1002_3028_amd import build
        build.build()
    return lbm.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 30
    from paper_1002_3028_amd import lbm
    for n in names:
        assert hasattr(lib, n), n
        assert n in lbm.exported_names(), n


def test_tile_shapes_listed(lib):
    from paper_1002_3028_amd import lbm
    shapes = lbm.tile_shapes()
    assert len(shapes) >= 4
    for bx, by, ny, nx in shapes:
        assert bx % 64 == 0 and bx * by <= 1024 and ny >= 1 and nx in (1, 2, 4, 8)


def _params(**kw):
    from paper_1002_3028_amd import inputs
    p = inputs.jet_params(64, 16, cs=0.1, table_seed=0)
    p.update(kw)
    return p


@pytest.mark.parametrize("bad", [
    dict(tau_nu=0.5), dict(tau_alpha=0.4), dict(pr_t=0.0), dict(nx=1), dict(nr=1),
    dict(r0=1.0),  # an axis must sit at r = 0
    dict(bc=("periodic", "outflow", "axis", "freeslip")),
    dict(bc=("inlet", "outflow", "freeslip", "axis")),
    dict(cs=-0.1), dict(hoop=2), dict(rho0=0.0), dict(T0=math.nan),
])
def test_invalid_configs_rejected(lib, bad):
    from paper_1002_3028_amd import lbm
    cfg, keep = lbm.make_config(_params(**bad))
    n = ctypes.c_size_t()
    assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.EINVAL
    h = ctypes.c_void_p(1)
    assert lib.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == lbm.EINVAL
    assert not h.value


def test_buffer_offset_limit(lib):
    """Buffers address their planes with 32-bit byte offsets: the largest
    grids that fit are accepted (8192 x 4096, 1.8 GB per FP32 buffer), one
    past the limit is refused before anything is allocated."""
    from paper_1002_3028_amd import lbm
    n = ctypes.c_size_t()
    cfg, keep = lbm.make_config(_params(nx=8192, nr=4096))
    assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.OK
    assert 2 * 13 * 4 * 8192 * 4096 < n.value < 2 * (1 << 31)
    for nx, nr in ((10000, 5000), (1 << 20, 512), (64, 1 << 22)):
        cfg, keep = lbm.make_config(_params(nx=nx, nr=nr))
        assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.EINVAL
        h = ctypes.c_void_p(1)
        assert lib.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == lbm.EINVAL
        assert not h.value


def test_precision_validated(lib):
    from paper_1002_3028_amd import lbm
    cfg, keep = lbm.make_config(_params(), precision=0)  # FP64 is the checker's, not ours
    n = ctypes.c_size_t()
    assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.EINVAL


def test_bytes_required(lib):
    """Two buffers of 13 planes; a plane holds nr + 2 rows (ghost rows) of a
    pitch that leaves 64 leading elements, the ghost column and vector slack."""
    from paper_1002_3028_amd import lbm
    p = _params(nx=100, nr=30)
    pitch = 192  # 64 + 100 + 1 + 8 rounded up to 64
    rows = 32
    assert lbm.bytes_required(p, "fp32") == 2 * ((13 * pitch * rows * 4 + 255) // 256 * 256)
    assert lbm.bytes_required(p, "fp16") == 2 * ((13 * pitch * rows * 2 + 255) // 256 * 256)


def test_strerror(lib):
    from paper_1002_3028_amd import lbm
    assert "unstable" in lbm.strerror(lbm.EUNSTABLE)
    assert lbm.strerror(12345) == "unknown error"


def test_null_safety(lib):
    lib.lbm_destroy(None)
    lib.lbm_batch_destroy(None)
    assert lib.lbm_step_count(None) == -1
    assert lib.lbm_step(None, 1) == -1


def test_layout_validated_and_single_buffer_is_half(lib):
    """One buffer updated in place takes exactly half the bytes of two;
    an unknown layout or an older config version is rejected."""
    from paper_1002_3028_amd import lbm
    for prec in ("fp32", "fp16"):
        n2 = lbm.bytes_required(_params(), prec, layout="two")
        n1 = lbm.bytes_required(_params(), prec, layout="single")
        assert n2 == 2 * n1
    for bad in (2, -1):
        cfg, keep = lbm.make_config(_params(), layout=bad)
        n = ctypes.c_size_t()
        assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.EINVAL
    cfg, keep = lbm.make_config(_params())
    cfg.abi_version = 1
    n = ctypes.c_size_t()
    assert lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)) == lbm.EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message (before
    touching any device)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_library_loads_after_torch():
    """The binding imports torch before it loads the library, so that the
    library binds to the HIP runtime that torch carries (a fresh interpreter
    whose first call loads the library)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1002_3028_amd import lbm\n"
            "assert 'torch' not in sys.modules\n"
            "lbm.tile_shape_infos()\n"
            "assert 'torch' in sys.modules\n"
            "print('ok')\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]


# ---- the same five calls in the FP64 oracle library -----------------------

@pytest.fixture(scope="module")
def ref_abi():
    import oracle
    import abi
    oracle.load()  # builds it if needed
    return abi.load(oracle.oracle.LIB_PATH)


def test_both_libraries_export_the_abi(lib, ref_abi):
    """The HIP library and the oracle export the five calls of the method's
    statement of the problem (and the state extras) under the same names,
    so one test body can drive either."""
    import abi
    from paper_1002_3028_amd import lbm
    hip = abi.load(lbm.LIB_PATH)
    for n in abi.FIVE + abi.EXTRAS:
        assert hasattr(hip, n), n
        assert hasattr(ref_abi, n), n


def _abi_case():
    from paper_1002_3028_amd import inputs
    p = inputs.jet_params(40, 12, cs=0.15, table_seed=0)
    inlet = inputs.inlet_rows(12, 4.0, 0.05, 0.9, T_amb=0.1, n_t=7, noise=0.05, seed=5)
    return p, inlet


@pytest.mark.parametrize("case", ["jet", "closed", "annulus", "eq", "xwalls", "substrate",
                                  "slab"])
def test_oracle_abi_is_the_oracle(ref, ref_abi, case):
    """Driving the oracle through the shared ABI gives bit-for-bit the result
    of its own lbm_ref_* calls on every edge-rule case: every field of the
    configuration (radius offset, walls and their temperatures, equilibrium
    sides, body force, tables, hoop form) reaches the oracle where it should;
    a shifted or dropped field would change the result."""
    import abi
    from gpu_common import noisy_inlet, tiny_params
    from paper_1002_3028_amd import inputs
    p = tiny_params(40, 12, case, hoop=1 if case != "closed" else 0)
    inlet = noisy_inlet(12, 7, 5)
    st = inputs.perturbed_state(40, 12, 3, r0=p["r0"])
    codes, m = abi.run_jet(ref_abi, p, "fp64", inlet, 23, state=st)
    assert all(v == 0 for k, v in codes.items() if k != "lbm_step_count"), codes
    assert codes["lbm_step_count"] == 23
    with ref.RefSolver(p) as s:
        s.set_state(*st)
        s.set_inlet(*inlet)
        s.step(23)
        mr = s.moments()
    for k in mr:
        np.testing.assert_array_equal(m[k], mr[k])


@pytest.mark.parametrize("change", ["fp32", "version", "layout"])
def test_oracle_abi_rejects_what_it_cannot_honour(ref_abi, change):
    import abi
    p, _ = _abi_case()
    cfg, keep = abi.config(p, "fp32" if change == "fp32" else "fp64")
    if change == "version":
        cfg.abi_version = 1
    if change == "layout":
        cfg.layout = 2
    h = ctypes.c_void_p(1)
    assert ref_abi.lbm_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert not h.value
    ref_abi.lbm_destroy(None)
    assert ref_abi.lbm_step(None, 1) == -1
