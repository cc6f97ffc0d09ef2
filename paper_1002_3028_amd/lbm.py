"""Python binding of liblbm_hip.so (include/lbm.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of the library.  PyTorch
supplies device memory (population buffers) and the HIP stream; nothing here
computes any part of the method.  If the library is missing this module
raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

ABI_VERSION = 2
OK, EINVAL, ENOMEM, EUNSTABLE, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
PRECISION = {"fp32": 1, "fp16": 2, "bf16": 3, "fp16sr": 4}
BC = {"inlet": 0, "outflow": 1, "periodic": 2, "axis": 3, "freeslip": 4, "wall": 5, "eq": 6}
LAYOUT = {"two": 0, "single": 1}  # two buffers, or one updated in place


class LbmError(RuntimeError):
    def __init__(self, code, what, msg=""):
        super().__init__(f"{what}: {msg} (code {code})")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("r0", ctypes.c_double),
        ("tau_nu", ctypes.c_double), ("tau_alpha", ctypes.c_double),
        ("cs", ctypes.c_double), ("delta", ctypes.c_double), ("pr_t", ctypes.c_double),
        ("table_n", ctypes.c_int32),
        ("nu_mult", ctypes.POINTER(ctypes.c_double)),
        ("alpha_mult", ctypes.POINTER(ctypes.c_double)),
        ("t_lo", ctypes.c_double), ("t_hi", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4),
        ("wall_T", ctypes.c_double * 4),
        ("eq_state", (ctypes.c_double * 4) * 4),
        ("body_force_x", ctypes.c_double),
        ("rho0", ctypes.c_double), ("ux0", ctypes.c_double),
        ("ur0", ctypes.c_double), ("T0", ctypes.c_double),
        ("hoop", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("rho_ref", ctypes.c_double), ("g_ref", ctypes.c_double),
        ("layout", ctypes.c_int32),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_lib = None

# name -> (argtypes, restype)
_SIGS = {
    "lbm_bytes_required": ([ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lbm_create": ([ctypes.POINTER(_Config), ctypes.POINTER(_vp)], ctypes.c_int),
    "lbm_create_in": ([ctypes.POINTER(_Config), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
                      ctypes.c_int),
    "lbm_set_inlet": ([_vp, ctypes.c_int32, _dp, _dp, _dp], ctypes.c_int),
    "lbm_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "lbm_moments": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_destroy": ([_vp], None),
    "lbm_step_count": ([_vp], ctypes.c_int64),
    "lbm_stream": ([_vp], _vp),
    "lbm_sync": ([_vp], ctypes.c_int),
    "lbm_set_graph_steps": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_set_state": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_get_populations": ([_vp, _dp, _dp], ctypes.c_int),
    "lbm_set_populations": ([_vp, _dp, _dp, ctypes.c_int64], ctypes.c_int),
    "lbm_conservation": ([_vp, _dp, _dp], ctypes.c_int),
    "lbm_conservation_noalloc": ([_vp, _dp, _dp], ctypes.c_int),
    "lbm_profiles": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "lbm_probe_copy": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "lbm_batch_create": ([ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.POINTER(_vp)],
                         ctypes.c_int),
    "lbm_batch_admit": ([_vp, ctypes.POINTER(_Config), ctypes.c_int32, _dp, _dp, _dp,
                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "lbm_batch_run": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_wait": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_poll": ([_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "lbm_batch_profiles": ([_vp, ctypes.c_int32, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_batch_moments": ([_vp, ctypes.c_int32, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_batch_retire": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_sync": ([_vp], ctypes.c_int),
    "lbm_batch_device_time": ([_vp, _dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "lbm_batch_jet_bytes": ([_vp, ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)],
                            ctypes.c_int),
    "lbm_batch_active": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t)],
                         ctypes.c_int),
    "lbm_batch_set_launch": ([_vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_set_cohort_bytes": ([_vp, ctypes.c_size_t], ctypes.c_int),
    "lbm_batch_set_streams": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_set_layout": ([_vp, ctypes.c_int32], ctypes.c_int),
    "lbm_batch_destroy": ([_vp], None),
    "lbm_tile_shape_count": ([], ctypes.c_int),
    "lbm_tile_shape": ([ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 4, ctypes.c_int),
    "lbm_tile_shape_info": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
                            ctypes.c_int),
    "lbm_set_tile_shape": ([_vp, ctypes.c_int32], ctypes.c_int),
}


def exported_names():
    return list(_SIGS)


def load():
    """Load liblbm_hip.so; raise if it is not built.

    torch is imported first.  The binding takes device memory and streams
    from torch, whose wheel carries its own HIP runtime, and the library must
    bind to that one: loaded first, the library would bring in the runtime
    under /opt/rocm and torch its own, and memory that one runtime allocated
    is unknown to the other (solver creation then fails, and the process can
    crash later)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (its HIP runtime, before the library's)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m "
                           "paper_1002_3028_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(code):
    return load().lbm_strerror(int(code)).decode()


def _check(rc, what):
    if rc != OK:
        raise LbmError(rc, what, strerror(rc))


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def make_config(p: dict, precision: str = "fp32", rho_ref: float = 1.0, g_ref: float = 0.0,
                layout: str = "two"):
    """Parameter dict -> lbm_config (plus arrays that must stay alive)."""
    c = _Config()
    c.abi_version = ABI_VERSION
    c.nx, c.nr = int(p["nx"]), int(p["nr"])
    c.r0 = float(p.get("r0", 0.0))
    c.tau_nu, c.tau_alpha = float(p["tau_nu"]), float(p["tau_alpha"])
    c.cs = float(p.get("cs", 0.0))
    c.delta = float(p.get("delta", 1.0))
    c.pr_t = float(p.get("pr_t", 0.3))
    keep = []
    if p.get("nu_mult") is not None:
        a, b = _f64(p["nu_mult"]), _f64(p["alpha_mult"])
        keep += [a, b]
        c.table_n = a.size
        c.nu_mult, c.alpha_mult = _ptr(a), _ptr(b)
    else:
        c.table_n = 0
    c.t_lo = float(p.get("t_lo", 0.0))
    c.t_hi = float(p.get("t_hi", 1.0))
    for s in range(4):
        v = p["bc"][s]
        c.bc[s] = BC[v] if isinstance(v, str) else int(v)
    wt = p.get("wall_T", [math.nan] * 4)
    eq = p.get("eq_state", [[1.0, 0.0, 0.0, 0.0]] * 4)
    for s in range(4):
        c.wall_T[s] = float(wt[s])
        for q in range(4):
            c.eq_state[s][q] = float(eq[s][q])
    c.body_force_x = float(p.get("body_force_x", 0.0))
    c.rho0 = float(p.get("rho0", 1.0))
    c.ux0 = float(p.get("ux0", 0.0))
    c.ur0 = float(p.get("ur0", 0.0))
    c.T0 = float(p.get("T0", 0.0))
    c.hoop = int(p.get("hoop", 1))
    c.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    c.rho_ref = float(rho_ref)
    c.g_ref = float(g_ref)
    c.layout = LAYOUT[layout] if isinstance(layout, str) else int(layout)
    return c, keep


def bytes_required(p: dict, precision="fp32", layout="two") -> int:
    cfg, keep = make_config(p, precision, layout=layout)
    n = ctypes.c_size_t()
    _check(load().lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)), "lbm_bytes_required")
    return int(n.value)


def tile_shapes():
    lib = load()
    out = []
    for q in range(lib.lbm_tile_shape_count()):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib.lbm_tile_shape(q, *[ctypes.byref(x) for x in v]), "lbm_tile_shape")
        out.append(tuple(x.value for x in v))
    return out


SHAPE_FIELDS = ("bx", "by", "ny", "nx", "waves", "cache", "steps", "lds")


def tile_shape_info(q: int) -> dict:
    """Every property of compiled shape q (see lbm_tile_shape_info)."""
    v = (ctypes.c_int32 * len(SHAPE_FIELDS))()
    _check(load().lbm_tile_shape_info(int(q), v, len(SHAPE_FIELDS)), "lbm_tile_shape_info")
    return dict(zip(SHAPE_FIELDS, (int(x) for x in v)))


def tile_shape_infos() -> list:
    return [tile_shape_info(q) for q in range(load().lbm_tile_shape_count())]


class Solver:
    """One jet on the current HIP device.

    Population buffers come from a torch uint8 tensor and work runs on a torch
    stream (default priority) unless ``stream`` is given.  layout="single"
    keeps one buffer updated in place (half the memory, same results).
    """

    def __init__(self, params: dict, precision: str = "fp32", rho_ref: float = 1.0,
                 g_ref: float = 0.0, stream=None, graph_steps: int = 0, tile_shape=None,
                 layout: str = "two"):
        import torch

        lib = load()
        self.lib = lib
        self.nx, self.nr = int(params["nx"]), int(params["nr"])
        self.precision = precision
        cfg, keep = make_config(params, precision, rho_ref, g_ref, layout)
        n = ctypes.c_size_t()
        _check(lib.lbm_bytes_required(ctypes.byref(cfg), ctypes.byref(n)), "lbm_bytes_required")
        self.mem = torch.empty(int(n.value), dtype=torch.uint8, device="cuda")
        self.torch_stream = stream if stream is not None else torch.cuda.Stream()
        h = _vp()
        rc = lib.lbm_create_in(ctypes.byref(cfg), _vp(self.mem.data_ptr()), n.value,
                               _vp(self.torch_stream.cuda_stream), ctypes.byref(h))
        _check(rc, "lbm_create_in")
        self.h = h
        del keep
        if tile_shape is not None and int(tile_shape) >= 0:
            _check(lib.lbm_set_tile_shape(self.h, int(tile_shape)), "lbm_set_tile_shape")
        if graph_steps:
            _check(lib.lbm_set_graph_steps(self.h, int(graph_steps)), "lbm_set_graph_steps")

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def step_count(self) -> int:
        return int(self.lib.lbm_step_count(self.h))

    @property
    def stream_handle(self) -> int:
        return int(self.lib.lbm_stream(self.h) or 0)

    def set_inlet(self, ux, ur, T):
        ux = _f64(ux).reshape(-1, self.nr)
        n_t = ux.shape[0]
        ur, T = _f64(ur, ux.size), _f64(T, ux.size)
        _check(self.lib.lbm_set_inlet(self.h, n_t, _ptr(ux), _ptr(ur), _ptr(T)), "lbm_set_inlet")

    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.h, int(n)), "lbm_step")

    def try_step(self, n: int = 1) -> int:
        return int(self.lib.lbm_step(self.h, int(n)))

    def sync(self):
        _check(self.lib.lbm_sync(self.h), "lbm_sync")

    def try_sync(self) -> int:
        return int(self.lib.lbm_sync(self.h))

    def set_graph_steps(self, k: int):
        _check(self.lib.lbm_set_graph_steps(self.h, int(k)), "lbm_set_graph_steps")

    def set_tile_shape(self, q: int):
        _check(self.lib.lbm_set_tile_shape(self.h, int(q)), "lbm_set_tile_shape")

    def moments(self):
        out = [np.empty((self.nr, self.nx)) for _ in range(4)]
        _check(self.lib.lbm_moments(self.h, *[_ptr(a) for a in out]), "lbm_moments")
        return dict(zip(("rho", "ux", "ur", "T"), out))

    def try_moments(self):
        out = [np.empty((self.nr, self.nx)) for _ in range(4)]
        rc = self.lib.lbm_moments(self.h, *[_ptr(a) for a in out])
        return int(rc), dict(zip(("rho", "ux", "ur", "T"), out))

    def profiles(self):
        a, b = np.empty(self.nx), np.empty(self.nx)
        c, d = np.empty(self.nr), np.empty(self.nr)
        _check(self.lib.lbm_profiles(self.h, _ptr(a), _ptr(b), _ptr(c), _ptr(d)), "lbm_profiles")
        return {"ux_axis": a, "T_axis": b, "ux_exit": c, "T_exit": d}

    def conservation(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.lbm_conservation(self.h, ctypes.byref(m), ctypes.byref(e)),
               "lbm_conservation")
        return m.value, e.value

    def conservation_noalloc(self):
        """conservation() with the library's fixed per-device partial sums."""
        m, e = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.lbm_conservation_noalloc(self.h, ctypes.byref(m), ctypes.byref(e)),
               "lbm_conservation_noalloc")
        return m.value, e.value

    def set_state(self, rho, ux, ur, T):
        n = self.nx * self.nr
        arrs = [_f64(a, n) for a in (rho, ux, ur, T)]
        _check(self.lib.lbm_set_state(self.h, *[_ptr(a) for a in arrs]), "lbm_set_state")

    def get_populations(self):
        f = np.empty((9, self.nr, self.nx))
        g = np.empty((4, self.nr, self.nx))
        _check(self.lib.lbm_get_populations(self.h, _ptr(f), _ptr(g)), "lbm_get_populations")
        return f, g

    def set_populations(self, f, g, step: int):
        n = self.nx * self.nr
        f, g = _f64(f, 9 * n), _f64(g, 4 * n)
        _check(self.lib.lbm_set_populations(self.h, _ptr(f), _ptr(g), int(step)),
               "lbm_set_populations")


class Batch:
    """Many resident jets advanced by one persistent launch per step."""

    def __init__(self, budget_bytes: int, max_slots: int, precision: str = "fp32", stream=None,
                 layout: str = "two"):
        lib = load()
        self.lib = lib
        self.precision = precision
        # without a caller's stream the library creates its own streams, back
        # to back, so that they sit on distinct hardware queues
        self.torch_stream = stream
        b = _vp()
        _check(lib.lbm_batch_create(int(budget_bytes), int(max_slots), PRECISION[precision],
                                    _vp(stream.cuda_stream) if stream is not None else None,
                                    ctypes.byref(b)),
               "lbm_batch_create")
        self.b = b
        self.shapes = {}
        if layout != "two":
            _check(lib.lbm_batch_set_layout(self.b, LAYOUT[layout]), "lbm_batch_set_layout")

    def close(self):
        if getattr(self, "b", None):
            self.lib.lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def jet_bytes(self, params: dict, precision: str | None = None) -> int:
        """Budget bytes of a jet in `precision` (default: the batch's)."""
        cfg, keep = make_config(params, precision or self.precision)
        n = ctypes.c_size_t()
        _check(self.lib.lbm_batch_jet_bytes(self.b, ctypes.byref(cfg), ctypes.byref(n)),
               "lbm_batch_jet_bytes")
        return int(n.value)

    def try_admit(self, params: dict, inlet, target_steps: int, rho_ref=1.0, g_ref=0.0,
                  precision: str | None = None):
        """Returns (code, slot).  precision: the jet's storage form (default:
        the batch's); a batch holds jets of several forms, each form in
        cohorts of its own."""
        cfg, keep = make_config(params, precision or self.precision, rho_ref, g_ref)
        slot = ctypes.c_int32(-1)
        if inlet is None:
            rc = self.lib.lbm_batch_admit(self.b, ctypes.byref(cfg), 0, None, None, None,
                                          int(target_steps), ctypes.byref(slot))
        else:
            ux, ur, T = inlet
            ux = _f64(ux).reshape(-1, int(params["nr"]))
            ur, T = _f64(ur, ux.size), _f64(T, ux.size)
            rc = self.lib.lbm_batch_admit(self.b, ctypes.byref(cfg), ux.shape[0], _ptr(ux),
                                          _ptr(ur), _ptr(T), int(target_steps),
                                          ctypes.byref(slot))
        if rc == OK:
            self.shapes[slot.value] = (int(params["nx"]), int(params["nr"]))
        return int(rc), int(slot.value)

    def admit(self, params: dict, inlet, target_steps: int, **kw) -> int:
        rc, slot = self.try_admit(params, inlet, target_steps, **kw)
        _check(rc, "lbm_batch_admit")
        return slot

    def run(self, k: int):
        _check(self.lib.lbm_batch_run(self.b, int(k)), "lbm_batch_run")

    def wait(self, in_flight: int = 0):
        """Wait until at most `in_flight` queued groups are unfinished."""
        _check(self.lib.lbm_batch_wait(self.b, int(in_flight)), "lbm_batch_wait")

    def poll(self, slot: int) -> int:
        n = ctypes.c_int64()
        _check(self.lib.lbm_batch_poll(self.b, int(slot), ctypes.byref(n)), "lbm_batch_poll")
        return int(n.value)

    def profiles(self, slot: int):
        nx, nr = self.shapes[slot]
        a, b = np.empty(nx), np.empty(nx)
        c, d = np.empty(nr), np.empty(nr)
        _check(self.lib.lbm_batch_profiles(self.b, int(slot), _ptr(a), _ptr(b), _ptr(c), _ptr(d)),
               "lbm_batch_profiles")
        return {"ux_axis": a, "T_axis": b, "ux_exit": c, "T_exit": d}

    def moments(self, slot: int):
        nx, nr = self.shapes[slot]
        out = [np.empty((nr, nx)) for _ in range(4)]
        _check(self.lib.lbm_batch_moments(self.b, int(slot), *[_ptr(a) for a in out]),
               "lbm_batch_moments")
        return dict(zip(("rho", "ux", "ur", "T"), out))

    def retire(self, slot: int):
        _check(self.lib.lbm_batch_retire(self.b, int(slot)), "lbm_batch_retire")
        self.shapes.pop(slot, None)

    def sync(self):
        _check(self.lib.lbm_batch_sync(self.b), "lbm_batch_sync")

    def device_time(self):
        """(milliseconds, groups): device time of the groups found complete
        by wait() or sync()."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.lbm_batch_device_time(self.b, ctypes.byref(ms), ctypes.byref(n)),
               "lbm_batch_device_time")
        return ms.value, n.value

    def active(self):
        n, used = ctypes.c_int32(), ctypes.c_size_t()
        _check(self.lib.lbm_batch_active(self.b, ctypes.byref(n), ctypes.byref(used)),
               "lbm_batch_active")
        return int(n.value), int(used.value)

    def set_cohort_bytes(self, nbytes: int):
        _check(self.lib.lbm_batch_set_cohort_bytes(self.b, int(nbytes)), "lbm_batch_set_cohort_bytes")

    def set_streams(self, n: int):
        """Spread each run's cohorts over 1 to 4 streams (default 2)."""
        _check(self.lib.lbm_batch_set_streams(self.b, int(n)), "lbm_batch_set_streams")

    def set_launch(self, tile_shape: int = -1, workgroups: int = 0):
        _check(self.lib.lbm_batch_set_launch(self.b, int(tile_shape), int(workgroups)),
               "lbm_batch_set_launch")


def probe_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_handle: int):
    _check(load().lbm_probe_copy(_vp(dst_ptr), _vp(src_ptr), int(nbytes), _vp(stream_handle)),
           "lbm_probe_copy")
