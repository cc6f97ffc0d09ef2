"""The solver C-ABI of include/lbm.h as ctypes signatures, for driving either
library that exports it through one test body: the HIP library
(paper_1002_3028_amd/liblbm_hip.so) or the FP64 oracle (oracle/liblbm_ref.so,
whose lbm_create takes precision 0, FP64).  Argument marshalling only (no
test functions here)."""
import ctypes
import math

import numpy as np

ABI_VERSION = 2
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp16sr": 4}
BC = {"inlet": 0, "outflow": 1, "periodic": 2, "axis": 3, "freeslip": 4, "wall": 5, "eq": 6}
FIVE = ("lbm_create", "lbm_set_inlet", "lbm_step", "lbm_moments", "lbm_destroy")
EXTRAS = ("lbm_step_count", "lbm_sync", "lbm_set_state", "lbm_get_populations",
          "lbm_set_populations", "lbm_conservation", "lbm_profiles", "lbm_strerror")


class Config(ctypes.Structure):
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
SIGS = {
    "lbm_create": ([ctypes.POINTER(Config), ctypes.POINTER(_vp)], ctypes.c_int),
    "lbm_set_inlet": ([_vp, ctypes.c_int32, _dp, _dp, _dp], ctypes.c_int),
    "lbm_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "lbm_moments": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_destroy": ([_vp], None),
    "lbm_step_count": ([_vp], ctypes.c_int64),
    "lbm_sync": ([_vp], ctypes.c_int),
    "lbm_set_state": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_get_populations": ([_vp, _dp, _dp], ctypes.c_int),
    "lbm_set_populations": ([_vp, _dp, _dp, ctypes.c_int64], ctypes.c_int),
    "lbm_conservation": ([_vp, _dp, _dp], ctypes.c_int),
    "lbm_profiles": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
    "lbm_strerror": ([ctypes.c_int], ctypes.c_char_p),
}


def load(path):
    """A CDLL of `path` with the ABI's signatures set (RTLD_LOCAL: the two
    libraries export the same names and each handle resolves its own)."""
    lib = ctypes.CDLL(path)
    for name, (args, res) in SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def config(p, precision):
    """(Config, arrays to keep alive) from a parameter dict."""
    c = Config()
    c.abi_version = ABI_VERSION
    c.nx, c.nr = int(p["nx"]), int(p["nr"])
    c.r0 = float(p.get("r0", 0.0))
    c.tau_nu, c.tau_alpha = float(p["tau_nu"]), float(p["tau_alpha"])
    c.cs, c.delta, c.pr_t = float(p.get("cs", 0.0)), float(p.get("delta", 1.0)), \
        float(p.get("pr_t", 0.3))
    keep = []
    if p.get("nu_mult") is not None:
        a, b = _f64(p["nu_mult"]), _f64(p["alpha_mult"])
        keep += [a, b]
        c.table_n, c.nu_mult, c.alpha_mult = a.size, _ptr(a), _ptr(b)
    c.t_lo, c.t_hi = float(p.get("t_lo", 0.0)), float(p.get("t_hi", 1.0))
    wt = p.get("wall_T", [math.nan] * 4)
    eq = p.get("eq_state", [[1.0, 0.0, 0.0, 0.0]] * 4)
    for s in range(4):
        v = p["bc"][s]
        c.bc[s] = BC[v] if isinstance(v, str) else int(v)
        c.wall_T[s] = float(wt[s])
        for q in range(4):
            c.eq_state[s][q] = float(eq[s][q])
    c.body_force_x = float(p.get("body_force_x", 0.0))
    c.rho0, c.ux0 = float(p.get("rho0", 1.0)), float(p.get("ux0", 0.0))
    c.ur0, c.T0 = float(p.get("ur0", 0.0)), float(p.get("T0", 0.0))
    c.hoop = int(p.get("hoop", 1))
    c.precision = PREC[precision]
    c.rho_ref, c.g_ref, c.layout = 1.0, 0.0, 0
    return c, keep


def run_jet(lib, p, precision, inlet, steps, state=None):
    """The five calls in order on `lib`: create, set_inlet, step, moments,
    destroy (plus set_state when a starting state is given).  Returns the
    return codes and the moment fields."""
    cfg, keep = config(p, precision)
    h = _vp()
    codes = {"lbm_create": lib.lbm_create(ctypes.byref(cfg), ctypes.byref(h))}
    if codes["lbm_create"] != 0:
        return codes, None
    try:
        if state is not None:
            arrs = [_f64(a) for a in state]
            codes["lbm_set_state"] = lib.lbm_set_state(h, *[_ptr(a) for a in arrs])
        if inlet is not None:
            ux, ur, T = (_f64(a).reshape(-1, int(p["nr"])) for a in inlet)
            codes["lbm_set_inlet"] = lib.lbm_set_inlet(h, ux.shape[0], _ptr(ux), _ptr(ur),
                                                       _ptr(T))
        codes["lbm_step"] = lib.lbm_step(h, int(steps))
        out = [np.empty((int(p["nr"]), int(p["nx"]))) for _ in range(4)]
        codes["lbm_moments"] = lib.lbm_moments(h, *[_ptr(a) for a in out])
        codes["lbm_step_count"] = lib.lbm_step_count(h)
    finally:
        lib.lbm_destroy(h)
    return codes, dict(zip(("rho", "ux", "ur", "T"), out))
