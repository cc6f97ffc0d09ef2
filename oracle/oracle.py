"""ctypes binding of the FP64 CPU oracle (``liblbm_ref.so``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark; never by the product package.  It
shares no code with the HIP path: it has its own C header, its own struct and
its own enum values.

A solver is configured with a plain ``dict`` of parameters whose names follow
the paper's notation (see ``lbm_ref.h``); the same dict can be handed to the
GPU binding, which translates it to its own structure.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_REF_LIB") or os.path.join(_HERE, "liblbm_ref.so")
SOURCES = [os.path.join(_HERE, "lbm_ref.c"), os.path.join(_HERE, "lbm_ref_abi.c")]

OK, EINVAL, ENOMEM, EUNSTABLE, ESTATE = 0, -1, -2, -3, -5
BC = {"inlet": 0, "outflow": 1, "periodic": 2, "axis": 3, "freeslip": 4,
      "wall": 5, "eq": 6}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def build(verbose: bool = False) -> str:
    """Compile liblbm_ref.so with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fopenmp", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp"] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Config(ctypes.Structure):
    _fields_ = [
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
        ("threads", ctypes.c_int32),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    h = ctypes.c_void_p
    lib.lbm_ref_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(h)]
    lib.lbm_ref_destroy.argtypes = [h]
    lib.lbm_ref_destroy.restype = None
    lib.lbm_ref_set_inlet.argtypes = [h, ctypes.c_int32, _dp, _dp, _dp]
    lib.lbm_ref_step.argtypes = [h, ctypes.c_int64]
    lib.lbm_ref_step_count.argtypes = [h]
    lib.lbm_ref_step_count.restype = ctypes.c_int64
    lib.lbm_ref_moments.argtypes = [h, _dp, _dp, _dp, _dp]
    lib.lbm_ref_conservation.argtypes = [h, _dp, _dp]
    lib.lbm_ref_profiles.argtypes = [h, _dp, _dp, _dp, _dp]
    lib.lbm_ref_set_state.argtypes = [h, _dp, _dp, _dp, _dp]
    lib.lbm_ref_get_populations.argtypes = [h, _dp, _dp]
    lib.lbm_ref_set_populations.argtypes = [h, _dp, _dp, ctypes.c_int64]
    lib.lbm_ref_feq.argtypes = [ctypes.c_double] * 3 + [_dp]
    lib.lbm_ref_feq.restype = None
    lib.lbm_ref_geq.argtypes = [ctypes.c_double] * 3 + [_dp]
    lib.lbm_ref_geq.restype = None
    lib.lbm_ref_table_lookup.argtypes = [_dp, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double]
    lib.lbm_ref_table_lookup.restype = ctypes.c_double
    lib.lbm_ref_collide_node.argtypes = [h, _dp, _dp, ctypes.c_double, _dp, _dp, _dp]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _bc_code(v):
    return BC[v] if isinstance(v, str) else int(v)


def make_config(p: dict, threads: int = 0):
    """Translate a parameter dict into the oracle's C structure.

    Returns (struct, keepalive) -- the tables must outlive the create call.
    """
    c = _Config()
    c.nx, c.nr = int(p["nx"]), int(p["nr"])
    c.r0 = float(p.get("r0", 0.0))
    c.tau_nu, c.tau_alpha = float(p["tau_nu"]), float(p["tau_alpha"])
    c.cs = float(p.get("cs", 0.0))
    c.delta = float(p.get("delta", 1.0))
    c.pr_t = float(p.get("pr_t", 0.3))
    keep = []
    nu_t, al_t = p.get("nu_mult"), p.get("alpha_mult")
    if nu_t is not None:
        a, b = _f64(nu_t), _f64(al_t)
        keep += [a, b]
        c.table_n = a.size
        c.nu_mult, c.alpha_mult = _ptr(a), _ptr(b)
    else:
        c.table_n = 0
    c.t_lo = float(p.get("t_lo", 0.0))
    c.t_hi = float(p.get("t_hi", 1.0))
    bc = p["bc"]
    for s in range(4):
        c.bc[s] = _bc_code(bc[s])
    wt = p.get("wall_T", [math.nan] * 4)
    for s in range(4):
        c.wall_T[s] = float(wt[s])
    eq = p.get("eq_state", [[1.0, 0.0, 0.0, 0.0]] * 4)
    for s in range(4):
        for q in range(4):
            c.eq_state[s][q] = float(eq[s][q])
    c.body_force_x = float(p.get("body_force_x", 0.0))
    c.rho0 = float(p.get("rho0", 1.0))
    c.ux0 = float(p.get("ux0", 0.0))
    c.ur0 = float(p.get("ur0", 0.0))
    c.T0 = float(p.get("T0", 0.0))
    c.hoop = int(p.get("hoop", 0))
    c.threads = int(threads)
    return c, keep


class RefSolver:
    """One oracle solver handle (FP64, CPU)."""

    def __init__(self, params: dict, threads: int = 0):
        lib = load()
        self.lib = lib
        self.nx, self.nr = int(params["nx"]), int(params["nr"])
        self.r0 = float(params.get("r0", 0.0))
        cfg, keep = make_config(params, threads)
        h = ctypes.c_void_p()
        rc = lib.lbm_ref_create(ctypes.byref(cfg), ctypes.byref(h))
        del keep
        if rc != OK:
            raise OracleError(rc, "lbm_ref_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_ref_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what):
        if rc != OK:
            raise OracleError(rc, what)

    @property
    def step_count(self):
        return int(self.lib.lbm_ref_step_count(self.h))

    def set_inlet(self, ux, ur, T):
        ux = _f64(ux).reshape(-1, self.nr)
        n_t = ux.shape[0]
        ur = _f64(ur, n_t * self.nr)
        T = _f64(T, n_t * self.nr)
        self._check(self.lib.lbm_ref_set_inlet(self.h, n_t, _ptr(ux), _ptr(ur), _ptr(T)),
                    "lbm_ref_set_inlet")

    def step(self, n=1):
        rc = self.lib.lbm_ref_step(self.h, int(n))
        self._check(rc, "lbm_ref_step")

    def try_step(self, n=1):
        return int(self.lib.lbm_ref_step(self.h, int(n)))

    def moments(self):
        shape = (self.nr, self.nx)
        out = [np.empty(shape) for _ in range(4)]
        rc = self.lib.lbm_ref_moments(self.h, *[_ptr(a) for a in out])
        self._check(rc, "lbm_ref_moments")
        return dict(zip(("rho", "ux", "ur", "T"), out))

    def conservation(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.lbm_ref_conservation(self.h, ctypes.byref(m), ctypes.byref(e)),
                    "lbm_ref_conservation")
        return m.value, e.value

    def profiles(self):
        a, b = np.empty(self.nx), np.empty(self.nx)
        c, d = np.empty(self.nr), np.empty(self.nr)
        self._check(self.lib.lbm_ref_profiles(self.h, _ptr(a), _ptr(b), _ptr(c), _ptr(d)),
                    "lbm_ref_profiles")
        return {"ux_axis": a, "T_axis": b, "ux_exit": c, "T_exit": d}

    def set_state(self, rho, ux, ur, T):
        n = self.nx * self.nr
        arrs = [_f64(a, n) for a in (rho, ux, ur, T)]
        self._check(self.lib.lbm_ref_set_state(self.h, *[_ptr(a) for a in arrs]),
                    "lbm_ref_set_state")

    def get_populations(self):
        f = np.empty((9, self.nr, self.nx))
        g = np.empty((4, self.nr, self.nx))
        self._check(self.lib.lbm_ref_get_populations(self.h, _ptr(f), _ptr(g)),
                    "lbm_ref_get_populations")
        return f, g

    def set_populations(self, f, g, step):
        n = self.nx * self.nr
        f = _f64(f, 9 * n)
        g = _f64(g, 4 * n)
        self._check(self.lib.lbm_ref_set_populations(self.h, _ptr(f), _ptr(g), int(step)),
                    "lbm_ref_set_populations")

    def collide_node(self, f, g, r):
        f = _f64(f, 9)
        g = _f64(g, 4)
        fo, go, d = np.empty(9), np.empty(4), np.empty(20)
        self._check(self.lib.lbm_ref_collide_node(self.h, _ptr(f), _ptr(g), float(r),
                                                  _ptr(fo), _ptr(go), _ptr(d)),
                    "lbm_ref_collide_node")
        names = ("rho", "ux", "ur", "T", "nu", "alpha", "tau_nu", "qxx", "qxr", "qrr",
                 "qnorm", "tau", "nu_tot", "nu_t", "alpha_tot", "tau_a", "theta",
                 "Fx", "Fr", "S")
        return fo, go, dict(zip(names, d))


def feq(rho, ux, ur):
    out = np.empty(9)
    load().lbm_ref_feq(rho, ux, ur, _ptr(out))
    return out


def geq(T, ux, ur):
    out = np.empty(4)
    load().lbm_ref_geq(T, ux, ur, _ptr(out))
    return out


def table_lookup(tab, t_lo, t_hi, T):
    tab = _f64(tab)
    return float(load().lbm_ref_table_lookup(_ptr(tab), tab.size, t_lo, t_hi, T))
