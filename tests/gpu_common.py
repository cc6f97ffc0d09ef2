"""Shared helpers of the GPU tests (no test functions here)."""
import math
import os

import numpy as np
import pytest

NAN = math.nan


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1002_3028_amd import lbm
    lbm.load()  # raises if the library is missing: no fallback


def host_threads():
    return max(1, min(16, os.cpu_count() or 1))


def rel_err(a, b):
    """max |a - b| / max |b| (the error relative to the field's scale)."""
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def speed(m):
    return np.hypot(m["ux"], m["ur"])


def tiny_params(nx, nr, case, hoop):
    """Parameter dicts that exercise every edge rule (and corner) on small
    grids; values of the paper's jet regime (tau 0.6, C_s 0.17, tables)."""
    from paper_1002_3028_amd import inputs
    nu_m, al_m = inputs.property_tables(0)
    p = dict(nx=nx, nr=nr, r0=0.0, tau_nu=0.6, tau_alpha=0.62, cs=0.17, delta=1.0, pr_t=0.3,
             nu_mult=nu_m, alpha_mult=al_m, t_lo=0.0, t_hi=1.0,
             bc=("inlet", "outflow", "axis", "freeslip"), wall_T=[NAN] * 4,
             eq_state=[[1.0, 0.0, 0.0, 0.0]] * 4, body_force_x=0.0, rho0=1.0, ux0=0.0,
             ur0=0.0, T0=0.0, hoop=hoop)
    if case == "jet":
        pass
    elif case == "closed":
        p["bc"] = ("periodic", "periodic", "axis", "wall")
        p["body_force_x"] = 1e-5
    elif case == "annulus":
        p.update(r0=5.0, bc=("periodic", "periodic", "wall", "wall"),
                 wall_T=[NAN, NAN, 1.0, 0.2])
    elif case == "eq":
        p.update(r0=3.0, bc=("eq", "eq", "eq", "eq"),
                 eq_state=[[1.01, 0.03, 0.0, 0.9], [0.99, 0.02, 0.01, 0.1],
                           [1.0, 0.01, 0.05, 0.7], [1.0, 0.0, 0.01, 0.3]])
    elif case == "xwalls":
        p.update(bc=("wall", "wall", "axis", "freeslip"), wall_T=[0.8, NAN, NAN, NAN])
    elif case == "substrate":
        p.update(bc=("inlet", "wall", "axis", "freeslip"), wall_T=[NAN, 0.3, NAN, NAN])
    elif case == "slab":
        p.update(r0=2.0, bc=("inlet", "outflow", "freeslip", "wall"),
                 wall_T=[NAN, NAN, NAN, 0.5])
    else:
        raise ValueError(case)
    return p


CASES = ["jet", "closed", "annulus", "eq", "xwalls", "substrate", "slab"]


def noisy_inlet(nr, n_t, seed):
    from paper_1002_3028_amd import inputs
    return inputs.inlet_rows(nr, max(2.0, nr / 2), 0.06, 0.9, T_amb=0.1, n_t=n_t, noise=0.05,
                             seed=seed)
