"""Seeded synthetic inputs for the axisymmetric thermal LBM-LES jet solver.

This module holds no arithmetic of the method itself: it only draws the
inputs that both the GPU path and its checker consume (property tables,
inlet rows, jet parameter draws, arrival traces) and returns them as plain
numpy arrays and parameter dicts.

Workload shapes follow the paper's setting (section 2.4: a half plane,
uniform lattice, an inlet edge with the profiles of eq. (7); section 2.3:
temperature-dependent properties).  The paper's own N2-Ar property curves and
its 200 x 96 physical run are not reproducible (their data are not given), so
seeded stand-ins of the same structure are used:

* property tables: 256 entries on T in [0, 1], monotone cubic (PCHIP through
  8 knots with random positive increments), nu rising 1x -> 8x and alpha
  1x -> 20x;
* inlet: parabolic axial velocity u_in = U_max (1 - (r/R)^2) for r < R (first
  line of eq. 7), uniform T_in inside the nozzle, ambient outside; optional
  multiplicative white noise per (step, node);
* batches and serving traces: jet sizes and inlet parameters drawn from
  numpy generators with fixed seeds.
"""
from __future__ import annotations

import math

import numpy as np

TABLE_N = 256


def property_tables(seed: int, n: int = TABLE_N):
    """(nu_mult, alpha_mult): monotone cubic multiplier tables over T in [0, 1].

    Children of SeedSequence(seed): 0 -> nu, 1 -> alpha, 2 -> reserved for the
    inlet noise of the same workload.
    """
    from scipy.interpolate import PchipInterpolator

    kids = np.random.SeedSequence(seed).spawn(3)
    knots_x = np.linspace(0.0, 1.0, 8)
    out = []
    for kid, top in ((kids[0], 8.0), (kids[1], 20.0)):
        rng = np.random.default_rng(kid)
        inc = rng.uniform(0.2, 1.0, 7)
        h = np.concatenate([[0.0], np.cumsum(inc)]) / inc.sum()
        knots_y = 1.0 + (top - 1.0) * h
        out.append(PchipInterpolator(knots_x, knots_y)(np.linspace(0.0, 1.0, n)))
    return out[0], out[1]


def inlet_rows(nr: int, radius: float, u_max: float, T_in: float = 1.0,
               T_amb: float = 0.0, r0: float = 0.0, n_t: int = 1,
               noise: float = 0.0, seed: int | None = None, t_profile: str = "flat"):
    """Inlet rows (ux, ur, T), each (n_t, nr), for the nodes r_j = r0 + j + 1/2.

    Nozzle nodes (r_j < radius) carry u_max (1 - (r_j/radius)^2) (eq. 7, first
    line) and, with t_profile = "flat", T_in; with t_profile = "cubic" they
    carry T_amb + (T_in - T_amb)(1 - (r_j/radius)^3) (eq. 7, second line, with
    T_min = T_amb and T_max = T_in).  The rest of the inlet face carries u = 0
    and T_amb.  With noise > 0, u is multiplied by (1 + noise * xi),
    xi ~ N(0, 1) independent per (row, node), drawn from child 2 of
    SeedSequence(seed).
    """
    r = r0 + np.arange(nr) + 0.5
    inside = r < radius
    prof = np.where(inside, u_max * (1.0 - (r / radius) ** 2), 0.0)
    ux = np.tile(prof, (n_t, 1))
    if noise > 0.0:
        rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
        ux = ux * (1.0 + noise * rng.standard_normal((n_t, nr)))
    ur = np.zeros((n_t, nr))
    if t_profile == "cubic":
        t_face = np.where(inside, T_amb + (T_in - T_amb) * (1.0 - (r / radius) ** 3), T_amb)
    elif t_profile == "flat":
        t_face = np.where(inside, T_in, T_amb)
    else:
        raise ValueError(t_profile)
    T = np.tile(t_face, (n_t, 1))
    return ux, ur, T


def jet_params(nx: int, nr: int, *, cs: float, table_seed: int | None,
               tau_nu: float = 0.6, tau_alpha: float = 0.6, pr_t: float = 0.3,
               hoop: int = 1) -> dict:
    """Parameter dict of a free jet: inlet at x0, outflow at x1, symmetry axis
    at r0 = 0 and a free-slip outer edge; ambient rho = 1, u = 0, T = 0."""
    p = dict(nx=nx, nr=nr, r0=0.0, tau_nu=tau_nu, tau_alpha=tau_alpha, cs=cs,
             delta=1.0, pr_t=pr_t, t_lo=0.0, t_hi=1.0,
             bc=("inlet", "outflow", "axis", "freeslip"),
             wall_T=[math.nan] * 4, eq_state=[[1.0, 0.0, 0.0, 0.0]] * 4,
             body_force_x=0.0, rho0=1.0, ux0=0.0, ur0=0.0, T0=0.0, hoop=hoop)
    if table_seed is not None:
        p["nu_mult"], p["alpha_mult"] = property_tables(table_seed)
    return p


def workload_small(hoop: int = 1):
    """128 x 32 jet, 500 steps: inlet radius 8, u_in = 0.05 (1 - (r/8)^2),
    T_in = 1, C_s = 0.1, tau_nu = tau_alpha = 0.6, tables from seed 0."""
    p = jet_params(128, 32, cs=0.1, table_seed=0, hoop=hoop)
    inlet = inlet_rows(32, 8.0, 0.05, 1.0)
    return p, inlet, 500


def workload_single(n_t: int = 20000, hoop: int = 1):
    """2048 x 512 jet, 20000 steps: inlet radius 32, U_max = 0.08 with 1 %
    white noise (one row per step), T_in = 1, C_s = 0.17, tables seed 1."""
    p = jet_params(2048, 512, cs=0.17, table_seed=1, hoop=hoop)
    inlet = inlet_rows(512, 32.0, 0.08, 1.0, n_t=n_t, noise=0.01, seed=1)
    return p, inlet, 20000


def workload_large(nx: int = 4096, nr: int = 1024, n_t: int = 20000, hoop: int = 1):
    """4096 x 1024 jet (inlet radius nr / 16 = 64), physics as the 2048 x 512
    jet; nx = 1024, nr = 256 gives its downscaled twin (radius 16)."""
    p = jet_params(nx, nr, cs=0.17, table_seed=1, hoop=hoop)
    inlet = inlet_rows(nr, nr / 16.0, 0.08, 1.0, n_t=n_t, noise=0.01, seed=1)
    return p, inlet, 20000


def workload_substrate(nx: int = 2048, nr: int = 512, n_t: int = 20000, T_wall: float = 0.0,
                       hoop: int = 1):
    """The 2048 x 512 jet impinging on a substrate (the paper's second case,
    section 4.2): physics and inlet of workload_single, with a no-slip wall at
    x = nx (the target plane) held at T_wall in place of the outflow.  The
    initial state is a formed jet column: along the whole axis the inlet
    profile u_x = U_max (1 - (r/R)^2), T = T_in for r < R, ambient outside,
    so that the column meets the plate at once (from rest the jet would need
    some 25 000 steps to cross 2048 nodes).  Returns (params, inlet, state)
    with state = (rho, ux, ur, T), each (nr, nx)."""
    p = jet_params(nx, nr, cs=0.17, table_seed=1, hoop=hoop)
    p["bc"] = ("inlet", "wall", "axis", "freeslip")
    p["wall_T"] = [math.nan, T_wall, math.nan, math.nan]
    radius = nr / 16.0
    inlet = inlet_rows(nr, radius, 0.08, 1.0, n_t=n_t, noise=0.01, seed=1)
    col_u, _, col_T = inlet_rows(nr, radius, 0.08, 1.0)
    ux = np.tile(col_u[0][:, None], (1, nx))
    T = np.tile(col_T[0][:, None], (1, nx))
    return p, inlet, (np.ones((nr, nx)), ux, np.zeros((nr, nx)), T)


def batch_jets(n: int = 64, seed: int = 2, steps: int = 5000, hoop: int = 1):
    """n independent jets of uneven sizes: nx in {256..2048 step 128}, nr in
    {64..512 step 32}, inlet radius nr/16, U_max ~ U[0.03, 0.1],
    T_in ~ U[0.5, 1], C_s ~ U[0.1, 0.2]; tables from seed 0."""
    rng = np.random.default_rng(seed)
    nu_m, al_m = property_tables(0)
    jets = []
    for _ in range(n):
        nx = int(rng.choice(np.arange(256, 2049, 128)))
        nr = int(rng.choice(np.arange(64, 513, 32)))
        u_in = float(rng.uniform(0.03, 0.1))
        T_in = float(rng.uniform(0.5, 1.0))
        cs = float(rng.uniform(0.1, 0.2))
        p = jet_params(nx, nr, cs=cs, table_seed=None, hoop=hoop)
        p["nu_mult"], p["alpha_mult"] = nu_m, al_m
        jets.append((p, inlet_rows(nr, nr / 16.0, u_in, T_in), steps))
    return jets


def umax_sweep(u_max_values=(0.03, 0.05, 0.07, 0.09), nx: int = 512, nr: int = 128,
               steps: int = 3000, hoop: int = 1):
    """Jets that differ only in the maximum inlet velocity (the paper's Fig. 7
    setting): inlet radius nr/8, both profiles of eq. (7) (parabolic u, cubic
    T), T_in = 1 into T = 0, C_s = 0.18, Pr_t = 0.3 (the validation values of
    Figs. 2-3), tables seed 0."""
    nu_m, al_m = property_tables(0)
    out = []
    for u in u_max_values:
        p = jet_params(nx, nr, cs=0.18, table_seed=None, hoop=hoop)
        p["nu_mult"], p["alpha_mult"] = nu_m, al_m
        out.append((p, inlet_rows(nr, nr / 8.0, u, 1.0, t_profile="cubic"), steps))
    return out


def arrival_trace(n: int = 2000, seed: int = 3, rate: float = 10.0, hoop: int = 1):
    """Poisson arrivals of jet-solve requests.

    Per request, in order: inter-arrival ~ Exp(1/rate); s = exp(U(0, ln 16)),
    nx = clip(16 round(8 s), 128, 2048), nr = nx / 4 (so 128 x 32 ... 2048 x
    512, log-uniform); steps ~ U{1000..10000}; U_max, T_in, C_s as in
    batch_jets; inlet radius nr / 16.  Returns a list of
    (arrival_time_s, params, inlet, steps).
    """
    rng = np.random.default_rng(seed)
    nu_m, al_m = property_tables(0)
    t = 0.0
    out = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate))
        s = math.exp(float(rng.uniform(0.0, math.log(16.0))))
        nx = int(min(max(16 * round(8 * s), 128), 2048))
        nr = nx // 4
        steps = int(rng.integers(1000, 10001))
        u_in = float(rng.uniform(0.03, 0.1))
        T_in = float(rng.uniform(0.5, 1.0))
        cs = float(rng.uniform(0.1, 0.2))
        p = jet_params(nx, nr, cs=cs, table_seed=None, hoop=hoop)
        p["nu_mult"], p["alpha_mult"] = nu_m, al_m
        out.append((t, p, inlet_rows(nr, nr / 16.0, u_in, T_in), steps))
    return out


def perturbed_state(nx: int, nr: int, seed: int, r0: float = 0.0, amp: float = 0.02,
                    T_mean: float = 0.5, T_amp: float = 0.2, noise: float = 0.0):
    """Smooth random non-uniform state (rho, ux, ur, T), each (nr, nx): a few
    random Fourier modes in x times smooth radial bumps; ur vanishes towards
    the axis.  Used for the closed-domain and parity checks.  noise > 0 adds
    independent Gaussian values of noise times each field's amplitude at
    every node (drawn after the modes, so the smooth part does not change),
    which makes every node differ from its neighbours."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    r = (np.arange(nr) + 0.5) / nr
    X, R = np.meshgrid(x, r)

    def field(a):
        out = np.zeros_like(X)
        for _ in range(3):
            kx = rng.integers(1, 4)
            kr = rng.integers(1, 4)
            ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
            out += a * rng.uniform(-1, 1) * np.sin(2 * np.pi * kx * X + ph1) * \
                np.cos(np.pi * kr * R + ph2)
        return out

    rho = 1.0 + field(amp)
    ux = field(amp)
    ur = field(amp) * R
    T = T_mean + field(T_amp)
    if noise > 0.0:  # (ur's noise also scaled by R)
        for a, scale in ((rho, amp), (ux, amp), (ur, amp * R), (T, T_amp)):
            a += (noise * scale) * rng.standard_normal(a.shape)
    return rho, ux, ur, T
