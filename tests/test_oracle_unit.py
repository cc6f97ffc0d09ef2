"""Node-level pins of the FP64 oracle.

Each check compares the oracle against something the paper or the mathematics
fixes independently of the oracle's own code: moment identities of the
equilibria (eq. 2), eq. (3) against the closed form of eq. (4), plain limits,
the collision invariants that the source terms must satisfy, and the table
lookup against numpy's linear interpolation.
"""
import math

import numpy as np
import pytest

from paper_1002_3028_amd import inputs

EX9 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
ER9 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
EX4 = np.array([1, 0, -1, 0])
ER4 = np.array([0, 1, 0, -1])


def _params(**kw):
    p = inputs.jet_params(8, 4, cs=0.15, table_seed=0)
    p.update(kw)
    return p


def test_equilibrium_moments(ref):
    """Eq. (2) moments of f^eq and g^eq: sum = rho (T), first moment = rho u
    (T u), second moment of f^eq = rho/3 I + rho u u; to 1e-13."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.2, 0.2, 2)
        T = rng.uniform(-1.0, 3.0)
        f = ref.feq(rho, u[0], u[1])
        g = ref.geq(T, u[0], u[1])
        assert abs(f.sum() - rho) <= 1e-13 * rho
        assert abs((EX9 * f).sum() - rho * u[0]) <= 1e-13 * rho
        assert abs((ER9 * f).sum() - rho * u[1]) <= 1e-13 * rho
        pxx = (EX9 * EX9 * f).sum()
        pxr = (EX9 * ER9 * f).sum()
        prr = (ER9 * ER9 * f).sum()
        assert abs(pxx - (rho / 3 + rho * u[0] ** 2)) <= 1e-13 * rho
        assert abs(pxr - rho * u[0] * u[1]) <= 1e-13 * rho
        assert abs(prr - (rho / 3 + rho * u[1] ** 2)) <= 1e-13 * rho
        scale = max(1.0, abs(T))
        assert abs(g.sum() - T) <= 1e-13 * scale
        assert abs((EX4 * g).sum() - T * u[0]) <= 1e-13 * scale
        assert abs((ER4 * g).sum() - T * u[1]) <= 1e-13 * scale
        # D2Q4 second moment: T c_s^2 I with c_s^2 = 1/2 (alpha = (tau-1/2)/2)
        assert abs((EX4 * EX4 * g).sum() - T / 2) <= 1e-13 * scale


def test_rest_equilibrium_is_weights(ref):
    f = ref.feq(1.0, 0.0, 0.0)
    np.testing.assert_allclose(f, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)
    np.testing.assert_allclose(ref.geq(1.0, 0.0, 0.0), [0.25] * 4, rtol=0, atol=1e-16)


def _random_pre(rng, rho=1.0, amp=0.02):
    u = rng.uniform(-0.08, 0.08, 2)
    f = ref_feq_np(rho, u) * (1 + amp * rng.standard_normal(9))
    g = 0.25 * rng.uniform(0.0, 1.0) * (1 + 2 * (EX4 * u[0] + ER4 * u[1])) * \
        (1 + amp * rng.standard_normal(4))
    return f, g


def ref_feq_np(rho, u):
    import oracle
    return oracle.feq(rho, u[0], u[1])


@pytest.mark.parametrize("cs", [0.1, 0.17, 0.5])
def test_quadratic_tau_solves_eq3(ref, cs):
    """Eq. (4) is the positive root of eq. (3): with S = -3 Q / (2 rho tau_tot)
    and |S| = sqrt(2 S:S), (tau_tot - 1/2)/3 = nu(T) + (C_s Delta)^2 |S|."""
    rng = np.random.default_rng(5)
    p = _params(cs=cs)
    nu_tab = p["nu_mult"]
    with ref.RefSolver(p) as s:
        for _ in range(100):
            f, g = _random_pre(rng)
            _, _, d = s.collide_node(f, g, r=3.5)
            rho = f.sum()
            feq = ref.feq(rho, (EX9 * f).sum() / rho, (ER9 * f).sum() / rho)
            q = np.array([[(EX9 * EX9 * (f - feq)).sum(), (EX9 * ER9 * (f - feq)).sum()],
                          [(EX9 * ER9 * (f - feq)).sum(), (ER9 * ER9 * (f - feq)).sum()]])
            tau = d["tau"]
            sbar = -3.0 * q / (2.0 * rho * tau)
            snorm = math.sqrt(2.0 * (sbar * sbar).sum())
            T = g.sum()
            nu = (p["tau_nu"] - 0.5) / 3.0 * np.interp(T, np.linspace(0, 1, nu_tab.size), nu_tab)
            lhs = (tau - 0.5) / 3.0
            rhs = nu + (cs * 1.0) ** 2 * snorm
            assert abs(lhs - rhs) <= 1e-13 * max(lhs, 1e-3)
            # eq. (5): alpha_tot = alpha + nu_t / Pr_t, tau_alpha from alpha_tot
            assert abs(d["nu_t"] - (cs ** 2) * snorm) <= 1e-13
            assert abs((d["tau_a"] - 0.5) / 2.0 - d["alpha_tot"]) <= 1e-14
            assert abs(d["alpha_tot"] - d["alpha"] - d["nu_t"] / p["pr_t"]) <= 1e-13


def test_cs_zero_gives_plain_bgk(ref):
    """C_s = 0: tau_tot = tau_nu(T) and tau_alpha_tot = tau_alpha(T)."""
    rng = np.random.default_rng(6)
    ones = np.ones(256)
    p = _params(cs=0.0, nu_mult=ones, alpha_mult=ones)
    with ref.RefSolver(p) as s:
        for _ in range(20):
            f, g = _random_pre(rng)
            _, _, d = s.collide_node(f, g, r=2.5)
            assert d["tau"] == p["tau_nu"]
            assert d["nu_t"] == 0.0
            assert abs(d["tau_a"] - p["tau_alpha"]) <= 1e-15


def test_collision_invariants_give_sources(ref):
    """Eq. (1): collisions conserve mass, momentum and T, so the change of the
    zeroth and first moments across one collision is exactly the sources:
    sum_k (f* - f) = theta (F1 split by weights), sum_k e_k (f* - f) = F
    (the e_ki F_2i / 6 weighting; sum_k e_kx^2 = 6), sum_k (g* - g) = S."""
    rng = np.random.default_rng(7)
    with ref.RefSolver(_params(cs=0.17, body_force_x=1e-4)) as s:
        for r in (0.5, 1.5, 7.5, 100.5):
            f, g = _random_pre(rng)
            fo, go, d = s.collide_node(f, g, r=r)
            assert abs((fo - f).sum() - d["theta"]) <= 1e-15
            assert abs((EX9 * (fo - f)).sum() - d["Fx"]) <= 1e-15
            assert abs((ER9 * (fo - f)).sum() - d["Fr"]) <= 1e-15
            assert abs((go - g).sum() - d["S"]) <= 1e-15
            # the mass source is the axisymmetric continuity term -rho u_r / r
            assert abs(d["theta"] + d["rho"] * d["ur"] / r) <= 1e-16


def test_sources_vanish_at_rest(ref):
    with ref.RefSolver(_params()) as s:
        f = ref.feq(1.0, 0.0, 0.0)
        g = ref.geq(0.7, 0.0, 0.0)
        fo, go, d = s.collide_node(f, g, r=0.5)
        # exact zero up to the rounding of rho = sum_k w_k
        for key in ("theta", "Fx", "Fr", "S"):
            assert abs(d[key]) <= 1e-15
        np.testing.assert_allclose(fo, f, rtol=0, atol=1e-15)
        np.testing.assert_allclose(go, g, rtol=0, atol=1e-17)


def test_table_lookup_matches_linear_interp(ref):
    """Eq. (6) tables: piecewise-linear on a uniform grid, clamped outside."""
    nu, al = inputs.property_tables(0)
    grid = np.linspace(0.0, 1.0, nu.size)
    # knots are exact
    for i in (0, 1, 17, 128, 254, 255):
        assert ref.table_lookup(nu, 0.0, 1.0, grid[i]) == pytest.approx(nu[i], abs=1e-15)
    rng = np.random.default_rng(3)
    for T in rng.uniform(-0.5, 1.5, 500):
        want = np.interp(T, grid, al)
        assert abs(ref.table_lookup(al, 0.0, 1.0, T) - want) <= 1e-13 * want
    # a table spanning another interval
    assert ref.table_lookup(np.array([1.0, 3.0]), 2.0, 4.0, 3.0) == pytest.approx(2.0)


def test_property_tables_shape():
    """Seeded stand-in for the N2-Ar curves: monotone, 1x -> 8x and 1x -> 20x."""
    nu, al = inputs.property_tables(0)
    assert nu.size == 256 and al.size == 256
    assert nu[0] == pytest.approx(1.0) and nu[-1] == pytest.approx(8.0)
    assert al[0] == pytest.approx(1.0) and al[-1] == pytest.approx(20.0)
    assert np.all(np.diff(nu) >= 0) and np.all(np.diff(al) >= 0)
    nu1, _ = inputs.property_tables(1)
    assert not np.allclose(nu, nu1)


def test_relaxation_relations(ref):
    """Text after eq. (1): nu = (tau_nu - 1/2)/3 and alpha = (tau_alpha - 1/2)/2
    (table multiplier 1 at T = t_lo)."""
    p = _params(tau_nu=0.8, tau_alpha=0.7, cs=0.0)
    with ref.RefSolver(p) as s:
        f = ref.feq(1.0, 0.01, 0.0)
        g = ref.geq(0.0, 0.01, 0.0)
        _, _, d = s.collide_node(f, g, r=4.5)
        assert d["nu"] == pytest.approx(0.1, abs=1e-15)
        assert d["alpha"] == pytest.approx(0.1, abs=1e-15)
        assert d["tau_nu"] == pytest.approx(0.8, abs=1e-15)
