"""Degenerate inputs of the method against the FP64 oracle, through every
kernel (one step per launch, two steps per launch, single buffer):

* C_s = 0 (plain LBGK, eq. 4 reduces to tau_nu), constant properties
  (no table), both, and tau close to 1/2;
* the smallest grid, 2 x 2, where every node is an edge node of both
  directions and every corner rule applies, for every edge-rule case;
* zero steps change nothing; a batch jet with a zero target stays at its
  initial state.
"""
import numpy as np
import pytest

from gpu_common import CASES, host_threads, noisy_inlet, rel_err, require_gpu, tiny_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _kernels(p):
    """(kwargs of lbm.Solver) for the three kernels."""
    from paper_1002_3028_amd import lbm
    infos = lbm.tile_shape_infos()
    pair = [q for q, i in enumerate(infos) if i["steps"] == 2 and i["cache"] == 8][0]
    return [dict(tile_shape=0), dict(layout="single"), dict(tile_shape=pair, graph_steps=4)]


def _compare(p, inlet, steps, tol):
    import oracle
    from paper_1002_3028_amd import inputs, lbm
    st = inputs.perturbed_state(p["nx"], p["nr"], seed=5, r0=p["r0"], amp=0.02, T_mean=0.5,
                                T_amp=0.2)
    with oracle.RefSolver(p, threads=host_threads()) as r:
        if inlet is not None:
            r.set_inlet(*inlet)
        r.set_state(*st)
        r.step(steps)
        fr, gr = r.get_populations()
    got = []
    for kw in _kernels(p):
        with lbm.Solver(p, "fp32", **kw) as s:
            if inlet is not None:
                s.set_inlet(*inlet)
            s.set_state(*st)
            s.step(steps)
            got.append(s.get_populations())
    for kw, (f, g) in zip(_kernels(p), got):
        ef, eg = rel_err(f, fr), rel_err(g, gr)
        print(f"{p['nx']}x{p['nr']} {p['bc']} {kw}: f {ef:.2e} g {eg:.2e}", flush=True)
        assert ef < tol and eg < tol, kw
        # the kernels agree with each other bit for bit
        assert np.array_equal(f, got[0][0]) and np.array_equal(g, got[0][1]), kw


@pytest.mark.parametrize("variant", ["no_les", "no_table", "neither", "tau_near_half"])
def test_degenerate_physics(variant):
    p = tiny_params(130, 33, "jet", 1)
    if variant in ("no_les", "neither"):
        p["cs"] = 0.0
    if variant in ("no_table", "neither"):
        p["nu_mult"] = p["alpha_mult"] = None
    if variant == "tau_near_half":
        p.update(tau_nu=0.505, tau_alpha=0.51)
    _compare(p, noisy_inlet(33, 3, 7), 20, 1e-5)


@pytest.mark.parametrize("case", CASES)
def test_smallest_grid(case):
    p = tiny_params(2, 2, case, 1)
    inlet = noisy_inlet(2, 3, 1) if p["bc"][0] == "inlet" else None
    _compare(p, inlet, 30, 1e-5)


def test_zero_steps_change_nothing():
    from paper_1002_3028_amd import lbm
    p = tiny_params(70, 12, "jet", 1)
    for kw in _kernels(p):
        with lbm.Solver(p, "fp32", **kw) as s:
            s.set_inlet(*noisy_inlet(12, 2, 3))
            s.step(5)
            f0, g0 = s.get_populations()
            s.step(0)
            f1, g1 = s.get_populations()
            assert s.step_count == 5
        assert np.array_equal(f0, f1) and np.array_equal(g0, g1), kw
    with lbm.Batch(1 << 26, 2, "fp32") as b:
        slot = b.admit(p, None, 0)
        b.run(10)
        assert b.poll(slot) == 0
        m = b.moments(slot)
        assert np.allclose(m["rho"], 1.0) and np.all(m["ux"] == 0.0)
