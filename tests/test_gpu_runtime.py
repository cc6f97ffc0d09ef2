"""GPU runtime behaviour: launch variants give bitwise-identical results,
determinism, checkpoint/restart, error reporting."""
import numpy as np
import pytest

from gpu_common import noisy_inlet, require_gpu, tiny_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _run(p, inlet, steps, **kw):
    from paper_1002_3028_amd import lbm
    with lbm.Solver(p, "fp32", **kw) as s:
        s.set_inlet(*inlet)
        s.step(steps)
        return s.get_populations()


def test_tile_shapes_and_graphs_bitwise_identical():
    """The per-node arithmetic does not depend on the tile shape or on graph
    grouping, so every launch variant gives the same bits."""
    from paper_1002_3028_amd import lbm
    p = tiny_params(200, 45, "jet", 1)
    inlet = noisy_inlet(45, 5, 1)
    f0, g0 = _run(p, inlet, 37)
    for q in range(len(lbm.tile_shapes())):
        f, g = _run(p, inlet, 37, tile_shape=q)
        assert np.array_equal(f, f0) and np.array_equal(g, g0), q
    for k in (1, 8, 16):
        f, g = _run(p, inlet, 37, graph_steps=k)
        assert np.array_equal(f, f0) and np.array_equal(g, g0), k


@pytest.mark.parametrize("precision", ["fp32", "fp16sr"])
def test_step_calls_of_any_length(precision):
    """Calls of odd and even lengths, shorter and longer than a graph, with
    reads, an inlet change and a graph-size change in between: directly
    launched steps leave the device descriptor behind and pass the
    difference as arguments, graph replays catch it up first; the result is
    that of one call of one-step launches."""
    from paper_1002_3028_amd import lbm
    p = tiny_params(200, 45, "jet", 1)
    inlet, inlet2 = noisy_inlet(45, 5, 1), noisy_inlet(45, 3, 2)
    calls = (1, 3, 20, 50, 7, 2, 41, 1, 60, 5)
    assert lbm.tile_shape_info(0)["steps"] == 1  # the reference: one step per launch

    def ref():
        with lbm.Solver(p, precision, tile_shape=0) as s:
            s.set_inlet(*inlet)
            s.step(sum(calls[:5]))
            s.set_inlet(*inlet2)
            s.step(sum(calls[5:]))
            return s.get_populations()

    f0, g0 = ref()
    pair = [q for q, inf in enumerate(lbm.tile_shape_infos()) if inf["steps"] == 2][0]
    with lbm.Solver(p, precision, graph_steps=20, tile_shape=pair) as s:
        s.set_inlet(*inlet)
        for q, n in enumerate(calls):
            if q == 5:
                s.set_inlet(*inlet2)
            if q == 7:
                s.set_graph_steps(16)
            s.step(n)
            if q in (2, 6):
                s.conservation()
                s.profiles()
        assert s.step_count == sum(calls)
        f, g = s.get_populations()
    assert np.array_equal(f, f0) and np.array_equal(g, g0)


def test_deterministic_repeat():
    p = tiny_params(300, 64, "jet", 0)
    inlet = noisy_inlet(64, 3, 2)
    a = _run(p, inlet, 100, graph_steps=20)
    b = _run(p, inlet, 100, graph_steps=20)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_checkpoint_restart_bitwise():
    """2n steps == n steps, save populations, reload into a new solver, n steps."""
    from paper_1002_3028_amd import lbm
    p = tiny_params(96, 24, "jet", 1)
    inlet = noisy_inlet(24, 9, 3)
    full = _run(p, inlet, 60)
    with lbm.Solver(p, "fp32") as a:
        a.set_inlet(*inlet)
        a.step(30)
        f, g = a.get_populations()
    with lbm.Solver(p, "fp32") as b:
        b.set_inlet(*inlet)
        b.set_populations(f, g, 30)
        b.step(30)
        assert b.step_count == 60
        f2, g2 = b.get_populations()
    assert np.array_equal(f2, full[0]) and np.array_equal(g2, full[1])


def test_profiles_are_moment_slices():
    from paper_1002_3028_amd import lbm
    p = tiny_params(150, 40, "jet", 1)
    with lbm.Solver(p, "fp32") as s:
        s.set_inlet(*noisy_inlet(40, 1, 4))
        s.step(80)
        m, pr = s.moments(), s.profiles()
    np.testing.assert_allclose(pr["ux_axis"], m["ux"][0], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(pr["T_axis"], m["T"][0], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(pr["ux_exit"], m["ux"][:, -1], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(pr["T_exit"], m["T"][:, -1], rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("kernel", ["one_step", "two_steps", "single_buffer"])
def test_runaway_inlet_reports_unstable(kernel):
    """A supersonic inlet blows the jet up; every kernel (one or two steps
    per launch, single buffer) flags it and the next synchronising call
    reports LBM_EUNSTABLE, sticky until a new state."""
    from paper_1002_3028_amd import inputs, lbm
    p = tiny_params(64, 16, "jet", 0)
    pair = [q for q, i in enumerate(lbm.tile_shape_infos()) if i["steps"] == 2][0]
    kw = {"one_step": dict(tile_shape=0), "two_steps": dict(tile_shape=pair, graph_steps=10),
          "single_buffer": dict(layout="single")}[kernel]
    with lbm.Solver(p, "fp32", **kw) as s:
        s.set_inlet(*inputs.inlet_rows(16, 8.0, 0.9, 5.0))
        s.step(400)
        assert s.try_sync() == lbm.EUNSTABLE
        assert s.try_step(1) == lbm.EUNSTABLE
        rc, _ = s.try_moments()
        assert rc == lbm.EUNSTABLE
        n = 64 * 16
        s.set_state(np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n))
        assert s.try_step(1) == lbm.OK
        s.sync()


def test_rejects_nonfinite_state():
    from paper_1002_3028_amd import lbm
    p = tiny_params(16, 8, "jet", 0)
    with lbm.Solver(p, "fp32") as s:
        bad = np.ones(128)
        bad[5] = np.nan
        with pytest.raises(lbm.LbmError) as e:
            s.set_state(bad, np.zeros(128), np.zeros(128), np.zeros(128))
        assert e.value.code == lbm.EINVAL
