"""One population buffer updated in place (AA pattern).

Every step does the one-step kernel's arithmetic on the same pulled values,
so the single-buffer layout must give exactly the bits of the two-buffer
scheme (shape 0): on every edge rule (periodic and equilibrium sides
included) and corner, in every precision, after odd and even step counts
(the two layouts of the buffer), with and without graphs.  Inlet rows, a
new state or populations loaded in either layout continue exactly;
checkpoints move between the layouts.  A batch in the single layout gives
each jet's two-buffer result and takes half the memory.  Direct parity with
the FP64 oracle as for the two-buffer path.
"""
import numpy as np
import pytest

from gpu_common import CASES, host_threads, noisy_inlet, rel_err, require_gpu, tiny_params

pytestmark = pytest.mark.gpu

GRIDS = [(200, 45), (40, 5), (65, 13)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _state0(p):
    from paper_1002_3028_amd import inputs
    return inputs.perturbed_state(p["nx"], p["nr"], seed=p["nx"] + 7 * p["nr"], r0=p["r0"],
                                  amp=0.02, T_mean=0.5, T_amp=0.2)


def _run(p, inlet, steps, precision, layout, **kw):
    from paper_1002_3028_amd import lbm
    with lbm.Solver(p, precision, layout=layout, **kw) as s:
        s.set_state(*_state0(p))
        if inlet is not None:
            s.set_inlet(*inlet)
        s.step(steps)
        f, g = s.get_populations()
        return f, g, s.moments(), s.profiles(), s.conservation()


def _same(a, b, what):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), what
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k]), (what, k)
    for k in a[3]:
        assert np.array_equal(a[3][k], b[3][k]), (what, k)
    assert a[4] == b[4], what


def _inlet(p, seed):
    return noisy_inlet(p["nr"], 5, seed) if p["bc"][0] == "inlet" else None


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16", "fp16sr"])
@pytest.mark.parametrize("case", CASES)
def test_single_equals_two_buffers(case, precision):
    for nx, nr in GRIDS:
        p = tiny_params(nx, nr, case, (nx + nr) % 2)
        inlet = _inlet(p, nx)
        for steps in (36, 37):
            ref = _run(p, inlet, steps, precision, "two", tile_shape=0)
            for gk in (0, 8):
                got = _run(p, inlet, steps, precision, "single", graph_steps=gk)
                _same(got, ref, (case, precision, nx, nr, steps, gk))


def test_single_buffer_takes_half_the_memory():
    from paper_1002_3028_amd import lbm
    p = tiny_params(300, 70, "jet", 1)
    for prec in ("fp32", "fp16"):
        assert 2 * lbm.bytes_required(p, prec, "single") == lbm.bytes_required(p, prec, "two")


def test_single_buffer_refuses_other_shapes():
    from paper_1002_3028_amd import lbm
    p = tiny_params(64, 16, "jet", 1)
    with lbm.Solver(p, "fp32", layout="single") as s:
        s.set_tile_shape(0)
        for q in range(1, len(lbm.tile_shapes())):
            with pytest.raises(lbm.LbmError) as e:
                s.set_tile_shape(q)
            assert e.value.code == lbm.EINVAL


@pytest.mark.parametrize("at", [30, 31])
@pytest.mark.parametrize("case", ["jet", "closed", "eq", "substrate"])
def test_checkpoints_between_layouts(case, at):
    """Populations saved after `at` steps in one layout, loaded into the other
    and run on: the same bits as an uninterrupted two-buffer run."""
    from paper_1002_3028_amd import lbm
    p = tiny_params(150, 30, case, 1)
    inlet = _inlet(p, 9)
    full = _run(p, inlet, at + 25, "fp32", "two", tile_shape=0)
    for src, dst in (("single", "two"), ("two", "single")):
        kw = {"tile_shape": 0} if src == "two" else {}
        with lbm.Solver(p, "fp32", layout=src, graph_steps=7, **kw) as a:
            a.set_state(*_state0(p))
            if inlet is not None:
                a.set_inlet(*inlet)
            a.step(at)
            f, g = a.get_populations()
        kw = {"tile_shape": 0} if dst == "two" else {}
        with lbm.Solver(p, "fp32", layout=dst, **kw) as b:
            if inlet is not None:
                b.set_inlet(*inlet)
            b.set_populations(f, g, at)
            b.step(25)
            f2, g2 = b.get_populations()
        assert np.array_equal(f2, full[0]) and np.array_equal(g2, full[1]), (src, dst)


@pytest.mark.parametrize("at", [12, 13])
def test_new_inlet_and_state_mid_run(at):
    """set_inlet and set_state after an even or odd number of steps (the
    buffer in either layout) continue exactly as with two buffers."""
    from paper_1002_3028_amd import inputs, lbm
    p = tiny_params(130, 33, "jet", 1)
    a_in, b_in = noisy_inlet(33, 4, 1), noisy_inlet(33, 6, 2)
    st2 = inputs.perturbed_state(130, 33, seed=77, amp=0.03, T_mean=0.4, T_amp=0.2)
    out = {}
    for layout in ("two", "single"):
        kw = {"tile_shape": 0} if layout == "two" else {}
        with lbm.Solver(p, "fp32", layout=layout, **kw) as s:
            s.set_state(*_state0(p))
            s.set_inlet(*a_in)
            s.step(at)
            s.set_inlet(*b_in)
            s.step(at + 3)
            s.set_state(*st2)
            s.step(9)
            out[layout] = s.get_populations()
    assert np.array_equal(out["two"][0], out["single"][0])
    assert np.array_equal(out["two"][1], out["single"][1])


def test_single_buffer_matches_oracle():
    import oracle
    from paper_1002_3028_amd import inputs, lbm
    p = tiny_params(200, 45, "jet", 1)
    inlet = noisy_inlet(45, 7, 3)
    st = inputs.perturbed_state(200, 45, seed=11, amp=0.02, T_mean=0.5, T_amp=0.2)
    with lbm.Solver(p, "fp32", layout="single", graph_steps=10) as g, \
            oracle.RefSolver(p, threads=host_threads()) as r:
        for s in (g, r):
            s.set_inlet(*inlet)
            s.set_state(*st)
            s.step(50)
        fg, gg = g.get_populations()
        fr, gr = r.get_populations()
    assert rel_err(fg, fr) < 3e-5 and rel_err(gg, gr) < 3e-5


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_batch_single_layout(precision):
    """Uneven jets (periodic and equilibrium sides among them) with odd and
    even targets in a single-layout batch: each equals itself alone in a
    two-buffer batch with one step per launch, at half the bytes per jet."""
    from paper_1002_3028_amd import lbm
    jets = []
    for q, (nx, nr, case, steps) in enumerate([(200, 45, "jet", 61), (64, 16, "closed", 62),
                                                (130, 33, "eq", 77), (90, 20, "annulus", 50),
                                                (70, 12, "xwalls", 41)]):
        p = tiny_params(nx, nr, case, q % 2)
        jets.append((p, _inlet(p, q), steps))
    refs = []
    for p, inlet, steps in jets:
        with lbm.Batch(1 << 28, 1, precision) as alone:
            alone.set_launch(0, 0)
            s = alone.admit(p, inlet, steps)
            alone.run(steps)
            refs.append(alone.moments(s))
    with lbm.Batch(1 << 30, 8, precision, layout="single") as b:
        with lbm.Batch(1 << 20, 1, precision) as two:
            assert 2 * b.jet_bytes(jets[0][0]) == two.jet_bytes(jets[0][0])
        slots = [b.admit(p, inlet, steps) for p, inlet, steps in jets[:3]]
        for _ in range(3):
            b.run(9)
        slots += [b.admit(p, inlet, steps) for p, inlet, steps in jets[3:]]
        for _ in range(10):
            b.run(7)
        assert [b.poll(s) for s in slots] == [st for _, _, st in jets]
        got = [b.moments(s) for s in slots]
    for n, (m, r) in enumerate(zip(got, refs)):
        for k in r:
            assert np.array_equal(m[k], r[k]), (n, k)
