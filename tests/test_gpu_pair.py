"""Two time steps per launch (LDS-blocked kernel).

The intermediate state is rounded through the storage codec, so a pair of
steps must give exactly the bits of two one-step launches (shape 0): on every
edge rule and corner (periodic x edges included: the frame wraps to the other
end of the domain, more than once on grids narrower than the frame), in every
precision, on grids with ragged tiles in both directions and grids smaller
than one tile, for odd step counts (a final single step), with and without
graphs, in a batch whose jets stop mid-pair, and across a checkpoint taken
after an odd number of steps.  The pair path is also compared with the FP64
oracle directly, at the one-step kernel's tolerance.
"""
import numpy as np
import pytest

from gpu_common import CASES, host_threads, noisy_inlet, rel_err, require_gpu, tiny_params

pytestmark = pytest.mark.gpu

# (nx, nr): ragged in x and r; narrower and lower than one tile; exact tiles;
# narrower than a third of the frame (a periodic frame wraps more than once)
GRIDS = [(200, 45), (40, 5), (128, 24), (65, 13), (20, 9)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _pair_shapes():
    from paper_1002_3028_amd import lbm
    return [q for q, inf in enumerate(lbm.tile_shape_infos()) if inf["steps"] == 2]


def _state(p, inlet, steps, precision, **kw):
    from paper_1002_3028_amd import inputs, lbm
    with lbm.Solver(p, precision, **kw) as s:
        st = inputs.perturbed_state(p["nx"], p["nr"], seed=p["nx"] + 7 * p["nr"], amp=0.02,
                                    T_mean=0.5, T_amp=0.2)
        s.set_state(*st)
        if inlet is not None:
            s.set_inlet(*inlet)
        s.step(steps)
        f, g = s.get_populations()
        m = s.moments()
        pr = s.profiles()
        mass = s.conservation()
    return f, g, m, pr, mass


def _same(a, b, what):
    fa, ga, ma, pa, ca = a
    fb, gb, mb, pb, cb = b
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb), what
    for k in ma:
        assert np.array_equal(ma[k], mb[k]), (what, k)
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), (what, k)
    assert ca == cb, what


def test_pair_shapes_compiled():
    from paper_1002_3028_amd import lbm
    infos = lbm.tile_shape_infos()
    pairs = _pair_shapes()
    assert len(pairs) >= 3
    for q in pairs:
        inf = infos[q]
        assert inf["bx"] == 64 and inf["by"] in (4, 8) and inf["nx"] == 1
        planes = 12 if inf["cache"] & 8 else 13  # bit 3: f_0 kept in registers
        assert inf["lds"] == planes * (inf["by"] * inf["ny"] + 2) * 66 * 4


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16", "fp16sr"])
@pytest.mark.parametrize("case", CASES)
def test_pair_equals_single(case, precision):
    for nx, nr in GRIDS:
        p = tiny_params(nx, nr, case, (nx + nr) % 2)
        inlet = noisy_inlet(nr, 5, nx) if p["bc"][0] == "inlet" else None
        ref = _state(p, inlet, 37, precision, tile_shape=0)
        for q in _pair_shapes():
            for gk in (0, 10):
                got = _state(p, inlet, 37, precision, tile_shape=q, graph_steps=gk)
                _same(got, ref, (case, precision, nx, nr, q, gk))


def test_pair_matches_oracle():
    """200 x 45 jet from a perturbed state, 50 steps with two steps per
    launch: populations within the one-step kernel's 50-step bound."""
    import oracle
    from paper_1002_3028_amd import inputs, lbm
    p = tiny_params(200, 45, "jet", 1)
    inlet = noisy_inlet(45, 7, 3)
    st = inputs.perturbed_state(200, 45, seed=11, amp=0.02, T_mean=0.5, T_amp=0.2)
    for q in _pair_shapes():
        with lbm.Solver(p, "fp32", tile_shape=q, graph_steps=10) as g, \
                oracle.RefSolver(p, threads=host_threads()) as r:
            for s in (g, r):
                s.set_inlet(*inlet)
                s.set_state(*st)
                s.step(50)
            fg, gg = g.get_populations()
            fr, gr = r.get_populations()
        assert rel_err(fg, fr) < 3e-5 and rel_err(gg, gr) < 3e-5, q


def test_pair_checkpoint_after_odd_steps():
    """31 steps, save, reload in a fresh solver at step 31, 30 more steps ==
    61 steps straight (both with two steps per launch)."""
    from paper_1002_3028_amd import lbm
    q = _pair_shapes()[0]
    p = tiny_params(150, 30, "substrate", 1)
    inlet = noisy_inlet(30, 9, 4)
    with lbm.Solver(p, "fp32", tile_shape=q, graph_steps=8) as a:
        a.set_inlet(*inlet)
        a.step(61)
        full = a.get_populations()
    with lbm.Solver(p, "fp32", tile_shape=q, graph_steps=8) as a:
        a.set_inlet(*inlet)
        a.step(31)
        f, g = a.get_populations()
    with lbm.Solver(p, "fp32", tile_shape=q) as b:
        b.set_inlet(*inlet)
        b.set_populations(f, g, 31)
        b.step(30)
        f2, g2 = b.get_populations()
    assert np.array_equal(f2, full[0]) and np.array_equal(g2, full[1])


def test_switch_shapes_mid_run():
    """Alternating one- and two-step shapes between calls keeps the bits."""
    from paper_1002_3028_amd import lbm
    p = tiny_params(100, 20, "jet", 0)
    inlet = noisy_inlet(20, 3, 5)
    ref = _state(p, inlet, 45, "fp32", tile_shape=0)
    qs = [0] + _pair_shapes()
    with lbm.Solver(p, "fp32", graph_steps=6) as s:
        from paper_1002_3028_amd import inputs
        s.set_state(*inputs.perturbed_state(100, 20, seed=100 + 140, amp=0.02, T_mean=0.5,
                                            T_amp=0.2))
        s.set_inlet(*inlet)
        done, k = 0, 0
        for n in (5, 7, 1, 12, 3, 17):
            s.set_tile_shape(qs[k % len(qs)])
            k += 1
            s.step(n)
            done += n
        assert done == 45
        got = s.get_populations()
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_batch_pairs_with_uneven_targets(precision):
    """Jets with odd and even targets, advanced in groups of 10 and 7 steps
    with a two-step shape: each jet equals itself alone (one-step kernel),
    a periodic jet admitted later included."""
    from paper_1002_3028_amd import lbm
    jets = []
    for q, (nx, nr, case, steps) in enumerate([(200, 45, "jet", 61), (64, 16, "xwalls", 62),
                                                (130, 33, "substrate", 77), (90, 20, "slab", 90),
                                                (70, 12, "closed", 41)]):
        p = tiny_params(nx, nr, case, q % 2)
        inlet = noisy_inlet(nr, 3 + q, q) if p["bc"][0] == "inlet" else None
        jets.append((p, inlet, steps))
    refs = []
    for p, inlet, steps in jets:
        with lbm.Batch(1 << 28, 1, precision) as alone:
            alone.set_launch(0, 0)
            s = alone.admit(p, inlet, steps)
            alone.run(steps)
            refs.append(alone.moments(s))
    for q in _pair_shapes():
        with lbm.Batch(1 << 30, 8, precision) as b:
            b.set_launch(q, 0)
            slots = [b.admit(p, inlet, steps) for p, inlet, steps in jets[:4]]
            for _ in range(4):
                b.run(10)
            late = b.admit(*jets[4])  # periodic
            for _ in range(8):
                b.run(7)
            got = [b.moments(s) for s in slots + [late]]
            assert [b.poll(s) for s in slots + [late]] == [st for _, _, st in jets]
        for n, (m, r) in enumerate(zip(got, refs)):
            for k in r:
                assert np.array_equal(m[k], r[k]), (q, n, k)
