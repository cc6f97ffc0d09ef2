"""Many jets in one persistent launch: each jet's result is bitwise the same
alone and in the mix (same kernel, no cross-jet arithmetic), jets finish at
their own step counts, admission respects the HBM budget, and jets admitted
while others run (continuous batching) are unaffected by their neighbours.
"""
import numpy as np
import pytest

from gpu_common import host_threads, noisy_inlet, rel_err, require_gpu, speed, tiny_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _jets():
    from paper_1002_3028_amd import inputs
    out = []
    for q, (nx, nr) in enumerate([(200, 45), (64, 16), (333, 70), (128, 32)]):
        p = tiny_params(nx, nr, "jet", q % 2)
        p["cs"] = 0.1 + 0.03 * q
        out.append((p, noisy_inlet(nr, 3 + q, q), 60 + 17 * q))
    p, inlet, _ = inputs.workload_small()
    out.append((p, inlet, 90))
    return out


def _moments_after(batch, slots):
    return {s: batch.moments(s) for s in slots}


@pytest.mark.parametrize("precision,cohort,streams", [
    ("fp32", 0, 2), ("fp16", 0, 2), ("fp32", 1 << 20, 1), ("fp32", 1 << 20, 2),
    ("fp32", 1 << 20, 3), ("fp16", 3 << 20, 1), ("fp16", 3 << 20, 2), ("fp16", 1 << 20, 4),
    ("fp16sr", 1 << 20, 2)])
def test_alone_equals_in_mix(precision, cohort, streams):
    """cohort = 0 puts every jet in one launch; a small cohort limit splits
    them into several cache-sized cohorts, run one after another on one
    stream or two at a time on two."""
    from paper_1002_3028_amd import lbm
    jets = _jets()
    with lbm.Batch(1 << 30, 16, precision) as mix:
        mix.set_cohort_bytes(cohort)
        mix.set_streams(streams)
        slots = [mix.admit(p, inlet, steps) for p, inlet, steps in jets]
        for _ in range(12):
            mix.run(10)
        assert [mix.poll(s) for s in slots] == [steps for _, _, steps in jets]
        mixed = _moments_after(mix, slots)
    for q, (p, inlet, steps) in enumerate(jets):
        with lbm.Batch(1 << 28, 2, precision) as alone:
            s = alone.admit(p, inlet, steps)
            alone.run(steps + 5)
            assert alone.poll(s) == steps
            m = alone.moments(s)
        for key in m:
            assert np.array_equal(m[key], mixed[slots[q]][key]), (q, key)


@pytest.mark.parametrize("cohort", [0, 1 << 20])
def test_storage_forms_mixed_in_one_batch(cohort):
    """Jets of four storage forms in one batch (its own FP16 and three
    others, admitted in interleaved order): each form runs in cohorts of its
    own, and every jet's result is bitwise the same as alone in a batch of
    its form."""
    from paper_1002_3028_amd import lbm
    jets = _jets()
    forms = ["fp32", "fp16sr", "fp16", "bf16", "fp16sr"]
    with lbm.Batch(1 << 30, 16, "fp16") as mix:
        mix.set_cohort_bytes(cohort)
        slots = [mix.admit(p, inlet, steps, precision=forms[q])
                 for q, (p, inlet, steps) in enumerate(jets)]
        for _ in range(12):
            mix.run(10)
        assert [mix.poll(s) for s in slots] == [steps for _, _, steps in jets]
        mixed = _moments_after(mix, slots)
    for q, (p, inlet, steps) in enumerate(jets):
        with lbm.Batch(1 << 28, 2, forms[q]) as alone:
            s = alone.admit(p, inlet, steps)
            alone.run(steps + 5)
            m = alone.moments(s)
        for key in m:
            assert np.array_equal(m[key], mixed[slots[q]][key]), (q, forms[q], key)


def test_batch_matches_single_solver_and_oracle():
    """A batched jet equals the single-jet solver bitwise and the oracle to
    the FP32 tolerance."""
    import oracle
    from paper_1002_3028_amd import lbm
    p, inlet, steps = _jets()[2]
    with lbm.Batch(1 << 28, 4, "fp32") as b:
        s = b.admit(p, inlet, steps)
        b.run(steps)
        mb = b.moments(s)
        pb = b.profiles(s)
    with lbm.Solver(p, "fp32") as g:
        g.set_inlet(*inlet)
        g.step(steps)
        mg = g.moments()
    for key in mg:
        assert np.array_equal(mb[key], mg[key]), key
    with oracle.RefSolver(p, threads=host_threads()) as r:
        r.set_inlet(*inlet)
        r.step(steps)
        mr = r.moments()
    assert rel_err(speed(mb), speed(mr)) < 1e-4 and rel_err(mb["T"], mr["T"]) < 1e-4
    np.testing.assert_array_equal(pb["ux_axis"], mb["ux"][0])
    np.testing.assert_array_equal(pb["T_exit"], mb["T"][:, -1])


def test_continuous_admission_and_retire():
    """Jets admitted while others are mid-run and slots reused after
    retirement give the same result as each jet alone."""
    from paper_1002_3028_amd import lbm
    jets = _jets()
    refs = []
    for p, inlet, steps in jets:
        with lbm.Batch(1 << 28, 2, "fp32") as alone:
            s = alone.admit(p, inlet, steps)
            alone.run(steps)
            refs.append(alone.moments(s))
    with lbm.Batch(1 << 30, 3, "fp32") as b:
        b.set_cohort_bytes(1 << 20)  # several cohorts, on the default two streams
        pending = list(range(len(jets)))
        live = {}
        done = {}
        rounds = 0
        while (pending or live) and rounds < 200:
            rounds += 1
            while pending:
                q = pending[0]
                p, inlet, steps = jets[q]
                rc, slot = b.try_admit(p, inlet, steps)
                if rc == lbm.ENOMEM:
                    break
                assert rc == lbm.OK
                live[slot] = q
                pending.pop(0)
            b.run(7)
            for slot, q in list(live.items()):
                if b.poll(slot) == jets[q][2]:
                    done[q] = b.moments(slot)
                    b.retire(slot)
                    del live[slot]
        assert len(done) == len(jets)
    for q in range(len(jets)):
        for key in refs[q]:
            assert np.array_equal(done[q][key], refs[q][key]), (q, key)


def test_stream_count_validated():
    from paper_1002_3028_amd import lbm
    with lbm.Batch(1 << 24, 2, "fp32") as b:
        for n in (0, 5, -1):
            with pytest.raises(lbm.LbmError) as e:
                b.set_streams(n)
            assert e.value.code == lbm.EINVAL
        for n in (1, 4, 2):
            b.set_streams(n)


def test_budget_admission():
    from paper_1002_3028_amd import lbm
    p = tiny_params(256, 64, "jet", 1)
    with lbm.Batch(1 << 24, 8, "fp32") as b:
        need = b.jet_bytes(p)
        n_fit = (1 << 24) // need
        slots = []
        for _ in range(n_fit):
            rc, s = b.try_admit(p, None, 10)
            assert rc == lbm.OK
            slots.append(s)
        rc, s = b.try_admit(p, None, 10)
        assert rc == lbm.ENOMEM and s == -1
        n_act, used = b.active()
        assert n_act == n_fit and used == n_fit * need
        b.retire(slots[0])
        rc, s = b.try_admit(p, None, 10)
        assert rc == lbm.OK
    with lbm.Batch(1 << 30, 2, "fp32") as b:
        b.admit(p, None, 5)
        b.admit(p, None, 5)
        rc, _ = b.try_admit(p, None, 5)
        assert rc == lbm.ENOMEM  # slot table full


def test_unstable_jet_fails_alone():
    """A runaway jet is flagged for its own slot only; its batch mates'
    results are unchanged."""
    from paper_1002_3028_amd import inputs, lbm
    good = _jets()[1]
    bad_p = tiny_params(64, 16, "jet", 0)
    bad_inlet = inputs.inlet_rows(16, 8.0, 0.9, 5.0)
    with lbm.Batch(1 << 28, 2, "fp32") as alone:
        s = alone.admit(*good)
        alone.run(good[2])
        ref = alone.moments(s)
    with lbm.Batch(1 << 28, 4, "fp32") as b:
        sg = b.admit(*good)
        sb = b.admit(bad_p, bad_inlet, 400)
        for _ in range(40):
            b.run(10)
        m = b.moments(sg)
        with pytest.raises(lbm.LbmError) as e:
            b.moments(sb)
        assert e.value.code == lbm.EUNSTABLE
    for key in ref:
        assert np.array_equal(m[key], ref[key])


@pytest.mark.parametrize("layout,steps_per_launch", [("two", 1), ("two", 2), ("single", 1)])
def test_any_grid_size(layout, steps_per_launch):
    """The tile walk hands every tile to exactly one workgroup whatever the grid
    size is against the tile count: grids from 8 workgroups (one per XCD, each
    walking its XCD's whole share) to 4096 (most of them idle) give the bits of
    the default grid, for the one-step, two-step and single-buffer kernels."""
    from paper_1002_3028_amd import lbm
    infos = lbm.tile_shape_infos()
    shape = [q for q, i in enumerate(infos) if i["steps"] == steps_per_launch][0]
    jets = _jets()
    runs = []
    for grid in (0, 8, 24, 136, 1288, 4096):
        with lbm.Batch(1 << 28, 8, "fp32", layout=layout) as b:
            b.set_launch(shape, grid)
            slots = [b.admit(p, inlet, steps) for p, inlet, steps in jets]
            for _ in range(4):
                b.run(30)
            assert [b.poll(s) for s in slots] == [steps for _, _, steps in jets], grid
            runs.append((grid, [b.moments(s) for s in slots]))
    base = runs[0][1]
    for grid, ms in runs[1:]:
        for q, (m, m0) in enumerate(zip(ms, base)):
            for key in m0:
                assert np.array_equal(m[key], m0[key]), (grid, q, key)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_tuned_batch_equals_default(tmp_path, monkeypatch, precision):
    """The batch tuner searches tile shape, grid, cohort size and streams on a
    set of jets, caches its pick under the set's key (a second call returns
    it without timing), and the tuned batch gives bitwise the moments of the
    batch with its default configuration."""
    from paper_1002_3028_amd import autotune, lbm
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    jets = _jets()
    infos = lbm.tile_shape_infos()
    # a quick search: the defaults' shapes plus one of each kind
    one = [q for q, i in enumerate(infos) if i["steps"] == 1][:2]
    two = [q for q, i in enumerate(infos) if i["steps"] == 2][-2:]
    cfg = autotune.tune_batch([(p, inlet) for p, inlet, _ in jets], precision, k_steps=10,
                              rounds=1, shapes=one + two)
    assert cfg["shape"] in one + two and cfg["trials"] > 10
    again = autotune.tune_batch([(p, inlet) for p, inlet, _ in jets], precision)
    assert {k: again[k] for k in ("shape", "workgroups", "cohort_mib", "streams")} == \
        {k: cfg[k] for k in ("shape", "workgroups", "cohort_mib", "streams")}
    assert "trials" in again  # read from the cache, not retimed
    out = []
    for c in (cfg, None):
        with lbm.Batch(1 << 30, 16, precision) as b:
            if c is not None:
                autotune.apply_batch(b, c)
            slots = [b.admit(p, inlet, steps) for p, inlet, steps in jets]
            for _ in range(10):
                b.run(11)
            out.append([b.moments(s) for s in slots])
    for q in range(len(jets)):
        for key in out[1][q]:
            assert np.array_equal(out[0][q][key], out[1][q][key]), (q, key)


def test_device_time_of_groups():
    """Every group queued and then waited on is timed once: the device time
    is positive and no more than the wall time around the groups."""
    import time
    from paper_1002_3028_amd import lbm
    jets = _jets()
    with lbm.Batch(1 << 30, 16, "fp32") as b:
        for p, inlet, steps in jets:
            b.admit(p, inlet, steps + 1000)
        b.run(10)
        b.sync()
        ms0, n0 = b.device_time()
        t0 = time.perf_counter()
        for _ in range(6):
            b.run(10)
            b.wait(1)
        b.sync()
        wall_ms = (time.perf_counter() - t0) * 1e3
        ms, n = b.device_time()
    assert n0 == 1 and n == 7
    assert 0.0 < ms - ms0 <= wall_ms, (ms - ms0, wall_ms)
