"""FP16 storage with stochastic rounding (fp16sr), through the C-ABI: values
written with lbm_set_populations are encoded by the device codec and read
back with lbm_get_populations.  The temperature planes with g_ref = 0 store
the value itself (zero offset), so the stored binary16 number is seen
directly.  Properties checked:

* every stored value is one of the two binary16 neighbours of the value
  (rounded toward zero, or one spacing away from zero);
* values that binary16 holds are stored unchanged (2^16 of them, normal and
  subnormal, both signs);
* the number of values rounded up matches the sum of their discarded
  fractions within 5 standard deviations of that binomial sum (unbiased);
* the rounding key is the node's and the step's: one value stored at every
  node rounds up at a share of them equal to its discarded fraction, writing
  the same data for the same step gives the same bits, and writing it for
  another step draws new keys (reproducible, and independent over steps);
* bit for bit, the stored number is what an independent model of the rule
  gives: the node and step hashed by the lowbias32 mixer, rotated by 7 bits
  per population, xor the value's FP32 bits; the top 13 bits r of that
  operand round the magnitude up when its discarded fraction of the binary16
  spacing plus r / 2^13 reaches one (normal and subnormal binary16 alike).
"""
import numpy as np
import pytest

from gpu_common import require_gpu, tiny_params

pytestmark = pytest.mark.gpu

NX, NR = 128, 128
N = 4 * NX * NR  # values per round trip (four g planes)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def solver():
    from paper_1002_3028_amd import lbm
    p = tiny_params(NX, NR, "jet", hoop=1)
    with lbm.Solver(p, "fp16sr", rho_ref=1.0, g_ref=0.0) as s:
        yield s


def _round_trip(s, g_values, step=0):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = np.broadcast_to(w[:, None, None], (9, NR, NX)).copy()
    s.set_populations(f, np.asarray(g_values, np.float64).reshape(4, NR, NX), step)
    return s.get_populations()[1].reshape(-1)


def _neighbours(v):
    """binary16 value of v rounded toward zero, and the next one away from zero."""
    h = v.astype(np.float16)
    lo = np.where(np.abs(h.astype(np.float64)) > np.abs(v), np.nextafter(h, np.float16(0)), h)
    hi = np.nextafter(lo, np.where(v < 0, np.float16(-np.inf), np.float16(np.inf)).astype(np.float16))
    return lo.astype(np.float64), hi.astype(np.float64)


def test_representable_values_unchanged(solver):
    rng = np.random.default_rng(11)
    m = rng.integers(1024, 2048, N)
    e = rng.integers(-14, 0, N)
    v = m * 2.0 ** (e - 10)
    sub = rng.random(N) < 0.25  # a quarter subnormal: n * 2^-24
    v[sub] = rng.integers(0, 1024, int(sub.sum())) * 2.0 ** -24
    v *= np.where(rng.integers(0, 2, N) == 1, -1.0, 1.0)
    got = _round_trip(solver, v)
    assert np.array_equal(got, v), int(np.sum(got != v))


def test_neighbours_and_unbiased(solver):
    rng = np.random.default_rng(12)
    # magnitudes log-uniform over [2^-20, 2^-2] (normal and subnormal binary16),
    # first rounded to FP32 so that the device sees the same value
    v = (2.0 ** rng.uniform(-20, -2, N) * np.where(rng.integers(0, 2, N) == 1, -1.0, 1.0))
    v = v.astype(np.float32).astype(np.float64)
    got = _round_trip(solver, v)
    lo, hi = _neighbours(v)
    assert np.all((got == lo) | (got == hi))
    up = got == hi
    phi = (np.abs(v) - np.abs(lo)) / (np.abs(hi) - np.abs(lo))
    normal = np.abs(lo) >= 2.0 ** -14
    for sel in (normal, ~normal):
        dev = float(np.sum(up[sel]) - np.sum(phi[sel]))
        sd = float(np.sqrt(np.sum(phi[sel] * (1 - phi[sel]))))
        print(f"{int(sel.sum())} values: {int(up[sel].sum())} up, expected {phi[sel].sum():.1f} "
              f"+- {sd:.1f}")
        # (below 2^-14 the offset steps are 2^-13 of the spacing: allow that)
        assert abs(dev) < 5 * sd + 2.0 ** -13 * sel.sum()


@pytest.mark.parametrize("phi", [j / 16 for j in range(1, 16)])
def test_fixed_fraction(solver, phi):
    """Values that all sit the same fraction phi of a spacing above a binary16
    number (every mantissa of 14 binades, both signs: 28 672 distinct values)
    round up in a fraction phi of cases."""
    m, e, sg = np.meshgrid(np.arange(1024, 2048), np.arange(-14, 0), [1.0, -1.0], indexing="ij")
    v = (sg * (m + phi) * 2.0 ** (e - 10)).reshape(-1)
    n = v.size
    up = (np.abs(_round_trip(solver, np.resize(v, N))) > np.abs(np.resize(v, N)))[:n]
    sd = np.sqrt(phi * (1 - phi) / n)
    print(f"phi {phi}: {up.mean():.4f} up of {n} (sd {sd:.4f})")
    assert abs(up.mean() - phi) < 5 * sd


@pytest.mark.parametrize("phi", [0.125, 0.5, 0.8125])
def test_one_value_everywhere(solver, phi):
    """One value at every node of the four planes: the share rounded up is
    its discarded fraction (the keys of 65 536 positions)."""
    v = (1024 + 301 + phi) * 2.0 ** -16  # a normal binary16 spacing of 2^-16
    got = _round_trip(solver, np.full(N, v))
    lo, hi = (1024 + 301) * 2.0 ** -16, (1024 + 302) * 2.0 ** -16
    assert np.all((got == lo) | (got == hi))
    up = float(np.mean(got == hi))
    sd = np.sqrt(phi * (1 - phi) / N)
    print(f"phi {phi}: {up:.4f} up of {N} (sd {sd:.4f})")
    assert abs(up - phi) < 5 * sd


def _lowbias32(x):
    """The lowbias32 integer mixer (C. Wellons, hash-prospector), on uint64
    arrays holding 32-bit values."""
    m = np.uint64(0xFFFFFFFF)
    x = x ^ (x >> np.uint64(16))
    x = (x * np.uint64(0x7FEB352D)) & m
    x = x ^ (x >> np.uint64(15))
    x = (x * np.uint64(0x846CA68B)) & m
    return x ^ (x >> np.uint64(16))


def _model_sr(v32, plane, step):
    """Binary16 value that stochastic rounding stores for FP32 values v32 of
    one population plane (shape NR x NX, node (i, j) at [j, i]) written for
    `step`, with a zero offset."""
    m = np.uint64(0xFFFFFFFF)
    j, i = np.meshgrid(np.arange(NR, dtype=np.uint64), np.arange(NX, dtype=np.uint64),
                       indexing="ij")
    key = _lowbias32(((j << np.uint64(16)) | i) ^ ((np.uint64(step) * np.uint64(0x9E3779B9)) & m))
    s = np.uint64((7 * plane) % 32)
    key = ((key >> s) | (key << (np.uint64(32) - s))) & m if s else key
    bits = v32.view(np.uint32).astype(np.uint64)
    r = ((bits ^ key) >> np.uint64(19)).astype(np.float64)
    a = np.abs(v32.astype(np.float64))
    # binary16 spacing at |v|: 2^(e - 10) in the normal range, 2^-24 below it
    e = np.frexp(a)[1] - 1  # a = 1.m * 2^e
    spacing = np.where(a >= 2.0 ** -14, np.ldexp(1.0, e - 10), 2.0 ** -24)
    lo = np.floor(a / spacing) * spacing
    up = (a - lo) / spacing + r / 8192.0 >= 1.0
    return np.sign(v32.astype(np.float64)) * (lo + up * spacing)


@pytest.mark.parametrize("step", [0, 7, 123457])
def test_rounding_rule_bitwise(solver, step):
    rng = np.random.default_rng(14 + step)
    v = 2.0 ** rng.uniform(-26, -1, N) * np.where(rng.integers(0, 2, N) == 1, -1.0, 1.0)
    v32 = v.astype(np.float32).reshape(4, NR, NX)
    got = _round_trip(solver, v32.astype(np.float64), step).reshape(4, NR, NX)
    for k in range(4):
        want = _model_sr(v32[k], 9 + k, step)
        bad = int(np.sum(got[k] != want))
        assert bad == 0, (k, bad)


def test_reproducible(solver):
    rng = np.random.default_rng(13)
    v = rng.uniform(-0.3, 0.3, N).astype(np.float32).astype(np.float64)
    a = _round_trip(solver, v, step=5)
    assert np.array_equal(_round_trip(solver, v, step=5), a)
    # another step, other keys: about half the values that do not sit on a
    # binary16 number round the other way (independent draws)
    b = _round_trip(solver, v, step=6)
    lo, hi = _neighbours(v)
    inexact = lo != v
    phi = (np.abs(v) - np.abs(lo)) / (np.abs(hi) - np.abs(lo))
    expect = float(np.sum((2 * phi * (1 - phi))[inexact]))
    differ = int(np.sum((a != b)[inexact]))
    print(f"{differ} of {int(inexact.sum())} differ, expected {expect:.0f}")
    assert abs(differ - expect) < 5 * np.sqrt(expect)
