"""The seeded input generators shared by the oracle and the GPU path (no
method arithmetic): the node-level noise option of perturbed_state leaves the
smooth part alone and has the stated size and radial scaling."""
import numpy as np

from paper_1002_3028_amd import inputs


def test_noise_zero_is_the_smooth_state():
    a = inputs.perturbed_state(40, 12, seed=5)
    b = inputs.perturbed_state(40, 12, seed=5, noise=0.0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_noise_adds_node_level_gaussian_terms():
    nx, nr, amp, t_amp, noise = 400, 100, 0.02, 0.2, 0.5
    smooth = inputs.perturbed_state(nx, nr, seed=8, amp=amp, T_amp=t_amp)
    rough = inputs.perturbed_state(nx, nr, seed=8, amp=amp, T_amp=t_amp, noise=noise)
    r = ((np.arange(nr) + 0.5) / nr)[:, None]
    scales = (amp, amp, amp * r, t_amp)
    for x, y, s in zip(rough, smooth, scales):
        z = (x - y) / (noise * s)  # standard normal draws
        assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02
        # independent from node to node: neighbours are uncorrelated
        assert abs(np.corrcoef(z[:, 1:].ravel(), z[:, :-1].ravel())[0, 1]) < 0.02
    # u_r keeps vanishing towards the axis
    assert np.abs(rough[2][0]).max() < np.abs(rough[2][-1]).max() / 20


def test_noise_is_seeded():
    a = inputs.perturbed_state(30, 10, seed=3, noise=0.3)
    b = inputs.perturbed_state(30, 10, seed=3, noise=0.3)
    c = inputs.perturbed_state(30, 10, seed=4, noise=0.3)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])


def test_serving_route():
    """Only FP16 requests longer than the step limit change storage (by
    default every one); a negative limit turns routing off."""
    from paper_1002_3028_amd import serve
    lim = serve.FP16_STEP_LIMIT
    assert serve.route("fp16", lim + 1) == "fp16sr"
    assert serve.route("fp16", 1000) == "fp16sr"
    assert serve.route("fp16", 4000, long_after=4000) == "fp16"
    assert serve.route("fp16", 4001, long_after=4000) == "fp16sr"
    assert serve.route("fp16", 10000, long_after=-1) == "fp16"
    assert serve.route("fp16", 10000, long_after=4000, long_storage="fp32") == "fp32"
    for prec in ("fp32", "bf16", "fp16sr"):
        assert serve.route(prec, 10000) == prec
