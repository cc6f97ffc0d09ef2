"""The single-jet tuner: best_shape returns a compiled shape of the asked
kind, caches it under the GPU architecture, precision and size class, and a
second call reads the cache instead of timing again."""
import json
import time

import pytest

from gpu_common import require_gpu, tiny_params

pytestmark = pytest.mark.gpu


def test_best_shape_picks_and_caches(tmp_path, monkeypatch):
    require_gpu()
    from paper_1002_3028_amd import autotune, lbm
    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(cache))
    p = tiny_params(256, 64, "jet", hoop=1)
    infos = lbm.tile_shape_infos()
    for steps in (1, 2):
        q = autotune.best_shape(p, None, "fp32", steps=steps)
        assert 0 <= q < len(infos) and infos[q]["steps"] == steps
        db = json.loads(cache.read_text())
        hit = [v for k, v in db.items() if k.endswith(f"/fp32/small/steps{steps}")]
        assert len(hit) == 1 and hit[0]["info"] == infos[q] and hit[0]["s_per_step"] > 0
        t0 = time.perf_counter()
        assert autotune.best_shape(p, None, "fp32", steps=steps) == q
        assert time.perf_counter() - t0 < 0.5  # read from the cache, not retimed
