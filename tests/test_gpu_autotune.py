"""The launch-configuration autotuner: it returns one of its candidates,
caches per shape bucket, and the configuration it picks renders the same
values as the default one (launch configurations change speed only)."""
import numpy as np
import pytest
import torch

import scenes
from paper_2501_01677_amd.autotune import Autotuner, shape_key
from paper_2501_01677_amd.raster import Batch, RenderConfig
from gpu_common import device_scene

pytestmark = pytest.mark.gpu


def test_autotuner_picks_a_candidate_with_identical_outputs(tmp_path):
    print("[case] autotune", flush=True)
    subs = [scenes.small_scene(500 + k, n=300 + 200 * k, width=96, height=64, sh_degree=k % 4, n_views=2)
            for k in range(3)]
    sc = scenes.Scene([s.sets[0] for s in subs], [scenes.Render(k, rd.camera, rd.mask)
                                                  for k, s in enumerate(subs) for rd in s.renders])
    ref = device_scene(sc, RenderConfig(tile=16))
    ref.forward()
    tuner = Autotuner(cache_path=str(tmp_path / "tune.json"), steps=1)
    cfg, times = tuner.best(ref.sets, ref.renders)
    assert len(times) == len(tuner.candidates)
    assert any(cfg == c for c in tuner.candidates)
    assert shape_key(ref.sets, ref.renders) in tuner.cache
    # a second tuner reads the cache instead of tuning again
    cfg2, _ = Autotuner(cache_path=str(tmp_path / "tune.json")).best(ref.sets, ref.renders)
    assert cfg2 == cfg
    b = Batch(ref.sets, ref.renders, cfg)
    b.forward()
    torch.cuda.synchronize()
    for r in range(len(sc.renders)):
        for k in ("rgb", "normal", "dist", "depth", "alpha", "n_contrib"):
            assert torch.equal(b.out[r][k], ref.out[r][k]), (r, k, cfg)
