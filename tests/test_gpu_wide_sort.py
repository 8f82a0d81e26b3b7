"""GPU: the wide sort partitions (512-thread workgroups over 8192 keys) that
sorts of at least 2^23 32-bit keys use, against the 64-bit-key path (sort
variant 1, whose passes always run 256-thread workgroups over 4096 keys).

- Tile passes with generated keys and packed words, at over 2^23 tile keys.
- Depth passes, the packed last pass and its record gather, at over 2^23
  visible splats.

Keys, values, tile ranges, image, final transmittance and contributor counts
must agree bit for bit.  (The full-size workload, also on wide partitions, is
checked against the oracle on sampled pixels in the full-size tests.)
"""
import numpy as np
import pytest

from paper_2509_25626_amd import scenes as S
from tests.conftest import gpu_available
from tests.test_gpu_parity import R, gpu_render  # noqa: F401  (module fixture)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

WIDE_MIN = 1 << 23  # smallest sort run on wide partitions
WIDE_PART = 8192


def _same(R, scene, cam):
    a = gpu_render(R, scene, cam, sort_variant=1)
    b = gpu_render(R, scene, cam, sort_variant=2)
    assert a["K"] == b["K"]
    for k in ("keys", "values", "ranges", "image", "final_T", "n_contrib"):
        assert np.array_equal(a[k], b[k]), k
    return b


def test_wide_tile_passes(R):
    # large splats, ~700 tiles each: 20k of them give over 2^23 tile keys
    scene = S.scene_outdoor(30, 20_000, log_scale_mu=-1.2, log_scale_sigma=0.3)
    cam = S.orbit_camera(1237, 822, 4.0, 30.0, 0.0)
    b = _same(R, scene, cam)
    print(f"K={b['K']} n_vis={b['n_vis']}")
    assert b["K"] >= WIDE_MIN
    assert b["K"] % WIDE_PART != 0  # a ragged last partition


def test_wide_depth_passes(R):
    # 8.7M tiny splats, all in view: the depth sort runs over 2^23+ records
    rng = np.random.Generator(np.random.PCG64(32))
    n = 8_700_000
    means = rng.uniform(-2.0, 2.0, size=(3, n))
    scene = S.random_scene(rng, n, 0, means, -5.5, 0.3, 0.5, 1.5)
    cam = S.orbit_camera(512, 512, 10.0, 20.0, 10.0)
    b = _same(R, scene, cam)
    print(f"K={b['K']} n_vis={b['n_vis']}")
    assert b["n_vis"] >= WIDE_MIN
    assert b["n_vis"] % WIDE_PART != 0
