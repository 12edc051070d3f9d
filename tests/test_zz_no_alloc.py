"""The allocation-free trace entry point (grtx_trace_noalloc) against grtx_trace, through
the C ABI: three calls in a row on the same device scratch, each with fewer rays than the
one before (the last traces free rays and an image in one launch), each bit-identical to
grtx_trace's outputs, hit lists and blended counts (and rounds where no ray restarted
after a list compaction). Needs an MI355X."""
import sys

import numpy as np
import pytest

from paper_2601_20429_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_2601_20429_amd import grtx  # noqa: E402

AMIN = float(np.float32(1.0 / 255.0))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _outputs(R, cap, dev="cuda"):
    return dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=dev),
                depth=torch.empty(R, dtype=torch.float32, device=dev),
                opacity=torch.empty(R, dtype=torch.float32, device=dev),
                stats=torch.empty((R, grtx.STATS_FIELDS), dtype=torch.int32, device=dev),
                hit_ids=torch.full((R, cap), -1, dtype=torch.int32, device=dev),
                hit_counts=torch.empty(R, dtype=torch.int32, device=dev))


def same_counts(got, ref, label):
    # the counters that do not follow the scheduling (the others count work, which depends
    # on when a full checkpoint list was compacted)
    for f in (grtx.STAT_BLENDED, grtx.STAT_STACK_DROPS):
        assert torch.equal(got["stats"][:, f], ref["stats"][:, f]), (label, f)
    # rounds too, where neither launch restarted a ray from the root after a compaction
    ok = (got["stats"][:, grtx.STAT_FALLBACKS] == 0) & (ref["stats"][:, grtx.STAT_FALLBACKS] == 0)
    assert torch.equal(got["stats"][ok, grtx.STAT_ROUNDS], ref["stats"][ok, grtx.STAT_ROUNDS]), label


def test_noalloc_equals_trace_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    scene = inputs.cluster_scene(2, 100_000, 3)
    bvh = grtx.build(grtx.SceneTensors.from_scene(scene, "cuda"), alpha_min=AMIN)
    cases = [(inputs.orbit_camera(320, 240), grtx.CHECKPOINT), (inputs.orbit_camera(96, 64), grtx.RESTART)]
    for cam, mode in cases:
        say("noalloc", cam.width, cam.height, "mode", mode)
        o, d = grtx.pinhole_rays(cam)
        R = cam.n_rays
        ref = grtx.trace(bvh, o, d, k=16, T_min=1e-3, mode=mode, image_width=cam.width, stats=True,
                         hit_capacity=256)
        got = grtx.trace_noalloc(bvh, o, d, _outputs(R, 256), k=16, T_min=1e-3, mode=mode,
                                 image_width=cam.width)
        torch.cuda.synchronize()
        for key in ["rgb", "depth", "opacity", "hit_ids", "hit_counts"]:
            assert torch.equal(got[key], ref[key]), (cam.width, key)
        same_counts(got, ref, cam.width)
    # a third call, smaller still: 1000 free rays and a 64x48 image in one launch
    cam = inputs.orbit_camera(64, 48)
    say("noalloc", "1000 free rays +", cam.width, cam.height)
    po, pd = grtx.pinhole_rays(cam)
    fo, fd = (torch.from_numpy(a).cuda() for a in inputs.incoherent_rays(5, 1000))
    o, d = torch.cat([fo, po]), torch.cat([fd, pd])
    R = int(o.shape[0])
    ref = grtx.trace(bvh, o, d, k=16, T_min=1e-3, image_width=cam.width, image_begin=1000, stats=True,
                     hit_capacity=256)
    got = grtx.trace_noalloc(bvh, o, d, _outputs(R, 256), k=16, T_min=1e-3, image_width=cam.width,
                             image_begin=1000)
    torch.cuda.synchronize()
    for key in ["rgb", "depth", "opacity", "hit_ids", "hit_counts"]:
        assert torch.equal(got[key], ref[key]), ("one launch", key)
    same_counts(got, ref, "one launch")
    # list capacities beyond the scratch are refused before any launch
    o, d = grtx.pinhole_rays(inputs.orbit_camera(8, 8))
    with pytest.raises(grtx.GrtxError) as e:
        grtx.trace_noalloc(bvh, o, d, _outputs(64, 4), k=16, defer_capacity=1 << 20, evict_capacity=1 << 20)
    assert e.value.status == grtx.ERR_CAPACITY
