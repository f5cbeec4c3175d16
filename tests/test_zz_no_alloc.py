"""The render entry point that allocates nothing (art_render_noalloc: the
library's static device scratch instead of library allocations), called
through the C ABI, against art_render on the same inputs: level maps, images
(every plane) and statistics equal bitwise, on two calls in a row with the
second image smaller than the first (the scratch keeps the first call's
contents), in FP64 and in the reduced-precision policy; an image above the
scratch's limit is refused before any device work."""
import numpy as np
import pytest

import art_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


STAT_KEYS = ("rays", "interp_frac", "n_abs", "steps", "steps_emit", "status", "learned")


@pytest.mark.parametrize("precision", ["fp64", "mixed_geo"])
def test_noalloc_equals_render_twice_shrinking(art, precision):
    print("CASE no-allocation render", precision, flush=True)
    big = dict(art_inputs.batch_workload()[63], precision=precision)           # 2049^2, 4 levels
    small = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 33, 2), precision=precision)
    for cfg in (big, small):
        ref_img, ref_lev, _, ref_st = art.render(cfg)
        out = art.alloc(cfg)
        img, lev, _, st = art.render_noalloc(cfg, out)
        torch.cuda.synchronize()
        print(cfg["name"], tuple(img.shape), "rays", st["rays"], flush=True)
        assert torch.equal(lev, ref_lev)
        assert torch.equal(img, ref_img)
        for k in STAT_KEYS:
            assert st[k] == ref_st[k], k


def test_noalloc_refuses_images_above_the_limit(art):
    cfg = dict(art_inputs.batch_workload()[63], nx0=257, ny0=257)             # 4097^2
    out = (torch.empty((1, 1, 1), dtype=torch.float64, device="cuda"),
           torch.empty((1, 1), dtype=torch.int8, device="cuda"), None)
    with pytest.raises(art.ArtError) as e:
        art.render_noalloc(cfg, out)
    assert "no-allocation limit" in str(e.value)
