"""GPU batches: many images through one work queue per level.

A batched image must be bitwise equal to the same image rendered alone (the
FP64 per-ray arithmetic does not depend on scheduling), a captured hipGraph
must reproduce the eager render on every replay, and the launch shape
(grid size, block size, refill threshold) must not change any result.
"""
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


def small_batch(precision="fp64"):
    cfgs = []
    for k, (a, inc, nu) in enumerate([(0.94, 163.0, 230e9), (0.0, 17.0, 86e9),
                                      (-0.94, 60.0, 345e9), (0.5, 90.0, 690e9)]):
        c = art_inputs.reduced(art_inputs.workload("thermal_1025"), 17, 1 + (k % 3))
        c.update(a=a, inc_deg=inc, freq_hz=nu, precision=precision)
        cfgs.append(c)
    return cfgs


def test_batch_equals_single(art):
    print("CASE batch equals single", flush=True)
    cfgs = small_batch()
    B = art.Batch(cfgs)
    B.render()
    st = B.stats()
    torch.cuda.synchronize()
    total = 0
    for i, c in enumerate(cfgs):
        img, lev, _, s1 = art.render(c)
        assert torch.equal(img, B.images[i]), i
        assert torch.equal(lev, B.levels[i]), i
        si = B.stats(i)
        assert si["rays"] == s1["rays"] and si["traced"] == s1["traced"]
        total += s1["rays"]
    assert st["rays"] == total
    B.close()


def test_batch_of_mixed_base_grids_equals_single(art):
    """Images with different (and non-square) base grids in one batch: the
    base-list and estimator launches are sized for the largest image, every
    other image uses its own grid; each image equals its single render."""
    print("CASE mixed base grids", flush=True)
    cfgs = []
    for k, (nx0, ny0, lv) in enumerate([(17, 17, 2), (9, 13, 3), (13, 5, 1), (5, 9, 2), (2, 3, 3)]):
        c = art_inputs.reduced(art_inputs.workload("thermal_1025"), nx0, lv)
        c.update(ny0=ny0, a=(0.94, 0.0, -0.5, 0.5, 0.9)[k], inc_deg=(163.0, 60.0, 90.0, 17.0, 120.0)[k],
                 precision="fp64")
        cfgs.append(c)
    for groups in (1, 2):
        B = art.Batch(cfgs)
        B.set_launch(groups=groups)
        B.render()
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            img, lev, _, s1 = art.render(c)
            assert torch.equal(img, B.images[i]), (groups, i)
            assert torch.equal(lev, B.levels[i]), (groups, i)
            assert B.stats(i)["rays"] == s1["rays"]
        B.close()


def test_batch_graph_replays(art):
    print("CASE batch graph replays", flush=True)
    cfgs = small_batch("mixed")
    B = art.Batch(cfgs)
    B.render()
    torch.cuda.synchronize()
    ref = [im.clone() for im in B.images]
    ref_lev = [lv.clone() for lv in B.levels]
    s = torch.cuda.Stream()
    B.capture(s)
    for rep in range(3):
        for im in B.images:
            im.fill_(-1.0)                  # eager work between replays
        torch.cuda.synchronize()
        B.launch(s)
        s.synchronize()
        for i in range(len(cfgs)):
            assert torch.equal(B.images[i], ref[i]), (rep, i)
            assert torch.equal(B.levels[i], ref_lev[i]), (rep, i)
    B.close()


def test_launch_shape_does_not_change_results(art):
    print("CASE launch shapes", flush=True)
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), 17, 2)
    ref, rlev, _, _ = art.render(cfg)
    try:
        for blocks, threads, refill, rb, ls in ((7, 64, 1, 0, 0), (300, 128, 8, 0, 0), (64, 256, 64, 0, 0),
                                                (256, 256, 1, 3, 1), (5, 128, 1, 192, 65535), (96, 256, 4, 64, 300)):
            art.set_launch(blocks, threads, refill, refine_blocks=rb, long_steps=ls)
            img, lev, _, _ = art.render(cfg)
            assert torch.equal(img, ref) and torch.equal(lev, rlev), (blocks, threads, refill, rb, ls)
    finally:
        art.set_launch(0, 0, 0)


def test_batch_rejects_mixed_kinds(art):
    c1 = art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 1)
    c2 = dict(c1, nstokes=1)
    with pytest.raises(art.ArtError):
        art.Batch([c1, c2])
    with pytest.raises(art.ArtError):
        art.Batch([c1] * 65)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_image_groups_do_not_change_results(art, precision):
    """Images split into groups with their own streams, counters and list
    slices: every image and statistic is bitwise the same for any group count,
    eager and from a captured graph."""
    print("CASE image groups", precision, flush=True)
    cfgs = small_batch(precision) + small_batch(precision)[::-1] + small_batch(precision)[1:]
    B = art.Batch(cfgs)
    B.set_launch(groups=1)
    B.render()
    torch.cuda.synchronize()
    ref = [im.clone() for im in B.images]
    ref_lev = [lv.clone() for lv in B.levels]
    ref_st = [B.stats(i) for i in range(len(cfgs))]
    s = torch.cuda.Stream()
    for groups in (2, 3, 4, 8):
        B.set_launch(groups=groups)
        assert B.get_launch()["groups"] == groups
        for im in B.images:
            im.fill_(-1.0)
        B.render()
        torch.cuda.synchronize()
        for i in range(len(cfgs)):
            assert torch.equal(B.images[i], ref[i]), (groups, i)
            assert torch.equal(B.levels[i], ref_lev[i]), (groups, i)
            st = B.stats(i)
            assert st["rays"] == ref_st[i]["rays"] and st["traced"] == ref_st[i]["traced"], (groups, i)
        B.capture(s)
        for rep in range(2):
            for im in B.images:
                im.fill_(-1.0)
            torch.cuda.synchronize()
            B.launch(s)
            s.synchronize()
            for i in range(len(cfgs)):
                assert torch.equal(B.images[i], ref[i]), (groups, rep, i)
    B.close()


def test_two_batches_in_flight(art):
    """Two batches replayed alternately on two library streams (concurrently)
    give, on every replay, images bitwise equal to one eager render."""
    print("CASE two batches in flight", flush=True)
    cfgs = small_batch("mixed")
    ref = art.Batch(cfgs)
    ref.render()
    torch.cuda.synchronize()
    want = [im.clone() for im in ref.images]
    ref.close()
    S1, S2 = art.Stream(), art.Stream()
    A, B = art.Batch(cfgs), art.Batch(cfgs)
    for X in (A, B):
        X.set_launch(256, 256, 1, 1)
    A.capture(S1.torch)
    B.capture(S2.torch)
    for k in range(6):
        (A if k % 2 == 0 else B).launch(S1.torch if k % 2 == 0 else S2.torch)
        if k % 2 == 1:
            torch.cuda.synchronize()
            for X in (A, B):
                for w, g in zip(want, X.images):
                    assert torch.equal(w, g)
    A.close()
    B.close()
    S1.close()
    S2.close()
