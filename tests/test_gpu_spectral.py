"""GPU spectral cube (adaptive sampling along ln nu, the Sec. 6 extension of
the Sec. 3.2 rule) against the oracle.

- Thermal plasma, IQUV, 9 frequencies from 86 to 690 GHz (3 base, 2 spectral
  levels) on a 9^2 -> 33^2 grid, FP64: the oracle replays the GPU's level
  maps and every decision (spatial criterion and the axis check) its own
  rule takes differently must sit at a tie (margin < 1e-9); every image
  agrees with the replay to relative L2 1e-6; the same with the per-plane
  rule.
- A negative spectral tolerance reproduces plain adaptive renders at every
  frequency bitwise; statistics count spectral values and rays consistently;
  mixed precision stays within MSE 1e-3 of the FP64 oracle; invalid cubes
  are refused.
- Time: 5 snapshots of an evolving synthetic flow (gridded model) as a cube
  along t, against the oracle's cube on the same snapshots.
"""
import numpy as np
import pytest

import art_inputs
from gpu_helpers import ETA_FP64, ETA_MIXED, check_ties, nmse, rel_l2
from oracle import ray as oray
from oracle import spectral as osp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NU = (86e9, 690e9)


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def small_cfg(**kw):
    c = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 2), precision="fp64")
    c.update(kw)
    return c


def oracle_cube(cfg, n0, L, sr, forced=None):
    planes = cfg["nstokes"] + cfg.get("subrings", 0)
    fn_nu = lambda nu: (lambda x, y: oray.trace(dict(cfg, freq_hz=nu), x, y)[0])
    res, nus = osp.render_spectral(fn_nu, cfg["fov"], cfg["nx0"], cfg["ny0"], cfg["levels"], cfg["r_rel"],
                                   cfg["r_abs"], NU[0], NU[1], n0, L, sr[0], sr[1], cfg["abs_norm"], planes,
                                   all_planes=cfg.get("all_planes", False), forced_levels=forced)
    return res


@pytest.mark.parametrize("all_planes", [False, True])
def test_spectral_cube_parity(art, all_planes):
    print("CASE spectral cube parity", all_planes, flush=True)
    cfg = small_cfg(all_planes=all_planes)
    n0, L, sr = 3, 2, (0.01, 1e-3)
    imgs, levs, _, sts = art.render_spectral(cfg, NU[0], NU[1], n0, L, *sr)
    torch.cuda.synchronize()
    g = [i.cpu().numpy() for i in imgs]
    gl = [l.cpu().numpy() for l in levs]
    o = oracle_cube(cfg, n0, L, sr, forced=gl)
    for i in range(len(gl)):
        check_ties(o[i], gl[i], ETA_FP64, label=" (image %d)" % i)
    nspec = 0
    for i in range(len(g)):
        for s in range(4):
            assert rel_l2(g[i][s], o[i]["img"][s]) <= 1e-6, (i, s, rel_l2(g[i][s], o[i]["img"][s]))
        assert sts[i]["rays"] == int((gl[i] >= 0).sum()), i
        assert sts[i]["spectral"] == int((gl[i] == -3).sum()), i
        nspec += sts[i]["spectral"]
        if osp.spectral_level(i, L) == 0:
            assert sts[i]["spectral"] == 0
    assert nspec > 0


def test_negative_tolerance_is_plain_render(art):
    print("CASE spectral R=-1", flush=True)
    cfg = small_cfg(precision="mixed")
    imgs, levs, _, sts = art.render_spectral(cfg, NU[0], NU[1], 2, 2, -1.0, -1.0)
    nus = osp.frequencies(NU[0], NU[1], 2, 2)
    for i, nu in enumerate(nus):
        img, lev, _, st = art.render(dict(cfg, freq_hz=float(nu)))
        assert torch.equal(lev, levs[i]), i
        assert float((img - imgs[i]).abs().max()) <= 1e-12 * float(img.abs().max()), i
        assert sts[i]["spectral"] == 0 and sts[i]["rays"] == st["rays"]


def test_mixed_precision_cube(art):
    """Mixed-precision cube against the FP64 oracle: decisions off the
    oracle's own rule only at reduced-precision ties, every plane of every
    image within MSE 1e-3 of the oracle's replay and of its own cube."""
    print("CASE spectral mixed", flush=True)
    cfg = small_cfg()
    sr = (0.01, 1e-3)
    b, lv, _, s32 = art.render_spectral(dict(cfg, precision="mixed"), NU[0], NU[1], 3, 2, *sr)
    gl = [l.cpu().numpy() for l in lv]
    rep = oracle_cube(cfg, 3, 2, sr, forced=gl)
    own = oracle_cube(cfg, 3, 2, sr)
    for i, y in enumerate(b):
        check_ties(rep[i], gl[i], ETA_MIXED, label=" (image %d)" % i)
        y = y.cpu().numpy()
        for s in range(4):
            if np.abs(own[i]["img"][s]).max() > 0:
                e1, e2 = nmse(y[s], rep[i]["img"][s]), nmse(y[s], own[i]["img"][s])
                assert e1 <= 1e-3 and e2 <= 1e-3, (i, s, e1, e2)


def test_spectral_cube_saves_rays(art):
    print("CASE spectral saves rays", flush=True)
    cfg = small_cfg(precision="mixed")
    _, _, _, sa = art.render_spectral(cfg, NU[0], NU[1], 3, 2, 0.01, 1e-3)
    _, _, _, sp = art.render_spectral(cfg, NU[0], NU[1], 3, 2, -1.0, -1.0)
    assert sum(s["rays"] for s in sa) < sum(s["rays"] for s in sp)


def test_invalid_cubes(art):
    cfg = small_cfg()
    with pytest.raises(art.ArtError):
        art.render_spectral(cfg, NU[0], NU[1], 1, 2)
    with pytest.raises(art.ArtError):
        art.render_spectral(cfg, NU[0], NU[1], 9, 3)          # 65 images
    with pytest.raises(art.ArtError):
        art.render_spectral(cfg, NU[1], NU[0], 3, 1)


def test_time_cube_parity(art):
    """Adaptive sampling in time: 5 snapshots of the evolving synthetic flow
    (t = 0, 25, ..., 100 M; 3 base times, 1 level), gridded model, 17^2 ->
    65^2, FP64, against the oracle cube (ties replayed)."""
    from art_inputs import mks
    print("CASE time cube parity", flush=True)
    times = [0.0, 25.0, 50.0, 75.0, 100.0]
    grids, geo = mks.mks_movie(times, seed=2)
    gdev = [torch.from_numpy(g).cuda() for g in grids]
    base = dict(art_inputs.workload("grid_4097"), nx0=17, ny0=17, levels=2, nstokes=1, precision="fp64")
    cfgs = [dict(base, grid_dev=gd) for gd in gdev]
    sr = (0.05, 0.025)
    imgs, levs, _, sts = art.render_cube(cfgs, 3, 1, *sr)
    torch.cuda.synchronize()
    g = [i.cpu().numpy() for i in imgs]
    gl = [l.cpu().numpy() for l in levs]

    def oracle(forced=None):
        fn_k = lambda k: (lambda x, y: oray.trace(base, x, y, grid=grids[k])[0])
        return osp.render_cube(fn_k, base["fov"], base["nx0"], base["ny0"], base["levels"], base["r_rel"],
                               base["r_abs"], 3, 1, sr[0], sr[1], base["abs_norm"], 1, forced_levels=forced)
    o = oracle(forced=gl)
    for k in range(len(gl)):
        check_ties(o[k], gl[k], ETA_FP64, label=" (frame %d)" % k)
    for k in range(len(times)):
        assert rel_l2(g[k][0], o[k]["img"][0]) <= 1e-6, (k, rel_l2(g[k][0], o[k]["img"][0]))
        assert sts[k]["spectral"] == int((gl[k] == -3).sum())
    assert sum(s["spectral"] for s in sts) > 0


def test_cube_validation(art):
    cfg = small_cfg()
    with pytest.raises(art.ArtError):
        art.render_cube([cfg] * 4, 3, 1)                        # 4 != 5 images
    with pytest.raises(art.ArtError):
        art.render_cube([cfg] * 4 + [dict(cfg, nx0=11, ny0=11)], 3, 1)


def spectral_cfgs(cfg, n0, L):
    return [dict(cfg, freq_hz=float(nu)) for nu in osp.frequencies(NU[0], NU[1], n0, L)]


def test_cube_batch_equals_eager_cube(art):
    """The cube as a batch object (art_cube_create): an eager render, three
    graph replays and two cube batches in flight on two library streams all
    give the images, level maps and per-image statistics (axis order) of
    art_render_cube, bitwise."""
    print("CASE cube batch", flush=True)
    cfg = small_cfg(precision="mixed")
    n0, L, sr = 3, 2, (0.01, 1e-3)
    cfgs = spectral_cfgs(cfg, n0, L)
    want_i, want_l, _, want_s = art.render_cube(cfgs, n0, L, *sr)
    torch.cuda.synchronize()
    S1, S2 = art.Stream(), art.Stream()
    A = art.Batch(cfgs, cube=(n0, L) + sr)
    A.render(S1.torch)
    S1.torch.synchronize()
    for i in range(len(cfgs)):
        assert torch.equal(A.images[i], want_i[i]) and torch.equal(A.levels[i], want_l[i]), i
        st = A.stats(i, stream=S1.torch)
        assert st["rays"] == want_s[i]["rays"] and st["spectral"] == want_s[i]["spectral"], i
    B = art.Batch(cfgs, cube=(n0, L) + sr)
    for X, S in ((A, S1), (B, S2)):
        X.set_launch(256, 256, 1, 1)
        X.capture(S.torch)
    for rep in range(3):
        A.launch(S1.torch)
        B.launch(S2.torch)
        torch.cuda.synchronize()
        for X in (A, B):
            for i in range(len(cfgs)):
                assert torch.equal(X.images[i], want_i[i]) and torch.equal(X.levels[i], want_l[i]), (rep, i)
    assert A.stats(stream=S1.torch)["rays"] == sum(s["rays"] for s in want_s)
    A.close()
    B.close()
    S1.close()
    S2.close()


def test_cube_batch_rejects_network(art):
    cfg = small_cfg(precision="mixed")
    cfgs = spectral_cfgs(cfg, 3, 1)
    A = art.Batch(cfgs, cube=(3, 1, 0.01, 1e-3))
    net = art.Cnn(seed=1)
    with pytest.raises(art.ArtError):
        A.set_learned(net)
    A.close()
    net.close()
