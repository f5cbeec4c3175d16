"""Full-size parity of the timed configuration: the 64-image thermal batch at
1025^2 (base 129^2, 3 levels, IQUV, mixed precision), three batches in flight
on library streams with one image group and a 256 x 256 persistent grid per
batch (the in-flight launch shape the benchmark times).

- The three batches, replayed round robin, give bitwise equal images on every
  replay, and two of the images equal a single eager render of that image.
- Sampled traced points (base-level and refined, four images spanning spin,
  inclination and frequency) agree with the oracle's FP64 ray tracer point by
  point: relative L2 over the samples <= 1e-4 on every Stokes plane (the
  mixed-precision transfer is good to ~1e-6 per ray on this workload).
- Every pixel is either traced (level >= 0) or interpolated (-1), and the
  statistics count exactly the traced pixels.
"""
import numpy as np
import pytest

import art_inputs
from gpu_helpers import ETA_FP64, ETA_MIXED, check_adaptive, check_ties, nmse, oracle_adaptive, rel_l2
from oracle import ray as oray

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAUNCH = (256, 256, 1, 1)
DEPTH = 3
SAMPLED = (0, 21, 42, 63)


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


@pytest.fixture(scope="module")
def rendered(art):
    print("CASE full-size batch in flight", LAUNCH, DEPTH, flush=True)
    cfgs = art_inputs.batch_workload_1025(precision="mixed")
    streams = [art.Stream() for _ in range(DEPTH)]
    batches = [art.Batch(cfgs) for _ in range(DEPTH)]
    for B, S in zip(batches, streams):
        B.set_launch(*LAUNCH)
        B.capture(S.torch)
    ref, same = None, True
    for rep in range(2):
        for B, S in zip(batches, streams):
            B.launch(S.torch)
        torch.cuda.synchronize()
        if ref is None:
            ref = [im.clone() for im in batches[0].images]
        same = same and all(torch.equal(a, b) for B in batches for a, b in zip(ref, B.images))
    st = batches[0].stats(stream=streams[0].torch)
    levels = [lv.clone() for lv in batches[0].levels]
    yield cfgs, ref, same, levels, st
    for B in batches:
        B.close()
    for S in streams:
        S.close()


def test_in_flight_replays_bitwise_equal(rendered):
    _, _, same, _, _ = rendered
    assert same


def test_batch_equals_single_render(art, rendered):
    cfgs, ref, _, levels, _ = rendered
    for k in (5, 58):
        img, lev, _, _ = art.render(cfgs[k])
        torch.cuda.synchronize()
        assert torch.equal(lev, levels[k]), k
        assert torch.equal(img, ref[k]), k


def test_sampled_traced_points_match_oracle(rendered):
    cfgs, ref, _, levels, _ = rendered
    rng = np.random.default_rng(11)
    for k in SAMPLED:
        cfg = cfgs[k]
        lev = levels[k].cpu().numpy()
        img = ref[k].cpu().numpy()
        ny, nx = lev.shape
        step0 = 1 << cfg["levels"]
        pts = []
        for lvl in range(cfg["levels"] + 1):
            jj, ii = np.nonzero(lev == lvl)
            if lvl == 0:
                # base points lie on the coarse lattice
                assert np.all(jj % step0 == 0) and np.all(ii % step0 == 0)
            if len(ii):
                pick = rng.choice(len(ii), size=min(12, len(ii)), replace=False)
                pts += [(ii[p], jj[p]) for p in pick]
        ii = np.array([p[0] for p in pts])
        jj = np.array([p[1] for p in pts])
        x, y = oray.screen_coords(cfg["fov"], nx, ny, ii, jj)
        want, _ = oray.trace(cfg, x, y)
        got = img[:, jj, ii].T
        print("image", k, "samples", len(ii), flush=True)
        for s in range(cfg["nstokes"]):
            assert rel_l2(got[:, s], want[:, s]) <= 1e-4, (k, s, rel_l2(got[:, s], want[:, s]))


def test_levels_and_statistics(rendered):
    cfgs, ref, _, levels, st = rendered
    traced = 0
    for k, lev in enumerate(levels):
        lv = lev.cpu().numpy()
        assert lv.shape == (1025, 1025)
        assert np.all((lv >= -1) & (lv <= cfgs[k]["levels"])), k
        assert np.all(lv[::8, ::8] == 0), k
        traced += int((lv >= 0).sum())
    assert st["rays"] == traced
    for img in ref:
        assert bool(torch.isfinite(img).all())


# --------------------------------------------------------------------------
# Whole images at the timed size, thermal view (129^2 -> 1025^2): FP64 and
# both reduced-precision policies against the oracle.  The oracle replays the
# GPU's level map, tracing every ray itself; every decision its own rule
# (Sec. 3.2) takes differently from the GPU's must sit at a tie, and the whole
# image must agree with the replay: relative L2 <= 1e-6 per Stokes plane in
# FP64, normalised MSE <= 1e-3 per plane for the reduced-precision forms, which
# are also held to the oracle's own adaptive FP64 image.

@pytest.fixture(scope="module")
def thermal_oracle():
    cfg = art_inputs.workload("thermal_1025")
    return oracle_adaptive(cfg)


def test_thermal_1025_fp64_whole_image(art, thermal_oracle):
    print("CASE thermal_1025 FP64 whole image", flush=True)
    cfg = dict(art_inputs.workload("thermal_1025"), precision="fp64")
    g, gl, st, rep = check_adaptive(art, cfg, 1e-6)
    print("rays", st["rays"], "oracle's own render", thermal_oracle["rays"],
          "level-map differences", int((gl != thermal_oracle["level"]).sum()), flush=True)
    for s in range(4):
        print("plane", s, "rel L2 vs replay", rel_l2(g[s], rep["img"][s]), flush=True)


@pytest.mark.parametrize("precision", ["mixed", "mixed_geo"])
def test_thermal_1025_reduced_precision_whole_image(art, thermal_oracle, precision):
    print("CASE thermal_1025 whole image", precision, flush=True)
    cfg = dict(art_inputs.workload("thermal_1025"), precision=precision)
    g, gl, st, rep = check_adaptive(art, cfg, 1e-2, eta=ETA_MIXED)
    for s in range(4):
        e1, e2 = nmse(g[s], rep["img"][s]), nmse(g[s], thermal_oracle["img"][s])
        print("plane", s, "mse vs replay", e1, "vs oracle's own image", e2, flush=True)
        assert e1 <= 1e-3 and e2 <= 1e-3, (s, e1, e2)


# --------------------------------------------------------------------------
# The uneven batch: the same 64 combinations with 1 + (k mod 4) levels
# (257^2 ... 2049^2 final grids) in one captured graph, FP32 transfer with
# FP64 geodesic right-hand sides only in the sensitive zones (photon shell,
# horizon, theta turning points), three batches in flight at the launch
# shape the benchmark times.

UNEVEN_PRECISION = "mixed_geo"


@pytest.fixture(scope="module")
def uneven(art):
    print("CASE full-size uneven batch", UNEVEN_PRECISION, flush=True)
    cfgs = art_inputs.batch_workload(precision=UNEVEN_PRECISION)
    Ss = [art.Stream() for _ in range(DEPTH)]
    Bs = [art.Batch(cfgs) for _ in range(DEPTH)]
    for B, S in zip(Bs, Ss):
        B.set_launch(*LAUNCH)
        B.capture(S.torch)
    for B, S in zip(Bs, Ss):
        B.launch(S.torch)
    torch.cuda.synchronize()
    imgs = [im.clone() for im in Bs[0].images]
    levels = [lv.clone() for lv in Bs[0].levels]
    same = all(torch.equal(a, b) for B in Bs[1:] for a, b in zip(imgs, B.images))
    st = Bs[0].stats(stream=Ss[0].torch)
    for B in Bs:
        B.close()
    for S in Ss:
        S.close()
    yield cfgs, imgs, levels, st, same


def test_uneven_batch_in_flight_identical(uneven):
    assert uneven[4]


@pytest.mark.parametrize("chunk", range(4))
def test_uneven_batch_whole_images_vs_oracle(uneven, chunk):
    """Every image of the batch, whole: the oracle replays its level map; the
    decisions its own rule takes differently sit at reduced-precision ties
    and every Stokes plane is within MSE 1e-3 of the replay."""
    cfgs, imgs, levels, _, _ = uneven
    for k in range(16 * chunk, 16 * chunk + 16):
        gl = levels[k].cpu().numpy()
        g = imgs[k].cpu().numpy()
        print("image", k, cfgs[k]["name"], "levels", cfgs[k]["levels"], "rays", int((gl >= 0).sum()),
              flush=True)
        rep = oracle_adaptive(cfgs[k], forced=gl)
        check_ties(rep, gl, ETA_MIXED, label=" (image %d)" % k)
        for s in range(4):
            e = nmse(g[s], rep["img"][s])
            assert e <= 1e-3, (k, s, e)


def test_uneven_batch_2049_fp64_whole_image(art):
    """The batch's hardest view at 2049^2 (a = -0.94, i = 163 deg, 690 GHz,
    4 levels) in FP64: decisions up to ties of 1e-9, whole image within
    relative L2 1e-6 of the oracle's replay."""
    print("CASE uneven batch image 63 FP64 whole image", flush=True)
    cfg = dict(art_inputs.batch_workload()[63], precision="fp64")
    g, gl, st, rep = check_adaptive(art, cfg, 1e-6)
    assert gl.shape == (2049, 2049)


def test_uneven_batch_levels_and_sizes(art, uneven):
    cfgs, imgs, levels, st, _ = uneven
    traced = 0
    for k, (img, lev) in enumerate(zip(imgs, levels)):
        L = cfgs[k]["levels"]
        n = 128 * (1 << L) + 1
        assert tuple(img.shape) == (4, n, n) and tuple(lev.shape) == (n, n), k
        lv = lev.cpu().numpy()
        assert np.all((lv >= -1) & (lv <= L)), k
        assert np.all(lv[:: 1 << L, :: 1 << L] == 0), k
        traced += int((lv >= 0).sum())
        assert bool(torch.isfinite(img).all()), k
    assert st["rays"] == traced


def test_uneven_batch_equals_single_and_oracle(art, uneven):
    cfgs, imgs, levels, _, _ = uneven
    rng = np.random.default_rng(12)
    for k in (1, 22, 43, 60):                      # 2, 3, 4, 1 levels
        cfg = cfgs[k]
        img, lev, _, _ = art.render(cfg)
        torch.cuda.synchronize()
        assert torch.equal(lev, levels[k]), k
        assert torch.equal(img, imgs[k]), k
        lv = lev.cpu().numpy()
        g = img.cpu().numpy()
        ny, nx = lv.shape
        jj, ii = np.nonzero(lv >= 0)
        pick = rng.choice(len(ii), size=min(40, len(ii)), replace=False)
        ii, jj = ii[pick], jj[pick]
        x, y = oray.screen_coords(cfg["fov"], nx, ny, ii, jj)
        want, _ = oray.trace(cfg, x, y)
        got = g[:, jj, ii].T
        for s in range(4):
            assert rel_l2(got[:, s], want[:, s]) <= 1e-4, (k, s, rel_l2(got[:, s], want[:, s]))


@pytest.mark.parametrize("precision", ["mixed", "mixed_geo"])
def test_uneven_batch_image_error(art, precision):
    """Every image of the uneven batch within the 0.1 % bar (Eq. 9) of its
    uniform full-resolution render, plain criterion at R_rel = 0.005 (on this
    batch the plain criterion reaches the bar from R_rel = 0.0075 down; at
    0.01 its worst image sits at 1.08e-3).  Measured with MIXED_GEO: largest
    5.0e-4."""
    import bench
    print("CASE uneven batch image error", precision, flush=True)
    cfgs = [dict(c, r_rel=0.005) for c in art_inputs.batch_workload(precision=precision)]
    B = art.Batch(cfgs)
    B.render()
    truths = []
    for c in cfgs:
        t, _, _ = art.render_uniform(c)
        truths.append(t[0].clone())
        del t
    chk = bench.mse_check(art, cfgs, B.images, truths)
    print("mse max", chk["mse_max"], "worst", chk["worst"], "mean", chk["mse_mean"], flush=True)
    assert chk["mse_ok"] and chk["n_over_bar"] == 0, chk
    B.close()


# --------------------------------------------------------------------------
# What the trained network gains at the 0.1 % bar, with the benchmark's
# held-out protocol: on the held-out batch (other spins, inclinations and
# field phases, the same structure as the uneven batch) the plain criterion
# misses the bar even at the grid's tightest R_rel (one image keeps an error
# floor: features the base grid does not see), while the look-ahead forms
# (proposal threshold z = 4 with the criterion as fallback, and z = 2 with
# the criterion as judge only) pass at R_rel = 0.005; applied unchanged to
# the uneven batch they pass there too.  The network is trained on the
# batch-structured training set (four frequencies, both network levels).

def test_learned_operating_point_gain(art):
    from paper_2103_07417_amd import learn
    import bench
    print("CASE learned operating point (held-out protocol)", flush=True)
    S = art.Stream()
    s = S.torch
    net, _ = learn.train(art_inputs.training_workload_batch(precision="mixed", r_rel=bench.TRAIN_RREL),
                         steps=300, lr=3e-3, seed=4, stream=s)
    res = {}
    for name, cfgs in (("heldout", art_inputs.batch_workload_heldout(precision=UNEVEN_PRECISION)),
                       ("timed", art_inputs.batch_workload(precision=UNEVEN_PRECISION))):
        truths = []
        for c in cfgs:
            t, _, _ = art.render_uniform(c, stream=s)
            truths.append(t.clone())
            del t
        s.synchronize()
        for form, rr in (("plain", min(bench.OP_RREL)), ("lookahead", 0.005), ("judge", 0.005)):
            B = art.Batch([dict(c, r_rel=rr) for c in cfgs], feat=True)
            if form == "plain":
                B.set_learned(None)
            elif form == "lookahead":
                B.set_learned(net, z_propose=4.0, z_suppress=-float("inf"), fallback=True)
            else:
                B.set_learned(net, z_propose=2.0, z_suppress=-float("inf"), fallback=False)
            B.render(s)
            st = B.stats(stream=s)
            chk = bench.mse_check(art, cfgs, B.images, truths)
            res[(name, form)] = (st["rays"], chk["mse_max"], chk["mse_ok"], chk["worst"])
            print(name, form, rr, res[(name, form)], flush=True)
            B.close()
        del truths
    net.close()
    S.close()
    assert not res[("heldout", "plain")][2]
    assert res[("heldout", "lookahead")][2] and res[("heldout", "judge")][2]
    assert res[("timed", "lookahead")][2] and res[("timed", "judge")][2] and res[("timed", "plain")][2]


# --------------------------------------------------------------------------
# The gridded snapshot at its full sizes: 4097^2 IQUV (base 257^2, 4 levels,
# mixed precision) and 16385^2 Stokes I with subring planes n = 0..3 (6
# levels), single adaptive renders: sampled traced points of every level
# against the oracle's FP64 tracer on the same snapshot.

@pytest.fixture(scope="module")
def snapshot():
    from art_inputs import mks
    grid, _ = mks.mks_snapshot(seed=2)
    return grid, torch.from_numpy(grid).cuda()


def sampled_vs_oracle(cfg, img, lev, grid, per_level, seed, tol):
    rng = np.random.default_rng(seed)
    lv = lev.cpu().numpy()
    ny, nx = lv.shape
    ii, jj = [], []
    for lvl in range(cfg["levels"] + 1):
        j, i = np.nonzero(lv == lvl)
        if len(i):
            pick = rng.choice(len(i), size=min(per_level, len(i)), replace=False)
            ii += list(i[pick])
            jj += list(j[pick])
    ii, jj = np.array(ii), np.array(jj)
    got = img[:, jj, ii].cpu().numpy().T
    x, y = oray.screen_coords(cfg["fov"], nx, ny, ii, jj)
    want, _ = oray.trace(cfg, x, y, grid=grid)
    planes = cfg["nstokes"] + cfg.get("subrings", 0)
    for s in range(planes):
        err = rel_l2(got[:, s], want[:, s])
        print("plane", s, "samples", len(ii), "rel L2", err, flush=True)
        assert err <= tol, (s, err)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_grid_4097_whole_image(art, snapshot, precision):
    """The snapshot at 4097^2 (base 257^2, 4 levels, IQUV), whole image: the
    oracle replays the GPU's level map on the same snapshot; decisions off
    its own rule only at ties (1e-9 in FP64, reduced-precision ties in the
    mixed form); relative L2 <= 1e-6 per plane in FP64, MSE <= 1e-3 mixed."""
    print("CASE grid 4097 whole image", precision, flush=True)
    cfg = dict(art_inputs.workload("grid_4097"), grid_dev=snapshot[1], precision=precision)
    fp64 = precision == "fp64"
    g, gl, st, rep = check_adaptive(art, cfg, 1e-6 if fp64 else 1e-2, grid=snapshot[0],
                                    eta=ETA_FP64 if fp64 else ETA_MIXED)
    assert gl.shape == (4097, 4097)
    for s in range(4):
        e = nmse(g[s], rep["img"][s])
        print("plane", s, "mse vs replay", e, flush=True)
        assert e <= 1e-3


def test_grid_16385_subrings_sampled(art, snapshot):
    print("CASE grid 16385 subrings full size", flush=True)
    cfg = dict(art_inputs.workload("grid_16385"), grid_dev=snapshot[1], precision="mixed")
    img, lev, _, st = art.render(cfg)
    torch.cuda.synchronize()
    assert tuple(lev.shape) == (16385, 16385) and st["rays"] == int((lev >= 0).sum())
    # the subring planes add up to the image (every step's increment goes to
    # exactly one plane)
    tot = img[1:5].sum(dim=0)
    assert float((tot - img[0]).abs().max()) <= 1e-5 * float(img[0].abs().max())
    sampled_vs_oracle(cfg, img, lev, snapshot[0], 8, 14, 1e-4)
    del img, lev
    torch.cuda.empty_cache()
