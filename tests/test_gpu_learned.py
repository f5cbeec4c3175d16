"""Learned renders on the GPU (network look-ahead, the criterion of Sec. 3.2
as judge and fallback) against the oracle, and what training gains.

- Parity: the GPU image equals the oracle replayed with the GPU's level map
  (relative L2 <= 1e-6, FP64); every GPU decision that the oracle's own
  learned refinement (bf16-rounding network oracle), replayed on the GPU's
  level map, takes differently sits at a tie (criterion margin < 1e-9 or a
  logit within 0.05 of a threshold), and the judge counters agree with the
  unforced oracle's when the level maps are equal.
- A batch of learned renders equals the same images rendered one by one,
  and a captured graph replays them bitwise.
- Training on plain-criterion masks with the GPU's own forward/backward
  kernels lowers the loss; the trained network then renders held-out images
  with fewer trace passes than the plain method at image MSE <= 1e-3
  against the uniform truth, and misses fewer flagged points than the
  untrained network.
"""
import numpy as np
import pytest

import art_inputs
from gpu_helpers import ETA_FP64, check_ties, oracle_adaptive, rel_l2
from oracle import cnn as ocnn
from oracle import learned as olearned
from oracle import ray as oray

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# the GPU's BF16 network follows the BF16-rounding oracle network to relative
# L2 ~3e-3 on logits of size 1-10: a logit this close to a threshold is a tie
TAU_Z = 0.05


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def case(name, **kw):
    print("CASE", name, kw, flush=True)


def small_cfg(nx0=9, levels=4, **kw):
    c = art_inputs.reduced(art_inputs.workload("thermal_1025"), nx0, levels)
    c["nstokes"] = 1
    c.update(kw)
    return c


def net_params(seed):
    rng = np.random.default_rng(seed)
    W, b = ocnn.init_params(seed=seed)
    b = [rng.normal(0.0, 0.1, size=x.shape) for x in b]
    return ocnn.unflatten(ocnn.flatten((W, b)).astype(np.float32).astype(np.float64))


def thresholds(art, cfg, params):
    """z_propose / z_suppress at the 85th / 10th percentile of the level-0
    logits of the oracle network (the level-0 grid is the same in every render)."""
    img, lev, ft, st = art.render(cfg, feat=True)
    f = art.feat_numpy(ft)
    x = ocnn.features(img.cpu().numpy()[0], f["rmin"], f["ncross"], cfg["nx0"], cfg["ny0"],
                      cfg["levels"], 0, st["n_abs"])
    z, _ = ocnn.forward(params, x, bf16=True)
    lab, val = ocnn.labels(lev.cpu().numpy(), cfg["nx0"], cfg["ny0"], cfg["levels"], 0)
    zz = z[val > 0]
    return float(np.percentile(zz, 85)), float(np.percentile(zz, 10))


@pytest.mark.parametrize("fallback,cap", [(True, 0), (False, 0), (False, 1)])
def test_learned_render_parity(art, fallback, cap):
    """cap = 1: the network only at level 0, levels 3 and 4 by the criterion."""
    cfg = small_cfg()
    case("learned parity", fallback=fallback, level_cap=cap)
    params = net_params(7)
    net = art.Cnn()
    net.set_params(ocnn.flatten(params).astype(np.float32))
    zh, zl = thresholds(art, cfg, params)
    img, lev, ft, st = art.render_learned(cfg, net, z_propose=zh, z_suppress=zl, fallback=fallback,
                                          level_cap=cap)
    g = img.cpu().numpy()[0]
    gl = lev.cpu().numpy()
    assert gl.min() >= -1 and gl.max() <= cfg["levels"]
    assert st["rays"] == int((gl >= 0).sum())
    # the image is exactly what the level map says
    o = oracle_adaptive(cfg, forced=gl)
    assert rel_l2(g, o["img"][0]) <= 1e-6, rel_l2(g, o["img"][0])

    def ray_fn(x, y):
        S, f = oray.trace(cfg, x, y)
        return S, f["rmin"], f["ncross"]

    args = (ray_fn, cfg["fov"], cfg["nx0"], cfg["ny0"], cfg["levels"], cfg["r_rel"], cfg["r_abs"],
            cfg["abs_norm"], 1, lambda x: ocnn.forward(params, x, bf16=True)[0], zh, zl)
    # every decision of the GPU's level map that the oracle's own learned rule
    # (given the same history) takes differently sits at a tie: a criterion
    # margin below 1e-9 or a logit within TAU_Z of a threshold
    rep = olearned.refine_learned(*args, fallback=fallback, forced_level=gl, level_cap=cap)
    check_ties(rep, gl, ETA_FP64, tau_z=TAU_Z)
    ol = olearned.refine_learned(*args, fallback=fallback, level_cap=cap)
    flips = int((gl != ol["level"]).sum())
    print("level-map differences from the unforced oracle", flips, "judge gpu", st["learned"],
          "oracle", ol["judge"], flush=True)
    names = ("proposed_extra", "suppressed", "fallback", "missed", "lookahead")
    if flips == 0:
        for k, n in enumerate(names):
            assert st["learned"][n] == ol["judge"][k], (n, st["learned"][n], ol["judge"][k])
    assert st["learned"]["lookahead"] > 0 and st["learned"]["suppressed"] > 0
    assert st["trace_launches"] == ol["passes"]
    net.close()


@pytest.mark.parametrize("fallback", [True, False])
def test_learned_uneven_batch(art, fallback):
    """A learned batch whose images have 1 to 4 levels on one base grid: every
    image equals its single learned render bitwise, and against the oracle's
    learned refinement of that image (its own level count) every differing
    decision sits at a tie and the image equals the oracle's replay."""
    case("learned uneven batch", fallback=fallback)
    params = net_params(11)
    net = art.Cnn()
    net.set_params(ocnn.flatten(params).astype(np.float32))
    cfgs = [small_cfg(levels=L, a=a, inc_deg=inc) for L, a, inc in
            ((1, 0.94, 163.0), (2, 0.0, 60.0), (3, -0.5, 90.0), (4, 0.5, 30.0), (4, 0.94, 163.0))]
    opts = dict(z_propose=0.3, z_suppress=-2.0, fallback=fallback)
    b = art.Batch(cfgs, feat=True)
    b.set_learned(net, **opts)
    b.render()
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        img, lev, _, st = art.render_learned(c, net, **opts)
        torch.cuda.synchronize()
        assert torch.equal(b.levels[i], lev), i
        assert torch.equal(b.images[i], img), i
        assert b.stats(i)["learned"] == st["learned"], i
        gl = lev.cpu().numpy()

        def ray_fn(x, y, c=c):
            S, f = oray.trace(c, x, y)
            return S, f["rmin"], f["ncross"]
        rep = olearned.refine_learned(ray_fn, c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"],
                                      c["r_abs"], c["abs_norm"], 1,
                                      lambda x: ocnn.forward(params, x, bf16=True)[0], 0.3, -2.0,
                                      fallback=fallback, forced_level=gl)
        check_ties(rep, gl, ETA_FP64, tau_z=TAU_Z, label=" (image %d, %d levels)" % (i, c["levels"]))
        assert rel_l2(img.cpu().numpy()[0], rep["img"][0]) <= 1e-6, i
    b.close()
    net.close()


def test_learned_feature_records_up_to_the_last_network_level(art):
    """A learned render writes the feature records of interpolated points
    only on the levels the network reads (0..2 of a 4-level image: it runs at
    levels 0 and 2); deeper interpolated points keep what the buffer held,
    traced points always carry theirs.  A plain render writes every record."""
    case("learned feature records")
    params = net_params(5)
    net = art.Cnn()
    net.set_params(ocnn.flatten(params).astype(np.float32))
    c = small_cfg(levels=4)
    N = c["levels"]

    def level_of(x):
        tz = np.zeros_like(x)
        y = x.copy()
        for _ in range(N):
            odd = (y % 2 == 1) | (y == 0)
            tz += np.where(odd, 0, 1)
            y = np.where(odd, y, y // 2)
        return np.where(x == 0, 0, np.maximum(0, N - tz))

    for learned in (True, False):
        out = art.alloc(c, feat=True)
        out[2].fill_(-7)
        if learned:
            _, lev, ft, st = art.render_learned(c, net, out=out, z_propose=0.3, z_suppress=-2.0, fallback=True)
        else:
            _, lev, ft, st = art.render(c, out=out)
        torch.cuda.synchronize()
        f = art.feat_numpy(ft)
        L = lev.cpu().numpy()
        jj, ii = np.mgrid[0:L.shape[0], 0:L.shape[1]]
        pl = np.maximum(level_of(ii), level_of(jj))
        assert pl.max() == N and (pl == 0).sum() == c["nx0"] * c["ny0"]
        unset = f["status"] == -7
        traced = L >= 0
        assert not unset[traced].any()
        if learned:
            assert not unset[~traced & (pl <= 2)].any()
            assert unset[~traced & (pl > 2)].all() and (~traced & (pl > 2)).sum() > 0
        else:
            assert not unset.any()
    net.close()


def test_learned_batch_equals_single_and_graph(art):
    case("learned batch")
    params = net_params(3)
    net = art.Cnn()
    net.set_params(ocnn.flatten(params).astype(np.float32))
    cfgs = [small_cfg(a=a, inc_deg=inc) for a, inc in ((0.94, 163.0), (0.0, 60.0), (-0.5, 90.0))]
    opts = dict(z_propose=0.5, z_suppress=-3.0, fallback=True)
    singles = [art.render_learned(c, net, **opts) for c in cfgs]
    b = art.Batch(cfgs, feat=True)
    b.set_learned(net, **opts)
    for groups in (3, 1):              # one image per group, then one group
        b.set_launch(groups=groups)
        for x in b.images:
            x.zero_()
        b.render()
        torch.cuda.synchronize()
        for i, (img, lev, _, st) in enumerate(singles):
            assert torch.equal(b.images[i], img), (groups, i)
            assert torch.equal(b.levels[i], lev), (groups, i)
            assert b.stats(i)["learned"] == st["learned"], (groups, i)
    ref = [x.clone() for x in b.images]
    s = torch.cuda.Stream()
    b.capture(s)
    for _ in range(3):
        for x in b.images:
            x.zero_()
        torch.cuda.synchronize()
        b.launch(s)
        s.synchronize()
        for i in range(len(cfgs)):
            assert torch.equal(b.images[i], ref[i]), i
    b.close()
    net.close()


def train_configs():
    return [small_cfg(nx0=17, levels=4, a=a, inc_deg=inc)
            for a, inc in ((0.94, 163.0), (0.0, 17.0), (0.5, 90.0), (-0.94, 60.0), (0.94, 17.0))]


def training_set(art, cfgs):
    """Features and labels of plain renders at the levels the network runs
    at (l with l + 2 <= N), grouped by level."""
    by_level = {}
    for c in cfgs:
        img, lev, ft, st = art.render(c, feat=True)
        for l in range(0, c["levels"] - 1, 2):
            x = art.cnn_features(c, img, ft, l, st["n_abs"])
            y, v = art.cnn_labels(c, lev, l)
            by_level.setdefault(l, []).append((x, y, v))
    return {l: tuple(torch.cat([t[i] for t in items]) for i in range(3))
            for l, items in by_level.items()}


def test_training_gains_over_the_plain_method(art):
    case("learned training")
    torch.manual_seed(0)
    cfgs = train_configs()
    data = training_set(art, cfgs[:-1])
    pos = sum(float(y[v > 0].float().mean()) for (_, y, v) in data.values()) / len(data)
    pw = float(np.clip((1 - pos) / pos, 1.0, 20.0) ** 0.5)
    net = art.Cnn(seed=4)
    untrained = art.Cnn(seed=4)
    first = {l: net.gradients(*d, pos_weight=pw)[0] for l, d in data.items()}
    for it in range(400):
        for l, (x, y, v) in data.items():
            net.train_step(x, y, v, lr=3e-3, pos_weight=pw, want_loss=False)
    last = {l: net.gradients(*d, pos_weight=pw)[0] for l, d in data.items()}
    print("loss", first, "->", last, flush=True)
    for l in data:
        assert last[l] < 0.7 * first[l], (l, first[l], last[l])
    # held-out image
    c = cfgs[-1]
    truth, _, _ = art.render_uniform(c)
    img_p, lev_p, _, st_p = art.render(c, feat=True)
    _, mse_p = art.metrics(truth, img_p)
    res = {}
    for name, n in (("trained", net), ("untrained", untrained)):
        img, lev, _, st = art.render_learned(c, n, z_propose=-1.5, fallback=False)
        _, mse = art.metrics(truth, img)
        res[name] = (st, mse)
        print(name, "rays", st["rays"], "passes", st["trace_launches"], "mse", mse,
              "judge", st["learned"], flush=True)
    print("plain rays", st_p["rays"], "passes", st_p["trace_launches"], "mse", mse_p, flush=True)
    st_t, mse_t = res["trained"]
    st_u, _ = res["untrained"]
    assert st_t["trace_launches"] < st_p["trace_launches"]
    assert mse_t <= 1e-3
    assert st_t["learned"]["missed"] < st_u["learned"]["missed"]
    net.close()
    untrained.close()
