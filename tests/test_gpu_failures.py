"""Failure paths of the HIP library, each forced from the host so that every
kernel still ends normally.

- Step cap: with max_steps = 1 every ray stops with status STEP_CAP and no
  emission yet; with max_steps = 300 the rays still inside the flow stop
  there with the contribution gathered so far, equal to the oracle's
  (relative L2 1e-6 in FP64), and a render reports them in its status
  histogram.
- NaN in the fluid: a shell of snapshot cells with a NaN velocity makes the
  rays that sample it NaN; the GPU flags the same rays NAN as the oracle, and
  a render with statistics returns ART_ENUMERIC with those rays flagged in
  the feature buffer.
- Allocation: a batch whose trace list would exceed the allocation limit is
  refused with ART_ENOMEM; without the limit it renders.
"""
import numpy as np
import pytest

import art_inputs
from art_inputs import mks
from gpu_helpers import rel_l2
from oracle import ray as oray

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEP_CAP, NAN = 3, 5


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def points(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-15, 15, n), rng.uniform(-15, 15, n)


def gpu_points(art, cfg, al, be):
    S, ft = art.trace_points(cfg, torch.tensor(al, device="cuda"), torch.tensor(be, device="cuda"))
    torch.cuda.synchronize()
    return S.cpu().numpy(), art.feat_numpy(ft)


@pytest.mark.parametrize("max_steps", [1, 300])
def test_step_cap_keeps_the_contribution(art, max_steps):
    print("CASE step cap", max_steps, flush=True)
    cfg = dict(art_inputs.workload("thermal_1025"), max_steps=max_steps, precision="fp64")
    al, be = points(400, 21)
    g, gf = gpu_points(art, cfg, al, be)
    c, cf = oray.trace(cfg, al, be)
    capped = cf["status"] == STEP_CAP
    if max_steps == 1:
        assert np.all(gf["status"] == STEP_CAP) and np.all(capped)
        assert np.all(g == 0.0) and np.all(c == 0.0)
    else:
        assert 0.2 < capped.mean() < 1.0
        assert np.mean(gf["status"] == cf["status"]) > 0.99
        assert np.abs(c[capped, 0]).max() > 0          # they had started to collect light
        for s in range(4):
            assert rel_l2(g[:, s], c[:, s]) <= 1e-6, (s, rel_l2(g[:, s], c[:, s]))
        small = art_inputs.reduced(cfg, 17, 1)
        _, _, _, st = art.render(small)
        assert st["status"]["step_cap"] > 0


def test_nan_in_the_fluid_is_reported(art):
    print("CASE NaN velocity shell", flush=True)
    grid, geo = mks.mks_snapshot(seed=2)
    x1 = geo["x1_0"] + (np.arange(geo["n1"]) + 0.5) * geo["dx1"]
    shell = (np.exp(x1) > 9.0) & (np.exp(x1) < 10.0)
    grid = grid.copy()
    grid[:, :, shell, 2] = np.nan                       # radial velocity of a shell of cells
    gdev = torch.from_numpy(grid).cuda()
    cfg = dict(art_inputs.workload("grid_4097"), grid_dev=gdev, nstokes=1, precision="fp64")
    al, be = points(300, 22)
    g, gf = gpu_points(art, cfg, al, be)
    c, cf = oray.trace(cfg, al, be, grid=grid)
    gn, cn = gf["status"] == NAN, cf["status"] == NAN
    print("NaN rays: gpu", int(gn.sum()), "oracle", int(cn.sum()), flush=True)
    assert 0.05 < cn.mean() < 0.95
    assert np.mean(gn == cn) > 0.98
    assert np.all(np.isnan(g[gn, 0])) and np.all(np.isfinite(g[~gn, 0]))
    # a render with statistics returns ART_ENUMERIC; the rays are flagged
    rcfg = dict(cfg, nx0=33, ny0=33, levels=1)
    out = art.alloc(rcfg, feat=True)
    with pytest.raises(art.ArtError) as e:
        art.render(rcfg, out=out)
    assert "art error -4" in str(e.value) and "NaN" in str(e.value)
    f = art.feat_numpy(out[2])
    assert (f["status"] == NAN).sum() > 0


def test_allocation_limit_gives_enomem(art):
    print("CASE allocation limit", flush=True)
    cfgs = [art_inputs.reduced(art_inputs.workload("thermal_1025"), 65, 2)]      # 257^2 pixels
    art.set_alloc_limit(1 << 16)
    try:
        with pytest.raises(art.ArtError) as e:
            art.Batch(cfgs)
        assert "art error -2" in str(e.value)
    finally:
        art.set_alloc_limit(0)
    B = art.Batch(cfgs)
    B.render()
    assert B.stats(0)["rays"] > 0
    B.close()
