"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance (stated by the method's accuracy target): relative L2
sqrt(sum (gpu - cpu)^2 / sum cpu^2) <= 1e-6 per Stokes plane for the FP64
path; normalised image MSE <= 1e-3 against the FP64 oracle for the reduced-
precision forms.  Refinement decisions are audited by the oracle's replay of
the GPU's level map: every decision its own rule takes differently must sit
at a tie (margin below 1e-9 for FP64, see gpu_helpers); the image is compared
against that replay.
"""
import numpy as np
import pytest

import art_inputs
from gpu_helpers import ETA_MIXED, check_adaptive, nmse, oracle_adaptive, rel_l2
from oracle import ray as oray
from oracle import refine as oref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def gpu_points(art, cfg, al, be):
    a = torch.tensor(al, dtype=torch.float64, device="cuda")
    b = torch.tensor(be, dtype=torch.float64, device="cuda")
    S, ft = art.trace_points(cfg, a, b)
    torch.cuda.synchronize()
    return S.cpu().numpy(), art.feat_numpy(ft)


def print_case(name, **kw):
    print("CASE", name, kw, flush=True)


def test_toy_disk_uniform_64(art):
    cfg = art_inputs.workload("toy_disk_64")
    print_case("toy_disk_64")
    img, ft, st = art.render_uniform(cfg, feat=True)
    g = img.cpu().numpy()[0]
    f = art.feat_numpy(ft)
    truth = oref.uniform(lambda x, y: oray.trace(cfg, x, y)[0], cfg["fov"], 64, 64)[0]
    _, of = oray.trace(cfg, *oray.screen_coords(cfg["fov"], 64, 64, *np.meshgrid(np.arange(64), np.arange(64))))
    assert rel_l2(g, truth) <= 1e-6
    assert np.mean(f["status"].ravel() == of["status"]) > 0.99
    assert np.mean(f["steps"].ravel() == of["steps"]) > 0.95
    assert st["rays"] == 4096 and st["status"]["nan"] == 0


@pytest.mark.parametrize("name,nst", [("thermal_1025", 4), ("thermal_1025", 1)])
def test_thermal_points_fp64(art, name, nst):
    cfg = dict(art_inputs.workload(name), nstokes=nst)
    print_case("thermal points", nstokes=nst)
    rng = np.random.default_rng(5)
    al = rng.uniform(-20, 20, 768)
    be = rng.uniform(-20, 20, 768)
    g, gf = gpu_points(art, cfg, al, be)
    c, cf = oray.trace(cfg, al, be)
    for s in range(nst):
        assert rel_l2(g[:, s], c[:, s]) <= 1e-6, (s, rel_l2(g[:, s], c[:, s]))
    assert np.mean(gf["status"] == cf["status"]) > 0.99
    assert np.mean(gf["ncross"] == cf["ncross"]) > 0.98
    assert np.abs(gf["rmin"] - cf["rmin"]).max() < 1e-3


def test_screen_ring_adaptive(art):
    cfg = dict(a=0.0, r_cam=1000.0, inc_deg=60.0, fov=16.0, nx0=33, ny0=33, levels=3,
               model="screen_ring", mp=art_inputs.screen_ring_params(), nstokes=4,
               r_rel=0.01, r_abs=0.01, abs_norm="mean")
    print_case("screen ring adaptive")
    g, gl, st, o = check_adaptive(art, cfg, 1e-13)
    assert 0.5 < st["interp_frac"] < 0.99


def test_screen_rectangular_and_tiny_grids(art):
    for nx0, ny0, L in ((9, 5, 3), (2, 2, 3), (3, 2, 2), (5, 5, 0)):
        cfg = dict(a=0.0, r_cam=1000.0, inc_deg=60.0, fov=16.0, nx0=nx0, ny0=ny0, levels=L,
                   model="screen_ring", mp=art_inputs.screen_ring_params(), nstokes=1,
                   r_rel=0.02, r_abs=0.005, abs_norm="max")
        print_case("screen grid", nx0=nx0, ny0=ny0, levels=L)
        check_adaptive(art, cfg, 1e-13)


@pytest.mark.parametrize("nx0,levels", [(17, 3), (33, 2)])
def test_thermal_adaptive_fp64(art, nx0, levels):
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), nx0, levels)
    print_case("thermal adaptive", nx0=nx0, levels=levels)
    g, gl, st, o = check_adaptive(art, cfg, 1e-6)
    assert st["status"]["nan"] == 0


@pytest.mark.parametrize("precision", ["mixed", "mixed_geo"])
def test_thermal_mixed_precision(art, precision):
    """Reduced-precision uniform images against the FP64 oracle's uniform
    image (every ray traced by the oracle), per Stokes plane."""
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), 33, 2)
    print_case("mixed precision uniform vs oracle", precision=precision)
    g32, _, _ = art.render_uniform(dict(cfg, precision=precision))
    g32 = g32.cpu().numpy()
    truth = oref.uniform(lambda x, y: oray.trace(cfg, x, y)[0], cfg["fov"], 129, 129, 4)
    for s in range(4):
        e = nmse(g32[s], truth[s])
        print("stokes", s, "mse vs oracle", e)
        assert e <= 1e-3, (s, e)
    assert nmse(g32[0], truth[0]) <= 1e-8


@pytest.mark.parametrize("precision", ["mixed", "mixed_geo"])
def test_thermal_mixed_adaptive_vs_oracle(art, precision):
    """Reduced-precision adaptive render against the FP64 oracle: decisions
    that differ from the oracle's own rule sit at ties of the reduced-
    precision size; the image is within MSE 1e-3 of the oracle's replay of
    its level map and of the oracle's own adaptive image, per Stokes plane."""
    cfg = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 33, 2), precision=precision)
    print_case("mixed precision adaptive vs oracle", precision=precision)
    g, gl, st, rep = check_adaptive(art, cfg, 1e-2, eta=ETA_MIXED)
    own = oracle_adaptive(cfg)
    for s in range(4):
        e1, e2 = nmse(g[s], rep["img"][s]), nmse(g[s], own["img"][s])
        print("stokes", s, "mse vs replay", e1, "vs oracle's adaptive image", e2)
        assert e1 <= 1e-3 and e2 <= 1e-3, (s, e1, e2)


def test_precision_policy_zones(art):
    """FP32 geodesic steps change the image only through the steps outside the
    sensitive zones: with every point sensitive the policy equals the mixed
    form bitwise; with the default zones it differs from it."""
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), 33, 2)
    print_case("precision policy zones")
    mixed, _, _ = art.render_uniform(dict(cfg, precision="mixed"))
    all64, _, _ = art.render_uniform(dict(cfg, precision="mixed_geo", fp64_radius=1e9))
    geo, _, _ = art.render_uniform(dict(cfg, precision="mixed_geo"))
    assert torch.equal(mixed, all64)
    assert not torch.equal(mixed, geo)


def test_device_metrics(art):
    rng = np.random.default_rng(9)
    t = rng.uniform(0, 1, 100003)
    a = t + rng.normal(0, 0.01, t.size)
    fe, mse = art.metrics(torch.tensor(t, device="cuda"), torch.tensor(a, device="cuda"))
    assert fe == pytest.approx(abs(t.sum() - a.sum()) / t.sum(), rel=1e-10)
    assert mse == pytest.approx(((t - a) ** 2).sum() / (t * t).sum(), rel=1e-10)


def test_determinism(art):
    cfg = art_inputs.reduced(art_inputs.workload("thermal_1025"), 17, 2)
    a, la, _, _ = art.render(cfg)
    b, lb, _, _ = art.render(cfg)
    assert torch.equal(a, b) and torch.equal(la, lb)


def test_invalid_arguments(art):
    base = art_inputs.reduced(art_inputs.workload("thermal_1025"), 17, 1)
    for bad in (dict(a=1.0), dict(nx0=1), dict(fov=0.0), dict(nstokes=3), dict(eps=0.0),
                dict(r_cam=1.0), dict(inc_deg=0.0)):
        with pytest.raises(art.ArtError):
            art.render(dict(base, **bad))


@pytest.mark.parametrize("interp,all_planes,subrings", [("nearest", False, 0), ("nearest", True, 0),
                                                       ("linear", True, 0), ("linear", True, 3),
                                                       ("nearest", True, 3), ("linear", "own", 0),
                                                       ("linear", "own", 3)])
def test_refinement_variants(art, interp, all_planes, subrings):
    """Nearest branch of Eqs. 5-6 and the per-plane criterion (Stokes and
    subring planes) against the oracle: decisions up to floating-point ties,
    images to 1e-6 after the mask-forced replay."""
    from gpu_helpers import check_adaptive
    print_case("refinement variant", interp=interp, all_planes=all_planes, subrings=subrings)
    cfg = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 3), interp=interp,
               all_planes=all_planes, subrings=subrings, r_rel=0.05, r_abs=0.01)
    g, gl, st, o = check_adaptive(art, cfg, 1e-6)
    assert 0.0 < st["interp_frac"] < 1.0
    if all_planes:
        one = art.render(dict(cfg, all_planes=False))[3]
        assert st["rays"] >= one["rays"]
    if all_planes == "own":
        shared = art.render(dict(cfg, all_planes=True))[3]
        assert st["rays"] > shared["rays"]


def test_own_normalisation_rejected_where_undefined(art):
    """The per-plane normalisation is defined for the linear branch of
    spatial refinement only: the nearest branch and axis-sampled cubes refuse it."""
    base = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 2), all_planes="own")
    with pytest.raises(art.ArtError):
        art.render(dict(base, interp="nearest"))
    cfgs = [dict(base, freq_hz=f) for f in (86e9, 150e9, 230e9)]
    with pytest.raises(art.ArtError):
        art.render_cube(cfgs, 2, 1)
