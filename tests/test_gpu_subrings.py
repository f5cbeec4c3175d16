"""GPU subring decomposition (Sec. 5.1) against the oracle.

- Per-ray planes (Stokes, then the subring planes of I) within relative L2
  1e-6 of the oracle in FP64, polarised and unpolarised.
- The planes sum to I on the GPU (each step's increment goes to one plane),
  also after interpolation in an adaptive render, and the adaptive image of
  every plane equals the oracle replayed with the GPU's level map.
- The thin-disk flux ratio of successive subrings is e^-pi at a = 0.
"""
import numpy as np
import pytest

import art_inputs
from gpu_helpers import ETA_FP64, check_ties, nmse, rel_l2
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


def thin_disk(subrings, inc=1.0, a=0.0):
    return dict(art_inputs.workload("toy_disk_64"), a=a, inc_deg=inc, nstokes=1, subrings=subrings,
                mp=art_inputs.toy_disk_params(r_in=2.0, h_over_r=0.02))


def gpu_points(art, cfg, al, be):
    S, _ = art.trace_points(cfg, torch.tensor(al, dtype=torch.float64, device="cuda"),
                            torch.tensor(be, dtype=torch.float64, device="cuda"), feat=False)
    torch.cuda.synchronize()
    return S.cpu().numpy()


@pytest.mark.parametrize("nst", [4, 1])
def test_subring_points_fp64(art, nst):
    print("CASE subring points", nst, flush=True)
    cfg = dict(art_inputs.workload("thermal_1025"), nstokes=nst, subrings=4)
    rng = np.random.default_rng(12)
    al = rng.uniform(-9, 9, 512)
    be = rng.uniform(-9, 9, 512)
    g = gpu_points(art, cfg, al, be)
    c, _ = oray.trace(cfg, al, be)
    assert g.shape == c.shape == (512, nst + 4)
    for s in range(nst + 4):
        if np.abs(c[:, s]).max() > 0:
            assert rel_l2(g[:, s], c[:, s]) <= 1e-6, (s, rel_l2(g[:, s], c[:, s]))
        else:
            assert np.abs(g[:, s]).max() == 0.0, s
    assert np.abs(g[:, nst:].sum(1) - g[:, 0]).max() <= 1e-13 * np.abs(g[:, 0]).max()


def test_subring_flux_ratio_gpu(art):
    print("CASE subring flux ratio", flush=True)
    bc = np.sqrt(27.0)
    al = np.unique(np.concatenate([np.linspace(4.0, 7.0, 6001), bc + np.linspace(-0.2, 0.3, 20000)]))
    g = gpu_points(art, thin_disk(5), al, np.zeros_like(al))
    F = [np.trapezoid(g[:, 1 + n], al) for n in range(5)]
    assert abs(F[3] / F[2] / np.exp(-np.pi) - 1.0) < 0.05, F


def test_subring_adaptive_render(art):
    print("CASE subring adaptive", flush=True)
    cfg = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 9, 3), nstokes=4, subrings=3)
    img, lev, _, st = art.render(cfg)
    g = img.cpu().numpy()
    gl = lev.cpu().numpy()
    assert g.shape[0] == 7
    # planes sum to I everywhere (interpolation is linear, with the same weights)
    assert np.abs(g[4:].sum(0) - g[0]).max() <= 1e-13 * np.abs(g[0]).max()
    fn = lambda x, y: oray.trace(cfg, x, y)[0]
    o = oref.refine(fn, cfg["fov"], 9, 9, 3, cfg["r_rel"], cfg["r_abs"], cfg["abs_norm"], 7,
                    forced_level=gl)
    check_ties(o, gl, ETA_FP64)
    for s in range(7):
        if np.abs(o["img"][s]).max() > 0:
            assert rel_l2(g[s], o["img"][s]) <= 1e-6, (s, rel_l2(g[s], o["img"][s]))


def test_subring_mixed_precision(art):
    """Mixed-precision subring planes against the FP64 oracle's (uniform)."""
    print("CASE subring mixed", flush=True)
    cfg = dict(art_inputs.reduced(art_inputs.workload("thermal_1025"), 33, 1), nstokes=4, subrings=4)
    g32, _, _ = art.render_uniform(dict(cfg, precision="mixed"))
    a = g32.cpu().numpy()
    truth = oref.uniform(lambda x, y: oray.trace(cfg, x, y)[0], cfg["fov"], 65, 65, 8)
    for s in range(8):
        if np.abs(truth[s]).max() > 0:
            e = nmse(a[s], truth[s])
            print("plane", s, "mse vs oracle", e, flush=True)
            assert e <= 1e-3, (s, e)
    assert np.abs(a[4:].sum(0) - a[0]).max() <= 1e-5 * np.abs(a[0]).max()
