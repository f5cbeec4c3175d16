"""GPU visibilities (Sec. 4.3) against the oracle.

Element by element on seeded synthetic images (ring + blobs + noise) at
sizes that span several 64 x 64 tiles and 16-wide chunks with ragged tails,
both stage orders (rows first when the u list is the shorter), axis cuts,
non-uniform and negative baselines, several planes, the taper, an empty
image and empty baseline lists; at the deployment size (16385^2, the 2D
window |u|, |v| <= 1000 G-lambda for a Sgr A*-like mass and distance) on
sampled baselines computed one by one by the oracle, plus Hermitian symmetry
of the full window.  Tolerance: |V_gpu - V_oracle| <= 1e-12 sum |g I| dx^2
(the error scale of an FP64 sum of that many terms).
"""
import numpy as np
import pytest

import art_inputs
from oracle import vis as ovis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def art():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07417_amd import art as a
    a.lib()
    return a


def l1_scale(img, dx, fwhm):
    ny, nx = img.shape[-2:]
    g = ovis.taper(ny, dx, fwhm)[:, None] * ovis.taper(nx, dx, fwhm)[None, :]
    return float(np.abs(img * g).sum(axis=(-2, -1)).max()) * dx * dx


def run(art, img, dx, u, v, fwhm):
    V = art.visibility(torch.from_numpy(img).cuda(), dx, u, v, fwhm=fwhm)
    torch.cuda.synchronize()
    return V.cpu().numpy()


CASES = [
    # name, ny, nx, planes, u, v, fwhm
    ("rows_first", 150, 203, 2, np.linspace(-3.0, 4.0, 23), np.linspace(-2.5, 2.5, 37), 9.0),
    ("cols_first", 150, 203, 2, np.linspace(-3.0, 4.0, 37), np.linspace(-2.5, 2.5, 23), 9.0),
    ("u_cut", 129, 257, 1, np.linspace(0.0, 6.0, 301), [0.0], 0.0),
    ("v_cut", 257, 129, 1, [0.0], np.linspace(-6.0, 0.0, 77), 5.0),
    ("nonuniform", 97, 65, 3, np.sort(np.random.default_rng(3).uniform(-5, 5, 70)),
     np.random.default_rng(4).uniform(-5, 5, 65), 0.0),
    ("single_tile", 16, 16, 1, [0.25, -1.0], [0.5], 4.0),
    ("tiny", 1, 3, 1, np.linspace(-1, 1, 5), np.linspace(-1, 1, 3), 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_visibility_parity(art, case):
    name, ny, nx, P, u, v, fwhm = case
    print("CASE vis", name, ny, nx, P, len(u), len(v), flush=True)
    fov = 40.0
    img = art_inputs.vis_image(ny, nx, fov, seed=len(name), planes=P)
    dx = fov / max(nx - 1, 1)
    g = run(art, img, dx, u, v, fwhm)
    o = ovis.visibility(img, dx, u, v, fwhm=fwhm)
    assert g.shape == o.shape == (P, len(v), len(u))
    err = np.abs(g - o).max()
    assert err <= 1e-12 * l1_scale(img, dx, fwhm), (name, err, l1_scale(img, dx, fwhm))


def test_visibility_empty_cases(art):
    print("CASE vis empty", flush=True)
    img = torch.zeros((1, 0, 7), dtype=torch.float64, device="cuda")
    V = art.visibility(img, 0.1, [0.0, 1.0], [0.5], fwhm=1.0)
    torch.cuda.synchronize()
    assert V.shape == (1, 1, 2) and float(V.abs().max()) == 0.0
    img = torch.ones((2, 5, 7), dtype=torch.float64, device="cuda")
    V = art.visibility(img, 0.1, [], [0.5])
    assert V.shape == (2, 1, 0)
    with pytest.raises(art.ArtError):
        art.visibility(img, 0.0, [1.0], [1.0])
    with pytest.raises(art.ArtError):
        art.visibility(img.float(), 0.1, [1.0], [1.0])


def test_visibility_plane_zero_and_hermitian(art):
    print("CASE vis zero baseline", flush=True)
    img = art_inputs.vis_image(200, 180, 40.0, seed=11, planes=1)
    dx = 40.0 / 179
    u = np.linspace(-2.0, 2.0, 41)
    V = run(art, img, dx, u, u, 10.0)[0]
    scale = l1_scale(img, dx, 10.0)
    g = ovis.taper(200, dx, 10.0)[:, None] * ovis.taper(180, dx, 10.0)[None, :]
    assert abs(V[20, 20] - (img[0] * g).sum() * dx * dx) <= 1e-12 * scale
    assert np.abs(V[::-1, ::-1] - np.conj(V)).max() <= 1e-12 * scale


def test_visibility_deployment_size(art):
    """16385^2 image over a 40 M field (the 16385^2 snapshot render's grid),
    baselines |u|, |v| <= 1000 G-lambda on the 1/FOV grid (u >= 0 half plane),
    taper FWHM = FOV / 4: sampled outputs against the oracle one by one."""
    n, fov = 16385, 40.0
    dx = fov / (n - 1)
    umax = art_inputs.glambda_to_inv_m(1000.0)
    half, full = ovis.grid_frequencies(fov, umax)
    print("CASE vis 16385^2", half.size, full.size, flush=True)
    img = art_inputs.vis_image(n, n, fov, seed=7, planes=1)
    V = run(art, img, dx, half, full, fov / 4)[0]
    assert V.shape == (full.size, half.size)
    scale = l1_scale(img, dx, fov / 4)
    rng = np.random.default_rng(2)
    picks = [(full.size // 2, 0), (0, half.size - 1), (full.size - 1, half.size // 3)]
    picks += [(int(rng.integers(full.size)), int(rng.integers(half.size))) for _ in range(3)]
    for l, m in picks:
        o = ovis.visibility_at(img[0], dx, half[m], full[l], fwhm=fov / 4)
        assert abs(V[l, m] - o) <= 1e-12 * scale, (l, m, V[l, m], o)
    # on the u = 0 column the visibility is Hermitian in v
    c = V[:, 0]
    assert np.abs(c[::-1] - np.conj(c)).max() <= 1e-12 * scale
