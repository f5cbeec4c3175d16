"""Pins of the oracle's visibilities (Sec. 4.3).

- On the transform grid u_k = k / (nx dx), v_l = l / (ny dx) the pixel sum is
  numpy's FFT times the phase of the centred origin (non-square, asymmetric
  image: a swapped axis, sign or index fails).
- Closed forms: an offset circular Gaussian transforms to a Gaussian times
  the shift phase; the taper alone (a uniform field) transforms to the
  Gaussian of its FWHM; a thin ring of diameter d gives J0(pi d rho), whose
  zeros along a baseline are spaced 1/d (the ring period of Sec. 4.3.1).
- Hermitian symmetry, V(0, 0) = tapered flux, linearity (residual
  visibilities), the shift theorem.
- The doubled field keeps the pixel size and holds the original grid as its
  central block.
"""
import numpy as np
import pytest
from scipy.special import j0

from oracle import ray as oray
from oracle import vis


def test_grid_frequencies_equal_fft():
    rng = np.random.default_rng(5)
    ny, nx, dx = 24, 37, 0.3
    img = rng.standard_normal((ny, nx)) + np.linspace(0, 1, nx)[None, :]
    u = np.arange(nx) / (nx * dx)
    v = np.arange(ny) / (ny * dx)
    V = vis.visibility(img, dx, u, v)
    cx, cy = 0.5 * (nx - 1), 0.5 * (ny - 1)
    k = np.arange(nx)[None, :]
    l = np.arange(ny)[:, None]
    F = np.fft.fft2(img) * np.exp(2j * np.pi * (k * cx / nx + l * cy / ny)) * dx * dx
    assert np.abs(V - F).max() <= 1e-12 * np.abs(img).sum() * dx * dx


def test_offset_gaussian_closed_form():
    nx, ny, dx = 161, 141, 0.05
    x = vis.axis_coords(nx, dx)[None, :]
    y = vis.axis_coords(ny, dx)[:, None]
    xc, yc, sig, F0 = 0.7, -0.45, 0.4, 3.0
    img = F0 / (2 * np.pi * sig ** 2) * np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2 * sig ** 2))
    u = np.linspace(-1.5, 2.0, 15)
    v = np.linspace(-1.0, 1.2, 9)
    V = vis.visibility(img, dx, u, v)
    U, W = np.meshgrid(u, v)
    ref = F0 * np.exp(-2 * np.pi ** 2 * sig ** 2 * (U ** 2 + W ** 2)) * np.exp(-2j * np.pi * (U * xc + W * yc))
    assert np.abs(V - ref).max() <= 1e-10 * F0


def test_taper_of_uniform_field_is_its_gaussian():
    n, dx, fwhm = 601, 0.02, 1.5
    img = np.ones((n, n))
    rho = np.linspace(0.0, 1.2, 13)
    V = vis.visibility(img, dx, rho, [0.0], fwhm=fwhm)[0]
    c = np.pi * fwhm ** 2 / (4 * np.log(2))
    ref = c * np.exp(-np.pi ** 2 * fwhm ** 2 * rho ** 2 / (4 * np.log(2)))
    assert np.abs(V - ref).max() <= 1e-10 * c
    # the taper is halved at FWHM / 2 from the centre
    g = vis.taper(n, dx, fwhm)
    x = vis.axis_coords(n, dx)
    assert abs(np.interp(fwhm / 2, x, g) - 0.5) < 1e-4


def test_thin_ring_period_is_one_over_diameter():
    n, dx, r0, w = 1201, 0.01, 2.5, 0.02
    x = vis.axis_coords(n, dx)
    r = np.hypot(x[None, :], x[:, None])
    img = np.exp(-(r - r0) ** 2 / (2 * w * w))
    u = np.linspace(0.05, 4.0, 3000)
    V = vis.visibility(img, dx, u, [0.0])[0]
    amp = 2 * np.pi * r0 * np.sqrt(2 * np.pi) * w
    ref = amp * j0(2 * np.pi * r0 * u) * np.exp(-2 * np.pi ** 2 * w * w * u * u)
    assert np.abs(V.imag).max() <= 1e-9 * amp          # centred, symmetric ring
    assert np.abs(V.real - ref).max() <= 2e-3 * amp
    zeros = u[:-1][np.sign(V.real[:-1]) != np.sign(V.real[1:])]
    spacing = np.diff(zeros)[3:]                       # asymptotic regime
    assert abs(spacing.mean() * (2 * r0) - 1.0) < 0.01


def test_symmetries_linearity_shift():
    rng = np.random.default_rng(8)
    ny, nx, dx = 30, 44, 0.1
    a = np.zeros((ny, nx))
    a[5:25, 6:30] = rng.random((20, 24))
    b = rng.random((ny, nx))
    u = np.linspace(-2.0, 2.0, 11)
    v = np.linspace(-1.5, 1.5, 7)
    Va = vis.visibility(a, dx, u, v, fwhm=2.0)
    # Hermitian: V(-u, -v) = conj V(u, v) for a real image
    assert np.abs(Va[::-1, ::-1] - np.conj(Va)).max() <= 1e-13 * np.abs(a).sum()
    # V(0, 0) is the tapered flux
    V0 = vis.visibility(a, dx, [0.0], [0.0], fwhm=2.0)[0, 0]
    g = vis.taper(ny, dx, 2.0)[:, None] * vis.taper(nx, dx, 2.0)[None, :]
    assert abs(V0 - (g * a).sum() * dx * dx) <= 1e-13 * a.sum()
    # linearity: the residual's visibility is the difference of visibilities
    Vb = vis.visibility(b, dx, u, v, fwhm=2.0)
    Vd = vis.visibility(a - 0.5 * b, dx, u, v, fwhm=2.0)
    assert np.abs(Vd - (Va - 0.5 * Vb)).max() <= 1e-12 * np.abs(b).sum()
    # shift theorem (no taper, nothing leaves the frame): 3 pixels in +x
    s = np.roll(a, 3, axis=1)
    Vs = vis.visibility(s, dx, u, v)
    V1 = vis.visibility(a, dx, u, v)
    assert np.abs(Vs - V1 * np.exp(-2j * np.pi * u[None, :] * 3 * dx)).max() <= 1e-12 * a.sum()


def test_visibility_at_matches_grid():
    rng = np.random.default_rng(9)
    img = rng.random((21, 33))
    u = np.array([-0.7, 0.0, 1.3])
    v = np.array([0.4, -2.2])
    V = vis.visibility(img, 0.2, u, v, fwhm=3.0)
    for l in range(2):
        for k in range(3):
            assert abs(vis.visibility_at(img, 0.2, u[k], v[l], fwhm=3.0) - V[l, k]) <= 1e-13 * img.sum()


def test_grid_frequencies_and_doubled_field():
    half, full = vis.grid_frequencies(40.0, 1.0)
    assert half[0] == 0.0 and np.isclose(half[1], 1 / 40.0) and half[-1] <= 1.0 < half[-1] + 1 / 40.0
    assert full.size == 2 * half.size - 1 and np.allclose(full[half.size - 1:], half)
    cfg = dict(fov=40.0, nx0=257, ny0=257, levels=2)
    d = vis.doubled_field(cfg)
    assert d["nx0"] == 513 and d["fov"] == 80.0 and d["levels"] == 2
    n, n2 = 4 * 256 + 1, 4 * 512 + 1
    x, _ = oray.screen_coords(cfg["fov"], n, n, np.arange(n), np.zeros(n))
    x2, _ = oray.screen_coords(d["fov"], n2, n2, np.arange(n2), np.zeros(n2))
    off = (n2 - n) // 2
    assert np.allclose(x2[off:off + n], x, rtol=0, atol=1e-12)
    assert np.allclose(vis.axis_coords(n, x[1] - x[0]), x, atol=1e-12)


@pytest.mark.parametrize("fwhm", [0.0, -1.0])
def test_no_taper(fwhm):
    assert np.array_equal(vis.taper(7, 0.1, fwhm), np.ones(7))
