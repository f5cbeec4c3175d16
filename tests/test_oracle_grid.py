"""Pins of the oracle's gridded-snapshot sampler and electron temperature.

- cell-centre values are returned exactly; fields linear in (x1, theta) are
  reproduced exactly between centres (trilinear interpolation is exact on
  them); phi is periodic; a theta beyond the pole equals the reflected point
  on the opposite meridian;
- the R_high temperature prescription on a uniform grid, computed by hand.
"""
import ctypes

import numpy as np
import pytest

from art_inputs import mks
from oracle import ray


def sample(cfg, grid, r, th, ph):
    p = ray.make_params(cfg, grid)
    out = np.zeros(8)
    ray.lib().or_grid_sample.argtypes = [ctypes.POINTER(ray.OrParams)] + [ctypes.c_double] * 3 + \
        [ctypes.POINTER(ctypes.c_double)]
    ray.lib().or_grid_sample(ctypes.byref(p), r, th, ph, ray._dp(out))
    return out


def small_grid(fn, n1=12, n2=10, n3=8, h=0.3):
    geo = mks.mks_snapshot_geometry(n1=n1, n2=n2, n3=n3, r_in=1.5, r_out=60.0, hslope=h)
    x1 = geo["x1_0"] + (np.arange(n1) + 0.5) * geo["dx1"]
    th = mks.theta_of_x2((np.arange(n2) + 0.5) / n2, h)
    ph = 2 * np.pi * (np.arange(n3) + 0.5) / n3
    P, T, X = np.meshgrid(ph, th, x1, indexing="ij")
    g = np.zeros((n3, n2, n1, 8), dtype=np.float32)
    for q in range(8):
        g[..., q] = fn(q, X, T, P)
    cfg = dict(a=0.5, r_cam=1000.0, inc_deg=60.0, model="grid", mp=mks.grid_params(geo))
    return cfg, np.ascontiguousarray(g), geo, x1, th, ph


def test_cell_centres_exact():
    rng = np.random.default_rng(1)
    vals = rng.uniform(0.5, 2.0, size=(8, 10, 12, 8)).astype(np.float32)
    cfg, g, geo, x1, th, ph = small_grid(lambda q, X, T, P: 0.0)
    g[...] = vals
    for (k, j, i) in [(0, 0, 0), (3, 4, 5), (7, 9, 11), (5, 2, 8)]:
        out = sample(cfg, g, np.exp(x1[i]), th[j], ph[k])
        assert np.allclose(out, vals[k, j, i], rtol=0, atol=1e-12)


def test_linear_fields_interpolated_exactly():
    fn = lambda q, X, T, P: (q + 1) * 0.1 + 0.3 * X - 0.2 * q * T
    cfg, g, geo, x1, th, ph = small_grid(fn)
    rng = np.random.default_rng(2)
    for _ in range(50):
        xs = rng.uniform(x1[0], x1[-1])
        ts = rng.uniform(th[0], th[-1])
        out = sample(cfg, g, np.exp(xs), ts, rng.uniform(0, 2 * np.pi))
        exp = np.array([(q + 1) * 0.1 + 0.3 * xs - 0.2 * q * ts for q in range(8)])
        # the grid holds FP32 values
        assert np.allclose(out, exp, rtol=0, atol=2e-6)


def test_periodic_phi_and_pole_reflection():
    rng = np.random.default_rng(3)
    cfg, g, geo, x1, th, ph = small_grid(lambda q, X, T, P: 0.0)
    g[...] = rng.uniform(0, 1, size=g.shape).astype(np.float32)
    for _ in range(20):
        r = np.exp(rng.uniform(x1[0], x1[-1]))
        t = rng.uniform(0.05, 1.0)
        p = rng.uniform(0, 2 * np.pi)
        a = sample(cfg, g, r, t, p)
        assert np.allclose(a, sample(cfg, g, r, t, p + 2 * np.pi), atol=1e-12)
        assert np.allclose(a, sample(cfg, g, r, t, p - 4 * np.pi), atol=1e-12)
        # theta = -t is the point at theta = t on the meridian phi + pi
        assert np.allclose(sample(cfg, g, r, -t, p + np.pi), a, atol=1e-12)
        t2 = np.pi - t
        assert np.allclose(sample(cfg, g, r, 2 * np.pi - t2, p + np.pi), sample(cfg, g, r, t2, p),
                           atol=1e-12)


def grid_plasma(cfg, grid, r, th, ph):
    p = ray.make_params(cfg, grid)
    out = np.zeros(3)
    L = ray.lib()
    L.or_grid_plasma.argtypes = [ctypes.POINTER(ray.OrParams)] + [ctypes.c_double] * 3 + \
        [ctypes.POINTER(ctypes.c_double)]
    L.or_grid_plasma.restype = ctypes.c_int
    ok = L.or_grid_plasma(ctypes.byref(p), r, th, ph, ray._dp(out))
    return ok, out


@pytest.mark.parametrize("rho,u,B", [(2.0, 0.3, 0.2), (1.0, 0.05, 0.5), (0.5, 0.4, 0.01)])
def test_rhigh_temperature_by_hand(rho, u, B):
    """Uniform cell, numbers worked by hand from the R_high prescription:
    Theta_e = (m_p/m_e) p/rho / (1 + T_i/T_e), T_i/T_e = (R_high b^2 + R_low)/(1 + b^2),
    b = p / (|B|^2/2); n_e = rho n_unit; |B|_G = |B| c sqrt(4 pi n_unit m_p)."""
    fn = lambda q, X, T, P: [rho, u, 0.0, 0.0, 0.0, 0.0, 0.0, B][q]
    cfg, g, geo, x1, th, ph = small_grid(fn)
    gam = cfg["mp"][3]
    nu = cfg["mp"][0]
    pg = (gam - 1) * u
    beta = pg / (0.5 * B * B)
    tr = (20.0 * beta ** 2 + 1.0) / (1.0 + beta ** 2)
    theta_e = (1.67262192369e-24 / 9.1093837015e-28) * pg / rho / (1 + tr)
    ok, out = grid_plasma(cfg, g, 5.0, 1.0, 0.3)
    assert ok == (B * B / rho <= cfg["mp"][4])
    if ok:
        assert out[0] == pytest.approx(rho * nu, rel=1e-7)
        assert out[1] == pytest.approx(theta_e, rel=1e-6)
        assert out[2] == pytest.approx(B * 2.99792458e10 * np.sqrt(4 * np.pi * nu * 1.67262192369e-24), rel=1e-6)


def test_sigma_cut():
    fn = lambda q, X, T, P: [0.1, 0.3, 0.0, 0.0, 0.0, 0.0, 0.0, 0.5][q]   # sigma = 2.5 > 1
    cfg, g, geo, x1, th, ph = small_grid(fn)
    ok, _ = grid_plasma(cfg, g, 5.0, 1.0, 0.3)
    assert ok == 0


def test_camera_azimuth_equals_rotated_snapshot():
    """A camera at azimuth k dphi sees a snapshot rotated by k cells exactly as
    a camera at 0 sees the original (the same sample positions up to the
    rounding of phi); an axisymmetric model ignores the azimuth bitwise; the
    snapshot itself is not axisymmetric (the azimuth changes its image)."""
    import art_inputs
    grid, geo = mks.mks_snapshot(seed=2, n1=48, n2=32, n3=32)
    cfg = dict(art_inputs.workload("grid_4097"), mp=mks.grid_params(geo), nstokes=4)
    k = 5
    rot = np.ascontiguousarray(np.roll(grid, k, axis=0))         # rot[i3] = grid[i3 - k]
    rng = np.random.default_rng(6)
    al = rng.uniform(-15, 15, 160)
    be = rng.uniform(-15, 15, 160)
    S0, _ = ray.trace(cfg, al, be, grid=grid)
    S1, _ = ray.trace(dict(cfg, phi_deg=k * 360.0 / 32), al, be, grid=rot)
    scale = np.abs(S0[:, 0]).max()
    assert scale > 0
    assert np.abs(S1 - S0).max() <= 1e-8 * scale
    S2, _ = ray.trace(dict(cfg, phi_deg=k * 360.0 / 32), al, be, grid=grid)
    assert np.abs(S2 - S0).max() > 1e-3 * scale
    th = dict(art_inputs.workload("thermal_1025"))
    A, _ = ray.trace(th, al, be)
    B, _ = ray.trace(dict(th, phi_deg=37.0), al, be)
    assert np.array_equal(A, B)
