"""Pins of the oracle's subring decomposition (Sec. 5.1).

- The subring planes split Stokes I: their sum equals I (each step's
  increment of I goes to exactly one plane).
- Self-similar demagnification: for a thin, optically thin equatorial disk
  around a Schwarzschild hole seen face-on, the flux of successive subrings
  falls by e^-gamma with the Lyapunov exponent gamma = pi (Sec. 5.1, a = 0),
  checked on n = 2 -> 3 (5 %) and n = 3 -> 4 (15 %) with a radial scan that
  resolves the rings around the critical radius sqrt(27) M.
- One subring plane reproduces I; emission before the first theta turning
  point (the direct image) lands in plane 0.
"""
import numpy as np

import art_inputs
from oracle import ray as oray


def thin_disk(subrings, inc=1.0, a=0.0):
    return dict(art_inputs.workload("toy_disk_64"), a=a, inc_deg=inc, nstokes=1, subrings=subrings,
                mp=art_inputs.toy_disk_params(r_in=2.0, h_over_r=0.02))


def radial_scan():
    bc = np.sqrt(27.0)
    return np.unique(np.concatenate([np.linspace(4.0, 7.0, 6001), bc + np.linspace(-0.2, 0.3, 20000)]))


def test_subring_planes_sum_to_stokes_i():
    cfg = thin_disk(5, inc=30.0, a=0.5)
    rng = np.random.default_rng(3)
    al = rng.uniform(-8, 8, 400)
    be = rng.uniform(-8, 8, 400)
    S, _ = oray.trace(cfg, al, be)
    assert S.shape == (400, 6)
    assert np.abs(S[:, 1:].sum(1) - S[:, 0]).max() <= 1e-14 * np.abs(S[:, 0]).max()
    assert (S[:, 2:] > 0).any()            # lensed light exists


def test_single_plane_is_stokes_i():
    cfg = thin_disk(1, inc=60.0, a=0.9)
    al = np.linspace(-7, 7, 101)
    S, _ = oray.trace(cfg, al, 0.3 * al)
    assert np.array_equal(S[:, 1], S[:, 0])


def test_polarised_planes_sum_to_stokes_i():
    cfg = dict(art_inputs.workload("thermal_1025"), subrings=4)
    rng = np.random.default_rng(4)
    al = rng.uniform(-10, 10, 64)
    be = rng.uniform(-10, 10, 64)
    S, _ = oray.trace(cfg, al, be)
    assert S.shape == (64, 8)
    assert np.abs(S[:, 4:].sum(1) - S[:, 0]).max() <= 1e-13 * np.abs(S[:, 0]).max()


def test_subring_flux_ratio_is_exp_minus_gamma():
    al = radial_scan()
    S, _ = oray.trace(thin_disk(5), al, np.zeros_like(al))
    F = [np.trapezoid(S[:, 1 + n], al) for n in range(5)]
    g = np.exp(-np.pi)
    assert abs(F[3] / F[2] / g - 1.0) < 0.05, F
    assert abs(F[4] / F[3] / g - 1.0) < 0.15, F
    # higher subrings live only near the critical radius
    for n in (3, 4):
        far = np.abs(al - np.sqrt(27.0)) > 0.1
        assert np.all(S[far, 1 + n] == 0.0), n


def test_direct_image_is_plane_zero():
    cfg = thin_disk(4, inc=1.0)
    al = np.linspace(7.5, 12.0, 50)           # far outside the photon ring: direct disk light only
    S, _ = oray.trace(cfg, al, np.zeros_like(al))
    assert np.array_equal(S[:, 1], S[:, 0]) and np.all(S[:, 2:] == 0.0)
