"""Seeded synthetic GRMHD-like snapshot on a modified Kerr-Schild (MKS) grid.

Pure input data for the gridded emission model (no arithmetic of the method):
a 288 x 128 x 128 grid (the SANE library resolution, Sec. 6) with x1 = ln r,
theta = pi x2 + (1 - h)/2 sin(2 pi x2) (zones compressed toward the midplane),
x3 = phi; fields per cell centre, FP32, interleaved [i3][i2][i1][8]:

  0 rho   analytic torus (Gaussian cross-section about r_c) plus a weak
          atmosphere, times seeded log-normal turbulence exp(s G - s^2/2),
          G a unit Gaussian random field with shell spectrum E(k) ~ k^-5/3,
          s = 0.0998 so that std(rho / rho_mean) = 0.1
  1 u     internal energy, pressure p = (gamma - 1) u = rho / (3 r)
  2-4     fluid 3-velocity in the local ZAMO frame (r, theta, phi components):
          v_phi = min(0.7, r^-1/2) sin(theta), v_r = -0.1 r^-1/2, v_theta = 0
  5-7     magnetic field in the ZAMO frame, |B|^2 = 2 p / beta with beta = 10,
          direction 0.3 e_r + 0.954 e_phi (mostly toroidal)
"""
import numpy as np

FIELDS = ("rho", "u", "U1", "U2", "U3", "B1", "B2", "B3")


def theta_of_x2(x2, hslope):
    return np.pi * x2 + 0.5 * (1.0 - hslope) * np.sin(2.0 * np.pi * x2)


def gaussian_field(shape, rng, slope=-5.0 / 3.0):
    """Unit-variance Gaussian random field with shell spectrum E(k) ~ k^slope
    (3D power ~ k^(slope - 2)) on the index grid."""
    kz = np.fft.fftfreq(shape[0])[:, None, None]
    ky = np.fft.fftfreq(shape[1])[None, :, None]
    kx = np.fft.rfftfreq(shape[2])[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** ((slope - 2.0) / 2.0)
    noise = rng.normal(size=shape[:2] + (shape[2] // 2 + 1,)) + \
        1j * rng.normal(size=shape[:2] + (shape[2] // 2 + 1,))
    g = np.fft.irfftn(noise * amp, s=shape, axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def mks_snapshot(seed=2, n1=288, n2=128, n3=128, r_in=1.2, r_out=1000.0, hslope=0.3,
                 r_c=12.0, width=3.0, atmosphere=1e-4, sigma_turb=0.0998, beta=10.0,
                 gamma_ad=13.0 / 9.0, turb=None):
    """Returns (grid float32 [n3][n2][n1][8], geometry dict).  turb: optional
    unit Gaussian field [n3][n2][n1] replacing the seeded one."""
    rng = np.random.default_rng(seed)
    x1_0 = np.log(r_in)
    dx1 = (np.log(r_out) - x1_0) / n1
    x1 = x1_0 + (np.arange(n1) + 0.5) * dx1
    x2 = (np.arange(n2) + 0.5) / n2
    r = np.exp(x1)[None, None, :]
    th = theta_of_x2(x2, hslope)[None, :, None]
    R = r * np.sin(th)
    z = r * np.cos(th)
    rho_bar = np.exp(-((R - r_c) ** 2 + z ** 2) / (2.0 * width ** 2)) + atmosphere * (r / r_c) ** -1.5
    G = gaussian_field((n3, n2, n1), rng) if turb is None else turb
    rho = rho_bar * np.exp(sigma_turb * G - 0.5 * sigma_turb ** 2)
    p = rho / (3.0 * r)
    u = p / (gamma_ad - 1.0)
    vphi = np.minimum(0.7, r ** -0.5) * np.sin(th)
    vr = -0.1 * r ** -0.5
    bmag = np.sqrt(2.0 * p / beta)
    dirn = np.array([0.3, 0.0, np.sqrt(1.0 - 0.09)])
    grid = np.empty((n3, n2, n1, 8), dtype=np.float32)
    grid[..., 0] = rho
    grid[..., 1] = u
    grid[..., 2] = np.broadcast_to(vr, rho.shape)
    grid[..., 3] = 0.0
    grid[..., 4] = np.broadcast_to(vphi, rho.shape)
    grid[..., 5] = bmag * dirn[0]
    grid[..., 6] = bmag * dirn[1]
    grid[..., 7] = bmag * dirn[2]
    geo = dict(x1_0=x1_0, dx1=dx1, hslope=hslope, n1=n1, n2=n2, n3=n3, gamma_ad=gamma_ad)
    return grid, geo


def mks_movie(times, seed=2, t_mix=200.0, n1=288, n2=128, n3=128, r_in=1.2, r_out=1000.0, **kw):
    """Snapshots of an evolving flow at the given times [M] (a movie for
    adaptive sampling in time): the turbulence field is carried around in phi
    at the Keplerian rate Omega(r) = r^-3/2 (periodic linear interpolation
    along x3, a different shift per radial zone) and turned into an
    independent field over t_mix (G_t = cos(w t) G_a + sin(w t) G_b,
    w = pi / (2 t_mix)).  At t = 0 the snapshot equals mks_snapshot(seed).
    Returns (list of float32 grids, geometry dict)."""
    rng = np.random.default_rng(seed)
    Ga = gaussian_field((n3, n2, n1), rng)
    Gb = gaussian_field((n3, n2, n1), np.random.default_rng([seed, 1]))
    x1_0 = np.log(r_in)
    dx1 = (np.log(r_out) - x1_0) / n1
    r = np.exp(x1_0 + (np.arange(n1) + 0.5) * dx1)
    i3 = np.arange(n3)[:, None]
    grids = []
    geo = None
    for t in times:
        shift = (r ** -1.5) * float(t) / (2.0 * np.pi / n3)        # cells per radial zone
        k = np.floor(shift).astype(np.int64)
        f = shift - k
        lo = (i3 - k[None, :]) % n3                                 # [n3, n1]
        hi = (lo - 1) % n3

        def carry(G):
            g_lo = np.take_along_axis(G, np.broadcast_to(lo[:, None, :], G.shape), axis=0)
            g_hi = np.take_along_axis(G, np.broadcast_to(hi[:, None, :], G.shape), axis=0)
            return (1.0 - f)[None, None, :] * g_lo + f[None, None, :] * g_hi
        w = 0.5 * np.pi * float(t) / t_mix
        G = np.cos(w) * carry(Ga) + np.sin(w) * carry(Gb) if t != 0 else Ga
        grid, geo = mks_snapshot(seed, n1, n2, n3, r_in, r_out, turb=G, **kw)
        grids.append(grid)
    return grids, geo


def mks_snapshot_geometry(n1=288, n2=128, n3=128, r_in=1.2, r_out=1000.0, hslope=0.3,
                          gamma_ad=13.0 / 9.0):
    """Geometry dictionary of mks_snapshot without generating the fields."""
    x1_0 = np.log(r_in)
    return dict(x1_0=x1_0, dx1=(np.log(r_out) - x1_0) / n1, hslope=hslope, n1=n1, n2=n2, n3=n3,
                gamma_ad=gamma_ad)


def grid_params(geo, n_unit=3.0e7, r_high=20.0, r_low=1.0, sigma_cut=1.0, r_emit=50.0):
    """Model-parameter vector of the gridded model: [0] density unit n_e per
    code rho [cm^-3], [1] R_high, [2] R_low, [3] adiabatic index, [4] sigma
    cut, [5] outer emission radius, [6] x1 of the first cell edge, [7] dx1,
    [8] h (theta compression), [9..11] n1, n2, n3."""
    mp = [0.0] * 16
    mp[0], mp[1], mp[2], mp[3], mp[4], mp[5] = n_unit, r_high, r_low, geo["gamma_ad"], sigma_cut, r_emit
    mp[6], mp[7], mp[8] = geo["x1_0"], geo["dx1"], geo["hslope"]
    mp[9], mp[10], mp[11] = geo["n1"], geo["n2"], geo["n3"]
    return mp
