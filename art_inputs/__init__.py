"""Seeded synthetic inputs and workload definitions shared by the oracle and
the HIP path.

This module holds no arithmetic of the method: only workload parameters and
the random numbers the models draw (the magnetic-field phase of the thermal
model, the turbulence of the gridded snapshot).  Both sides receive these as
inputs.
"""
import numpy as np

SGRA_MASS_MSUN = 4.0e6       # Sec. 3.1 semi-analytic model: M = 4e6 Msun, D = 7.78 kpc
SGRA_DIST_PC = 7780.0


def theta_m_rad(mass_msun=SGRA_MASS_MSUN, dist_pc=SGRA_DIST_PC):
    """Angular size of one gravitational radius GM / (c^2 D) in radians."""
    G, c, msun, pc = 6.67430e-8, 2.99792458e10, 1.98847e33, 3.0856775814913673e18
    return G * mass_msun * msun / (c * c) / (dist_pc * pc)


def glambda_to_inv_m(u_glambda, mass_msun=SGRA_MASS_MSUN, dist_pc=SGRA_DIST_PC):
    """Baseline length in G-lambda -> cycles per gravitational radius on the screen."""
    return float(u_glambda) * 1e9 * theta_m_rad(mass_msun, dist_pc)


def thermal_params(seed=1, n0=2.0e6, theta0=100.0, beta_ref=10.0, r_ref=10.0,
                   r_emit=50.0, ne_index=1.1, th_index=0.84, b_index=1.0):
    """Model-parameter vector of the semi-analytic thermal plasma:
    n_e = n0 r^-1.1, Theta_e = Theta0 r^-0.84, |B| ~ r^-1 with plasma beta
    beta_ref at r_ref, field phase psi0 = 2 pi U(0,1) drawn from `seed`."""
    rng = np.random.default_rng(seed)
    psi0 = 2.0 * np.pi * rng.uniform()
    mp = [0.0] * 16
    mp[0], mp[1], mp[2], mp[3] = n0, theta0, beta_ref, r_ref
    mp[4], mp[5] = psi0, r_emit
    mp[6], mp[7], mp[8] = ne_index, th_index, b_index
    return mp


def toy_disk_params(r_in=2.0, h_over_r=0.3):
    """j = r^-2 exp(-z^2 / (2 (h r)^2)) outside r_in, no absorption."""
    mp = [0.0] * 16
    mp[0], mp[1] = r_in, h_over_r
    return mp


def screen_ring_params(radius=5.0, width=0.35, diffuse=0.05, diffuse_scale=6.0):
    """Closed-form screen intensity (refinement tests without ray tracing)."""
    mp = [0.0] * 16
    mp[0], mp[1], mp[2], mp[3] = radius, width, diffuse, diffuse_scale
    return mp


def screen_poly_params(c):
    mp = [0.0] * 16
    for i, v in enumerate(c):
        mp[i] = float(v)
    return mp


def workload(name):
    """Workload dictionaries.  Vertex-grid convention: a 'k^2 base' is k cells,
    i.e. (k+1)^2 vertices, so 128^2 -> 1024^2 is 129^2 -> 1025^2."""
    common = dict(r_cam=1000.0, r_out=1000.0, fov=40.0, eps=0.03, max_steps=100000,
                  mass_msun=SGRA_MASS_MSUN)
    if name == "toy_disk_64":
        return dict(common, name=name, a=0.0, inc_deg=17.0, model="toy_disk",
                    mp=toy_disk_params(), nstokes=1, nx0=64, ny0=64, levels=0,
                    r_rel=-1.0, r_abs=-1.0, abs_norm="mean", freq_hz=230e9)
    if name == "thermal_1025":
        return dict(common, name=name, a=0.94, inc_deg=163.0, model="thermal",
                    mp=thermal_params(seed=1), nstokes=4, nx0=129, ny0=129, levels=3,
                    r_rel=0.01, r_abs=1e-3, abs_norm="max", freq_hz=230e9)
    if name == "grid_4097":
        # gridded snapshot, paper's GRMHD tolerances (Sec. 4.1): R_rel = 1e-3, R_abs = 0.025
        from . import mks
        geo = mks.mks_snapshot_geometry()
        return dict(common, name=name, a=0.94, inc_deg=163.0, model="grid",
                    mp=mks.grid_params(geo), nstokes=4, nx0=257, ny0=257, levels=4,
                    r_rel=1e-3, r_abs=0.025, abs_norm="mean", freq_hz=230e9, snapshot_seed=2)
    if name == "grid_16385":
        # the snapshot refined 6 levels from 257^2 to 16385^2, Stokes I split
        # into subrings n = 0..3 (the learned proposal's deployment size)
        return dict(workload("grid_4097"), name=name, levels=6, nstokes=1, subrings=4)
    if name == "thermal_1025_mixed":
        return dict(workload("thermal_1025"), name=name, precision="mixed")
    raise KeyError(name)


BATCH_SPINS = (0.0, 0.5, 0.94, -0.94)
BATCH_INCS = (17.0, 60.0, 90.0, 163.0)
BATCH_FREQS = (86e9, 230e9, 345e9, 690e9)


def batch_workload(precision="mixed", base=129):
    """64 thermal-plasma images: spin x inclination x frequency in
    lexicographic order, image k refined 1 + (k mod 4) levels
    (129^2 -> 257^2, 513^2, 1025^2, 2049^2)."""
    cfgs = []
    k = 0
    for a in BATCH_SPINS:
        for inc in BATCH_INCS:
            for nu in BATCH_FREQS:
                c = dict(workload("thermal_1025"), name="batch_%02d" % k, a=a, inc_deg=inc,
                         freq_hz=nu, levels=1 + (k % 4), precision=precision,
                         nx0=base, ny0=base)
                cfgs.append(c)
                k += 1
    return cfgs


HELDOUT_SPINS = (0.2, 0.7, 0.9, -0.6)
HELDOUT_INCS = (30.0, 45.0, 115.0, 150.0)


def batch_workload_heldout(precision="mixed", base=129):
    """A batch of the same structure as batch_workload (64 thermal images,
    the same four frequencies, image k refined 1 + (k mod 4) levels) at
    spins, inclinations and field phases (seeds 201..264) disjoint from it
    and from the training images: the batch on which tolerances are chosen
    before they are applied, unchanged, to batch_workload."""
    cfgs = []
    k = 0
    for a in HELDOUT_SPINS:
        for inc in HELDOUT_INCS:
            for nu in BATCH_FREQS:
                cfgs.append(dict(workload("thermal_1025"), name="heldout_%02d" % k, a=a, inc_deg=inc,
                                 freq_hz=nu, levels=1 + (k % 4), precision=precision,
                                 mp=thermal_params(seed=201 + k), nx0=base, ny0=base))
                k += 1
    return cfgs


def batch_workload_1025(precision="mixed"):
    """64 images of the thermal_1025 kind (base 129^2, 3 levels -> 1025^2):
    spin x inclination x frequency in lexicographic order, one level count
    for the whole batch (the learned form's batch)."""
    cfgs = []
    k = 0
    for a in BATCH_SPINS:
        for inc in BATCH_INCS:
            for nu in BATCH_FREQS:
                cfgs.append(dict(workload("thermal_1025"), name="b1025_%02d" % k, a=a, inc_deg=inc,
                                 freq_hz=nu, precision=precision))
                k += 1
    return cfgs


TRAIN_SPINS = (0.3, 0.7, -0.5, 0.99)
TRAIN_INCS = (30.0, 75.0, 120.0, 150.0)


def training_workload(precision="mixed", nx0=129, levels=3):
    """Training images of the learned proposal: thermal plasma at spins and
    inclinations disjoint from the benchmark batch, 230 GHz, plasma field
    phases from seeds 11.., same grid as the images it will refine."""
    cfgs = []
    k = 0
    for a in TRAIN_SPINS:
        for inc in TRAIN_INCS:
            cfgs.append(dict(workload("thermal_1025"), name="train_%02d" % k, a=a, inc_deg=inc,
                             mp=thermal_params(seed=11 + k), precision=precision, nx0=nx0,
                             ny0=nx0, levels=levels))
            k += 1
    return cfgs


BATCH_TRAIN_SPINS = (0.3, -0.3, 0.8, -0.8)
BATCH_TRAIN_INCS = (25.0, 75.0, 105.0, 140.0)


def training_workload_batch(precision="mixed", r_rel=0.005, base=129, levels=4):
    """Training images of the learned proposal for the batched workload: 16
    thermal images on its base grid with four levels (so the network sees the
    grids of both levels it runs at, 129^2 and 513^2), spins, inclinations and
    field phases (seeds 401..416) disjoint from batch_workload and
    batch_workload_heldout, each of the four frequencies at every spin;
    labels come from the criterion at r_rel."""
    cfgs = []
    k = 0
    for a in BATCH_TRAIN_SPINS:
        for inc in BATCH_TRAIN_INCS:
            cfgs.append(dict(workload("thermal_1025"), name="btrain_%02d" % k, a=a, inc_deg=inc,
                             freq_hz=BATCH_FREQS[(k + k // 4) % 4], mp=thermal_params(seed=401 + k),
                             precision=precision, nx0=base, ny0=base, levels=levels, r_rel=r_rel))
            k += 1
    return cfgs


GRID_TRAIN_VIEWS = ((0.94, 17.0), (0.94, 60.0), (0.94, 120.0), (0.5, 163.0))


def grid_training_workload(grid_dev, precision="mixed"):
    """Training images of the snapshot (base 257^2, 4 levels, Stokes I) seen
    from inclinations / spins other than the deployment view (a = 0.94,
    i = 163 deg)."""
    return [dict(workload("grid_4097"), name="gtrain_%d" % k, a=a, inc_deg=inc, nstokes=1,
                 grid_dev=grid_dev, precision=precision)
            for k, (a, inc) in enumerate(GRID_TRAIN_VIEWS)]


def reduced(cfg, nx0, levels):
    """Same physics on a smaller vertex grid (parity-test sizes)."""
    c = dict(cfg)
    c["nx0"] = c["ny0"] = nx0
    c["levels"] = levels
    return c


def vis_image(ny, nx, fov, seed=0, planes=1, ring_radius=None, width=None):
    """Seeded synthetic screen images for visibility tests, float64 numpy
    [planes, ny, nx] on the vertex grid of `fov` (pixel dx = fov / (nx - 1)):
    a thin Gaussian-profile ring with a brightness asymmetry, a few Gaussian
    blobs and a low-amplitude noise floor, different per plane (evaluated with
    torch CPU tensors in bands of rows, for speed at 16385^2)."""
    import torch
    rng = np.random.default_rng(seed)
    dx = fov / (nx - 1)
    x = torch.from_numpy((np.arange(nx) - 0.5 * (nx - 1)) * dx)
    y = torch.from_numpy((np.arange(ny) - 0.5 * (ny - 1)) * dx)
    out = np.empty((planes, ny, nx))
    for p in range(planes):
        r0 = ring_radius if ring_radius is not None else 0.13 * fov * (1.0 + 0.1 * p)
        w = width if width is not None else max(3.0 * dx, 0.01 * fov)
        phase = rng.uniform(0, 6.3)
        blobs = [(rng.uniform(-0.25, 0.25, 2) * fov, rng.uniform(0.02, 0.08) * fov, rng.uniform(0.2, 1.0))
                 for _ in range(3)]
        noise = np.random.default_rng([seed, p])
        for j0 in range(0, ny, 1024):
            yy = y[j0:j0 + 1024]
            Y = yy[:, None].expand(yy.numel(), nx)
            X = x[None, :].expand(yy.numel(), nx)
            r = torch.hypot(X, Y)
            img = torch.exp(-0.5 * ((r - r0) / w) ** 2) * (1.0 + 0.6 * torch.cos(torch.atan2(Y, X) - phase))
            for (cx, cy), s, amp in blobs:
                img += amp * torch.exp(-0.5 * ((X - cx) ** 2 + (Y - cy) ** 2) / (s * s))
            out[p, j0:j0 + 1024] = img.numpy() + 0.01 * noise.random((yy.numel(), nx))
    return out
