"""Pins of the oracle's adaptive sampling along frequency (Sec. 6 extension of
the Sec. 3.2 recursion).

- Cube geometry: n = 2^L (n0 - 1) + 1 images equally spaced in ln nu, the
  spectral level and stencil of every index.
- R = -1 on the spectral axis reproduces independent plain adaptive renders
  at every frequency (bitwise); R = +inf takes the spectral mean wherever a
  continuation exists (no rays there).
- A spectrum linear in ln nu has D = 0: no point of a new frequency is
  traced and its base points equal the truth; a quadratic one has
  D = 16 A h^2 in the two-sided and both one-sided forms, i.e. the estimate
  D/8 is twice the true interpolation error A h^2 (as for the spatial axis).
- Monotone in the tolerance; a mask-forced replay reproduces every image;
  the per-plane option sees a spectral feature only in the second plane.
"""
import numpy as np
import pytest

from oracle import refine as oref
from oracle import spectral as osp

NU0 = 230e9


def ring(x, y):
    r = np.hypot(x, y)
    return np.exp(-0.5 * ((r - 5.0) / 0.6) ** 2) + 0.05 * np.exp(-0.5 * (r / 6.0) ** 2)


def make_fn(A=0.3, B=0.0, second=None, tilt=0.1, btilt=0.0):
    """I(x, y, nu) = ring(x, y) (1 + A (1 + tilt x) u + B (1 + btilt x) u^2), u = ln(nu / NU0)."""
    def fn_nu(nu):
        u = np.log(nu / NU0)

        def fn(x, y):
            x = np.asarray(x, dtype=float)
            y = np.asarray(y, dtype=float)
            base = ring(x, y)
            p0 = base * (1.0 + A * (1.0 + tilt * x) * u + B * (1.0 + btilt * x) * u * u)
            if second is None:
                return p0[:, None]
            return np.stack([p0, second(x, y, u)], axis=1)
        return fn
    return fn_nu


COMMON = dict(fov=20.0, nx0=9, ny0=9, levels=2, r_rel=0.01, r_abs=1e-3, nu_min=86e9, nu_max=690e9)


def cube(fn_nu, n0=3, slevels=2, sr=(1e-3, 1e-3), nstokes=1, all_planes=False, forced=None):
    c = COMMON
    return osp.render_spectral(fn_nu, c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"],
                               c["nu_min"], c["nu_max"], n0, slevels, sr[0], sr[1], nstokes=nstokes,
                               all_planes=all_planes, forced_levels=forced)


def test_cube_geometry():
    assert osp.cube_size(3, 2) == 9 and osp.cube_size(2, 0) == 2
    nus = osp.frequencies(86e9, 690e9, 3, 2)
    assert nus.size == 9 and np.isclose(nus[0], 86e9) and np.isclose(nus[-1], 690e9)
    assert np.allclose(np.diff(np.log(nus)), np.log(690 / 86) / 8)
    assert [osp.spectral_level(i, 2) for i in range(9)] == [0, 2, 1, 2, 0, 2, 1, 2, 0]
    assert osp.neighbours(0, 9, 2) is None
    assert osp.neighbours(2, 9, 2) == (None, 0, 4, 8)
    assert osp.neighbours(6, 9, 2) == (0, 4, 8, None)
    assert osp.neighbours(3, 9, 2) == (0, 2, 4, 6)
    assert osp.neighbours(1, 9, 2) == (None, 0, 2, 4)


def test_negative_tolerance_is_plain_per_frequency():
    fn = make_fn(A=0.4, B=0.5)
    res, nus = cube(fn, sr=(-1.0, -1.0))
    c = COMMON
    for i, nu in enumerate(nus):
        ref = oref.refine(fn(nu), c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"])
        assert np.array_equal(res[i]["img"], ref["img"]), i
        assert np.array_equal(res[i]["level"], ref["level"]), i
        assert res[i]["spectral"] == 0


def test_linear_spectrum_traces_nothing_new():
    # separable: the same spatial decisions at every frequency, so every
    # stencil sees values exactly linear in ln nu
    fn = make_fn(A=0.3, B=0.0, tilt=0.0)
    res, nus = cube(fn, n0=3, slevels=2)
    st0 = 1 << COMMON["levels"]
    for i, nu in enumerate(nus):
        if osp.spectral_level(i, 2) == 0:
            continue
        assert res[i]["rays"] == 0, (i, res[i]["traced"])
        assert res[i]["spectral"] > 0
        img = res[i]["img"][0]
        jj, ii = np.meshgrid(np.arange(9) * st0, np.arange(9) * st0, indexing="ij")
        from oracle.ray import screen_coords
        x, y = screen_coords(COMMON["fov"], img.shape[1], img.shape[0], ii.ravel(), jj.ravel())
        truth = fn(nu)(x, y)[:, 0].reshape(9, 9)
        assert np.abs(img[jj, ii] - truth).max() <= 1e-12 * np.abs(truth).max()


def test_quadratic_second_difference():
    A, h, u0 = 0.7, 0.13, 0.4
    f = lambda u: A * u * u * np.ones(3)
    a, b, c, d = f(u0 - 3 * h), f(u0 - h), f(u0 + h), f(u0 + 3 * h)
    err = 0.5 * (b + c) - f(u0)
    assert np.allclose(err, A * h * h)
    for args in ((a, b, c, d), (None, b, c, d), (a, b, c, None)):
        D, inf = osp.second_difference(*args)
        assert not inf.any()
        assert np.allclose(D, 16 * A * h * h, rtol=1e-12)
        assert np.allclose(D / 8.0, 2.0 * err)
    D, inf = osp.second_difference(None, b, c, None)
    assert inf.all()


def test_infinite_tolerance_takes_the_spectral_mean():
    fn = make_fn(A=0.5, B=2.0)
    res, nus = cube(fn, n0=3, slevels=2, sr=(np.inf, np.inf))
    st0 = 1 << COMMON["levels"]
    jj, ii = np.meshgrid(np.arange(9) * st0, np.arange(9) * st0, indexing="ij")
    for i in range(9):
        nb = osp.neighbours(i, 9, 2)
        if nb is None:
            continue
        assert res[i]["rays"] == 0
        _, b, c, _ = nb
        assert np.array_equal(res[i]["img"][:, jj, ii], 0.5 * (res[b]["img"][:, jj, ii] + res[c]["img"][:, jj, ii]))
        assert (res[i]["level"][jj, ii] == oref.SPECTRAL).all()


def test_two_base_frequencies_trace_the_first_level():
    # n0 = 2: the level-1 image has no continuation on either side
    fn = make_fn(A=0.3)
    res, nus = cube(fn, n0=2, slevels=1, sr=(np.inf, np.inf))
    c = COMMON
    ref = oref.refine(fn(nus[1]), c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"])
    assert res[1]["spectral"] == 0 and res[1]["traced"][0] == 81
    assert np.array_equal(res[1]["img"], ref["img"]) and np.array_equal(res[1]["level"], ref["level"])


def test_monotone_in_tolerance():
    fn = make_fn(A=0.5, B=1.5)
    rays = []
    for sr in (1e-4, 1e-3, 1e-2, 1e-1):
        res, _ = cube(fn, sr=(sr, sr))
        rays.append(sum(r["rays"] for r in res))
    assert all(x >= y for x, y in zip(rays, rays[1:])), rays
    assert rays[0] > rays[-1]


def test_forced_replay_reproduces_the_cube():
    fn = make_fn(A=0.5, B=1.5)
    res, _ = cube(fn, sr=(3e-3, 3e-3))
    rep, _ = cube(fn, sr=(3e-3, 3e-3), forced=[r["level"] for r in res])
    for r, q in zip(res, rep):
        assert np.array_equal(r["img"], q["img"]) and np.array_equal(r["level"], q["level"])


def test_per_plane_check_sees_the_second_plane():
    second = lambda x, y, u: ring(x, y) * np.cos(3.0 * u)       # strongly curved in ln nu
    fn = make_fn(A=0.3, B=0.0, second=second, tilt=0.0)
    res1, _ = cube(fn, nstokes=2, all_planes=False)
    res2, _ = cube(fn, nstokes=2, all_planes=True)
    new = [i for i in range(9) if osp.spectral_level(i, 2) > 0]
    assert sum(res1[i]["rays"] for i in new) == 0
    assert sum(res2[i]["rays"] for i in new) > 0


def test_threshold_is_twice_the_true_error_against_the_bracketing_norm():
    # I = ring(x, y) (1 + B u^2): at the middle frequency of 4 base ones the
    # spectral mean misses by ring B h^2 exactly, the estimate is twice that,
    # and a base point is traced iff 2 ring B h^2 > R_abs N_abs, N_abs the mean
    # of the two bracketing images' level-0 means (R_rel = 0: relative test off)
    from oracle.ray import screen_coords
    B = 0.8
    fn = make_fn(A=0.0, B=B, tilt=0.0)
    c = COMMON
    n0, L = 4, 1
    nus = osp.frequencies(c["nu_min"], c["nu_max"], n0, L)
    h = np.log(nus[1] / nus[0])
    st0 = 1 << c["levels"]
    nx = st0 * (c["nx0"] - 1) + 1
    jj, ii = np.meshgrid(np.arange(c["ny0"]) * st0, np.arange(c["nx0"]) * st0, indexing="ij")
    x, y = screen_coords(c["fov"], nx, nx, ii.ravel(), jj.ravel())
    rg = ring(x, y).reshape(c["ny0"], c["nx0"])
    w = np.ones(c["nx0"])
    w[0] = w[-1] = 0.5
    ring_mean = (w[:, None] * w[None, :] * rg).sum() / ((c["nx0"] - 1) * (c["ny0"] - 1))
    s = lambda nu: 1.0 + B * np.log(nu / NU0) ** 2
    n_abs = 0.5 * (s(nus[2]) + s(nus[4])) * ring_mean
    est = 2.0 * rg * B * h * h
    r_abs = float(np.median(est[est > 1e-3 * est.max()]) / n_abs)
    res, _ = osp.render_spectral(fn, c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"],
                                 c["nu_min"], c["nu_max"], n0, L, 0.0, r_abs)
    traced = res[3]["level"][jj, ii] == 0
    want = est > r_abs * n_abs
    assert 0 < want.sum() < want.size
    assert np.array_equal(traced, want)


def test_relative_threshold_is_twice_the_true_relative_error():
    # B varies across the screen, R_abs = 0 (absolute test on): a base point of
    # the middle frequency is traced iff 2 |B(x)| h^2 ring / ((b + c)/2) > R_rel
    from oracle.ray import screen_coords
    c = COMMON
    B0, bt = 0.8, 0.08
    fn = make_fn(A=0.0, B=B0, tilt=0.0, btilt=bt)
    n0, L = 4, 1
    nus = osp.frequencies(c["nu_min"], c["nu_max"], n0, L)
    h = np.log(nus[1] / nus[0])
    st0 = 1 << c["levels"]
    nx = st0 * (c["nx0"] - 1) + 1
    jj, ii = np.meshgrid(np.arange(c["ny0"]) * st0, np.arange(c["nx0"]) * st0, indexing="ij")
    x, y = screen_coords(c["fov"], nx, nx, ii.ravel(), jj.ravel())
    x = x.reshape(c["ny0"], c["nx0"])
    Bx = B0 * (1.0 + bt * x)
    ub, uc = np.log(nus[2] / NU0), np.log(nus[4] / NU0)
    mean_bc = 0.5 * ((1.0 + Bx * ub * ub) + (1.0 + Bx * uc * uc))
    est = 2.0 * np.abs(Bx) * h * h / mean_bc
    u = np.unique(est)
    r_rel = float(0.5 * (u[u.size // 2] + u[u.size // 2 + 1]))     # between two distinct values
    res, _ = osp.render_spectral(fn, c["fov"], c["nx0"], c["ny0"], c["levels"], c["r_rel"], c["r_abs"],
                                 c["nu_min"], c["nu_max"], n0, L, r_rel, 0.0)
    traced = res[3]["level"][jj, ii] == 0
    want = est > r_rel
    assert 0 < want.sum() < want.size
    assert np.array_equal(traced, want)
