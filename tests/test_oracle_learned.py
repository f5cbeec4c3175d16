"""Pins of the learned-refinement oracle (oracle/learned.py) by special cases
that reduce to the paper's method or to brute force:

- a network that proposes nothing and suppresses nothing gives exactly the
  plain refinement of Sec. 3.2 (image, level map, ray count), with every
  level-(l+2) point the criterion flags counted as a fallback trace;
- a network that proposes everything traces every point: the uniform image;
- a network that suppresses everything leaves bilinear interpolation of the
  base grid (the R = infinity case);
- with fallback off, every flagged point that was not traced is counted;
- interpolated points inherit the minimum radius of their neighbours.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import cnn, learned, refine


def ring(x, y):
    r = np.hypot(x, y)
    return np.stack([np.exp(-((r - 8.0) / 1.2) ** 2) + 0.05 * np.exp(-r / 10.0)], -1)


def ray_fn(x, y):
    return ring(x, y), np.hypot(x, y), (np.hypot(x, y) < 8.0).astype(np.int64)


def const_logits(v):
    return lambda x: np.full((15,) + x.shape[1:], float(v))


ARGS = dict(fov=40.0, nx0=9, ny0=7, r_rel=0.01, r_abs=0.01, abs_norm="mean", nstokes=1)


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_silent_network_is_the_plain_method(levels):
    out = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(0.0), z_hi=1.0,
                                 z_lo=-1.0, **ARGS)
    plain = refine.refine(lambda x, y: ring(x, y), ARGS["fov"], ARGS["nx0"], ARGS["ny0"], levels,
                          ARGS["r_rel"], ARGS["r_abs"], "mean", 1)
    assert np.array_equal(out["img"], plain["img"])
    assert np.array_equal(out["level"], plain["level"])
    assert out["rays"] == plain["rays"]
    assert out["judge"][0] == out["judge"][1] == out["judge"][3] == out["judge"][4] == 0
    # the fallback pass traces exactly what the criterion flags at levels l+2
    assert out["judge"][2] == sum(plain["traced"][l + 2] for l in range(0, levels - 1, 2))
    assert out["passes"] == levels + 1


def test_proposing_everything_is_uniform():
    levels = 3
    out = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(10.0), z_hi=1.0,
                                 z_lo=-1.0, all_levels=True, **ARGS)
    nx, ny = refine.grid_size(9, levels), refine.grid_size(7, levels)
    uni = refine.uniform(lambda x, y: ring(x, y), ARGS["fov"], nx, ny)
    assert np.array_equal(out["img"], uni)
    assert (out["level"] >= 0).all()
    # base, levels 1+2 in one pass, the (empty) fallback pass of level 2, level 3
    assert out["passes"] == 4
    off = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(10.0), z_hi=1.0,
                                 z_lo=-1.0, all_levels=True, fallback=False, **ARGS)
    assert np.array_equal(off["img"], uni)
    assert off["passes"] == 3 and off["judge"][3] == 0


def test_suppressing_everything_is_bilinear():
    levels = 2
    out = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(-10.0), z_hi=1.0,
                                 z_lo=-1.0, **ARGS)
    n0x, n0y = ARGS["nx0"], ARGS["ny0"]
    nx, ny = refine.grid_size(n0x, levels), refine.grid_size(n0y, levels)
    dx = 40.0 / (nx - 1)
    xs0 = -20.0 + np.arange(n0x) * dx * 4
    ys0 = -0.5 * dx * (ny - 1) + np.arange(n0y) * dx * 4
    X0, Y0 = np.meshgrid(xs0, ys0)
    rgi = RegularGridInterpolator((ys0, xs0), ring(X0, Y0)[..., 0])
    X, Y = np.meshgrid(-20.0 + np.arange(nx) * dx, -0.5 * dx * (ny - 1) + np.arange(ny) * dx)
    ref = rgi(np.stack([Y.ravel(), X.ravel()], -1)).reshape(ny, nx)
    assert np.abs(out["img"][0] - ref).max() < 1e-14
    assert out["rays"] == n0x * n0y
    assert out["judge"][1] > 0 and out["judge"][2] == 0


def test_judge_counts_missed_points_without_fallback():
    levels = 2
    on = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(0.0), z_hi=1.0,
                                z_lo=-1.0, fallback=True, **ARGS)
    off = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(0.0), z_hi=1.0,
                                 z_lo=-1.0, fallback=False, **ARGS)
    assert off["judge"][3] == on["judge"][2] > 0
    assert off["rays"] == on["rays"] - on["judge"][2]
    assert off["passes"] == on["passes"] - 1


def test_interpolated_points_inherit_neighbour_features():
    levels = 2
    out = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(-10.0), z_hi=1.0,
                                 z_lo=-1.0, **ARGS)
    rm = out["rmin"]
    lev = out["level"]
    # level-1 edge midpoint between two base points: min of the two
    s = 2
    p, q = 1, 0                        # level-1 units
    assert lev[q * s, p * s] == -1
    assert rm[q * s, p * s] == min(rm[0, 0], rm[0, 2 * s])
    # level-1 centre: min of four corners
    p, q = 1, 1
    corners = [rm[0, 0], rm[0, 2 * s], rm[2 * s, 0], rm[2 * s, 2 * s]]
    assert rm[q * s, p * s] == min(corners)


def test_level_cap_hands_deeper_levels_to_the_criterion():
    """With level_cap = 1 a network that proposes everything traces the
    level-2 grid completely (one look-ahead pass) and the criterion alone
    refines levels 3 and 4: the plain method started from the level-2 grid
    (with R_abs = 0 the normalisation, which differs between the two, plays
    no part).  A cap at or above the deepest network level changes nothing."""
    levels = 4
    a = dict(ARGS, r_abs=0.0)
    out = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(10.0), z_hi=1.0, z_lo=-1.0,
                                 level_cap=1, **a)
    nx0b, ny0b = refine.grid_size(9, 2), refine.grid_size(7, 2)
    plain = refine.refine(lambda x, y: ring(x, y), a["fov"], nx0b, ny0b, 2, a["r_rel"], 0.0, "mean", 1)
    assert np.array_equal(out["img"], plain["img"])
    deeper = plain["level"] >= 1
    assert np.array_equal(out["level"][deeper], plain["level"][deeper] + 2)
    assert np.all((out["level"][~deeper] >= 0) & (out["level"][~deeper] <= 2) | (plain["level"][~deeper] < 0))
    assert out["passes"] == 5 and plain["rays"] > plain["traced"][0]
    assert all(np.all(np.isinf(x["zmargin"])) for x in out["audit"][-2:])
    full = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(3.0), z_hi=1.0, z_lo=-1.0, **ARGS)
    capped = learned.refine_learned(ray_fn, levels=levels, logits_fn=const_logits(3.0), z_hi=1.0, z_lo=-1.0,
                                    level_cap=3, **ARGS)
    assert np.array_equal(full["level"], capped["level"]) and np.array_equal(full["img"], capped["img"])
