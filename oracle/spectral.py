"""Adaptive sampling along frequency or time (test oracle).

Test infrastructure only.  The paper closes (Sec. 6) by proposing to extend
the recursive subdivision of Sec. 3.2 to the frequency and time domains.
The cube below is written for frequency; the same rule along any equally
spaced sequence axis (snapshots of a movie at a fixed cadence) is
render_cube.
This module is this project's reading of that extension, built from the
paper's own one-axis rule:

* A spectral cube has n = 2^L (n0 - 1) + 1 images at frequencies equally
  spaced in ln nu between nu_min and nu_max (the grid-size equation of
  Sec. 3.2 along a third axis).  Images at indices k 2^L are the base
  frequencies; spectral level s adds the indices that are odd multiples of
  h = 2^(L-s), midway (in ln nu) between two images of the coarser levels.
* Base-frequency images are plain adaptive renders (Sec. 3.2).
* An image of spectral level s is an adaptive render whose points may take a
  cheaper value than a ray: for every base point and every point the spatial
  criterion flags, the one-axis criterion of Sec. 3.2 (categories 2-3) is
  evaluated along ln nu at the same pixel, with the bracketing images b, c
  (indices i -+ h) and the continuations a, d (indices i -+ 3h) of the
  finished coarser levels:
      D = (a + d) - (b + c)     (both continuations; the same edge reading as
                                 the spatial criterion: twice the one-sided
                                 second difference if one is missing, trace if
                                 both are),
      trace iff |D| > 8 R_abs N_abs  and  |D| > 4 R_rel |b + c|,
  with N_abs the mean of the two bracketing images' own N_abs; otherwise the
  point takes (b + c) / 2 on every plane (level-map mark SPECTRAL).  With the
  per-plane option the check is the OR over planes, as for the spatial
  criterion.
"""
import numpy as np

from . import refine as oref
from .refine import _axis_terms


def cube_size(n0, levels):
    return (1 << levels) * (n0 - 1) + 1


def frequencies(nu_min, nu_max, n0, levels):
    """Frequencies of the cube, equally spaced in ln nu."""
    n = cube_size(n0, levels)
    if n == 1:
        return np.array([float(nu_min)])
    t = np.arange(n) / (n - 1.0)
    return float(nu_min) * (float(nu_max) / float(nu_min)) ** t


def spectral_level(i, levels):
    """Spectral level of cube index i (0 for base frequencies)."""
    if i % (1 << levels) == 0:
        return 0
    s = levels
    while i % 2 == 0:
        i //= 2
        s -= 1
    return s


def neighbours(i, n, levels):
    """(a, b, c, d) cube indices of image i's spectral stencil (None outside)."""
    s = spectral_level(i, levels)
    if s == 0:
        return None
    h = 1 << (levels - s)

    def ok(k):
        return k if 0 <= k < n else None
    return ok(i - 3 * h), ok(i - h), ok(i + h), ok(i + 3 * h)


def second_difference(a, b, c, d, with_mag=False):
    """The spectral D of the stencil (arrays; a or d may be None); with_mag
    also the magnitude sum of its terms."""
    has_a = a is not None
    has_d = d is not None
    z = np.zeros_like(b)
    out = _axis_terms(b, c, a if has_a else z, d if has_d else z,
                      np.full(b.shape, has_a), np.full(b.shape, has_d), with_mag)
    return out[1:] if with_mag else (out[1], out[2])


def spectral_alt(imgs, nabs, stencil, r_rel, r_abs, all_planes=False):
    """alt(i, j) for oracle.refine: the spectral check and value at final-grid
    points (i, j) from the finished images of the stencil (a, b, c, d), with
    the tie margin of the check (see oracle.refine.and_margin)."""
    ia, ib, ic, id_ = stencil
    n_abs = 0.5 * (nabs[ib] + nabs[ic])
    thrA = 8.0 * r_abs * n_abs
    crel = 4.0 * r_rel

    def alt(ii, jj):
        ii = np.asarray(ii)
        jj = np.asarray(jj)
        b = imgs[ib][:, jj, ii]
        c = imgs[ic][:, jj, ii]
        a = imgs[ia][:, jj, ii] if ia is not None else None
        d = imgs[id_][:, jj, ii] if id_ is not None else None
        S = b + c
        magS = np.abs(b[0]) + np.abs(c[0])
        planes = range(b.shape[0]) if all_planes else range(1)
        decs, margins = [], []
        with np.errstate(invalid="ignore"):
            for st in planes:
                Dp, inf, mag = second_difference(a[st] if a is not None else None, b[st], c[st],
                                                 d[st] if d is not None else None, with_mag=True)
                dd, mg = oref.linear_margin(Dp, S[0], mag, magS, thrA, crel)
                forced = inf | np.isnan(Dp)
                decs.append(dd | forced)
                margins.append(np.where(forced, np.inf, mg))
            bad, margin = oref.or_margin(decs, margins)
            nan0 = np.isnan(S[0])
            bad = bad | nan0
            margin = np.where(nan0, np.inf, margin)
        return ~bad, S * 0.5, margin
    return alt


def render_cube(ray_fn_k, fov, nx0, ny0, levels, r_rel, r_abs, n0, slevels, sr_rel, sr_abs,
                abs_norm="mean", nstokes=1, all_planes=False, forced_levels=None):
    """Cube along any equally spaced sequence axis (time, ln nu, ...).

    ray_fn_k(k) -> ray_fn(x, y) of cube image k.  Returns results[k] =
    oracle.refine's dict of image k, in axis order.  forced_levels: optional
    list of final-grid level maps (mask-forced replay of every image)."""
    n = cube_size(n0, slevels)
    res = [None] * n
    order = [i for i in range(n) if spectral_level(i, slevels) == 0]
    for s in range(1, slevels + 1):
        order += [i for i in range(n) if spectral_level(i, slevels) == s]
    for i in order:
        fl = forced_levels[i] if forced_levels is not None else None
        alt = None
        st = neighbours(i, n, slevels)
        if st is not None:
            imgs = {k: res[k]["img"] for k in st if k is not None}
            nabs = {k: res[k]["n_abs"] for k in st if k is not None}
            alt = spectral_alt(imgs, nabs, st, sr_rel, sr_abs, all_planes)
        res[i] = oref.refine(ray_fn_k(i), fov, nx0, ny0, levels, r_rel, r_abs, abs_norm, nstokes,
                             forced_level=fl, all_planes=all_planes, alt=alt)
    return res


def render_spectral(ray_fn_nu, fov, nx0, ny0, levels, r_rel, r_abs, nu_min, nu_max, n0, slevels,
                    sr_rel, sr_abs, abs_norm="mean", nstokes=1, all_planes=False, forced_levels=None):
    """Spectral cube: the cube along ln nu.  ray_fn_nu(nu) -> ray_fn(x, y) of
    that frequency.  Returns (results, frequencies)."""
    nus = frequencies(nu_min, nu_max, n0, slevels)
    res = render_cube(lambda k: ray_fn_nu(nus[k]), fov, nx0, ny0, levels, r_rel, r_abs, n0, slevels,
                      sr_rel, sr_abs, abs_norm, nstokes, all_planes, forced_levels)
    return res, nus
