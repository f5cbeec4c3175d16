"""Level-by-level adaptive refinement, written from the paper (test oracle).

Test infrastructure only.  Follows Gelles et al. 2021:

* Sec. 3.2 ("Adaptive Ray-Tracing by Recursive Subdivision"): trace an
  n0x x n0y vertex grid, then refine by factors of two, (n) -> (2n-1) points
  per axis, N times, giving n_x = 2^N (n0x - 1) + 1 (the grid-size equation).
* Decision rule (Sec. 3.2, after Eqs. 3-4): a new point is ray traced iff the
  estimated absolute error exceeds R_abs AND the estimated relative error
  exceeds R_rel; otherwise it is interpolated.
* Point categories 1-4 (Sec. 3.2, Fig. 2 list): already computed / between
  two points above and below / between left and right / centre of four
  corners.  Estimates use the level-n values only.
* Linear branch of Eqs. 5-6 (and App. A.2): with the four corners and the
  four continuations on the two diagonals,
      eps_abs = |(I5+I6+I7+I8) - (I1+I2+I3+I4)| / (16 Ibar_int)
      eps_rel = |(I5+I6+I7+I8) - (I1+I2+I3+I4)| / (4 (I1+I2+I3+I4)),
  and the interpolated value is the corner mean (Eq. 14).  Categories 2-3 are
  the one-axis simplification (App. A), read here as
      eps_abs = |a+d-b-c| / (8 Ibar_int),  eps_rel = |a+d-b-c| / (4 |b+c|).
* Ibar_int (Sec. 3.2, after Eq. 6): average of the level-0 interpolant, i.e.
  the trapezoid-weighted mean of the base grid, fixed after the first pass.
  Alternatively the level-0 maximum (a "1e-3 max I" tolerance).

Readings where the paper is silent (App. A last paragraph: "appropriate
modifications" at the edge): per axis, if one continuation point falls outside
the image, the available one-sided second difference counts twice; if both
fall outside, the axis is unavailable.  A centre point (category 4) with one
diagonal unavailable uses twice the other diagonal's term; a point with no
available axis is traced.  A NaN anywhere in the stencil traces.
The decision is evaluated without division: trace iff
|D| > (4 m R_abs) N_abs  and  |D| > (4 R_rel) |S|, m = 2 (1D) or 4 (2D).

Nearest branch of Eqs. 5-6: eps_abs = G / Ibar_int, eps_rel = G / |I_nn| with
G = sqrt(((I4-I1)/2)^2 + ((I3-I2)/2)^2) and I_nn = I1 (the nearest neighbour
"chosen arbitrarily" as I1); in 1D G = |c-b|/2 and I_nn = b (reading).  The
interpolated value is I_nn.  Per-plane criterion (option, A11 reading): the
OR of the criterion over every plane, each plane's estimate compared with
N_abs and with |Stokes I| (S or I_nn of plane 0).
"""
import numpy as np

from .ray import screen_coords


def grid_size(n0, levels):
    """n = 2^N (n0 - 1) + 1 (Sec. 3.2)."""
    return (1 << levels) * (n0 - 1) + 1


def trapezoid_mean(I0):
    """Mean of the bilinear interpolant of the base grid over the field of view
    (trapezoid weights: 1/2 on edges, 1/4 in corners)."""
    ny, nx = I0.shape
    wx = np.ones(nx)
    wx[0] = wx[-1] = 0.5
    wy = np.ones(ny)
    wy[0] = wy[-1] = 0.5
    return float((wy[:, None] * wx[None, :] * I0).sum() / ((nx - 1) * (ny - 1)))


def _axis_terms(lo_in, hi_in, lo_out, hi_out, has_lo, has_hi, with_mag=False):
    """Pair sum P = in_lo + in_hi and second-difference sum D for one axis.

    D = (out_lo + out_hi) - P with both continuations present; twice the
    available one-sided second difference if one is missing.  `inf` marks an
    axis with both continuations outside the image (unavailable).  With
    with_mag, also the sum of the magnitudes of the terms of D (what a
    relative perturbation of the values can move D by, per unit).
    """
    P = lo_in + hi_in
    both = has_lo & has_hi
    D = np.where(both, (lo_out + hi_out) - P, 0.0)
    only_hi = ~has_lo & has_hi      # low continuation outside: use high side
    D = np.where(only_hi, 2.0 * ((hi_out - 2.0 * hi_in) + lo_in), D)
    only_lo = has_lo & ~has_hi
    D = np.where(only_lo, 2.0 * ((lo_out - 2.0 * lo_in) + hi_in), D)
    inf = ~has_lo & ~has_hi
    if not with_mag:
        return P, D, inf
    a = np.abs
    mag = np.where(both, a(lo_out) + a(hi_out) + a(lo_in) + a(hi_in), 0.0)
    mag = np.where(only_hi, 2.0 * (a(hi_out) + 2.0 * a(hi_in) + a(lo_in)), mag)
    mag = np.where(only_lo, 2.0 * (a(lo_out) + 2.0 * a(lo_in) + a(hi_in)), mag)
    return P, D, inf, mag


def and_margin(gaps, scales):
    """Decision of an AND of tests `gap_k > 0` and its tie margin: the
    smallest relative perturbation of the inputs that can change it, given
    that a relative perturbation eta moves gap_k by at most eta * scale_k.
    True decision: the easiest test to break; false: every failing test has
    to pass."""
    with np.errstate(invalid="ignore", divide="ignore"):
        eta = [np.where(sc > 0, np.abs(g) / sc, np.inf) for g, sc in zip(gaps, scales)]
        ok = [g > 0 for g in gaps]
    dec = np.logical_and.reduce(ok)
    m_true = np.minimum.reduce(eta)
    m_false = np.maximum.reduce([np.where(o, 0.0, e) for o, e in zip(ok, eta)])
    return dec, np.where(dec, m_true, m_false)


def or_margin(decs, margins):
    """OR over planes: true flips only if every true plane flips (largest of
    their margins); false flips if any plane turns true (smallest margin)."""
    dec = np.logical_or.reduce(decs)
    m_true = np.maximum.reduce([np.where(d, m, 0.0) for d, m in zip(decs, margins)])
    m_false = np.minimum.reduce(margins)
    return dec, np.where(dec, m_true, m_false)


def linear_margin(D, S, magD, magS, thrA, crel):
    """The linear-branch test |D| > thrA and |D| > crel |S| (Eqs. 5-6 without
    division) with its tie margin; thrA moves with N_abs (a mean or maximum
    of level-0 values), crel |S| with the neighbour magnitudes magS."""
    absD = np.abs(D)
    return and_margin([absD - thrA, absD - crel * np.abs(S)],
                      [magD + thrA, magD + crel * magS])


def level_stencil(img, nx0, ny0, l, s, nstokes, all_planes=False, with_mag=False, mag_all=False):
    """Stencil sums for every new point of level l+1 (Sec. 3.2 categories 2-4).

    img holds the level-l values at multiples of 2s (final-grid units).
    Returns the new points' level-(l+1) indices (p, q), the neighbour sums
    S per Stokes plane, the second-difference sum D of Stokes I (of every
    plane, shape (nstokes, n), with all_planes), the no-available-axis flag
    and the neighbour count m.  with_mag adds the magnitude sums of D's terms
    (same shape as D) and of Stokes I's neighbours (for tie margins; of every
    plane's neighbours, shape (nstokes, n), with mag_all).
    """
    nxl, nyl = grid_size(nx0, l + 1), grid_size(ny0, l + 1)
    q, p = np.meshgrid(np.arange(nyl), np.arange(nxl), indexing="ij")
    new = (p % 2 == 1) | (q % 2 == 1)
    p, q = p[new], q[new]
    cat2 = (p % 2 == 0) & (q % 2 == 1)   # between below/above (y axis)
    cat3 = (p % 2 == 1) & (q % 2 == 0)   # between left/right (x axis)
    cat4 = (p % 2 == 1) & (q % 2 == 1)   # centre of four corners

    def val(pp, qq, st):
        ok = (pp >= 0) & (pp < nxl) & (qq >= 0) & (qq < nyl)
        pc = np.clip(pp, 0, nxl - 1) * s
        qc = np.clip(qq, 0, nyl - 1) * s
        return img[st, qc, pc], ok

    npt = p.size
    S_all = np.zeros((nstokes, npt))
    nd = nstokes if all_planes else 1
    D = np.zeros((nd, npt))
    magD = np.zeros((nd, npt))
    magS = np.zeros((nstokes, npt))
    inf = np.zeros(npt, dtype=bool)
    m = np.where(cat4, 4.0, 2.0)
    # categories 2 and 3: one axis (dx, dy) = (0, 1) or (1, 0)
    for cat, (dx, dy) in ((cat2, (0, 1)), (cat3, (1, 0))):
        pc, qc = p[cat], q[cat]
        for st in range(nstokes):
            lo_in, _ = val(pc - dx, qc - dy, st)
            hi_in, _ = val(pc + dx, qc + dy, st)
            S_all[st, cat] = lo_in + hi_in
            magS[st, cat] = np.abs(lo_in) + np.abs(hi_in)
        for st in range(nd):
            lo_in, _ = val(pc - dx, qc - dy, st)
            hi_in, _ = val(pc + dx, qc + dy, st)
            lo_out, has_lo = val(pc - 3 * dx, qc - 3 * dy, st)
            hi_out, has_hi = val(pc + 3 * dx, qc + 3 * dy, st)
            _, Dc, infc, mc = _axis_terms(lo_in, hi_in, lo_out, hi_out, has_lo, has_hi, True)
            D[st, cat] = Dc
            magD[st, cat] = mc
            inf[cat] = infc
    # category 4: diagonals x' (I1 -> I4, outer I5, I8), y' (I2 -> I3, outer I6, I7)
    pc, qc = p[cat4], q[cat4]
    for st in range(nstokes):
        i1, _ = val(pc - 1, qc - 1, st)
        i4, _ = val(pc + 1, qc + 1, st)
        i2, _ = val(pc + 1, qc - 1, st)
        i3, _ = val(pc - 1, qc + 1, st)
        S_all[st, cat4] = (i1 + i4) + (i2 + i3)
        magS[st, cat4] = np.abs(i1) + np.abs(i4) + np.abs(i2) + np.abs(i3)
    for st in range(nd):
        i1, _ = val(pc - 1, qc - 1, st)
        i4, _ = val(pc + 1, qc + 1, st)
        i2, _ = val(pc + 1, qc - 1, st)
        i3, _ = val(pc - 1, qc + 1, st)
        i5, h5 = val(pc - 3, qc - 3, st)
        i8, h8 = val(pc + 3, qc + 3, st)
        i6, h6 = val(pc + 3, qc - 3, st)
        i7, h7 = val(pc - 3, qc + 3, st)
        _, Dx, infx, mx = _axis_terms(i1, i4, i5, i8, h5, h8, True)
        _, Dy, infy, my = _axis_terms(i2, i3, i6, i7, h6, h7, True)
        D[st, cat4] = np.where(infx, 2.0 * Dy, np.where(infy, 2.0 * Dx, Dx + Dy))
        magD[st, cat4] = np.where(infx, 2.0 * my, np.where(infy, 2.0 * mx, mx + my))
        inf[cat4] = infx & infy
    out = (p, q, S_all, (D if all_planes else D[0]), inf, m)
    if with_mag:
        out = out + ((magD if all_planes else magD[0]), (magS if mag_all else magS[0]))
    return out


def nearest_stencil(img, nx0, ny0, l, s, nstokes):
    """Nearest-neighbour branch of Eqs. 5-6 for every new point of level l+1.

    The nearest neighbour is the point's lower-left level-l neighbour: b (the
    lower of the two neighbours on the point's axis) for categories 2-3, I1
    for category 4.  Returns (p, q), the nearest values per plane (the
    interpolated value) and the gradient magnitude per plane,
    G = |c - b| / 2 (1D) or sqrt(((I4 - I1)/2)^2 + ((I3 - I2)/2)^2) (2D).
    """
    nxl, nyl = grid_size(nx0, l + 1), grid_size(ny0, l + 1)
    q, p = np.meshgrid(np.arange(nyl), np.arange(nxl), indexing="ij")
    new = (p % 2 == 1) | (q % 2 == 1)
    p, q = p[new], q[new]
    cat2 = (p % 2 == 0) & (q % 2 == 1)   # between below (b) and above (c)
    cat3 = (p % 2 == 1) & (q % 2 == 0)   # between left (b) and right (c)
    cat4 = (p % 2 == 1) & (q % 2 == 1)   # corners I1 (-,-), I4 (+,+), I2 (+,-), I3 (-,+)
    Inn = np.zeros((nstokes, p.size))
    G = np.zeros((nstokes, p.size))
    for st in range(nstokes):
        def val(sel, dp, dq):
            return img[st, (q[sel] + dq) * s, (p[sel] + dp) * s]
        for sel, (dp, dq) in ((cat2, (0, 1)), (cat3, (1, 0))):
            b = val(sel, -dp, -dq)
            c = val(sel, dp, dq)
            Inn[st, sel] = b
            G[st, sel] = np.abs(c - b) / 2.0
        i1, i4 = val(cat4, -1, -1), val(cat4, 1, 1)
        i2, i3 = val(cat4, 1, -1), val(cat4, -1, 1)
        Inn[st, cat4] = i1
        G[st, cat4] = np.sqrt(((i4 - i1) / 2.0) ** 2 + ((i3 - i2) / 2.0) ** 2)
    return p, q, Inn, G


SPECTRAL = -3     # level-map mark: value taken from the spectral alternative


def refine(ray_fn, fov, nx0, ny0, levels, r_rel, r_abs, abs_norm="mean",
           nstokes=1, forced_level=None, interp="linear", all_planes=False, alt=None):
    """Adaptive image by recursive subdivision.

    ray_fn(x, y) -> (n, nstokes) array: traces screen points (nstokes = the
    number of image planes).
    forced_level: optional final-grid int array; if given, a candidate at
    level l+1 is traced iff forced_level == l+1 (mask-forced replay).
    interp: "linear" (Eqs. 5-6 linear branch, interpolation by the neighbour
    mean) or "nearest" (Eqs. 5-6 nearest branch, the nearest neighbour's
    value).  all_planes: the decision is the OR of the criterion over every
    plane, each plane's estimate measured against N_abs and |Stokes I|;
    all_planes="own": each plane measured against its own normalisation (the
    trapezoid mean, or with abs_norm="max" the maximum, of |plane| over the
    base grid) and its own neighbour sum |S_plane| (linear branch), so a
    faint plane (a high-order subring, polarisation) is refined where it has
    structure of its own.
    alt: optional cheaper source of values, alt(i, j) -> (ok, values) for
    final-grid points (i, j); it is consulted for every base point and for
    every point the criterion flags, and points where ok holds take its
    values (level-map mark SPECTRAL) instead of being traced.  An alt may
    also return (ok, values, margin).

    Returns dict(img=(nstokes, ny, nx), level=(ny, nx) int8 with -1 for
    interpolated and l for traced at level l, n_abs, ibar, imax0, per-level
    candidate and traced counts, and `audit`: per level (0 = the base
    points' alternative check, if any) the final-grid points (i, j) judged,
    the state this oracle's own rule gives them from its own values (-1
    interpolated, the level if traced, SPECTRAL) and the tie margin of that
    decision (the smallest relative perturbation of the values it reads
    that could change it; inf where no perturbation can).  In a forced
    replay the image follows forced_level while the audit records what the
    rule itself would have decided at each point, given the same history.
    """
    nx, ny = grid_size(nx0, levels), grid_size(ny0, levels)
    img = np.full((nstokes, ny, nx), np.nan)
    lev = np.full((ny, nx), -1, dtype=np.int8)
    audit = []
    st0 = 1 << levels
    jj, ii = np.meshgrid(np.arange(ny0) * st0, np.arange(nx0) * st0, indexing="ij")
    x, y = screen_coords(fov, nx, ny, ii.ravel(), jj.ravel())
    nspec = 0

    def alt_call(ii_, jj_):
        out = alt(ii_, jj_)
        if len(out) == 3:
            return out
        return out[0], out[1], np.full(np.shape(out[0]), np.inf)

    if alt is None:
        S0 = np.asarray(ray_fn(x, y)).reshape(-1, nstokes)
        for s in range(nstokes):
            img[s, jj, ii] = S0[:, s].reshape(ny0, nx0)
        lev[jj, ii] = 0
        ntr0 = nx0 * ny0
    else:
        bi, bj = ii.ravel(), jj.ravel()
        ok, vals, am = alt_call(bi, bj)
        audit.append(dict(i=bi, j=bj, own=np.where(ok, SPECTRAL, 0).astype(np.int8), margin=am))
        if forced_level is not None:
            ok = forced_level[bj, bi] == SPECTRAL
        for s in range(nstokes):
            img[s, bj[ok], bi[ok]] = vals[s][ok]
        lev[bj[ok], bi[ok]] = SPECTRAL
        tr = ~ok
        if tr.any():
            St = np.asarray(ray_fn(x[tr], y[tr])).reshape(-1, nstokes)
            for s in range(nstokes):
                img[s, bj[tr], bi[tr]] = St[:, s]
        lev[bj[tr], bi[tr]] = 0
        ntr0 = int(tr.sum())
        nspec += int(ok.sum())
    I0 = img[0, jj, ii]
    ibar = trapezoid_mean(I0)
    imax0 = float(I0.max())
    n_abs = ibar if abs_norm == "mean" else imax0
    own_norm = all_planes == "own"
    if own_norm and interp != "linear":
        raise ValueError("own-normalisation planes are defined for the linear branch")
    # every plane's normalisation (plane 0: Stokes I's, the usual one)
    n_abs_p = [n_abs] + [trapezoid_mean(np.abs(img[st, jj, ii])) if abs_norm == "mean"
                         else float(np.abs(img[st, jj, ii]).max()) for st in range(1, nstokes)]
    cand, traced = [nx0 * ny0], [ntr0]
    for l in range(levels):
        s = 1 << (levels - l - 1)          # spacing of the level-(l+1) grid
        planes = range(nstokes) if all_planes else range(1)
        if interp == "nearest":
            p, q, Inn, G = nearest_stencil(img, nx0, ny0, l, s, nstokes)
            npt = p.size
            decs, margins = [], []
            with np.errstate(invalid="ignore"):
                for st in planes:
                    # G moves by at most eta times the sum of the magnitudes it reads
                    mag = nearest_magnitude(img, nx0, ny0, l, s, st)
                    d, mg = and_margin([G[st] - r_abs * n_abs, G[st] - r_rel * np.abs(Inn[0])],
                                       [mag + r_abs * n_abs, mag + r_rel * np.abs(Inn[0])])
                    bad = np.isnan(G[st])
                    decs.append(d | bad)
                    margins.append(np.where(bad, np.inf, mg))
                dec, margin = or_margin(decs, margins)
                nan0 = np.isnan(Inn[0])
                dec = dec | nan0
                margin = np.where(nan0, np.inf, margin)
            interp_vals = Inn
        else:
            p, q, S_all, D, inf, m, magD, magSa = level_stencil(img, nx0, ny0, l, s, nstokes,
                                                                bool(all_planes), with_mag=True, mag_all=True)
            npt = p.size
            S = S_all[0]
            crel = 4.0 * r_rel
            Ds = D if all_planes else D[None, :]
            Ms = magD if all_planes else magD[None, :]
            with np.errstate(invalid="ignore"):
                decs, margins = [], []
                for st, (Dp, Mp) in enumerate(zip(Ds, Ms)):
                    pl = st if own_norm else 0
                    thrA = (4.0 * m * r_abs) * n_abs_p[pl]
                    d, mg = linear_margin(Dp, S_all[pl], Mp, magSa[pl], thrA, crel)
                    bad = np.isnan(Dp)
                    decs.append(d | bad)
                    margins.append(np.where(bad, np.inf, mg))
                dec, margin = or_margin(decs, margins)
                forced_trace = inf | np.isnan(S)
                dec = dec | forced_trace
                margin = np.where(forced_trace, np.inf, margin)
            interp_vals = S_all * (1.0 / m)
        spec = np.zeros(npt, dtype=bool)
        own = np.where(dec, l + 1, -1).astype(np.int8)
        if alt is not None:
            ok, avals, am = alt_call(p[dec] * s, q[dec] * s)
            spec[np.nonzero(dec)[0][ok]] = True
            own[np.nonzero(dec)[0][ok]] = SPECTRAL
            # a flagged point's state also depends on the alternative's check
            margin = margin.copy()
            margin[dec] = np.minimum(margin[dec], am)
        audit.append(dict(i=p * s, j=q * s, own=own, margin=margin))
        if forced_level is not None:
            fl = forced_level[q * s, p * s]
            dec = fl == l + 1
            spec = fl == SPECTRAL
        else:
            dec = dec & ~spec
        # interpolate everything first (level-l values only), then the
        # alternative's values, then trace
        for st in range(nstokes):
            img[st, q * s, p * s] = interp_vals[st]
        if spec.any():
            _, avals, _ = alt_call(p[spec] * s, q[spec] * s)
            for st in range(nstokes):
                img[st, q[spec] * s, p[spec] * s] = avals[st]
            lev[q[spec] * s, p[spec] * s] = SPECTRAL
            nspec += int(spec.sum())
        tp, tq = p[dec] * s, q[dec] * s
        if tp.size:
            xs, ys = screen_coords(fov, nx, ny, tp, tq)
            St = np.asarray(ray_fn(xs, ys)).reshape(-1, nstokes)
            for st in range(nstokes):
                img[st, tq, tp] = St[:, st]
        lev[tq, tp] = l + 1
        cand.append(int(npt))
        traced.append(int(dec.sum()))
    n_interp = int((lev < 0).sum())
    return dict(img=img, level=lev, n_abs=n_abs, n_abs_planes=n_abs_p, ibar=ibar, imax0=imax0,
                candidates=cand, traced=traced, rays=int(sum(traced)), spectral=nspec,
                interp_frac=n_interp / float(nx * ny), nx=nx, ny=ny, audit=audit)


def nearest_magnitude(img, nx0, ny0, l, s, st):
    """Sum of the magnitudes of the level-l values the nearest branch reads
    for each new point of level l+1 (bounds what a relative perturbation
    moves G by), in the order of nearest_stencil."""
    nxl, nyl = grid_size(nx0, l + 1), grid_size(ny0, l + 1)
    q, p = np.meshgrid(np.arange(nyl), np.arange(nxl), indexing="ij")
    new = (p % 2 == 1) | (q % 2 == 1)
    p, q = p[new], q[new]
    cat4 = (p % 2 == 1) & (q % 2 == 1)
    cat2 = (p % 2 == 0) & (q % 2 == 1)
    v = lambda pp, qq: np.abs(img[st, np.clip(qq, 0, nyl - 1) * s, np.clip(pp, 0, nxl - 1) * s])
    one = np.where(cat2, v(p, q - 1) + v(p, q + 1), v(p - 1, q) + v(p + 1, q))
    four = v(p - 1, q - 1) + v(p + 1, q + 1) + v(p + 1, q - 1) + v(p - 1, q + 1)
    return np.where(cat4, four, one)


def disagreements(res, level_map, state_of=None):
    """Points where a level map's decisions differ from the oracle's own rule
    in a forced replay (refine(..., forced_level=level_map)): returns
    (count, largest tie margin among them, list of (i, j, own, given,
    margin)) over every audited level."""
    rows = []
    for a in res["audit"]:
        given = level_map[a["j"], a["i"]]
        if state_of is not None:
            given = state_of(given)
        bad = np.nonzero(given != a["own"])[0]
        for k in bad:
            rows.append((int(a["i"][k]), int(a["j"][k]), int(a["own"][k]), int(given[k]),
                         float(a["margin"][k])))
    worst = max((r[4] for r in rows), default=0.0)
    return len(rows), worst, rows


def uniform(ray_fn, fov, nx, ny, nstokes=1):
    """Truth image: a ray through every vertex of the nx x ny grid."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x, y = screen_coords(fov, nx, ny, ii.ravel(), jj.ravel())
    S = np.asarray(ray_fn(x, y)).reshape(-1, nstokes)
    return np.stack([S[:, s].reshape(ny, nx) for s in range(nstokes)])
