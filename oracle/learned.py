"""Learned refinement proposal around the paper's criterion (test oracle).

Test infrastructure only.  The refinement of Sec. 3.2 (see refine.py) with a
network that looks ahead: at a level l where it can (l + 2 <= N, or also
l + 1 = N with all_levels), the network reads the level-l grid and gives a
logit for each of the 15 new points a level-l vertex owns (cnn.OWNED).

* logit > z_hi: a level-(l+1) point is traced; a level-(l+2) point is traced
  in the same pass as level l+1 (look-ahead);
* logit < z_lo: the point is suppressed (interpolated even if the criterion
  flags it);
* otherwise the criterion of Eqs. 5-6 decides.

Level l+1: traced = proposed or (flagged and not suppressed).  Level l+2
(after the look-ahead pass): look-ahead points stay traced; the criterion,
evaluated on the level-(l+1) values, flags points; a flagged point that is
neither traced nor suppressed is traced if `fallback`, else only counted.
Interpolated points inherit the smallest minimum radius and the largest
crossing count of the points they are interpolated from.

Judge counters (same meaning as the library's statistics):
  [0] proposed points the criterion would not have traced,
  [1] flagged points the network suppressed,
  [2] flagged points traced as fallback after a look-ahead pass,
  [3] flagged points left interpolated (fallback off),
  [4] look-ahead rays.
"""
import numpy as np

from . import cnn
from .ray import screen_coords
from .refine import grid_size, level_stencil, linear_margin, trapezoid_mean

UNSET, PROPOSE, SUPPRESS = 0, 1, 2


def _neighbours(p, q):
    """Interpolation neighbours (level-(l+1) units) of new points: the two
    points along the odd axis, or the four corners of a centre point."""
    cat4 = (p % 2 == 1) & (q % 2 == 1)
    cat2 = (p % 2 == 0) & (q % 2 == 1)
    nb = []
    for (ax, ay), (bx, by) in (((-1, -1), (1, 1)), ((1, -1), (-1, 1))):
        nb.append((np.where(cat4, p + ax, np.where(cat2, p, p - 1)),
                   np.where(cat4, q + ay, np.where(cat2, q - 1, q))))
        nb.append((np.where(cat4, p + bx, np.where(cat2, p, p + 1)),
                   np.where(cat4, q + by, np.where(cat2, q + 1, q))))
    return nb, cat4


def refine_learned(ray_fn, fov, nx0, ny0, levels, r_rel, r_abs, abs_norm, nstokes, logits_fn,
                   z_hi, z_lo, fallback=True, all_levels=False, forced_level=None, level_cap=0):
    """ray_fn(x, y) -> (S (n, nstokes), rmin (n,), ncross (n,)).
    level_cap > 0: the network runs only at levels l < level_cap; deeper
    levels take the criterion alone (as a plain render does).
    logits_fn(x) -> (15, H, W) for the features x (3, H, W) of a level.
    forced_level: optional final-grid level map to replay (a point new at
    level l+1 or l+2 of a network pass is traced iff the map says so).
    Returns dict(img, level, judge, passes, rays, n_abs, audit): audit lists,
    per decision pass, the final-grid points (i, j) judged, the state this
    oracle's own rule gives them from its own values and logits (-1 or the
    level traced at), the tie margin of the criterion's part of the decision
    (relative perturbation, see refine.and_margin) and the distance of the
    point's logit from the nearer of z_hi and z_lo (inf for points no logit
    decides).  In a forced replay the image follows forced_level."""
    nx, ny = grid_size(nx0, levels), grid_size(ny0, levels)
    img = np.full((nstokes, ny, nx), np.nan)
    lev = np.full((ny, nx), -1, dtype=np.int8)
    rmin = np.zeros((ny, nx))
    ncr = np.zeros((ny, nx), dtype=np.int64)
    judge = [0] * 5
    passes = 0
    audit = []

    def trace(tp, tq, level):
        if tp.size:
            xs, ys = screen_coords(fov, nx, ny, tp, tq)
            S, rm, nc = ray_fn(xs, ys)
            S = np.asarray(S).reshape(-1, nstokes)
            for st in range(nstokes):
                img[st, tq, tp] = S[:, st]
            rmin[tq, tp] = rm
            ncr[tq, tp] = nc
        lev[tq, tp] = level

    st0 = 1 << levels
    jj, ii = np.meshgrid(np.arange(ny0) * st0, np.arange(nx0) * st0, indexing="ij")
    trace(ii.ravel(), jj.ravel(), 0)
    passes += 1
    I0 = img[0, jj, ii]
    n_abs = trapezoid_mean(I0) if abs_norm == "mean" else float(I0.max())

    def criterion(l):
        """Points new at level l+1, their stencil sums, the criterion's flag
        and its tie margin."""
        s = 1 << (levels - l - 1)
        p, q, S_all, D, inf, m, magD, magS = level_stencil(img, nx0, ny0, l, s, nstokes,
                                                           with_mag=True)
        thrA = (4.0 * m * r_abs) * n_abs
        with np.errstate(invalid="ignore"):
            crit, margin = linear_margin(D, S_all[0], magD, magS, thrA, 4.0 * r_rel)
            forced = inf | np.isnan(D) | np.isnan(S_all[0])
            crit = crit | forced
            margin = np.where(forced, np.inf, margin)
        return p, q, s, S_all, m, crit, margin

    def interpolate(p, q, s, S_all, m, sel):
        pp, qq = p[sel], q[sel]
        for st in range(nstokes):
            img[st, qq * s, pp * s] = S_all[st][sel] / m[sel]
        nb, _ = _neighbours(pp, qq)
        cat4 = (pp % 2 == 1) & (qq % 2 == 1)
        r = np.full(pp.shape, np.inf)
        c = np.full(pp.shape, -1, dtype=np.int64)
        for k, (bx, by) in enumerate(nb):
            use = np.ones(pp.shape, dtype=bool) if k < 2 else cat4
            bxs, bys = np.clip(bx, 0, None) * s, np.clip(by, 0, None) * s
            r = np.where(use, np.minimum(r, rmin[bys, bxs]), r)
            c = np.where(use, np.maximum(c, ncr[bys, bxs]), c)
        rmin[qq * s, pp * s] = r
        ncr[qq * s, pp * s] = c
        lev[qq * s, pp * s] = -1

    def record(p, q, s, own_dec, level, cmargin, zmargin):
        audit.append(dict(i=p * s, j=q * s, own=np.where(own_dec, level, -1).astype(np.int8),
                          margin=cmargin, zmargin=zmargin))

    def forced_at(p, q, s, level):
        return forced_level[q * s, p * s] == level

    l = 0
    while l < levels:
        net_here = (level_cap <= 0 or l < level_cap) and (l + 2 <= levels or (all_levels and l + 1 <= levels))
        if not net_here:
            p, q, s, S_all, m, crit, cm = criterion(l)
            record(p, q, s, crit, l + 1, cm, np.full(p.shape, np.inf))
            dec = crit if forced_level is None else forced_at(p, q, s, l + 1)
            interpolate(p, q, s, S_all, m, ~dec)
            trace(p[dec] * s, q[dec] * s, l + 1)
            passes += 1
            l += 1
            continue
        z = logits_fn(cnn.features(img[0], rmin, ncr, nx0, ny0, levels, l, n_abs))
        mark = np.full((ny, nx), UNSET, dtype=np.int8)
        zgap = np.full((ny, nx), np.inf)
        ahead_p, ahead_q = [], []
        for k, (lv, fp, fq, ok) in enumerate(cnn.owned_points(nx0, ny0, levels, l)):
            hi = ok & (z[k] > z_hi)
            lo = ok & ~(z[k] > z_hi) & (z[k] < z_lo)
            zgap[fq[ok], fp[ok]] = np.minimum(np.abs(z[k] - z_hi), np.abs(z[k] - z_lo))[ok]
            if lv == l + 1:
                mark[fq[hi], fp[hi]] = PROPOSE
            else:
                ahead_p.append(fp[hi])
                ahead_q.append(fq[hi])
            mark[fq[lo], fp[lo]] = SUPPRESS
        ahead_p = np.concatenate(ahead_p) if ahead_p else np.zeros(0, dtype=np.int64)
        ahead_q = np.concatenate(ahead_q) if ahead_q else np.zeros(0, dtype=np.int64)
        # level l+1
        p, q, s, S_all, m, crit, cm = criterion(l)
        mk = mark[q * s, p * s]
        prop, sup = mk == PROPOSE, mk == SUPPRESS
        dec = prop | (crit & ~sup)
        record(p, q, s, dec, l + 1, cm, zgap[q * s, p * s])
        judge[0] += int((prop & ~crit).sum())
        judge[1] += int((crit & sup).sum())
        if forced_level is not None:
            dec = forced_at(p, q, s, l + 1)
            if l + 2 <= levels:
                fq2, fp2 = np.nonzero(forced_level == l + 2)
                ahead_p, ahead_q = fp2, fq2
        interpolate(p, q, s, S_all, m, ~dec)
        trace(np.concatenate([p[dec] * s, ahead_p]), np.concatenate([q[dec] * s, ahead_q]), l + 1)
        lev[ahead_q, ahead_p] = l + 2
        judge[4] += int(ahead_p.size)
        passes += 1
        if l + 2 > levels:
            l += 1
            continue
        # level l+2, judged by the criterion on the level-(l+1) values
        p, q, s, S_all, m, crit, cm = criterion(l + 1)
        keep = lev[q * s, p * s] == l + 2
        sup = mark[q * s, p * s] == SUPPRESS
        zg = zgap[q * s, p * s]
        if forced_level is None:
            want = crit & ~sup & ~keep
            record(p, q, s, keep | (want if fallback else np.zeros_like(want)), l + 2, cm, zg)
        else:
            # own rule: look-ahead proposals, then fallback on flagged points
            look = np.zeros((ny, nx), dtype=bool)
            for k, (lv, fp, fq, ok) in enumerate(cnn.owned_points(nx0, ny0, levels, l)):
                if lv == l + 2:
                    hi = ok & (z[k] > z_hi)
                    look[fq[hi], fp[hi]] = True
            la = look[q * s, p * s]
            own = la | ((crit & ~sup & ~la) if fallback else np.zeros_like(la))
            record(p, q, s, own, l + 2, cm, zg)
            want = np.zeros_like(keep)
        judge[1] += int((crit & sup & ~keep).sum())
        if fallback:
            judge[2] += int(want.sum())
        else:
            judge[3] += int(want.sum())
        dec = want if fallback else np.zeros_like(want)
        interpolate(p, q, s, S_all, m, ~keep & ~dec)
        if fallback:
            trace(p[dec] * s, q[dec] * s, l + 2)
            passes += 1
        l += 2
    return dict(img=img, level=lev, judge=judge, passes=passes, rays=int((lev >= 0).sum()),
                n_abs=n_abs, rmin=rmin, ncross=ncr, audit=audit)
