"""Pins of the oracle's refinement and metrics (Sec. 3.2, Eqs. 5-9, App. A-B).

- Grid sizes n = 2^N (n0-1)+1 and candidate counts.
- R = -1 reproduces the uniform image bitwise; R = +inf reproduces bilinear
  interpolation of the base grid (scipy RegularGridInterpolator), IF = 1 - n0^2/n^2.
- Quadratic images: the estimate equals twice the true residual (the printed
  final formulas of Eqs. 5-6); bilinear images give zero, harmonic x^2 - y^2
  gives zero at centre points.
- Power-law statistics (Sec. 3.2 and App. B): on fractional Brownian motion
  with structure function ~ x^(beta-2), the RMS ratio estimate/true error is
  2^(beta/2-2) (nearest) and 2^(beta/2-4) sqrt((1+2^(beta-1)-3^(beta-2))/(1-2^(beta-4)))
  (linear); linear/nearest true error ratio is sqrt(1-2^(beta-4)).
- Metamorphic: scaling by powers of two, transposition, tolerance monotonicity.
- A hand-worked 3x3 -> 5x5 example (tests/golden) and a brute-force per-pixel
  re-derivation on 9x9 -> 33x33.
- Metrics on hand-computed toy images (Eqs. 7-9).
"""
import json
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import metrics, refine

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def smooth(x, y):
    return np.stack([np.exp(-((x - 1) ** 2 + (y + 2) ** 2) / 30.0) + 0.3 * np.sin(0.4 * x) * np.cos(0.3 * y) + 1.0], -1)


def test_grid_sizes_and_counts():
    assert refine.grid_size(65, 4) == 1025 and refine.grid_size(65, 6) == 4097
    assert refine.grid_size(129, 3) == 1025 and refine.grid_size(257, 6) == 16385
    out = refine.refine(smooth, 40.0, 9, 7, 2, 0.01, 0.01)
    assert (out["nx"], out["ny"]) == (33, 25)
    assert out["candidates"] == [63, 17 * 13 - 63, 33 * 25 - 17 * 13]


def test_negative_tolerance_is_uniform_bitwise():
    out = refine.refine(smooth, 40.0, 9, 9, 2, -1.0, -1.0)
    uni = refine.uniform(smooth, 40.0, 33, 33)
    assert np.array_equal(out["img"], uni)
    assert out["interp_frac"] == 0.0


@pytest.mark.parametrize("n0,L", [(3, 2), (5, 3), (9, 2)])
def test_infinite_tolerance_is_bilinear(n0, L):
    out = refine.refine(smooth, 40.0, n0, n0, L, np.inf, np.inf)
    n = out["nx"]
    xs = np.linspace(-20, 20, n0)
    X0, Y0 = np.meshgrid(xs, xs, indexing="xy")
    rgi = RegularGridInterpolator((xs, xs), smooth(X0, Y0)[..., 0].T)
    X, Y = np.meshgrid(np.linspace(-20, 20, n), np.linspace(-20, 20, n))
    ref = rgi(np.stack([X.ravel(), Y.ravel()], -1)).reshape(n, n)
    assert np.abs(out["img"][0] - ref).max() < 1e-14
    assert out["interp_frac"] == pytest.approx(1 - n0 * n0 / n ** 2, abs=0, rel=1e-15)


def _stencil_on_truth(fn, n0, levels, l):
    """Stencil of level l+1 computed from the exact function at level-l points."""
    n = refine.grid_size(n0, levels)
    s = 1 << (levels - l - 1)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    img = fn(ii.astype(float), jj.astype(float))[None]
    p, q, S_all, D, inf, m = refine.level_stencil(img, n0, n0, l, s, 1)
    true = img[0, q * s, p * s]
    return p, q, S_all[0], D, inf, m, true, s


def _both_diagonals(p, q, nl):
    """False for centre points with a whole diagonal outside the image."""
    inside = lambda a, b: (a >= 0) & (a < nl) & (b >= 0) & (b < nl)
    cat4 = (p % 2 == 1) & (q % 2 == 1)
    xd = inside(p - 3, q - 3) | inside(p + 3, q + 3)
    yd = inside(p + 3, q - 3) | inside(p - 3, q + 3)
    return ~(cat4 & ~(xd & yd))


@pytest.mark.parametrize("l", [0, 1])
def test_quadratic_estimate_is_twice_true_residual(l):
    fn = lambda x, y: 0.3 * x * x - 0.2 * x * y + 0.5 * y * y + x + 2.0
    p, q, S, D, inf, m, true, s = _stencil_on_truth(fn, 9, 2, l)
    # the one-sided edge rule is exact for quadratics; a centre point whose
    # whole diagonal is missing borrows the other diagonal and is excluded
    ok = ~inf & _both_diagonals(p, q, refine.grid_size(9, l + 1))
    resid = np.abs(S / m - true)
    est = np.abs(D) / (4.0 * m)
    assert np.allclose(est[ok], 2.0 * resid[ok], rtol=1e-12, atol=1e-9)
    assert resid[ok].max() > 0


def test_bilinear_zero_and_harmonic_zero_at_centres():
    fb = lambda x, y: 3.0 + 0.5 * x - 0.25 * y + 0.125 * x * y
    p, q, S, D, inf, m, true, s = _stencil_on_truth(fb, 9, 2, 1)
    ok = ~inf & _both_diagonals(p, q, refine.grid_size(9, 2))
    assert np.abs(D[ok]).max() < 1e-12
    fh = lambda x, y: x * x - y * y + 100.0
    p, q, S, D, inf, m, true, s = _stencil_on_truth(fh, 9, 2, 1)
    nl = refine.grid_size(9, 2)
    centre = (p % 2 == 1) & (q % 2 == 1) & (p >= 3) & (q >= 3) & (p <= nl - 4) & (q <= nl - 4)
    assert centre.sum() > 0
    assert np.abs(D[centre]).max() < 1e-12


def fbm(n, H, rng):
    """Exact fractional Brownian motion by circulant embedding (Davies-Harte)."""
    k = np.arange(n + 1)
    g = 0.5 * (np.abs(k + 1) ** (2 * H) - 2 * np.abs(k) ** (2 * H) + np.abs(k - 1) ** (2 * H))
    row = np.concatenate([g, g[-2:0:-1]])
    lam = np.fft.fft(row).real
    assert lam.min() > -1e-9
    lam = np.clip(lam, 0, None)
    m = row.size
    z = rng.normal(size=m) + 1j * rng.normal(size=m)
    w = np.fft.fft(np.sqrt(lam / m) * z)
    return np.concatenate([[0.0], np.cumsum(w.real[:n])])


@pytest.mark.parametrize("beta", [2.5, 3.0])
def test_power_law_estimator_statistics(beta):
    rng = np.random.default_rng(2021)
    H = (beta - 2.0) / 2.0
    N = 1 << 19
    B = fbm(N, H, rng)
    # check the generator's structure function D(x) ~ x^(beta-2)
    d1 = np.mean((B[1:] - B[:-1]) ** 2)
    d4 = np.mean((B[4:] - B[:-4]) ** 2)
    assert d4 / d1 == pytest.approx(4 ** (beta - 2), rel=0.02)
    # linear estimator through the oracle's category-3 stencil on a 1-row image
    img = B[None, None, :]
    n0 = (N // 2) + 1
    p, q, S_all, D, inf, m = refine.level_stencil(img, n0, 1, 0, 1, 1)
    true = B[p]
    ok = ~inf
    ratio_lin = np.sqrt(np.mean((np.abs(D[ok]) / 8.0) ** 2) / np.mean((S_all[0, ok] / 2 - true[ok]) ** 2))
    pred_lin = 2 ** (beta / 2 - 4) * np.sqrt((1 + 2 ** (beta - 1) - 3 ** (beta - 2)) / (1 - 2 ** (beta - 4)))
    assert ratio_lin == pytest.approx(pred_lin, rel=0.02)
    if beta == 2.5:
        assert round(pred_lin, 2) == 0.27      # value printed in Sec. 3.2
    # nearest-neighbour estimate |c-b|/2 against |b - I| (nearest = b)
    b, c, I = B[p[ok] - 1], B[p[ok] + 1], true[ok]
    ratio_nn = np.sqrt(np.mean(((c - b) / 2) ** 2) / np.mean((b - I) ** 2))
    pred_nn = 2 ** (beta / 2 - 2)
    assert ratio_nn == pytest.approx(pred_nn, rel=0.02)
    if beta == 2.5:
        assert round(pred_nn, 2) == 0.59       # value printed in Sec. 3.2
    # App. B: linear / nearest true error = sqrt(1 - 2^(beta-4))
    r_lin_nn = np.sqrt(np.mean((S_all[0, ok] / 2 - I) ** 2) / np.mean((b - I) ** 2))
    assert r_lin_nn == pytest.approx(np.sqrt(1 - 2 ** (beta - 4)), rel=0.02)
    if beta == 2.5:
        assert round(np.sqrt(1 - 2 ** (beta - 4)), 1) == 0.8


def ring(x, y):
    rho = np.sqrt(x * x + y * y)
    return np.stack([np.exp(-0.5 * ((rho - 5) / 0.4) ** 2) * (1 + 0.3 * x / 7) + 0.05 * np.exp(-rho ** 2 / 60)], -1)


@pytest.mark.parametrize("c", [8.0, 0.25])
def test_scale_invariance(c):
    a = refine.refine(ring, 20.0, 17, 17, 3, 0.01, 0.01)
    b = refine.refine(lambda x, y: c * ring(x, y), 20.0, 17, 17, 3, 0.01, 0.01)
    assert np.array_equal(a["level"], b["level"])
    assert np.array_equal(a["img"] * c, b["img"])


def test_transpose_swaps_categories():
    a = refine.refine(ring, 20.0, 17, 17, 3, 0.01, 0.005)
    b = refine.refine(lambda x, y: ring(y, x), 20.0, 17, 17, 3, 0.01, 0.005)
    assert np.array_equal(a["level"].T, b["level"])
    assert np.array_equal(a["img"][0].T, b["img"][0])


def test_tolerance_monotone_first_level():
    a = refine.refine(ring, 20.0, 33, 33, 1, 0.01, 0.02)
    b = refine.refine(ring, 20.0, 33, 33, 1, 0.01, 0.005)
    c = refine.refine(ring, 20.0, 33, 33, 1, 0.002, 0.02)
    ta, tb, tc = a["level"] == 1, b["level"] == 1, c["level"] == 1
    assert np.all(tb[ta]) and np.all(tc[ta]) and tb.sum() > ta.sum()


def test_golden_3x3_to_5x5():
    g = json.load(open(os.path.join(GOLD, "refine_3x3_to_5x5.json")))
    T = np.array(g["truth"], dtype=float)

    def fn(x, y):
        i = np.rint(x + 2).astype(int)
        j = np.rint(y + 2).astype(int)
        return T[j, i][:, None]
    for case in g["cases"]:
        out = refine.refine(fn, g["fov"], g["n0"], g["n0"], g["levels"], case["r_rel"], case["r_abs"])
        assert out["ibar"] == case["ibar"]
        assert np.array_equal(out["level"], np.array(case["level"]))
        assert np.array_equal(out["img"][0], np.array(case["image"], dtype=float))


def _brute_force(img_fn, n0, levels, r_rel, r_abs, fov):
    """Per-pixel loop re-derivation of the refinement (independent of the
    vectorised oracle): returns (img, level)."""
    from oracle.ray import screen_coords
    n = refine.grid_size(n0, levels)
    img = np.full((n, n), np.nan)
    lev = -np.ones((n, n), dtype=int)
    val = lambda i, j: float(img_fn(*screen_coords(fov, n, n, np.array([i]), np.array([j])))[0, 0])
    st0 = 1 << levels
    for j in range(0, n, st0):
        for i in range(0, n, st0):
            img[j, i] = val(i, j)
            lev[j, i] = 0
    base = img[::st0, ::st0]
    w = np.ones(n0); w[0] = w[-1] = 0.5
    ibar = float((w[:, None] * w[None, :] * base).sum() / ((n0 - 1) ** 2))
    for l in range(levels):
        s = 1 << (levels - l - 1)
        nl = refine.grid_size(n0, l + 1)
        new = {}
        for qq in range(nl):
            for pp in range(nl):
                if pp % 2 == 0 and qq % 2 == 0:
                    continue
                get = lambda a, b: img[b * s, a * s] if (0 <= a < nl and 0 <= b < nl) else None
                if pp % 2 == 1 and qq % 2 == 1:
                    axes = [((-1, -1), (1, 1)), ((1, -1), (-1, 1))]
                    mm = 4
                else:
                    axes = [((-1, 0), (1, 0))] if pp % 2 == 1 else [((0, -1), (0, 1))]
                    mm = 2
                Ssum, Dsum, navail, Dlist = 0.0, 0.0, 0, []
                for (dlo, dhi) in axes:
                    lo, hi = get(pp + dlo[0], qq + dlo[1]), get(pp + dhi[0], qq + dhi[1])
                    Ssum += lo + hi
                    olo = get(pp + 3 * dlo[0], qq + 3 * dlo[1])
                    ohi = get(pp + 3 * dhi[0], qq + 3 * dhi[1])
                    if olo is not None and ohi is not None:
                        Dlist.append(olo + ohi - lo - hi)
                    elif ohi is not None:
                        Dlist.append(2 * (lo - 2 * hi + ohi))
                    elif olo is not None:
                        Dlist.append(2 * (olo - 2 * lo + hi))
                if not Dlist:
                    trace = True
                else:
                    Dv = sum(Dlist) * (len(axes) / len(Dlist))
                    trace = abs(Dv) / (4 * mm * ibar) > r_abs and abs(Dv) / (4 * abs(Ssum)) > r_rel
                new[(pp, qq)] = (trace, Ssum / mm)
        for (pp, qq), (trace, v) in new.items():
            if trace:
                img[qq * s, pp * s] = val(pp * s, qq * s)
                lev[qq * s, pp * s] = l + 1
            else:
                img[qq * s, pp * s] = v
    return img, lev


def test_brute_force_9_to_33():
    out = refine.refine(ring, 20.0, 9, 9, 2, 0.02, 0.01)
    img, lev = _brute_force(ring, 9, 2, 0.02, 0.01, 20.0)
    assert np.array_equal(out["level"], lev)
    assert np.allclose(out["img"][0], img, rtol=1e-14, atol=0)
    assert 0 < (lev > 0).sum() < (lev != 0).sum()


def test_metrics_hand_computed():
    t = np.array([[1.0, 2.0], [3.0, 4.0]])
    a = np.array([[1.0, 2.0], [3.0, 5.0]])
    assert metrics.flux_error(t, a) == pytest.approx(0.1, rel=1e-15)
    assert metrics.mse(t, a) == pytest.approx(1.0 / 30.0, rel=1e-15)
    assert metrics.interp_fraction(np.array([[0, -1], [-1, 2]])) == 0.5


# ------------------------------------------------ nearest branch, per-plane criterion

def test_nearest_infinite_tolerance_is_floor_upsampling():
    n0, L = 5, 3
    out = refine.refine(ring, 20.0, n0, n0, L, np.inf, np.inf, interp="nearest")
    S = 1 << L
    n = out["nx"]
    xs = np.linspace(-10, 10, n)
    X, Y = np.meshgrid(xs, xs)
    base = ring(X[::S, ::S], Y[::S, ::S])[..., 0]
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(out["img"][0], base[jj // S, ii // S])


def test_nearest_negative_tolerance_is_uniform():
    out = refine.refine(ring, 20.0, 9, 9, 2, -1.0, -1.0, interp="nearest")
    assert np.array_equal(out["img"], refine.uniform(ring, 20.0, 33, 33))


def _brute_force_nearest(fn, n0, L, r_rel, r_abs, fov):
    """Per-point loops over the nearest branch of Eqs. 5-6 (one plane)."""
    n = (1 << L) * (n0 - 1) + 1
    xs = np.linspace(-fov / 2, fov / 2, n)
    img = np.full((n, n), np.nan)
    lev = np.full((n, n), -1, dtype=np.int8)
    S0 = 1 << L
    for j in range(0, n, S0):
        for i in range(0, n, S0):
            img[j, i] = fn(np.array([xs[i]]), np.array([xs[j]]))[0, 0]
            lev[j, i] = 0
    b0 = img[::S0, ::S0]
    wx = np.ones(n0); wx[0] = wx[-1] = 0.5
    nabs = float((wx[:, None] * wx[None, :] * b0).sum() / (n0 - 1) ** 2)
    for l in range(L):
        s = 1 << (L - l - 1)
        nl = (1 << (l + 1)) * (n0 - 1) + 1
        dec = {}
        for q in range(nl):
            for p in range(nl):
                if p % 2 == 0 and q % 2 == 0:
                    continue
                v = lambda a, b: img[b * s, a * s]
                if p % 2 == 1 and q % 2 == 1:
                    i1, i4, i2, i3 = v(p - 1, q - 1), v(p + 1, q + 1), v(p + 1, q - 1), v(p - 1, q + 1)
                    G = np.sqrt(((i4 - i1) / 2) ** 2 + ((i3 - i2) / 2) ** 2)
                    nn = i1
                elif q % 2 == 1:
                    b, c = v(p, q - 1), v(p, q + 1)
                    G, nn = abs(c - b) / 2, b
                else:
                    b, c = v(p - 1, q), v(p + 1, q)
                    G, nn = abs(c - b) / 2, b
                dec[(p, q)] = (G / nabs > r_abs and G / abs(nn) > r_rel, nn)
        for (p, q), (t, nn) in dec.items():
            if t:
                img[q * s, p * s] = fn(np.array([xs[p * s]]), np.array([xs[q * s]]))[0, 0]
                lev[q * s, p * s] = l + 1
            else:
                img[q * s, p * s] = nn
    return img, lev


def test_nearest_brute_force_9_to_33():
    out = refine.refine(ring, 20.0, 9, 9, 2, 0.05, 0.02, interp="nearest")
    img, lev = _brute_force_nearest(ring, 9, 2, 0.05, 0.02, 20.0)
    assert np.array_equal(out["level"], lev)
    assert np.array_equal(out["img"][0], img)
    assert 0 < (lev > 0).sum() < (lev != 0).sum()


def _planes(fn2):
    return lambda x, y: np.concatenate([ring(x, y), fn2(x, y)], -1)


@pytest.mark.parametrize("interp", ["linear", "nearest"])
def test_all_planes_criterion(interp):
    args = (20.0, 9, 9, 2, 0.02, 0.01, "mean", 2)
    # a copy of I (or its negative, or zeros) as second plane changes nothing
    base = refine.refine(_planes(lambda x, y: ring(x, y)), *args, interp=interp)
    for fn2 in (lambda x, y: ring(x, y), lambda x, y: -ring(x, y), lambda x, y: 0 * ring(x, y)):
        o = refine.refine(_planes(fn2), *args, interp=interp, all_planes=True)
        assert np.array_equal(o["level"], base["level"])
    # a sharp feature only in the second plane adds traced points at level 1
    sharp = lambda x, y: np.stack([np.tanh((x - 1.3) / 0.2)], -1) * 0.5
    a = refine.refine(_planes(sharp), 20.0, 9, 9, 1, 0.02, 0.01, "mean", 2, interp=interp)
    b = refine.refine(_planes(sharp), 20.0, 9, 9, 1, 0.02, 0.01, "mean", 2, interp=interp, all_planes=True)
    ta, tb = a["level"] == 1, b["level"] == 1
    assert np.all(tb[ta]) and tb.sum() > ta.sum()


def test_own_norm_planes_criterion():
    """all_planes="own": every plane against its own normalisation and its own
    neighbour sum.  A copy of I (or its negative) as second plane changes
    nothing (the same test on the same magnitudes); scaling the second plane by
    a power of two changes no decision (both thresholds scale with the plane,
    exactly in binary); so a faint copy of a sharp feature is refined as fully
    as the feature itself, while the shared normalisation (all_planes=True)
    ignores it; a constant plane c has N_abs = |c| (trapezoid mean of |c|)."""
    args = (20.0, 9, 9, 2, 0.02, 0.01, "mean", 2)
    base = refine.refine(_planes(lambda x, y: ring(x, y)), *args)
    for fn2 in (lambda x, y: ring(x, y), lambda x, y: -ring(x, y)):
        o = refine.refine(_planes(fn2), *args, all_planes="own")
        assert np.array_equal(o["level"], base["level"])
    sharp = lambda x, y: np.stack([np.tanh((x - 1.3) / 0.2) + 1.5 * np.exp(-(x * x + (y - 2.0) ** 2))], -1)
    faint = lambda x, y: sharp(x, y) * 2.0 ** -12
    full = refine.refine(_planes(sharp), *args, all_planes="own")
    own = refine.refine(_planes(faint), *args, all_planes="own")
    assert np.array_equal(own["level"], full["level"])
    assert np.isclose(own["n_abs_planes"][1], full["n_abs_planes"][1] * 2.0 ** -12, rtol=0, atol=0)
    # one level (the same history for both): the shared normalisation's traced
    # points are a strict subset of the own normalisation's
    args1 = (20.0, 9, 9, 1, 0.02, 0.01, "mean", 2)
    own1 = refine.refine(_planes(faint), *args1, all_planes="own")
    shared1 = refine.refine(_planes(faint), *args1, all_planes=True)
    t_own, t_sh = own1["level"] > 0, shared1["level"] > 0
    assert np.all(t_own[t_sh]) and t_own.sum() >= t_sh.sum() + 5
    const = refine.refine(_planes(lambda x, y: np.full((np.size(x), 1), -0.75)), *args, all_planes="own")
    assert const["n_abs_planes"][1] == 0.75 and const["n_abs_planes"][0] == const["n_abs"]
    with pytest.raises(ValueError):
        refine.refine(_planes(sharp), *args, interp="nearest", all_planes="own")
