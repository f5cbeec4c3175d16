"""Pins of the oracle's geodesic integrator and camera against what the
physics fixes independently of the oracle's own code.

- Schwarzschild critical impact parameter sqrt(27) M (textbook).
- Kerr capture from the roots of the radial potential (textbook Kerr).
- Conservation of the Carter constant and of the null norm along rays.
- Schwarzschild orbit-equation (Binet) quadrature for the total sweep angle.
- Strong-deflection logarithm: sweep ~ -ln(b/b_c - 1), slope -1 at a = 0
  (Lyapunov exponent gamma = pi of Sec. 5.1 for a = 0).
- Camera: far-field Bardeen relations between screen point and (lambda, eta).
- Walker-Penrose constant: conserved under an independent parallel transport
  built from symbolic Christoffel symbols (sympy), and a 90-degree rotation
  of the polarisation vector multiplies it by +-i.
"""
import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import ray

BASE = dict(r_cam=1000.0, r_out=1000.0, max_steps=200000, nstokes=1,
            model="toy_disk", mp=[2.0, 0.3])


def cfg(**kw):
    c = dict(BASE)
    c.update(kw)
    return c


def camera(c, al, be):
    p = ray.make_params(c)
    y5 = np.zeros(5); kt = np.zeros(1); kph = np.zeros(1)
    kup = np.zeros(4); fup = np.zeros(4)
    import ctypes
    ray.lib().or_camera(ctypes.byref(p), al, be, ray._dp(y5), ray._dp(kt), ray._dp(kph),
                        ray._dp(kup), ray._dp(fup))
    return y5, kt[0], kph[0], kup, fup


def impact_b(c, al, be):
    """b = L/E from the initial covariant momentum (a = 0)."""
    y5, kt, kph, _, _ = camera(c, al, be)
    th = y5[1]
    return np.sqrt(y5[4] ** 2 + kph ** 2 / np.sin(th) ** 2) / kt


def test_schwarzschild_critical_impact_parameter():
    c = cfg(a=0.0, inc_deg=60.0, eps=0.01)
    lo, hi = 5.0, 5.4
    for _ in range(45):
        m = 0.5 * (lo + hi)
        _, f = ray.trace(c, np.array([m]), np.array([0.0]), nthreads=1)
        if f["status"][0] == 1:
            lo = m
        else:
            hi = m
    b = impact_b(c, 0.5 * (lo + hi), 0.0)
    assert abs(b - np.sqrt(27.0)) < 2e-6, b


def radial_capture(a, lam, eta, rh):
    """Textbook Kerr: a photon from infinity is captured iff
    R(r) = (r^2+a^2-a lam)^2 - Delta (eta + (lam-a)^2) has no real root r > r_+."""
    # R(r) = r^4 + (a^2 - lam^2 - eta) r^2 + 2 (eta + (lam - a)^2) r - a^2 eta
    coeffs = [1.0, 0.0, a * a - lam * lam - eta, 2.0 * (eta + (lam - a) ** 2), -a * a * eta]
    roots = np.roots(coeffs)
    real = roots[np.abs(roots.imag) < 1e-9].real
    return not np.any(real > rh), (real[real > rh].max() if np.any(real > rh) else None)


@pytest.mark.parametrize("a,inc", [(0.94, 163.0), (0.5, 60.0), (-0.94, 17.0)])
def test_kerr_capture_matches_radial_potential(a, inc):
    c = cfg(a=a, inc_deg=inc, eps=0.02)
    rng = np.random.default_rng(7)
    al = rng.uniform(-8, 8, 300)
    be = rng.uniform(-8, 8, 300)
    _, f = ray.trace(c, al, be)
    rh = 1.0 + np.sqrt(1 - a * a)
    checked = 0
    for k in range(al.size):
        y5, kt, kph, _, _ = camera(c, al[k], be[k])
        th = y5[1]
        lam = -kph / kt   # k is the reversed momentum: L/E = -k_phi/k_t
        eta = (y5[4] ** 2 + np.cos(th) ** 2 * (-a * a * kt * kt + kph ** 2 / np.sin(th) ** 2)) / kt ** 2
        cap, rt = radial_capture(a, lam, eta, rh)
        # near-critical rays are exponentially sensitive; exclude a margin
        # measured by how close a double root the potential has
        rr = np.roots([1.0, 0.0, a * a - lam * lam - eta, 2.0 * (eta + (lam - a) ** 2), -a * a * eta])
        dmin = np.min(np.abs(np.subtract.outer(rr, rr)) + np.eye(4) * 1e9)
        if dmin < 0.15:
            continue
        checked += 1
        assert (f["status"][k] == 1) == cap, (al[k], be[k], f[k], cap, rt)
    assert checked > 200


@pytest.mark.parametrize("a,inc,al,be", [(0.94, 163.0, 3.0, 2.0), (0.94, 17.0, -6.0, 1.0),
                                         (0.5, 90.0, 0.3, 5.5), (0.0, 60.0, 7.0, -3.0)])
def test_carter_constant_and_null_norm_conserved(a, inc, al, be):
    c = cfg(a=a, inc_deg=inc, eps=0.03)
    _, f, st, kt, kph = ray.trace_path(c, al, be)
    th = st[:, 1]
    Q = st[:, 4] ** 2 + np.cos(th) ** 2 * (-a * a * kt * kt + kph ** 2 / np.sin(th) ** 2)
    nn = np.array([ray.lib().or_null_norm(a, kt, kph, ray._dp(np.ascontiguousarray(s[:5])))
                   for s in st])
    scale = kt * kt * 30.0
    assert np.abs(Q - Q[0]).max() < 1e-5 * max(abs(Q[0]), scale)
    assert np.abs(nn).max() < 1e-4 * kt * kt
    # halving eps reduces the drift (consistent integrator)
    _, _, st2, _, _ = ray.trace_path(cfg(a=a, inc_deg=inc, eps=0.015), al, be)
    Q2 = st2[:, 4] ** 2 + np.cos(st2[:, 1]) ** 2 * (-a * a * kt * kt + kph ** 2 / np.sin(st2[:, 1]) ** 2)
    assert np.abs(Q2 - Q2[0]).max() <= np.abs(Q - Q[0]).max() + 1e-14


@pytest.mark.parametrize("al,be", [(-0.00244140625, 16.97509765625), (1e-4, 16.0), (-3e-3, -16.5)])
def test_near_polar_rays_keep_their_invariants(al, be):
    """Rays whose screen point lies almost on the projected spin axis pass a
    pole with a tiny k_phi: the centrifugal barrier turns them back at
    sin(theta) ~ |k_phi|/|k_theta|.  The step rule must resolve the turn
    (Carter constant and null norm conserved, no runaway)."""
    a = 0.94
    c = cfg(a=a, inc_deg=163.0, eps=0.03)
    _, f, st, kt, kph = ray.trace_path(c, al, be)
    assert f["status"] in (1, 2), f
    th = st[:, 1]
    assert np.abs(th).max() < 10.0
    Q = st[:, 4] ** 2 + np.cos(th) ** 2 * (-a * a * kt * kt + kph ** 2 / np.sin(th) ** 2)
    nn = np.array([ray.lib().or_null_norm(a, kt, kph, ray._dp(np.ascontiguousarray(s[:5])))
                   for s in st])
    assert np.abs(Q - Q[0]).max() < 1e-4 * abs(Q[0])
    assert np.abs(nn).max() < 1e-4 * kt * kt


def _binet_sweep(b, u_end_a, u_end_b):
    """Total orbital sweep of a Schwarzschild photon with impact parameter b
    between radii 1/u_end_a and 1/u_end_b through its turning point:
    (du/dpsi)^2 = 1/b^2 - u^2 + 2 u^3."""
    f = lambda u: 1.0 / b ** 2 - u * u + 2.0 * u ** 3
    ut = optimize.brentq(f, 1e-12, 1.0 / 3.0)  # turning point below the photon sphere u=1/3

    def leg(u0):
        # substitute u = ut - s^2 (sig = s^2): with f(ut) = 0,
        # f(ut - sig) = sig [(2ut - 6ut^2) + sig (6ut - 1) - 2 sig^2],
        # which removes the square-root endpoint singularity
        smax = np.sqrt(ut - u0)

        def g(s):
            sig = s * s
            return 2.0 / np.sqrt((2.0 * ut - 6.0 * ut * ut) + sig * (6.0 * ut - 1.0) - 2.0 * sig * sig)
        val, _ = integrate.quad(g, 0.0, smax, epsabs=1e-14, epsrel=1e-13, limit=200)
        return val
    return leg(u_end_a) + leg(u_end_b)


@pytest.mark.parametrize("alpha", [6.0, 8.0, 15.0])
def test_schwarzschild_sweep_matches_binet_quadrature(alpha):
    c = cfg(a=0.0, inc_deg=90.0, eps=0.005)
    _, f, st, kt, kph = ray.trace_path(c, alpha, 0.0)
    assert f["status"] == 2
    b = impact_b(c, alpha, 0.0)
    r0, th0, ph0 = st[0, 0], st[0, 1], st[0, 2]
    r1, th1, ph1 = st[-1, 0], st[-1, 1], st[-1, 2]
    v0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    v1 = np.array([np.sin(th1) * np.cos(ph1), np.sin(th1) * np.sin(ph1), np.cos(th1)])
    psi = np.arccos(np.clip(v0 @ v1, -1, 1))
    psi_b = _binet_sweep(b, 1.0 / r0, 1.0 / r1)
    # the sweep is below 2 pi for these b, arccos returns 2 pi - psi above pi
    psi_or = psi if psi_b <= np.pi else 2 * np.pi - psi
    assert abs(psi_or - psi_b) < 2e-6, (psi_or, psi_b)


def test_strong_deflection_log_slope_schwarzschild():
    """Near the critical curve the sweep grows like -ln(b - b_c) with unit
    slope at a = 0 (gamma = pi per half orbit, Sec. 5.1)."""
    c = cfg(a=0.0, inc_deg=90.0, eps=0.01)
    # screen alpha giving b = b_c (1 + d): b = alpha / sqrt(1 - 2/r_cam) to O(alpha^2/r^2)
    bc = np.sqrt(27.0)
    ds = np.array([1e-3, 1e-4, 1e-5, 1e-6])
    sweeps = []
    for d in ds:
        target = bc * (1 + d)
        al = optimize.brentq(lambda x: impact_b(c, x, 0.0) - target, 5.0, 5.4, xtol=1e-14)
        _, f, st, kt, kph = ray.trace_path(c, al, 0.0)
        assert f["status"] == 2
        sweeps.append(np.sum(np.abs(np.diff(np.unwrap(st[:, 2])))))
    slope = np.polyfit(np.log(ds), sweeps, 1)[0]
    assert abs(slope + 1.0) < 0.02, slope


@pytest.mark.parametrize("a,inc", [(0.94, 163.0), (0.0, 60.0), (-0.5, 30.0)])
def test_camera_far_field_bardeen_relations(a, inc):
    c = cfg(a=a, inc_deg=inc)
    i = np.deg2rad(inc)
    for al, be in [(4.0, 3.0), (-5.0, 1.0), (2.0, -6.0)]:
        y5, kt, kph, _, _ = camera(c, al, be)
        lam = -kph / kt   # k is the reversed momentum: L/E = -k_phi/k_t
        eta = (y5[4] ** 2 + np.cos(i) ** 2 * (-a * a * kt * kt + kph ** 2 / np.sin(i) ** 2)) / kt ** 2
        # Bardeen: alpha = -lam / sin i, beta^2 = eta + a^2 cos^2 i - lam^2 cot^2 i
        assert abs(-lam / np.sin(i) - al) < 0.02 * abs(al) + 0.02
        beta2 = eta + a * a * np.cos(i) ** 2 - lam ** 2 / np.tan(i) ** 2
        assert abs(np.sqrt(max(beta2, 0.0)) - abs(be)) < 0.02 * abs(be) + 0.02


@pytest.fixture(scope="module")
def christoffel_bl():
    import sympy as sp
    t, r, th, ph, a = sp.symbols("t r theta phi a", real=True)
    Sig = r ** 2 + a ** 2 * sp.cos(th) ** 2
    Del = r ** 2 - 2 * r + a ** 2
    g = sp.zeros(4, 4)
    g[0, 0] = -(1 - 2 * r / Sig)
    g[0, 3] = g[3, 0] = -2 * a * r * sp.sin(th) ** 2 / Sig
    g[1, 1] = Sig / Del
    g[2, 2] = Sig
    g[3, 3] = (r ** 2 + a ** 2 + 2 * a ** 2 * r * sp.sin(th) ** 2 / Sig) * sp.sin(th) ** 2
    X = [t, r, th, ph]
    gi = g.inv()
    dg = [[[sp.diff(g[m, n], X[k]) for k in range(4)] for n in range(4)] for m in range(4)]
    Gam = [[[sum(gi[l, m] * (dg[m][i][j] + dg[m][j][i] - dg[i][j][m]) for m in range(4)) / 2
             for j in range(4)] for i in range(4)] for l in range(4)]
    f = sp.lambdify((r, th, a), Gam, "numpy")
    return lambda rr, tt, aa: np.array(f(rr, tt, aa), dtype=float)


@pytest.mark.parametrize("a,inc,al,be", [(0.94, 163.0, 4.0, 3.0), (0.5, 60.0, -6.0, 2.0)])
def test_walker_penrose_conserved_under_parallel_transport(christoffel_bl, a, inc, al, be):
    c = cfg(a=a, inc_deg=inc)
    y5, kt, kph, kup, fup = camera(c, al, be)
    Gam = christoffel_bl

    def rhs(lam, Y):
        x, k, f = Y[0:4], Y[4:8], Y[8:12]
        G = Gam(x[1], x[2], a)
        dk = -np.einsum("lij,i,j->l", G, k, k)
        df = -np.einsum("lij,i,j->l", G, k, f)
        return np.concatenate([k, dk, df])

    def wp(x, k, f):
        out = np.zeros(2)
        ray.lib().or_walker_penrose(a, x[1], x[2], ray._dp(np.ascontiguousarray(k)),
                                    ray._dp(np.ascontiguousarray(f)), ray._dp(out))
        return out[0] + 1j * out[1]

    Y0 = np.concatenate([[0.0, y5[0], y5[1], 0.0], kup, fup])
    ev = lambda lam, Y: Y[1] - 4.0
    ev.terminal = True
    sol = integrate.solve_ivp(rhs, (0, 1100.0), Y0, rtol=1e-11, atol=1e-13, events=ev,
                              dense_output=False, max_step=5.0)
    k0 = wp(Y0[0:4], Y0[4:8], Y0[8:12])
    for Y in sol.y.T[:: max(1, sol.y.shape[1] // 20)]:
        kk = wp(Y[0:4], Y[4:8], Y[8:12])
        assert abs(kk - k0) < 1e-7 * abs(k0)
    assert sol.y[1].min() < 10.0   # the ray reached the strong-field region

    # rotating the camera polarisation vector by 90 degrees about the line of
    # sight multiplies kappa by +-i
    zr = np.zeros(5)
    from oracle.ray import make_params  # noqa: F401
    # build e2 = d x f in the camera's orthonormal frame via the metric
    # (the oracle returns contravariant BL components; convert with the ZAMO frame)
    r, th = y5[0], y5[1]
    Sig = r * r + a * a * np.cos(th) ** 2
    Del = r * r - 2 * r + a * a
    A = (r * r + a * a) ** 2 - a * a * Del * np.sin(th) ** 2
    al_z = np.sqrt(Sig * Del / A); om = 2 * a * r / A
    er, eh, ep = np.sqrt(Del / Sig), 1 / np.sqrt(Sig), 1 / (np.sqrt(A / Sig) * np.sin(th))
    f_hat = np.array([fup[1] / er, fup[2] / eh, fup[3] / ep])
    d_hat = np.array([kup[1] / er, kup[2] / eh, (kup[3] + om / al_z * 1.0) / ep])
    d_hat /= np.linalg.norm(d_hat)
    e2 = np.cross(d_hat, f_hat)
    f2 = np.array([0.0, e2[0] * er, e2[1] * eh, e2[2] * ep])
    ratio = wp(Y0[0:4], kup, f2) / k0
    assert abs(abs(ratio) - 1) < 1e-9 and abs(ratio.real) < 1e-9
    del zr
