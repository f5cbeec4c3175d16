"""Whole-ray pins of the oracle's invariant transfer: the redshift factors.

Each test traces one complete ray with the oracle and compares the observed
intensity with an independent computation that shares nothing with the
oracle's tracer except, where stated, its emissivity function (pinned on its
own in test_oracle_transfer.py):

- Toy disk, Schwarzschild, camera in the equatorial plane: the ray through
  (alpha, 0) stays in the plane, where the flow (Keplerian outside the ISCO,
  the ISCO's plunging geodesic inside) and the photon momentum have textbook
  closed forms.  I = integral of j g^2 over the affine parameter, g the ratio
  of observed to emitted frequency (Lorentz invariance of I_nu / nu^3), is
  computed by quadrature in r with d lambda = dr / |k^r|.
- Thermal power-law plasma, same geometry: the IQUV transfer equation
  dS/ds = j - K S in the emitter frame becomes, per unit affine length,
  J = L g^2 j and K_lambda = (L / g) K (ds = (L / g) d lambda; I_obs =
  g^3 I_em), integrated outward from the horizon to the camera by an ODE
  solver.  The pitch angle, the comoving field and the frequency shift are
  derived here from the ZAMO-frame flow and field; by reflection symmetry the
  projected field lies in the orbital plane (horizontal on the screen), so
  the polarisation angle is 90 degrees at every point.  Optically thin-to-
  moderate and optically thick (I -> g^3 B_nu) regimes are both covered.
- Circular emissivity j_V: the thermal (ultra-relativistic Maxwell-Juttner)
  average of the leading-order circularly polarised single-electron
  synchrotron emissivity for an isotropic pitch-angle distribution
  (Legg & Westfold 1968; Melrose 1971): per electron,
  (sqrt3 e^3 B sin th / (4 pi m c^2)) (4 cot th / (3 gamma)) H(nu / nu_c),
  H(y) = y K_{1/3}(y) + int_y^inf K_{1/3}(t) dt, nu_c = 3/2 gamma^2 nu_B sin th.

A wrong power of g in the emission (g^3 instead of g^2) or in the absorption
(K g instead of K / g), a Doppler factor of the wrong sign, or a wrong
pitch angle fails these by far more than their tolerances.
"""
import numpy as np
import pytest
from scipy import integrate, special

import art_inputs
from oracle import ray as oray

E_CGS, ME, C, H_PL = 4.80320471e-10, 9.1093837015e-28, 2.99792458e10, 6.62607015e-27


# ------------------------------------------------ Schwarzschild, equatorial
def photon_constants(r_cam, alpha):
    """Conserved k_t, k_phi of the backward ray leaving a static camera at
    (r_cam, theta = pi/2) toward screen point (alpha, 0): the direction in
    the camera frame is (-r_cam e_r + alpha e_phi) / norm and k = d - e_t,
    so k^(t) = -1, k_t = sqrt(1 - 2/r_cam), k_phi = r_cam * alpha / norm."""
    nrm = np.hypot(r_cam, alpha)
    return np.sqrt(1.0 - 2.0 / r_cam), r_cam * alpha / nrm


def k_r_contra(r, kt, kph):
    """|k^r| of a null ray in the equatorial plane (Schwarzschild, BL)."""
    return np.sqrt(kt * kt - (1.0 - 2.0 / r) * kph * kph / (r * r))


def flow_contra(r):
    """Equatorial flow, a = 0: circular Keplerian orbit outside r = 6
    (u^t = 1/sqrt(1-3/r), Omega = r^-3/2), the plunging geodesic with the ISCO's
    E = sqrt(8/9), L = 2 sqrt3 inside.  Returns (u^t, u^r, u^phi)."""
    if r >= 6.0:
        ut = 1.0 / np.sqrt(1.0 - 3.0 / r)
        return ut, 0.0, ut * r ** -1.5
    E, L = np.sqrt(8.0 / 9.0), 2.0 * np.sqrt(3.0)
    f = 1.0 - 2.0 / r
    ur = -np.sqrt(max(E * E - f * (1.0 + L * L / (r * r)), 0.0))
    return E / f, ur, L / (r * r)


def k_dot_u(r, kt, kph):
    """k.u for the inward backward ray (k^r < 0, covariant k_r = k^r / f)."""
    f = 1.0 - 2.0 / r
    ut, ur, up = flow_contra(r)
    kr_cov = -k_r_contra(r, kt, kph) / f
    return kt * ut + kr_cov * ur + kph * up


@pytest.mark.parametrize("alpha", [1.5, 3.5, 5.0])
def test_toy_disk_equatorial_ray_matches_quadrature(alpha):
    cfg = dict(art_inputs.workload("toy_disk_64"), inc_deg=90.0, eps=0.003)
    S, ft = oray.trace(cfg, np.array([alpha]), np.array([0.0]), nthreads=1)
    assert oray.STATUS[int(ft["status"][0])] == "captured"
    kt, kph = photon_constants(cfg["r_cam"], alpha)
    assert abs(kph / kt) < np.sqrt(27.0)           # captured: no turning point
    # emission j = r^-2 in the plane (cos theta = 0), J = j g^2 = j / (k.u)^2
    f = lambda r: 1.0 / (r * r) / k_dot_u(r, kt, kph) ** 2 / k_r_contra(r, kt, kph)
    r_end = 2.015                                  # the ray stops between 2.01 and 2.02
    pts = [6.0]
    I = integrate.quad(f, r_end, cfg["r_cam"], points=pts, limit=400, epsabs=0, epsrel=1e-12)[0]
    assert abs(S[0, 0] / I - 1.0) < 2e-5, (S[0, 0], I)


# ------------------------------------------------------- thermal plasma
def thermal_state(mp, r):
    """n_e, Theta_e, |B| of the power-law plasma (closed form)."""
    n0, th0, beta_ref, r_ref = mp[0], mp[1], mp[2], mp[3]
    ine, ith, ib = mp[6], mp[7], mp[8]
    ne, th = n0 * r ** -ine, th0 * r ** -ith
    ne_ref, th_ref = n0 * r_ref ** -ine, th0 * r_ref ** -ith
    b_ref = np.sqrt(8.0 * np.pi * ne_ref * ME * C * C * th_ref / beta_ref)
    return ne, th, b_ref * (r / r_ref) ** -ib


def equatorial_coefficients(cfg, r, kt, kph):
    """J (4) and K (4x4) per unit affine length at radius r on the inward
    equatorial ray, polarisation reference = screen up."""
    mp = cfg["mp"]
    f = 1.0 - 2.0 / r
    # orthonormal static-frame components (a = 0: the ZAMO is static)
    ut, ur, up = flow_contra(r)
    u_hat = np.array([ut * np.sqrt(f), ur / np.sqrt(f), 0.0, up * r])
    kr_cov = -k_r_contra(r, kt, kph) / f
    k_hat = np.array([kt / np.sqrt(f), kr_cov * np.sqrt(f), 0.0, kph / r])  # covariant
    eta = np.array([-1.0, 1.0, 1.0, 1.0])
    dot = lambda a, b: float(np.sum(eta * a * b))
    k_up = eta * k_hat
    ku = dot(k_up, u_hat)
    # field |B|(cos psi e_phi + sin psi e_r) in the static frame, made comoving
    psi = mp[4]
    Bh = np.array([0.0, np.sin(psi), 0.0, np.cos(psi)])
    q = dot(u_hat, Bh)
    b_hat = (Bh + q * u_hat) / np.sqrt(1.0 + q * q)
    cth = -dot(k_up, b_hat) / ku
    ne, th, B = thermal_state(mp, r)
    c = np.zeros(8)
    if r < mp[5]:
        oray.lib().or_thermal_coefs(ne, th, B, cfg["freq_hz"] * ku, cth, oray._dp(c))
    jI, jQ, jV, aI, aQ, aV, rQ, rV = c
    L = oray.length_unit_cm(cfg["mass_msun"])
    g = 1.0 / ku
    fJ, fK = L * g * g, L / g
    # field horizontal on the screen, reference vertical: cos 2chi = -1, sin 2chi = 0
    J = fJ * np.array([jI, -jQ, 0.0, jV])
    a_v = fK * np.array([-aQ, 0.0, aV])
    r_v = fK * np.array([-rQ, 0.0, rV])
    A_I = fK * aI
    K = np.array([[A_I, a_v[0], a_v[1], a_v[2]],
                  [a_v[0], A_I, r_v[2], -r_v[1]],
                  [a_v[1], -r_v[2], A_I, r_v[0]],
                  [a_v[2], r_v[1], -r_v[0], A_I]])
    return J, K


def transfer_ode(cfg, kt, kph, r_end, nstokes):
    """Forward transfer from the far end of the backward ray (the horizon) to
    the camera: dS/dr = (J - K S) / |k^r| (r increases along the photon)."""
    def rhs(r, S):
        J, K = equatorial_coefficients(cfg, r, kt, kph)
        if nstokes == 1:
            return [(J[0] - K[0, 0] * S[0]) / k_r_contra(r, kt, kph)]
        return (J - K @ S) / k_r_contra(r, kt, kph)
    sol = integrate.solve_ivp(rhs, (r_end, cfg["mp"][5]), np.zeros(nstokes), method="LSODA",
                              rtol=1e-10, atol=1e-30, first_step=1e-4, max_step=0.02)
    return sol.y[:, -1]


@pytest.mark.parametrize("nstokes", [1, 4])
@pytest.mark.parametrize("n0_scale,tol", [(1.0, 1e-5), (300.0, 1e-3)])
def test_thermal_equatorial_ray_matches_transfer_ode(nstokes, n0_scale, tol):
    """n0_scale 1: the workload's density (optical depth ~0.3 along this ray);
    300: optically thick with strong Faraday rotation and conversion.  The
    oracle's residual is its second-order discretisation (it falls 4x when
    the step halves); tol is set from it at eps = 0.003."""
    mp = art_inputs.thermal_params(seed=1)
    mp[0] *= n0_scale
    mp[4] = 0.4                     # field phase: toroidal and radial parts both present
    alpha = 3.5
    kt, kph = photon_constants(1000.0, alpha)
    errs = []
    for eps in (0.006, 0.003):
        cfg = dict(art_inputs.workload("thermal_1025"), a=0.0, inc_deg=90.0, eps=eps, mp=mp,
                   nstokes=nstokes)
        S, ft = oray.trace(cfg, np.array([alpha]), np.array([0.0]), nthreads=1)
        if eps == 0.006:
            want = transfer_ode(cfg, kt, kph, 2.015, nstokes)
            scale = abs(want[0])
            assert scale > 0
        errs.append(np.abs(S[0, :nstokes] - want).max() / scale)
    assert errs[-1] <= tol, (errs, S[0, :nstokes], want)
    assert errs[0] > 2.5 * errs[1], errs           # the residual is the step's


def test_thermal_thick_limit_is_redshifted_planck():
    """Deep inside an optically thick thermal emitter I_obs -> g^3 B_nu(nu_obs/g):
    a cold, dense, weakly emitting plasma (Rayleigh-Jeans regime at the
    photosphere) seen along the equatorial ray.  The photosphere sits where
    the optical depth first reaches ~1, so compare with g^3 B_nu at the radius
    where the independently computed depth is 1, within the spread of g^3
    B_nu over the radii where the depth lies between 0.1 and 10."""
    mp = art_inputs.thermal_params(seed=1)
    mp[0] *= 1e4
    mp[4] = 0.4
    alpha = 3.5
    cfg = dict(art_inputs.workload("thermal_1025"), a=0.0, inc_deg=90.0, eps=0.003, mp=mp, nstokes=1)
    S, ft = oray.trace(cfg, np.array([alpha]), np.array([0.0]), nthreads=1)
    kt, kph = photon_constants(cfg["r_cam"], alpha)
    rs = np.linspace(mp[5] - 1e-9, 2.05, 20000)
    K = np.array([equatorial_coefficients(cfg, r, kt, kph)[1][0, 0] / k_r_contra(r, kt, kph)
                  for r in rs])
    tau = np.concatenate([[0.0], np.cumsum(0.5 * (K[1:] + K[:-1]) * -np.diff(rs))])
    assert tau[-1] > 100.0

    def planck_obs(r):
        g = 1.0 / k_dot_u(r, kt, kph)
        th = thermal_state(mp, r)[1]
        nu_e = cfg["freq_hz"] / g
        return g ** 3 * 2 * H_PL * nu_e ** 3 / C ** 2 / np.expm1(H_PL * nu_e / (th * ME * C * C))
    band = (tau > 0.1) & (tau < 10.0)
    vals = np.array([planck_obs(r) for r in rs[band]])
    assert vals.min() <= S[0, 0] <= vals.max(), (S[0, 0], vals.min(), vals.max())
    r1 = rs[np.argmin(np.abs(tau - 1.0))]
    assert abs(S[0, 0] / planck_obs(r1) - 1.0) < 0.5


# -------------------------------------------------- circular emissivity
def h_circ(y):
    return y * special.kv(1.0 / 3.0, y) + integrate.quad(lambda t: special.kv(1.0 / 3.0, t), y,
                                                          np.inf, limit=200)[0]


def f_sync(y):
    return y * integrate.quad(lambda t: special.kv(5.0 / 3.0, t), y, np.inf, limit=200)[0]


def textbook_thermal(ne, th, B, nu, cth):
    """(j_I, j_V) from the single-electron emissivities integrated over the
    ultra-relativistic Maxwell-Juttner distribution N(gamma) = n gamma^2
    e^(-gamma/Theta) / (2 Theta^3), directly in gamma."""
    sth = np.sqrt(1.0 - cth * cth)
    nuB = E_CGS * B / (2 * np.pi * ME * C)
    P0 = np.sqrt(3.0) * E_CGS ** 3 * B * sth / (4 * np.pi * ME * C * C)

    def weight(gam):
        return ne * gam * gam * np.exp(-gam / th) / (2.0 * th ** 3)

    def y(gam):
        return nu / (1.5 * gam * gam * nuB * sth)
    # gamma = Theta z: the weight peaks near z = 2, the spectrum cuts off
    # below z ~ sqrt(nu / nu_c(Theta)); both lie inside [1e-3, 80] Theta
    xm = nu / (1.5 * th * th * nuB * sth)
    zs = sorted({0.5, 2.0, (2.0 * xm) ** (1.0 / 3.0), np.sqrt(xm)})
    pts = [th * z for z in zs if 1e-3 < z < 80.0]
    lo, hi = 1e-3 * th, 80.0 * th
    quad = lambda fn: integrate.quad(fn, lo, hi, points=pts, limit=800, epsrel=1e-10, epsabs=0)[0]
    jI = quad(lambda g: weight(g) * P0 * f_sync(y(g)))
    jV = quad(lambda g: weight(g) * P0 * (4.0 * cth / (3.0 * g * sth)) * h_circ(y(g)))
    return jI, jV


@pytest.mark.parametrize("xM", [0.5, 2.0, 10.0, 50.0, 300.0])
@pytest.mark.parametrize("cth", [0.3, -0.7])
def test_circular_emissivity_matches_textbook_integral(xM, cth):
    ne, th, B = 1e6, 30.0, 20.0
    sth = np.sqrt(1 - cth * cth)
    nuB = E_CGS * B / (2 * np.pi * ME * C)
    nu = xM * 3.0 * nuB * th * th * sth / 2.0
    c = np.zeros(8)
    oray.lib().or_thermal_coefs(ne, th, B, nu, cth, oray._dp(c))
    jI, jV = textbook_thermal(ne, th, B, nu, cth)
    # the fitting forms follow these integrals to a few parts in a thousand
    assert abs(c[0] / jI - 1) < 0.01, (c[0], jI)
    assert abs(c[2] / jV - 1) < 0.01, (c[2], jV)
