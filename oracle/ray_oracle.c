/*
 * ray_oracle.c -- plain, slow, scalar FP64 CPU oracle for the per-ray part of
 * adaptive black-hole ray tracing (Gelles et al. 2021, arXiv:2103.07417).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
 * load this file; only tests/, the smoke check and the bench's CPU-baseline leg
 * use it.  It shares no code with the HIP path: both implement the method
 * written out below independently.
 *
 * The paper delegates everything per ray to an external GRRT code (Sec. 4.1,
 * "Models and Implementation"); it only fixes that a ray is traced for each
 * sampled screen point and returns an intensity I(x) (Sec. 3, opening
 * paragraph) or Stokes (I,Q,U,V) (Sec. 6, last paragraph).  The discretisation
 * below is therefore this project's own method definition:
 *
 *   - Kerr spacetime, mass M = 1, spin a, spherical Kerr-Schild coordinates.
 *   - Null geodesic in Hamiltonian form H = g^{mu nu} k_mu k_nu / 2 with k_t,
 *     k_phi conserved exactly; state (r, theta, phi, k_r, k_theta); classical
 *     RK4 with the step rule h = eps * clamp(r/20, 1, 4) / (|dr|/r + |dtheta| +
 *     |dphi|), limited to half the coordinate distance to the horizon when
 *     moving inward.
 *   - k is the time-reversed photon momentum, normalised so that k.u_cam = +1.
 *   - Termination: r < 1.01 r_h (captured), r > r_out with dr/dlambda > 0
 *     (escaped), step cap, or transmission below 1e-12 (optically thick).
 *   - Plasma, coefficients and transfer are evaluated once per step at the
 *     arithmetic midpoint of the step's end states, with the step's length.
 *   - Polarised transfer: one-pass backward accumulation of the observer-side
 *     4x4 propagator O, S += O * Delta, O <- O * exp(-K h), where exp of the
 *     Lorentz-algebra part of K is evaluated in closed form.
 *   - Polarisation basis: Walker-Penrose constant of the camera's screen-up
 *     vector, compared at each point with that of the projected magnetic field.
 *
 * Pins (tests/test_oracle_*.py) tie each piece to something outside this
 * file: closed forms of Kerr geodesics and of constant-coefficient slabs,
 * textbook synchrotron integrals for j_I, j_Q and j_V, and whole equatorial
 * Schwarzschild rays whose intensity is recomputed by quadrature (toy disk)
 * or by an ODE solver of the transfer equation (thermal plasma), which fixes
 * the redshift factors g^2 of the emission and 1/g of the absorption.  The
 * sign convention of V (positive for cos th_B > 0) is a reading.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* Operation-count categories (used only by the instrumented build,
 * opcount.cpp): 0 geodesic, 1 plasma point, 2 transfer update. */
#ifndef OR_CAT
#define OR_CAT(c) ((void)0)
#endif
#ifndef OR_EMIT
#define OR_EMIT(e) ((void)0)
#endif

/* ----------------------------------------------------------------- consts */
#define OR_E      4.80320471e-10   /* electron charge [esu] */
#define OR_ME     9.1093837015e-28 /* electron mass [g] */
#define OR_C      2.99792458e10    /* speed of light [cm/s] */
#define OR_H      6.62607015e-27   /* Planck [erg s] */
#define OR_PI     3.14159265358979323846
#define OR_MP     1.67262192369e-24 /* proton mass [g] */

enum { OR_OK = 0, OR_CAPTURED = 1, OR_ESCAPED = 2, OR_STEPCAP = 3, OR_THICK = 4, OR_NAN = 5 };
enum { OR_MODEL_TOYDISK = 1, OR_MODEL_THERMAL = 2, OR_MODEL_GRID = 3,
       OR_MODEL_SCREEN_RING = 10, OR_MODEL_SCREEN_POLY = 11 };

typedef struct {
    double a;          /* spin, |a| < 1 */
    double r_cam;      /* camera radius [M] */
    double inc;        /* camera inclination [rad] */
    double r_out;      /* escape radius [M] */
    double eps;        /* step-rule accuracy */
    int32_t max_steps;
    int32_t nstokes;   /* 1 or 4 */
    int32_t model;
    int32_t nsub;      /* subring planes (0: none) */
    double freq;       /* observing frequency [Hz] */
    double L_cm;       /* length unit GM/c^2 [cm] */
    double mp[16];     /* model parameters (see or_model_*) */
    /* grid model (MKS snapshot), unused otherwise */
    const float* grid; /* [8][n3][n2][n1] fields rho,u,U1,U2,U3,B1,B2,B3 */
    int32_t n1, n2, n3, pad2;
    double gp[8];      /* x1 start, x1 stop, hslope, ... */
    double phi_cam;    /* camera azimuth [rad] */
} or_params;

#define OR_MAX_SUB 8

typedef struct { double re, im; } cplx;

/* ------------------------------------------------------------ Kerr in BL */
/* Boyer-Lindquist covariant metric components (textbook Kerr). */
typedef struct { double tt, tp, rr, hh, pp; } bl_cov;
typedef struct { double tt, tp, rr, hh, pp; } bl_con;

static void bl_metric(double a, double r, double th, bl_cov* g, bl_con* gi)
{
    double c = cos(th), s = sin(th);
    double s2 = s * s, c2 = c * c;
    double Sig = r * r + a * a * c2;
    double Del = r * r - 2.0 * r + a * a;
    double A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s2;
    if (g) {
        g->tt = -(1.0 - 2.0 * r / Sig);
        g->tp = -2.0 * a * r * s2 / Sig;
        g->rr = Sig / Del;
        g->hh = Sig;
        g->pp = (r * r + a * a + 2.0 * a * a * r * s2 / Sig) * s2;
    }
    if (gi) {
        gi->tt = -A / (Sig * Del);
        gi->tp = -2.0 * a * r / (Sig * Del);
        gi->rr = Del / Sig;
        gi->hh = 1.0 / Sig;
        gi->pp = (Del - a * a * s2) / (Sig * Del * s2);
    }
}

/* ZAMO (locally non-rotating) tetrad in BL: e_(t) = (1/al)(1,0,0,om),
 * e_(r) = sqrt(Del/Sig) d_r, e_(th) = d_th/sqrt(Sig), e_(ph) = d_ph/varpi. */
typedef struct { double al, om, er, eh, ep; } zamo;

static void zamo_frame(double a, double r, double th, zamo* z)
{
    double c = cos(th), s = sin(th);
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * r + a * a;
    double A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s * s;
    z->al = sqrt(Sig * Del / A);
    z->om = 2.0 * a * r / A;
    z->er = sqrt(Del / Sig);
    z->eh = 1.0 / sqrt(Sig);
    z->ep = 1.0 / (sqrt(A / Sig) * s);
}

static double horizon(double a) { return 1.0 + sqrt(1.0 - a * a); }

/* --------------------------------------------- geodesic RHS (KS, spherical)
 * Inverse KS metric: g^tt = -(1+2r/Sig), g^tr = 2r/Sig, g^rr = Del/Sig,
 * g^rph = a/Sig, g^thth = 1/Sig, g^phph = 1/(Sig sin^2).  With
 *   Qf = -2r kt^2 + 4r kt kr + Del kr^2 + 2a kr kph + kth^2 + kph^2/sin^2
 * one has 2H = -kt^2 + Qf/Sig.  Hamilton's equations give the RHS below.   */
static void geo_rhs(double a, double kt, double kph, const double* y, double* dy)
{
    double r = y[0], th = y[1], kr = y[3], kth = y[4];
    double c = cos(th), s = sin(th);
    double s2 = s * s;
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * r + a * a;
    double iS = 1.0 / Sig;
    double Lph = 0.0, Lph_over = 0.0, dQth = 0.0;
    if (kph != 0.0) {
        Lph = kph * kph / s2;
        Lph_over = kph / s2;
        dQth = -2.0 * kph * kph * c / (s2 * s);
    }
    double Qf = -2.0 * r * kt * kt + 4.0 * r * kt * kr + Del * kr * kr
                + 2.0 * a * kr * kph + kth * kth + Lph;
    double dQr = -2.0 * kt * kt + 4.0 * kt * kr + (2.0 * r - 2.0) * kr * kr;
    double dSth = -2.0 * a * a * c * s;
    dy[0] = (2.0 * r * kt + Del * kr + a * kph) * iS;
    dy[1] = kth * iS;
    dy[2] = (a * kr + Lph_over) * iS;
    dy[3] = -0.5 * (dQr * iS - Qf * 2.0 * r * iS * iS);
    dy[4] = -0.5 * (dQth * iS - Qf * dSth * iS * iS);
}

/* KS Hamiltonian 2H (null norm) for diagnostics. */
double or_null_norm(double a, double kt, double kph, const double* y)
{
    double r = y[0], th = y[1], kr = y[3], kth = y[4];
    double c = cos(th), s = sin(th);
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * r + a * a;
    double Qf = -2.0 * r * kt * kt + 4.0 * r * kt * kr + Del * kr * kr
                + 2.0 * a * kr * kph + kth * kth + (kph != 0.0 ? kph * kph / (s * s) : 0.0);
    return -kt * kt + Qf / Sig;
}

void or_geo_rhs(double a, double kt, double kph, const double* y, double* dy)
{
    geo_rhs(a, kt, kph, y, dy);
}

/* ------------------------------------------------------------------ camera
 * ZAMO camera at (r_cam, theta = inc, phi = 0).  The backward ray through
 * screen point (alpha, beta) [M, at the hole's distance] leaves the camera in
 * the direction d = (-r_cam e_r - beta e_th + alpha e_ph)/norm (beta up =
 * toward decreasing theta, alpha right = +phi).  k = d - e_(t), i.e. the
 * reversed photon momentum with k.u_cam = +1.  The polarisation reference is
 * screen-up (-e_th) projected orthogonal to d.                            */
typedef struct {
    double y[5];       /* r, th, ph, k_r(KS), k_th */
    double kt, kph;    /* conserved covariant components */
    double kup_bl[4];  /* contravariant BL momentum at the camera */
    double fup_bl[4];  /* contravariant BL polarisation reference */
} cam_ray;

static void camera_ray(const or_params* p, double alpha, double beta, cam_ray* cr)
{
    double a = p->a, r = p->r_cam, th = p->inc;
    zamo z; zamo_frame(a, r, th, &z);
    bl_cov g; bl_metric(a, r, th, &g, 0);
    double nrm = sqrt(r * r + alpha * alpha + beta * beta);
    double dr = -r / nrm, dh = -beta / nrm, dp = alpha / nrm;
    /* contravariant k = d - e_(t) */
    double ku_t = -1.0 / z.al;
    double ku_r = dr * z.er;
    double ku_h = dh * z.eh;
    double ku_p = dp * z.ep - z.om / z.al;
    double kt = g.tt * ku_t + g.tp * ku_p;
    double kr_bl = g.rr * ku_r;
    double kth = g.hh * ku_h;
    /* k_phi = k . d_phi = sqrt(g_phiphi) (k . e_(phi)): only the screen direction
     * contributes (the ZAMO observer has no angular momentum), so alpha = 0
     * gives k_phi = 0 exactly */
    double kph = dp * sqrt(g.pp);
    (void)ku_p;
    double Del = r * r - 2.0 * r + a * a;
    double kr_ks = kr_bl - (2.0 * r / Del) * kt - (a / Del) * kph;
    cr->y[0] = r; cr->y[1] = th; cr->y[2] = p->phi_cam; cr->y[3] = kr_ks; cr->y[4] = kth;
    cr->kt = kt; cr->kph = kph;
    cr->kup_bl[0] = ku_t; cr->kup_bl[1] = ku_r; cr->kup_bl[2] = ku_h; cr->kup_bl[3] = ku_p;
    /* f = -e_th projected orthogonal to d in the camera frame, normalised */
    double ux = 0.0, uy = -1.0, uz = 0.0;  /* -e_th in (r,th,ph) components */
    double dd = ux * dr + uy * dh + uz * dp;
    double fr = ux - dd * dr;
    double fh = uy - dd * dh, fp = uz - dd * dp;
    double fn = sqrt(fr * fr + fh * fh + fp * fp);
    fr /= fn; fh /= fn; fp /= fn;
    cr->fup_bl[0] = 0.0;
    cr->fup_bl[1] = fr * z.er;
    cr->fup_bl[2] = fh * z.eh;
    cr->fup_bl[3] = fp * z.ep;
}

void or_camera(const or_params* p, double alpha, double beta, double* y5,
               double* kt, double* kph, double* kup, double* fup)
{
    cam_ray cr; camera_ray(p, alpha, beta, &cr);
    memcpy(y5, cr.y, sizeof(cr.y));
    *kt = cr.kt; *kph = cr.kph;
    memcpy(kup, cr.kup_bl, sizeof(cr.kup_bl));
    memcpy(fup, cr.fup_bl, sizeof(cr.fup_bl));
}

/* ------------------------------------------------- Walker-Penrose constant
 * kappa = (A1 - i A2)(r - i a cos th), BL contravariant components:
 *   A1 = (k^t f^r - k^r f^t) + a sin^2 (k^r f^ph - k^ph f^r)
 *   A2 = [(r^2+a^2)(k^ph f^th - k^th f^ph) - a (k^t f^th - k^th f^t)] sin   */
static cplx walker_penrose(double a, double r, double th, const double* k, const double* f)
{
    double c = cos(th), s = sin(th);
    double A1 = (k[0] * f[1] - k[1] * f[0]) + a * s * s * (k[1] * f[3] - k[3] * f[1]);
    double A2 = ((r * r + a * a) * (k[3] * f[2] - k[2] * f[3]) - a * (k[0] * f[2] - k[2] * f[0])) * s;
    cplx z;
    z.re = A1 * r - A2 * a * c;
    z.im = -(A1 * a * c + A2 * r);
    return z;
}

void or_walker_penrose(double a, double r, double th, const double* k, const double* f, double* out)
{
    cplx z = walker_penrose(a, r, th, k, f);
    out[0] = z.re; out[1] = z.im;
}

/* ------------------------------------------------------------ fluid model */
/* Equatorial circular-orbit energy / angular momentum (orbit in +phi). */
static void circ_EL(double a, double r, double* E, double* L)
{
    double sr = sqrt(r), r34 = pow(r, 0.75);
    double den = r34 * sqrt(r * sr - 3.0 * sr + 2.0 * a);
    *E = (r * sr - 2.0 * sr + a) / den;
    *L = (r * r - 2.0 * a * sr + a * a) / den;
}

double or_r_isco(double a)
{
    double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    double z2 = sqrt(3.0 * a * a + z1 * z1);
    double sg = (a > 0.0) ? 1.0 : ((a < 0.0) ? -1.0 : 0.0);
    return 3.0 + z2 - sg * sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

/* ZAMO-frame 3-velocity (v_r, v_ph) of the equatorial flow at radius r:
 * Keplerian Omega = 1/(r^1.5 + a) outside the ISCO, the plunging geodesic
 * with the ISCO's E and L inside.  Applied unchanged at every theta.       */
static void flow_v3(double a, double r, double risco, double Eis, double Lis,
                    double* vr, double* vp)
{
    double Del = r * r - 2.0 * r + a * a;
    double A = (r * r + a * a) * (r * r + a * a) - a * a * Del;
    double al = sqrt(r * r * Del / A);
    double om = 2.0 * a * r / A;
    double vpi = sqrt(A) / r;
    if (r >= risco) {
        double Om = 1.0 / (r * sqrt(r) + a);
        *vp = vpi * (Om - om) / al;
        *vr = 0.0;
    } else {
        double Gam = (Eis - om * Lis) / al;
        *vp = (Lis / vpi) / Gam;
        double q = 1.0 - 1.0 / (Gam * Gam) - (*vp) * (*vp);
        *vr = -sqrt(q > 0.0 ? q : 0.0);
    }
}

/* 4-velocity (BL contravariant) of the model flow at (r, th). */
static void flow_u(double a, double r, double th, double risco, double Eis, double Lis,
                   double* u, double* Gam_out, double* vr_out, double* vp_out, zamo* zf)
{
    double vr, vp;
    flow_v3(a, r, risco, Eis, Lis, &vr, &vp);
    zamo z; zamo_frame(a, r, th, &z);
    double Gam = 1.0 / sqrt(1.0 - vr * vr - vp * vp);
    u[0] = Gam / z.al;
    u[1] = Gam * vr * z.er;
    u[2] = 0.0;
    u[3] = Gam * (z.om / z.al + vp * z.ep);
    if (Gam_out) *Gam_out = Gam;
    if (vr_out) *vr_out = vr;
    if (vp_out) *vp_out = vp;
    if (zf) *zf = z;
}

void or_flow_u(double a, double r, double th, double* u)
{
    double risco = or_r_isco(a), E, L;
    circ_EL(a, risco, &E, &L);
    flow_u(a, r, th, risco, E, L, u, 0, 0, 0, 0);
}

void or_circ_EL(double a, double r, double* E, double* L) { circ_EL(a, r, E, L); }

/* ------------------------------------------ thermal synchrotron coefficients
 * Ultra-relativistic thermal electrons, x = 2 nu / (3 nu_B Theta^2 sin th_B).
 * Emissivity integrals (forms of Dexter 2016, App. A; leading constant
 * 2 pi / sqrt 6 and exponent 3 * 2^(-2/3) follow from the saddle point of the
 * Maxwell-Juttner average of the single-electron synchrotron spectrum):
 *   I_I = 2.5651 (1 + 1.92 x^-1/3 + 0.9977 x^-2/3) exp(-1.8899 x^1/3)
 *   I_Q = 2.5651 (1 + 0.932 x^-1/3 + 0.4998 x^-2/3) exp(-1.8899 x^1/3)
 *   I_V = (1.8138/x + 3.423 x^-2/3 + 0.02955 x^-1/2 + 2.0377 x^-1/3) exp(-1.8899 x^1/3)
 *   j_I = n e^2 nu/(2 sqrt3 c Theta^2) I_I, j_Q likewise with I_Q,
 *   j_V = n e^2 nu/(2 sqrt3 c Theta^2) (4 cot th_B / (3 Theta)) I_V,
 * total polarised fraction capped at 0.99; absorption from Kirchhoff's law
 * alpha_S = j_S / B_nu(T_e); rotativities are the cold-plasma forms times
 *   g_V = ln(1+2 Theta)/(2 Theta^2 + ln(1+2 Theta)),  g_Q = 1/(1+2 Theta) + 6 Theta.
 * Signs in the frame whose Q axis is the projected field: j_Q, alpha_Q and
 * rho_Q negative; V terms carry sign(cos th_B).                            */
typedef struct { double jI, jQ, jV, aI, aQ, aV, rQ, rV; } coefs;

static void thermal_coefs(double ne, double Th, double B, double nu, double cth, coefs* c)
{
    memset(c, 0, sizeof(*c));
    double sth2 = 1.0 - cth * cth;
    if (sth2 < 0.0) sth2 = 0.0;
    double sth = sqrt(sth2);
    double nuB = OR_E * B / (2.0 * OR_PI * OR_ME * OR_C);
    double e2 = OR_E * OR_E;
    /* rotativities */
    double lg = log1p(2.0 * Th);
    double gV = lg / (2.0 * Th * Th + lg);
    double gQ = 1.0 / (1.0 + 2.0 * Th) + 6.0 * Th;
    c->rV = 2.0 * ne * e2 * nuB * cth / (OR_ME * OR_C * nu * nu) * gV;
    c->rQ = -ne * e2 * nuB * nuB * sth2 / (OR_ME * OR_C * nu * nu * nu) * gQ;
    if (sth < 1e-10) return;
    double x = 2.0 * nu / (3.0 * nuB * Th * Th * sth);
    double x13 = cbrt(x);
    double xm13 = 1.0 / x13, xm23 = xm13 * xm13;
    double ex = exp(-1.8899 * x13);
    double II = 2.5651 * (1.0 + 1.92 * xm13 + 0.9977 * xm23) * ex;
    double IQ = 2.5651 * (1.0 + 0.932 * xm13 + 0.4998 * xm23) * ex;
    double IV = (1.8138 / x + 3.423 * xm23 + 0.02955 / sqrt(x) + 2.0377 * xm13) * ex;
    double pref = ne * e2 * nu / (2.0 * sqrt(3.0) * OR_C * Th * Th);
    double jI = pref * II;
    double jQ = pref * IQ;
    double jV = pref * (4.0 * cth / (3.0 * Th * sth)) * IV;
    double P = sqrt(jQ * jQ + jV * jV);
    if (P > 0.99 * jI) {
        double sc = 0.99 * jI / P;
        jQ *= sc; jV *= sc;
    }
    double Bnu = 2.0 * OR_H * nu * nu * nu / (OR_C * OR_C)
                 / expm1(OR_H * nu / (Th * OR_ME * OR_C * OR_C));
    c->jI = jI; c->jQ = -jQ; c->jV = jV;
    c->aI = jI / Bnu; c->aQ = -jQ / Bnu; c->aV = jV / Bnu;
}

void or_thermal_coefs(double ne, double Th, double B, double nu, double cth, double* out8)
{
    coefs c; thermal_coefs(ne, Th, B, nu, cth, &c);
    out8[0] = c.jI; out8[1] = c.jQ; out8[2] = c.jV; out8[3] = c.aI;
    out8[4] = c.aQ; out8[5] = c.aV; out8[6] = c.rQ; out8[7] = c.rV;
}

/* -------------------------------------------------- transfer exponentials
 * M = exp(-aI x) exp(-A x) for the Lorentz-algebra part A of the transfer
 * matrix K = aI 1 + A with boost (aQ,aU,aV) and rotation (rQ,rU,rV):
 *   A = [[0,aQ,aU,aV],[aQ,0,rV,-rU],[aU,-rV,0,rQ],[aV,rU,-rQ,0]].
 * A has eigenvalues +-L1, +-i L2 with L1^2 - L2^2 = |a|^2 - |r|^2,
 * L1 L2 = a.r; then exp(yA) = c0 + c1 A + c2 A^2 + c3 A^3 with
 *   c0 = (L2^2 cosh yL1 + L1^2 cos yL2)/D, c2 = (cosh yL1 - cos yL2)/D,
 *   c1 = (L2^2 sinh(yL1)/L1 + L1^2 sin(yL2)/L2)/D,
 *   c3 = (sinh(yL1)/L1 - sin(yL2)/L2)/D,   D = L1^2 + L2^2,
 * evaluated below in forms free of cancellation and overflow.            */
static double shc_damped(double u, double w)   /* e^-w sinh(u)/u */
{
    if (u < 1.0) {
        double u2 = u * u;
        double s = 1.0 + u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0 * (1.0 + u2 / 72.0 * (1.0 + u2 / 110.0 * (1.0 + u2 / 156.0)))));
        return exp(-w) * s;
    }
    return (exp(u - w) - exp(-u - w)) / (2.0 * u);
}
static double sinc_(double v)                   /* sin(v)/v */
{
    if (v < 1.0) {
        double v2 = v * v;
        return 1.0 - v2 / 6.0 * (1.0 - v2 / 20.0 * (1.0 - v2 / 42.0 * (1.0 - v2 / 72.0 * (1.0 - v2 / 110.0 * (1.0 - v2 / 156.0)))));
    }
    return sin(v) / v;
}
static double gfun_damped(double u, double w)  /* e^-w (sinh(u)/u - 1)/u^2 */
{
    if (u < 1.0) {
        double u2 = u * u;
        double s = 1.0 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0 * (1.0 + u2 / 72.0 * (1.0 + u2 / 110.0 * (1.0 + u2 / 156.0 * (1.0 + u2 / 210.0))))));
        return exp(-w) * s;
    }
    return (shc_damped(u, w) - exp(-w)) / (u * u);
}
static double hfun(double v)                    /* (1 - sin(v)/v)/v^2 */
{
    if (v < 1.0) {
        double v2 = v * v;
        return 1.0 / 6.0 * (1.0 - v2 / 20.0 * (1.0 - v2 / 42.0 * (1.0 - v2 / 72.0 * (1.0 - v2 / 110.0 * (1.0 - v2 / 156.0 * (1.0 - v2 / 210.0))))));
    }
    return (1.0 - sin(v) / v) / (v * v);
}

static void matmul4(const double* A, const double* B, double* C)
{
    double T[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[i * 4 + k] * B[k * 4 + j];
            T[i * 4 + j] = s;
        }
    memcpy(C, T, sizeof(T));
}

/* out = exp(-aI x) exp(-A x); x >= 0. */
static void lorentz_exp(double aI, const double* av, const double* rv, double x, double* out)
{
    double A[16] = {
        0.0,    av[0],  av[1],  av[2],
        av[0],  0.0,    rv[2], -rv[1],
        av[1], -rv[2],  0.0,    rv[0],
        av[2],  rv[1], -rv[0],  0.0 };
    double a2 = av[0] * av[0] + av[1] * av[1] + av[2] * av[2];
    double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    double ad = av[0] * rv[0] + av[1] * rv[1] + av[2] * rv[2];
    double dlt = a2 - r2;
    double D = sqrt(dlt * dlt + 4.0 * ad * ad);
    double L1s = 0.5 * (D + dlt); if (L1s < 0.0) L1s = 0.0;
    double L2s = 0.5 * (D - dlt); if (L2s < 0.0) L2s = 0.0;
    double L1 = sqrt(L1s), L2 = sqrt(L2s);
    double u = x * L1, v = x * L2, w = x * aI;
    double ew = exp(-w);
    double ch = 0.5 * (exp(u - w) + exp(-u - w));
    double shc = shc_damped(u, w);
    double snc = sinc_(v);
    double c0, c1, c2, c3;
    if (D > 0.0) {
        double sh2 = shc_damped(0.5 * u, 0.5 * w);   /* e^-w/2 sinh(u/2)/(u/2) */
        double sn2 = sinc_(0.5 * v);
        c2 = 0.5 * x * x * (L1s * sh2 * sh2 + L2s * ew * sn2 * sn2) / D;
        c1 = -x * (L2s * shc + L1s * ew * snc) / D;
        c3 = -x * x * x * (L1s * gfun_damped(u, w) + L2s * ew * hfun(v)) / D;
    } else {
        c2 = 0.5 * x * x * ew;
        c1 = -x * ew;
        c3 = -x * x * x * ew / 6.0;
    }
    c0 = ch - L1s * c2;
    double A2[16], A3[16];
    matmul4(A, A, A2);
    matmul4(A2, A, A3);
    for (int i = 0; i < 16; ++i) out[i] = c1 * A[i] + c2 * A2[i] + c3 * A3[i];
    for (int i = 0; i < 4; ++i) out[i * 5] += c0;
}

void or_lorentz_exp(double aI, const double* av, const double* rv, double x, double* out)
{
    lorentz_exp(aI, av, rv, x, out);
}

static double phi1(double w)      /* (1 - e^-w)/w */
{
    if (w < 1e-4) return 1.0 - w / 2.0 + w * w / 6.0 - w * w * w / 24.0;
    return -expm1(-w) / w;
}
static double mean_depth(double w) /* 1/w - 1/(e^w - 1): emission-weighted depth / h */
{
    if (w < 0.1) { double w2 = w * w; return 0.5 - w / 12.0 + w * w2 / 720.0 - w * w2 * w2 / 30240.0; }
    return 1.0 / w - 1.0 / expm1(w);
}

/* One constant-coefficient step of length h (affine) for the IQUV vector.
 * K per unit affine length: aI, av[3], rv[3]; J per unit affine length.   */
static void transfer_step4(double* S, double* O, double aI, const double* av, const double* rv,
                           const double* J, double h)
{
    double E[16], G[16], d[4], od[4];
    lorentz_exp(aI, av, rv, h, E);
    double w = aI * h;
    double sbar = h * mean_depth(w);
    lorentz_exp(0.0, av, rv, sbar, G);
    double sc = h * phi1(w);
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += G[i * 4 + k] * J[k];
        d[i] = sc * s;
    }
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += O[i * 4 + k] * d[k];
        od[i] = s;
    }
    for (int i = 0; i < 4; ++i) S[i] += od[i];
    matmul4(O, E, O);
}

void or_transfer_step4(double* S, double* O, double aI, const double* av, const double* rv,
                       const double* J, double h)
{
    transfer_step4(S, O, aI, av, rv, J, h);
}

/* --------------------------------------------------- screen test functions
 * Closed-form "rays" for refinement tests: the intensity is a function of the
 * screen point only (Sec. 3: the method needs only samples of I(x)).       */
static void screen_fn(const or_params* p, double al, double be, double* S)
{
    double I;
    if (p->model == OR_MODEL_SCREEN_RING) {
        /* bright thin ring of radius mp0, width mp1, plus diffuse disk */
        double rho = sqrt(al * al + be * be);
        double d = (rho - p->mp[0]) / p->mp[1];
        I = exp(-0.5 * d * d) * (1.0 + 0.5 * al / (rho + 1.0)) + p->mp[2] * exp(-rho * rho / (2.0 * p->mp[3] * p->mp[3]));
    } else {
        /* quadratic c0 + c1 al + c2 be + c3 al^2 + c4 al be + c5 be^2 */
        I = p->mp[0] + p->mp[1] * al + p->mp[2] * be + p->mp[3] * al * al
            + p->mp[4] * al * be + p->mp[5] * be * be;
    }
    S[0] = I;
    S[1] = 0.5 * I * cos(0.3 * al);
    S[2] = 0.5 * I * sin(0.3 * be);
    S[3] = 0.1 * I;
}

/* ---------------------------------------------------------------- tracing */
typedef struct { float rmin; int32_t ncross; int32_t steps; int32_t status; } ray_feat;

/* ------------------------------------------------------ gridded snapshot
 * MKS cell centres: x1 = ln r at x1_0 + (i + 1/2) dx1, theta_j = theta(x2_j)
 * with x2_j = (j + 1/2)/n2 and theta(x2) = pi x2 + (1-h)/2 sin(2 pi x2),
 * phi_k = 2 pi (k + 1/2)/n3.  Fields are interpolated trilinearly in
 * (x1, theta, phi) between cell centres: clamped in x1 and theta, periodic in
 * phi.  A theta outside [0, pi] (pole passage) is reflected with phi + pi.   */
static double mks_theta(double x2, double h)
{
    return OR_PI * x2 + 0.5 * (1.0 - h) * sin(2.0 * OR_PI * x2);
}

static void grid_sample(const or_params* p, double r, double th, double ph, double* out)
{
    int n1 = (int)p->mp[9], n2 = (int)p->mp[10], n3 = (int)p->mp[11];
    double x1_0 = p->mp[6], dx1 = p->mp[7], h = p->mp[8];
    double tw = fmod(th, 2.0 * OR_PI);
    if (tw < 0.0) tw += 2.0 * OR_PI;
    if (tw > OR_PI) { tw = 2.0 * OR_PI - tw; ph += OR_PI; }
    double pw = ph - 2.0 * OR_PI * floor(ph / (2.0 * OR_PI));
    /* x1 */
    double f1 = (log(r) - x1_0) / dx1 - 0.5;
    int i1 = (int)floor(f1);
    double t1 = f1 - i1;
    if (i1 < 0) { i1 = 0; t1 = 0.0; }
    if (i1 > n1 - 2) { i1 = n1 - 2; t1 = 1.0; }
    /* theta by bisection over the cell-centre angles */
    int j;
    double t2;
    double th0 = mks_theta(0.5 / n2, h), thn = mks_theta((n2 - 0.5) / n2, h);
    if (tw <= th0) { j = 0; t2 = 0.0; }
    else if (tw >= thn) { j = n2 - 2; t2 = 1.0; }
    else {
        int lo = 0, hi = n2 - 1;
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (mks_theta((mid + 0.5) / n2, h) <= tw) lo = mid; else hi = mid;
        }
        j = lo;
        double ta = mks_theta((j + 0.5) / n2, h), tb = mks_theta((j + 1.5) / n2, h);
        t2 = (tw - ta) / (tb - ta);
    }
    /* phi, periodic */
    double f3 = pw * n3 / (2.0 * OR_PI) - 0.5;
    double fl3 = floor(f3);
    double t3 = f3 - fl3;
    int k0 = ((int)fl3 % n3 + n3) % n3, k1 = (k0 + 1) % n3;
    for (int q = 0; q < 8; ++q) out[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
        double w = (di ? t1 : 1.0 - t1) * (dj ? t2 : 1.0 - t2) * (dk ? t3 : 1.0 - t3);
        size_t idx = (((size_t)(dk ? k1 : k0) * n2 + (size_t)(j + dj)) * n1 + (size_t)(i1 + di)) * 8;
        for (int q = 0; q < 8; ++q) out[q] += w * (double)p->grid[idx + q];
    }
}

void or_grid_sample(const or_params* p, double r, double th, double ph, double* out8)
{
    grid_sample(p, r, th, ph, out8);
}

/* Electron density, temperature and field strength of the gridded model:
 * p = (gamma-1) u, plasma beta b = p / (|B|^2/2), T_i/T_e = (R_high b^2 +
 * R_low)/(1 + b^2), Theta_e = (m_p/m_e) (p/rho) / (1 + T_i/T_e),
 * n_e = rho n_unit, |B|_G = |B| c sqrt(4 pi n_unit m_p); nothing emits where
 * |B|^2/rho exceeds the sigma cut.  Returns 0 where nothing emits.        */
static int grid_plasma(const or_params* p, double r, double th, double ph, double* f,
                       double* ne, double* Th, double* Bmag)
{
    grid_sample(p, r, th, ph, f);
    double rho = f[0], uu = f[1];
    if (!(rho > 0.0)) return 0;
    double gam = p->mp[3];
    double pg = (gam - 1.0) * uu;
    double b2 = f[5] * f[5] + f[6] * f[6] + f[7] * f[7];
    if (b2 / rho > p->mp[4]) return 0;
    double bet = b2 > 0.0 ? pg / (0.5 * b2) : 1e30;
    double bet2 = bet * bet;
    double tratio = (p->mp[1] * bet2 + p->mp[2]) / (1.0 + bet2);
    *Th = (OR_MP / OR_ME) * pg / rho / (1.0 + tratio);
    if (!(*Th > 0.0)) return 0;
    double n_unit = p->mp[0];
    *ne = rho * n_unit;
    *Bmag = sqrt(b2) * OR_C * sqrt(4.0 * OR_PI * n_unit * OR_MP);
    if (!(*Bmag > 0.0)) return 0;
    return 1;
}

int or_grid_plasma(const or_params* p, double r, double th, double ph, double* out3)
{
    double f[8];
    int ok = grid_plasma(p, r, th, ph, f, &out3[0], &out3[1], &out3[2]);
    return ok;
}

static int plasma_point(const or_params* p, double r, double th, double ph, double kt, double kph,
                        double kr_ks, double kth, const cplx* kap0, double rh,
                        double risco, double Eis, double Lis,
                        double* J, double* aI, double* av, double* rv)
{
    /* returns 1 if emitting (J, K filled; per unit affine length), else 0 */
    double a = p->a;
    J[0] = J[1] = J[2] = J[3] = 0.0; *aI = 0.0;
    av[0] = av[1] = av[2] = 0.0; rv[0] = rv[1] = rv[2] = 0.0;
    if (r <= rh * 1.0001) return 0;
    double Del = r * r - 2.0 * r + a * a;
    double kr_bl = kr_ks + (2.0 * r / Del) * kt + (a / Del) * kph;
    double kcov[4] = { kt, kr_bl, kth, kph };
    bl_cov g; bl_con gi; bl_metric(a, r, th, &g, &gi);
    double kup[4];
    kup[0] = gi.tt * kcov[0] + gi.tp * kcov[3];
    kup[1] = gi.rr * kcov[1];
    kup[2] = gi.hh * kcov[2];
    kup[3] = gi.tp * kcov[0] + gi.pp * kcov[3];
    double u[4], Gam, vr, vp; zamo z;
    if (p->model == OR_MODEL_TOYDISK) {
        double rin = p->mp[0], hr = p->mp[1];
        if (r <= rin) return 0;
        flow_u(a, r, th, risco, Eis, Lis, u, &Gam, &vr, &vp, &z);
        double ku = kcov[0] * u[0] + kcov[1] * u[1] + kcov[2] * u[2] + kcov[3] * u[3];
        double cz = cos(th);
        double j = exp(-cz * cz / (2.0 * hr * hr)) / (r * r);
        J[0] = j / (ku * ku);
        return 1;
    }
    double ne, Th, Bmag;          /* n_e [cm^-3], Theta_e, |B| [G] */
    double v3[3], B3[3];          /* ZAMO-frame velocity and field (r, th, ph) */
    if (p->model == OR_MODEL_THERMAL) {
        if (r >= p->mp[5]) return 0;
        double vr_, vp_;
        flow_v3(a, r, risco, Eis, Lis, &vr_, &vp_);
        double n0 = p->mp[0], Th0 = p->mp[1], beta_ref = p->mp[2], r_ref = p->mp[3];
        double psi = p->mp[4];
        double ine = p->mp[6], ith = p->mp[7], ib = p->mp[8];
        ne = n0 * pow(r, -ine);
        Th = Th0 * pow(r, -ith);
        double ne_ref = n0 * pow(r_ref, -ine), Th_ref = Th0 * pow(r_ref, -ith);
        double Bref = sqrt(8.0 * OR_PI * ne_ref * OR_ME * OR_C * OR_C * Th_ref / beta_ref);
        Bmag = Bref * pow(r / r_ref, -ib);
        /* field |B|(cos psi e_ph + sin psi e_r) in the ZAMO frame */
        v3[0] = vr_; v3[1] = 0.0; v3[2] = vp_;
        B3[0] = sin(psi); B3[1] = 0.0; B3[2] = cos(psi);
    } else if (p->model == OR_MODEL_GRID) {
        if (r >= p->mp[5]) return 0;
        double f[8];
        if (!grid_plasma(p, r, th, ph, f, &ne, &Th, &Bmag)) return 0;
        v3[0] = f[2]; v3[1] = f[3]; v3[2] = f[4];
        B3[0] = f[5]; B3[1] = f[6]; B3[2] = f[7];
    } else {
        return 0;
    }
    /* common tail: fluid 4-velocity and unit comoving field direction from
     * their ZAMO-frame components; polarisation angle; coefficients */
    zamo_frame(a, r, th, &z);
    double vv = v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2];
    Gam = 1.0 / sqrt(1.0 - vv);
    u[0] = Gam / z.al;
    u[1] = Gam * v3[0] * z.er;
    u[2] = Gam * v3[1] * z.eh;
    u[3] = Gam * (z.om / z.al + v3[2] * z.ep);
    double ku = kcov[0] * u[0] + kcov[1] * u[1] + kcov[2] * u[2] + kcov[3] * u[3];
    double Bn = sqrt(B3[0] * B3[0] + B3[1] * B3[1] + B3[2] * B3[2]);
    double Bt[3] = { B3[0] / Bn, B3[1] / Bn, B3[2] / Bn };
    double Bdotu = Gam * (v3[0] * Bt[0] + v3[1] * Bt[1] + v3[2] * Bt[2]);
    double resc = 1.0 / sqrt(1.0 + Bdotu * Bdotu);
    double b[4];
    b[0] = (Bdotu * u[0]) * resc;
    b[1] = (Bt[0] * z.er + Bdotu * u[1]) * resc;
    b[2] = (Bt[1] * z.eh + Bdotu * u[2]) * resc;
    b[3] = (Bt[2] * z.ep + Bdotu * u[3]) * resc;
    double kb = kcov[0] * b[0] + kcov[1] * b[1] + kcov[2] * b[2] + kcov[3] * b[3];
    double nu = p->freq * ku;
    double cth = -kb / ku;
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    coefs c; thermal_coefs(ne, Th, Bmag, nu, cth, &c);
    /* polarisation angle: project b orthogonal to the photon direction */
    double n[4];
    for (int m = 0; m < 4; ++m) n[m] = kup[m] / ku - u[m];
    double bl[4];
    bl[0] = g.tt * b[0] + g.tp * b[3];
    bl[1] = g.rr * b[1];
    bl[2] = g.hh * b[2];
    bl[3] = g.tp * b[0] + g.pp * b[3];
    double bn = bl[0] * n[0] + bl[1] * n[1] + bl[2] * n[2] + bl[3] * n[3];
    double bp[4];
    for (int m = 0; m < 4; ++m) bp[m] = b[m] - bn * n[m];
    cplx kb_ = walker_penrose(a, r, th, kup, bp);
    /* z = kappa0 * conj(kappa_B) */
    double zr = kap0->re * kb_.re + kap0->im * kb_.im;
    double zi = kap0->im * kb_.re - kap0->re * kb_.im;
    double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;
    double zn = zr * zr + zi * zi;
    double c2x = 1.0, s2x = 0.0;
    if (zn > 0.0) { c2x = z2r / zn; s2x = z2i / zn; }
    double L = p->L_cm;
    double fJ = L / (ku * ku), fK = L * ku;
    J[0] = fJ * c.jI;
    J[1] = fJ * c.jQ * c2x;
    J[2] = fJ * c.jQ * s2x;
    J[3] = fJ * c.jV;
    *aI = fK * c.aI;
    av[0] = fK * c.aQ * c2x; av[1] = fK * c.aQ * s2x; av[2] = fK * c.aV;
    rv[0] = fK * c.rQ * c2x; rv[1] = fK * c.rQ * s2x; rv[2] = fK * c.rV;
    return 1;
}

/* Subring decomposition (Sec. 5.1): the emission of a step belongs to
 * subring n = the number of turning points of theta (sign changes of
 * k_theta) the backward ray has passed before the step, i.e. the number of
 * half-orbits between emission and reception; the last plane collects
 * n >= nsub - 1.  S[4 + n] accumulates the step's increment of Stokes I.   */
static void trace_one(const or_params* p, double al, double be, double* S, ray_feat* ft,
                      double* rec, int rec_cap, int* rec_n)
{
    for (int i = 0; i < 4 + OR_MAX_SUB; ++i) S[i] = 0.0;
    ft->rmin = 0.0f; ft->ncross = 0; ft->steps = 0; ft->status = OR_OK;
    if (p->model >= OR_MODEL_SCREEN_RING) {
        screen_fn(p, al, be, S);
        ft->rmin = (float)p->r_cam;
        return;
    }
    double a = p->a;
    double rh = horizon(a), rstop = 1.01 * rh;
    double risco = or_r_isco(a), Eis, Lis;
    circ_EL(a, risco, &Eis, &Lis);
    cam_ray cr; camera_ray(p, al, be, &cr);
    cplx kap0 = walker_penrose(a, cr.y[0], cr.y[1], cr.kup_bl, cr.fup_bl);
    double kt = cr.kt, kph = cr.kph;
    double y[5]; memcpy(y, cr.y, sizeof(y));
    double O[16] = { 1,0,0,0, 0,1,0,0, 0,0,1,0, 0,0,0,1 };
    double T1 = 1.0;   /* scalar transmission for the I-only path */
    double rmin = y[0];
    int ncross = 0, nstep = 0, status = OR_OK, nturn = 0;
    int pol = (p->nstokes == 4);
    for (;;) {
        double k1[5], k2[5], k3[5], k4[5], yt[5], yn[5];
        geo_rhs(a, kt, kph, y, k1);
        if (y[0] > p->r_out && k1[0] > 0.0) { status = OR_ESCAPED; break; }
        if (y[0] < rstop) { status = OR_CAPTURED; break; }
        if (nstep >= p->max_steps) { status = OR_STEPCAP; break; }
        if ((pol ? O[0] : T1) < 1e-12) { status = OR_THICK; break; }
        if (!(y[0] == y[0]) || !(y[3] == y[3])) { status = OR_NAN; break; }
        double rate = fabs(k1[0]) / y[0] + fabs(k1[1]) + fabs(k1[2]);
        /* pole control: within |sin theta| < 0.1 of a pole a ray with k_phi != 0
         * meets the centrifugal barrier; the theta step is limited to a fraction
         * of the distance to the pole so that no stage lands inside the barrier */
        if (kph != 0.0) {
            /* distance to the pole, floored at half the barrier's
             * sin theta ~ |k_phi| / |k_theta| */
            double se = fabs(sin(y[1]));
            double ka = fabs(y[4]);
            if (0.5 * fabs(kph) > se * ka) se = 0.5 * fabs(kph) / ka;
            if (se < 0.1) rate += fabs(k1[1]) * (1.0 / se - 10.0);
        }
        double far = y[0] / 20.0;
        if (far < 1.0) far = 1.0;
        if (far > 4.0) far = 4.0;
        double h = p->eps * far / rate;
        if (k1[0] < 0.0) {
            double hh = 0.5 * (y[0] - rh) / (-k1[0]);
            if (hh < h) h = hh;
        }
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        geo_rhs(a, kt, kph, yt, k2);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        geo_rhs(a, kt, kph, yt, k3);
        for (int i = 0; i < 5; ++i) yt[i] = y[i] + h * k3[i];
        geo_rhs(a, kt, kph, yt, k4);
        for (int i = 0; i < 5; ++i) yn[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        /* transfer over the step at the midpoint */
        double rm = 0.5 * (y[0] + yn[0]), thm = 0.5 * (y[1] + yn[1]), phm = 0.5 * (y[2] + yn[2]);
        double krm = 0.5 * (y[3] + yn[3]), kthm = 0.5 * (y[4] + yn[4]);
        double J[4], aI, av[3], rv[3];
        OR_CAT(1);
        int emits = plasma_point(p, rm, thm, phm, kt, kph, krm, kthm, &kap0, rh, risco, Eis, Lis, J, &aI, av, rv);
        OR_EMIT(emits);
        if (emits) {
            OR_CAT(2);
            double I0 = S[0];
            if (pol) {
                transfer_step4(S, O, aI, av, rv, J, h);
            } else {
                double w = aI * h;
                S[0] += T1 * h * phi1(w) * J[0];
                T1 *= exp(-w);
            }
            if (p->nsub > 0) {
                int nq = p->nsub < OR_MAX_SUB ? p->nsub : OR_MAX_SUB;
                int n = nturn < nq - 1 ? nturn : nq - 1;
                S[4 + n] += S[0] - I0;
            }
        }
        OR_CAT(0);
        if (cos(y[1]) * cos(yn[1]) < 0.0) ncross++;
        if (y[4] * yn[4] < 0.0) nturn++;
        if (rec && nstep < rec_cap) {
            for (int i = 0; i < 5; ++i) rec[nstep * 6 + i] = y[i];
            rec[nstep * 6 + 5] = h;
        }
        memcpy(y, yn, sizeof(y));
        if (y[0] < rmin) rmin = y[0];
        nstep++;
    }
    if (rec && nstep < rec_cap) {
        for (int i = 0; i < 5; ++i) rec[nstep * 6 + i] = y[i];
        rec[nstep * 6 + 5] = 0.0;
    }
    if (rec_n) *rec_n = nstep + 1;
    ft->rmin = (float)rmin;
    ft->ncross = ncross;
    ft->steps = nstep;
    ft->status = status;
    if (!(S[0] == S[0])) ft->status = OR_NAN;
}

/* ------------------------------------------------------- threaded driver */
typedef struct {
    const or_params* p;
    const double* al; const double* be;
    double* S; ray_feat* ft;
    int n, nstokes;
    volatile int* next;
} job_t;

static void* worker(void* arg)
{
    job_t* j = (job_t*)arg;
    for (;;) {
        int i = __atomic_fetch_add(j->next, 16, __ATOMIC_RELAXED);
        if (i >= j->n) break;
        int e = i + 16 < j->n ? i + 16 : j->n;
        for (int k = i; k < e; ++k) {
            double S[4 + OR_MAX_SUB];
            trace_one(j->p, j->al[k], j->be[k], S, &j->ft[k], 0, 0, 0);
            const int ns = j->nstokes, nq = j->p->nsub < OR_MAX_SUB ? j->p->nsub : OR_MAX_SUB;
            for (int s = 0; s < ns; ++s) j->S[(size_t)k * (ns + nq) + s] = S[s];
            for (int q = 0; q < nq; ++q) j->S[(size_t)k * (ns + nq) + ns + q] = S[4 + q];
        }
    }
    return 0;
}

/* Trace n screen points; S is n x (nstokes + nsub) (row-major: Stokes, then
 * the subring planes of I), ft is n features. */
int or_trace(const or_params* p, int n, const double* al, const double* be,
             double* S, void* feat, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    volatile int next = 0;
    job_t j = { p, al, be, S, (ray_feat*)feat, n, p->nstokes, &next };
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], 0, worker, &j);
    worker(&j);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], 0);
    return 0;
}

/* Trace one ray and record (r, th, ph, k_r, k_th, h) at every step start and
 * the final state (h = 0).  Returns the number of records written (<= cap). */
/* Plasma and transfer coefficients per unit affine length at one point of the
 * ray through screen point (al, be) (test and diagnosis helper): out = J[4],
 * alpha_I, alpha_{Q,U,V}, rho_{Q,U,V}.  Returns 1 where the plasma emits.   */
int or_plasma_point(const or_params* p, double al, double be, const double* y, double* out)
{
    double a = p->a, rh = 1.0 + sqrt(1.0 - a * a);
    double risco = or_r_isco(a), Eis, Lis;
    circ_EL(a, risco, &Eis, &Lis);
    cam_ray cr; camera_ray(p, al, be, &cr);
    cplx kap0 = walker_penrose(a, cr.y[0], cr.y[1], cr.kup_bl, cr.fup_bl);
    double J[4], aI, av[3], rv[3];
    int ok = plasma_point(p, y[0], y[1], y[2], cr.kt, cr.kph, y[3], y[4], &kap0, rh, risco, Eis, Lis,
                          J, &aI, av, rv);
    for (int i = 0; i < 4; ++i) out[i] = J[i];
    out[4] = aI;
    for (int i = 0; i < 3; ++i) { out[5 + i] = av[i]; out[8 + i] = rv[i]; }
    return ok;
}

int or_trace_path(const or_params* p, double al, double be, double* S, void* feat,
                  double* rec, int cap, double* kt_kph)
{
    int n = 0;
    trace_one(p, al, be, S, (ray_feat*)feat, rec, cap, &n);
    cam_ray cr; camera_ray(p, al, be, &cr);
    kt_kph[0] = cr.kt; kt_kph[1] = cr.kph;
    return n < cap ? n : cap;
}
