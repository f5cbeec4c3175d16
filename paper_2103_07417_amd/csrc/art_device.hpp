// art_device.hpp -- per-ray device physics for the adaptive black-hole ray
// tracer (gfx950).  One lane integrates one ray.
//
// The paper leaves everything per ray to an external GRRT code (Sec. 4.1,
// "Models and Implementation"); only "trace a ray per sampled screen point and
// return I (or I, Q, U, V)" is fixed (Sec. 3 opening paragraph; Sec. 6 last
// paragraph).  The discretisation implemented here is this project's method:
//   * Kerr spacetime (M = 1), spherical Kerr-Schild coordinates, Hamiltonian
//     geodesic with conserved k_t, k_phi; state (r, th, ph, k_r, k_th); RK4;
//     step h = eps clamp(r/20,1,4) / (|dr|/r + |dth| + |dph|), at most half the
//     coordinate distance to the horizon when moving inward.
//   * k = reversed photon momentum with k.u_cam = +1 (backward tracing).
//   * Termination: r < 1.01 r_h, r > r_out outgoing, step cap, or the
//     transmission of I below 1e-12.
//   * Plasma, coefficients and the transfer update once per step at the
//     arithmetic midpoint of the step's end states.
//   * Polarised transfer by one-pass backward accumulation of the observer
//     propagator O (S += O Delta, O <- O exp(-K h)), exp of the Lorentz-algebra
//     part of K in closed form; emission propagated to its optical-depth
//     weighted mean depth.
//   * Polarisation frame from the Walker-Penrose constant of the camera's
//     screen-up vector compared with that of the projected field.
// Geometry runs in FP64; the plasma model, coefficients and transfer run in
// the template type R (double, or float for the mixed-precision policy).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace art {

enum : int { RAY_OK = 0, RAY_CAPTURED = 1, RAY_ESCAPED = 2, RAY_STEPCAP = 3,
             RAY_THICK = 4, RAY_NAN = 5 };
enum : int { MODEL_TOY = 1, MODEL_THERMAL = 2, MODEL_GRID = 3, MODEL_SCREEN_RING = 10, MODEL_SCREEN_POLY = 11 };

// Kernel-side description of one render.  Filled on the host.
struct Params {
    double a, rh, rstop;
    double r_cam, th_cam, r_out, eps;
    double x0, y0, dx;             // screen coordinates of the final grid
    int32_t nx, ny;
    // ZAMO frame and BL metric at the camera
    double c_al, c_om, c_er, c_eh, c_ep;
    double c_gtt, c_gtp, c_grr, c_ghh, c_gpp, c_del;
    // per-image constants of the ray start: sin, cos of th_cam, 1/c_al,
    // 1/c_del, 1/c_ep (computed on the host once, not per ray)
    double s_cam, c_cam, ic_al, ic_del, ic_ep;
    // equatorial flow: ISCO radius, energy, angular momentum
    double risco, Eis, Lis;
    int32_t model, nstokes, max_steps, nsub;   // nsub: subring planes of I (0..8)
    double freq, L_cm;
    double mp[16];
    double Bref, lnr_ref, psi_c, psi_s;   // thermal: |B| at r_ref, ln r_ref, field phase
    const float* grid;             // gridded model: [n3][n2][n1][8] cell-centre fields
    const double* theta_tab;       // gridded model: theta of the n2 cell centres
    double B_unit;                 // gridded model: Gauss per code field unit
    int32_t g_n1, g_n2, g_n3, pad2;
    // precision policy: geodesic right-hand sides stay FP64 where r < r64
    // (photon shell, horizon) or |k_theta| < kth64 (theta turning points)
    double r64, kth64;
    double phi_cam;                // camera azimuth [rad]
};

constexpr int kMaxThetaCells = 256;

struct RayFeat { float rmin; int32_t ncross; int32_t steps; int32_t status; };

// --------------------------------------------------------------- constants
constexpr double kE  = 4.80320471e-10;     // electron charge [esu]
constexpr double kMe = 9.1093837015e-28;   // electron mass [g]
constexpr double kC  = 2.99792458e10;      // speed of light [cm/s]
constexpr double kH  = 6.62607015e-27;     // Planck constant [erg s]
constexpr double kPi = 3.14159265358979323846;
constexpr double kMp = 1.67262192369e-24;   // proton mass [g]

// math wrappers resolving to the precision of R.  FP64: the library
// functions.  FP32 (the transfer precision): the hardware units directly
// (v_exp_f32 = 2^x, v_log_f32 = log2 x, v_sqrt_f32, v_rsq_f32, each about one
// ulp) with the base change as one multiply, instead of the correctly rounded
// library sequences (four to fifteen times the instructions); the relative
// error of e^x is then about |x| 2^-24, far inside what FP32 transfer carries.
// log1p and expm1 compensate the rounding of u = 1 + x and u = e^x
// (Goldberg, "What every computer scientist should know about floating-point
// arithmetic", 1991, Theorem 4; Kahan's expm1 analogue), which keeps their
// relative accuracy for small |x| without a series.  fcbrt(float) takes
// x > 0 only.
__device__ __forceinline__ double fexp(double x) { return ::exp(x); }
__device__ __forceinline__ float  fexp(float x)  { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ double fsqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ float  fsqrt(float x)  { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double flog(double x) { return ::log(x); }
__device__ __forceinline__ float  flog(float x)  { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double fcbrt(double x) { return ::cbrt(x); }
__device__ __forceinline__ float  fcbrt(float x)  { return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f)); }
__device__ __forceinline__ double flog1p(double x) { return ::log1p(x); }
__device__ __forceinline__ double fexpm1(double x) { return ::expm1(x); }
__device__ __forceinline__ double fsin(double x) { return ::sin(x); }
__device__ __forceinline__ float  fsin(float x)  { return ::sinf(x); }
__device__ __forceinline__ double fabs_(double x) { return ::fabs(x); }
__device__ __forceinline__ float  fabs_(float x)  { return ::fabsf(x); }

// Reciprocals: hardware estimate refined by Newton steps (two in FP64, one in
// FP32) -- within an ulp or two of the correctly rounded quotient, at a third
// of the cost of an IEEE division sequence.
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = ::fma(::fma(-x, r, 1.0), r, r);
    r = ::fma(::fma(-x, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ float frcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return ::fmaf(::fmaf(-x, r, 1.0f), r, r);
}
// 1/sqrt(x): FP64 as the reciprocal of the square root, FP32 on v_rsq_f32.
__device__ __forceinline__ double frsq(double x) { return frcp(::sqrt(x)); }
__device__ __forceinline__ float  frsq(float x)  { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float flog1p(float x)
{
    const float u = 1.0f + x;
    return u == 1.0f ? x : flog(u) * (x * frcp(u - 1.0f));
}
// e^x - 1 given u = fexp(x) (the compensation above; FP64: the library).
__device__ __forceinline__ float fexpm1_u(float x, float u)
{
    if (u == 1.0f) return x;
    const float um = u - 1.0f;
    if (um == -1.0f || __builtin_isinf(u)) return um;
    return um * (x * frcp(flog(u)));
}
__device__ __forceinline__ double fexpm1_u(double x, double) { return ::expm1(x); }
__device__ __forceinline__ float fexpm1(float x) { return fexpm1_u(x, fexp(x)); }

// sin and cos of theta + d from sin, cos of theta for a small increment d
// (|d| <= 1/8: Taylor series of sin d to d^9 and of 1 - cos d to d^10, whose
// first omitted terms are below 2.5e-17 relative; then the angle-addition
// formulas).  The step rule keeps |h dtheta/dlambda| <= eps * 4, so the
// library branch is the exception.
__device__ __forceinline__ void rotate_sc(double s0, double c0, double d, double& s, double& c)
{
    if (::fabs(d) > 0.125) {
        double sd, cd;
        ::sincos(d, &sd, &cd);
        s = s0 * cd + c0 * sd;
        c = c0 * cd - s0 * sd;
        return;
    }
    const double d2 = d * d;
    const double sd = d * (1.0 - d2 * (1.0 / 6.0) * (1.0 - d2 * (1.0 / 20.0) * (1.0 - d2 * (1.0 / 42.0) * (1.0 - d2 * (1.0 / 72.0)))));
    const double cm = d2 * (1.0 / 2.0) * (1.0 - d2 * (1.0 / 12.0) * (1.0 - d2 * (1.0 / 30.0) * (1.0 - d2 * (1.0 / 56.0) * (1.0 - d2 * (1.0 / 90.0)))));
    // cos d = 1 - cm; keep the small correction separate for accuracy
    s = s0 + (c0 * sd - s0 * cm);
    c = c0 - (s0 * sd + c0 * cm);
}

// ------------------------------------------------------ geodesic right-hand side
// Inverse Kerr-Schild metric: g^tt = -(1+2r/S), g^tr = 2r/S, g^rr = D/S,
// g^rph = a/S, g^thth = 1/S, g^phph = 1/(S sin^2).  2H = -kt^2 + Qf/S with
// Qf = -2r kt^2 + 4r kt kr + D kr^2 + 2a kr kph + kth^2 + kph^2/sin^2.
// (s, c) = (sin, cos) of the evaluation point's theta, supplied by the caller.
template <typename T>
__device__ __forceinline__ void geo_rhs(T a, T kt, T kph, const T y[5], T s, T c, T dy[5])
{
    const T r = y[0], kr = y[3], kth = y[4];
    const T s2 = s * s;
    const T Sig = r * r + a * a * c * c;
    const T Del = r * r - T(2.0) * r + a * a;
    const T iS = frcp(Sig);
    T Lph = T(0.0), Lpo = T(0.0), dQth = T(0.0);
    if (kph != T(0.0)) {
        const T is2 = frcp(s2);
        Lpo = kph * is2;
        Lph = kph * Lpo;
        dQth = T(-2.0) * Lph * c * (s * is2);
    }
    const T kt2 = kt * kt;
    const T Qf = T(-2.0) * r * kt2 + T(4.0) * r * kt * kr + Del * kr * kr
                 + T(2.0) * a * kr * kph + kth * kth + Lph;
    const T dQr = T(-2.0) * kt2 + T(4.0) * kt * kr + (T(2.0) * r - T(2.0)) * kr * kr;
    const T dSth = T(-2.0) * a * a * c * s;
    const T QiS2 = Qf * iS * iS;
    dy[0] = (T(2.0) * r * kt + Del * kr + a * kph) * iS;
    dy[1] = kth * iS;
    dy[2] = (a * kr + Lpo) * iS;
    dy[3] = T(-0.5) * (dQr * iS - T(2.0) * r * QiS2);
    dy[4] = T(-0.5) * (dQth * iS - dSth * QiS2);
}

// Right-hand side in FP32 from an FP64 state (precision policy, outside the
// sensitive zones); the derivative is returned in FP64 for the RK4 sums.
__device__ __forceinline__ void geo_rhs32(double a, double kt, double kph, const double y[5], double s,
                                          double c, double dy[5])
{
    float yf[5], df[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) yf[i] = (float)y[i];
    geo_rhs<float>((float)a, (float)kt, (float)kph, yf, (float)s, (float)c, df);
#pragma unroll
    for (int i = 0; i < 5; ++i) dy[i] = (double)df[i];
}

// ------------------------------------------------------------ Walker-Penrose
// kappa = (A1 - i A2)(r - i a cos th) with (BL contravariant components)
//   A1 = (k^t f^r - k^r f^t) + a sin^2 (k^r f^ph - k^ph f^r)
//   A2 = [(r^2+a^2)(k^ph f^th - k^th f^ph) - a (k^t f^th - k^th f^t)] sin
template <typename T>
__device__ __forceinline__ void walker_penrose(T a, T r, T s, T c, const T k[4], const T f[4], T& re, T& im)
{
    const T A1 = (k[0] * f[1] - k[1] * f[0]) + a * s * s * (k[1] * f[3] - k[3] * f[1]);
    const T A2 = ((r * r + a * a) * (k[3] * f[2] - k[2] * f[3]) - a * (k[0] * f[2] - k[2] * f[0])) * s;
    re = A1 * r - A2 * a * c;
    im = -(A1 * a * c + A2 * r);
}

// --------------------------------------------------------------- ray start
struct RayStart {
    double y[5];
    double kt, kph;
    double k0r, k0i;      // Walker-Penrose constant of the polarisation reference
};

// Pinhole camera: backward direction d = (-r_cam e_r - beta e_th + alpha e_ph)/|.|
// in the ZAMO frame at (r_cam, th_cam, 0); k = d - e_(t); reference = screen up
// (-e_th) projected orthogonal to d.
__device__ __forceinline__ void camera_start(const Params& P, double al, double be, RayStart& R)
{
    const double r = P.r_cam;
    const double inrm = 1.0 / ::sqrt(r * r + al * al + be * be);
    const double dr = -r * inrm, dh = -be * inrm, dp = al * inrm;
    const double iual = P.ic_al;
    const double ku_t = -iual;
    const double ku_r = dr * P.c_er;
    const double ku_h = dh * P.c_eh;
    const double ku_p = dp * P.c_ep - P.c_om * iual;
    const double kt = P.c_gtt * ku_t + P.c_gtp * ku_p;
    const double kr_bl = P.c_grr * ku_r;
    const double kth = P.c_ghh * ku_h;
    // k_phi = sqrt(g_phiphi) (k . e_(phi)) = dp / e_phi: the ZAMO observer has no
    // angular momentum, so alpha = 0 gives k_phi = 0 exactly
    const double kph = dp * P.ic_ep;
    (void)ku_p;
    const double iD = P.ic_del;
    R.y[0] = r;
    R.y[1] = P.th_cam;
    R.y[2] = P.phi_cam;
    R.y[3] = kr_bl - (2.0 * r * iD) * kt - (P.a * iD) * kph;
    R.y[4] = kth;
    R.kt = kt;
    R.kph = kph;
    // polarisation reference: (0,-1,0) - (d.(0,-1,0)) d, normalised
    double fr = dh * dr, fh = -1.0 + dh * dh, fp = dh * dp;
    const double ifn = 1.0 / ::sqrt(fr * fr + fh * fh + fp * fp);
    fr *= ifn; fh *= ifn; fp *= ifn;
    const double kup[4] = { ku_t, ku_r, ku_h, ku_p };
    const double fup[4] = { 0.0, fr * P.c_er, fh * P.c_eh, fp * P.c_ep };
    walker_penrose(P.a, r, P.s_cam, P.c_cam, kup, fup, R.k0r, R.k0i);
}

// ------------------------------------------------------------- fluid model
// ZAMO-frame 3-velocity of the equatorial flow at radius r (Keplerian
// Omega = 1/(r^1.5 + a) outside the ISCO, the plunging geodesic with the ISCO
// energy and angular momentum inside), applied at every theta.
template <typename G>
__device__ __forceinline__ void flow_v3(const Params& P, G r, G dr, G& vr, G& vp)
{
    const G a = G(P.a);
    const G Del = dr * (r - G(2.0 - P.rh));          // (r - r+)(r - r-), dr = r - r+ from FP64
    const G A = (r * r + a * a) * (r * r + a * a) - a * a * Del;
    const G iA = frcp(A);
    const G al = fsqrt(r * r * Del * iA);
    const G ial = frcp(al);
    const G om = G(2) * a * r * iA;
    const G sA = fsqrt(A);
    const G ir = frcp(r);
    const G vpi = sA * ir;
    if (r >= G(P.risco)) {
        const G Om = frcp(r * fsqrt(r) + a);
        vp = vpi * (Om - om) * ial;
        vr = G(0);
    } else {
        const G Gam = (G(P.Eis) - om * G(P.Lis)) * ial;
        vp = (G(P.Lis) * r * frcp(sA)) * frcp(Gam);
        const G iG = frcp(Gam);
        const G q = G(1) - iG * iG - vp * vp;
        vr = -fsqrt(q > G(0) ? q : G(0));
    }
}

// Everything the transfer needs at one point, per unit affine length.
template <typename R>
struct Coef {
    R jI, jQ, jU, jV;     // emission (J)
    R aI, aQ, aU, aV;     // absorption
    R rQ, rU, rV;         // rotation
};

template <typename R>
__device__ __forceinline__ void thermal_coefs(R ne, R Th, R B, R nu, R cth,
                                              R& jI, R& jQ, R& jV, R& aI, R& aQ, R& aV,
                                              R& rQ, R& rV)
{
    const R e2 = R(kE * kE);
    const R sth2 = cth * cth < R(1) ? R(1) - cth * cth : R(0);
    const R sth = fsqrt(sth2);
    const R nuB = R(kE / (2.0 * kPi * kMe * kC)) * B;
    const R iTh = frcp(Th);
    const R inu = frcp(nu);
    const R lg = flog1p(R(2) * Th);
    const R gV = lg * frcp(R(2) * Th * Th + lg);
    const R gQ = frcp(R(1) + R(2) * Th) + R(6) * Th;
    const R imc = R(1.0 / (kMe * kC));
    const R nee = ne * e2;
    rV = R(2) * nee * nuB * cth * imc * (inu * inu) * gV;
    rQ = -nee * nuB * nuB * sth2 * imc * (inu * inu * inu) * gQ;
    jI = jQ = jV = aI = aQ = aV = R(0);
    if (sth < R(1e-10)) return;
    const R x = R(2) * nu * frcp(R(3) * nuB * Th * Th * sth);
    const R x13 = fcbrt(x);
    const R xm13 = frcp(x13), xm23 = xm13 * xm13;
    const R ex = fexp(R(-1.8899) * x13);
    const R II = R(2.5651) * (R(1) + R(1.92) * xm13 + R(0.9977) * xm23) * ex;
    const R IQ = R(2.5651) * (R(1) + R(0.932) * xm13 + R(0.4998) * xm23) * ex;
    const R IV = (R(1.8138) * (xm13 * xm23) + R(3.423) * xm23 + R(0.02955) * frsq(x)
                  + R(2.0377) * xm13) * ex;
    const R pref = nee * nu * (iTh * iTh) * R(1.0 / (2.0 * 1.7320508075688772 * kC));
    R jI_ = pref * II;
    R jQ_ = pref * IQ;
    R jV_ = pref * (R(4) * cth * frcp(R(3) * Th * sth)) * IV;
    const R P = fsqrt(jQ_ * jQ_ + jV_ * jV_);
    if (P > R(0.99) * jI_) {
        const R sc = R(0.99) * jI_ * frcp(P);
        jQ_ *= sc; jV_ *= sc;
    }
    // 1/B_nu = expm1(q) c^2 / (2 h nu^3) with q = h nu / (Theta m c^2), written as
    // (expm1(q)/q) / (2 Theta m nu^2) so that no factor leaves the FP32 range
    // (1/q and 1/(2 Theta m nu^2) from the reciprocals of Theta and nu:
    // nu^-2 >= 1e-26 and 1/m ~ 1e27 for the frequencies of the method)
    const R q = R(kH / (kMe * kC * kC)) * nu * iTh;
    const R phq = q < R(1e-6) ? R(1) + R(0.5) * q : fexpm1(q) * (Th * inu * R(kMe * kC * kC / kH));
    const R iBnu = phq * ((R(0.5 / kMe) * iTh) * (inu * inu));
    jI = jI_; jQ = -jQ_; jV = jV_;
    aI = jI_ * iBnu; aQ = -jQ_ * iBnu; aV = jV_ * iBnu;
}

// Gridded snapshot: trilinear interpolation in (x1 = ln r, theta, phi) between
// cell centres, clamped in x1 and theta, periodic in phi; theta outside
// [0, pi] is reflected with phi + pi.  The cell-centre angles come from the
// LDS table `tht` (bisection).  Fields are FP32 [n3][n2][n1][8].
template <typename R>
__device__ __forceinline__ void grid_sample(const Params& P, const double* tht, double r, double th,
                                            double ph, R f[8])
{
    const int n1 = P.g_n1, n2 = P.g_n2, n3 = P.g_n3;
    double tw = ::fmod(th, 2.0 * kPi);
    if (tw < 0.0) tw += 2.0 * kPi;
    if (tw > kPi) { tw = 2.0 * kPi - tw; ph += kPi; }
    const double pw = ph - 2.0 * kPi * ::floor(ph * (1.0 / (2.0 * kPi)));
    const double f1 = (::log(r) - P.mp[6]) * frcp(P.mp[7]) - 0.5;
    int i1 = (int)::floor(f1);
    double t1 = f1 - (double)i1;
    if (i1 < 0) { i1 = 0; t1 = 0.0; }
    if (i1 > n1 - 2) { i1 = n1 - 2; t1 = 1.0; }
    int j;
    double t2;
    if (tw <= tht[0]) { j = 0; t2 = 0.0; }
    else if (tw >= tht[n2 - 1]) { j = n2 - 2; t2 = 1.0; }
    else {
        int lo = 0, hi = n2 - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tht[mid] <= tw) lo = mid; else hi = mid;
        }
        j = lo;
        t2 = (tw - tht[j]) * frcp(tht[j + 1] - tht[j]);
    }
    const double f3 = pw * (double)n3 * (1.0 / (2.0 * kPi)) - 0.5;
    const double fl3 = ::floor(f3);
    const double t3 = f3 - fl3;
    const int k0 = (((int)fl3 % n3) + n3) % n3, k1 = (k0 + 1) % n3;
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = R(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
        const R w = R((di ? t1 : 1.0 - t1) * (dj ? t2 : 1.0 - t2) * (dk ? t3 : 1.0 - t3));
        const size_t idx = (((size_t)(dk ? k1 : k0) * n2 + (size_t)(j + dj)) * n1 + (size_t)(i1 + di)) * 8;
        const float4 lo = *reinterpret_cast<const float4*>(P.grid + idx);
        const float4 hi = *reinterpret_cast<const float4*>(P.grid + idx + 4);
        f[0] += w * R(lo.x); f[1] += w * R(lo.y); f[2] += w * R(lo.z); f[3] += w * R(lo.w);
        f[4] += w * R(hi.x); f[5] += w * R(hi.y); f[6] += w * R(hi.z); f[7] += w * R(hi.w);
    }
}

// Plasma and coefficients at a midpoint.  Returns false where nothing emits.
// (s, c) = (sin, cos) of th, supplied by the caller.  The emission-point
// geometry (ZAMO frame, fluid 4-velocity, comoving field, photon direction,
// polarisation angle) is evaluated in the transfer precision R; Delta is
// formed as (r - r+)(r - r-) from the FP64 distance to the horizon, so no
// cancellation is left near it.
template <typename R, int MODEL>
__device__ __forceinline__ bool plasma_point(const Params& P, const double* tht, double r_d, double th,
                                             double s_d, double c_d, double ph, double kt_d, double kph_d,
                                             double kr_ks_d, double kth_d, double k0r_d, double k0i_d,
                                             Coef<R>& C)
{
    if (r_d <= P.rh * 1.0001) return false;
    if constexpr (MODEL == MODEL_TOY) {
        if (r_d <= P.mp[0]) return false;
    } else {
        if (r_d >= P.mp[5]) return false;
    }
    using G = R;
    const G a = G(P.a), r = G(r_d), s = G(s_d), c = G(c_d);
    const G kt = G(kt_d), kph = G(kph_d), kth = G(kth_d);
    const G dr = G(r_d - P.rh);
    const G s2 = s * s;
    const G Sig = r * r + a * a * c * c;
    const G Del = dr * (r - G(2.0 - P.rh));
    const G A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s2;
    const G iD = frcp(Del);
    const G iS = frcp(Sig);
    const G iA = frcp(A);
    const G is = frcp(s);
    const G kr_bl = G(kr_ks_d) + (G(2) * r * iD) * kt + (a * iD) * kph;
    // ZAMO frame at (r, th)
    const G izal = frsq(Sig * Del * iA);
    const G zom = G(2) * a * r * iA;
    const G zer = fsqrt(Del * iS);
    const G zeh = fsqrt(iS);
    const G zep = fsqrt(Sig * iA) * is;
    if constexpr (MODEL == MODEL_TOY) {
        G vr, vp;
        flow_v3<G>(P, r, dr, vr, vp);
        const G Gam = frsq(G(1) - vr * vr - vp * vp);
        const G u0 = Gam * izal, u1 = Gam * vr * zer, u3 = Gam * (zom * izal + vp * zep);
        const G ku = kt * u0 + kr_bl * u1 + kph * u3;
        const G hr = G(P.mp[1]);
        const G iku = frcp(ku);
        const G j = fexp(-c * c * frcp(G(2) * hr * hr)) * frcp(r * r);
        C.jI = R(j * iku * iku);
        C.jQ = C.jU = C.jV = R(0);
        C.aI = C.aQ = C.aU = C.aV = R(0);
        C.rQ = C.rU = C.rV = R(0);
        return true;
    } else {
        R ne, Th, Bm;
        G v3[3], B3[3];
        if constexpr (MODEL == MODEL_THERMAL) {
            // power-law plasma: scalars in R
            const R lr = flog(R(r));
            ne = R(P.mp[0]) * fexp(-R(P.mp[6]) * lr);
            Th = R(P.mp[1]) * fexp(-R(P.mp[7]) * lr);
            Bm = R(P.Bref) * fexp(-R(P.mp[8]) * (lr - R(P.lnr_ref)));
            G vr, vp;
            flow_v3<G>(P, r, dr, vr, vp);
            v3[0] = vr; v3[1] = G(0); v3[2] = vp;
            B3[0] = G(P.psi_s); B3[1] = G(0); B3[2] = G(P.psi_c);
        } else {
            R f[8];
            grid_sample<R>(P, tht, r_d, th, ph, f);
            const R rho = f[0];
            if (!(rho > R(0))) return false;
            const R pg = (R(P.mp[3]) - R(1)) * f[1];
            const R b2 = f[5] * f[5] + f[6] * f[6] + f[7] * f[7];
            if (b2 > R(P.mp[4]) * rho) return false;           // sigma cut
            const R bet = b2 > R(0) ? pg * frcp(R(0.5) * b2) : R(1e30);
            const R bet2 = bet * bet;
            const R tratio = (R(P.mp[1]) * bet2 + R(P.mp[2])) * frcp(R(1) + bet2);
            Th = R(kMp / kMe) * pg * frcp(rho) * frcp(R(1) + tratio);
            if (!(Th > R(0))) return false;
            ne = rho * R(P.mp[0]);
            Bm = fsqrt(b2) * R(P.B_unit);
            if (!(Bm > R(0))) return false;
            v3[0] = G(f[2]); v3[1] = G(f[3]); v3[2] = G(f[4]);
            B3[0] = G(f[5]); B3[1] = G(f[6]); B3[2] = G(f[7]);
        }
        // fluid 4-velocity and unit comoving field direction from ZAMO components
        const G vv = v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2];
        const G Gam = frsq(G(1) - vv);
        const G u0 = Gam * izal, u1 = Gam * v3[0] * zer, u2 = Gam * v3[1] * zeh;
        const G u3 = Gam * (zom * izal + v3[2] * zep);
        const G ku = kt * u0 + kr_bl * u1 + kth * u2 + kph * u3;
        const G iBn = frsq(B3[0] * B3[0] + B3[1] * B3[1] + B3[2] * B3[2]);
        const G Bt0 = B3[0] * iBn, Bt1 = B3[1] * iBn, Bt2 = B3[2] * iBn;
        const G Bdu = Gam * (v3[0] * Bt0 + v3[1] * Bt1 + v3[2] * Bt2);
        const G resc = frsq(G(1) + Bdu * Bdu);
        const G b0 = Bdu * u0 * resc;
        const G b1 = (Bt0 * zer + Bdu * u1) * resc;
        const G b2_ = (Bt1 * zeh + Bdu * u2) * resc;
        const G b3 = (Bt2 * zep + Bdu * u3) * resc;
        const G kb = kt * b0 + kr_bl * b1 + kth * b2_ + kph * b3;
        const G iku = frcp(ku);
        G cth = -kb * iku;
        cth = cth > G(1) ? G(1) : (cth < G(-1) ? G(-1) : cth);
        // contravariant k (BL)
        const G iSD = iS * iD;
        const G gitt = -A * iSD, gitp = G(-2) * a * r * iSD;
        const G girr = Del * iS, gihh = iS, gipp = (Del - a * a * s2) * iSD * (is * is);
        const G kup[4] = { gitt * kt + gitp * kph, girr * kr_bl, gihh * kth, gitp * kt + gipp * kph };
        // photon direction n = k/ku - u; b_perp = b - (b.n) n
        const G n0 = kup[0] * iku - u0, n1 = kup[1] * iku - u1, n2 = kup[2] * iku - u2;
        const G n3 = kup[3] * iku - u3;
        const G gtt = -(G(1) - G(2) * r * iS), gtp = G(-2) * a * r * s2 * iS;
        const G grr = Sig * iD, ghh = Sig, gpp = (r * r + a * a + G(2) * a * a * r * s2 * iS) * s2;
        const G bl0 = gtt * b0 + gtp * b3, bl1 = grr * b1, bl2 = ghh * b2_, bl3 = gtp * b0 + gpp * b3;
        const G bn = bl0 * n0 + bl1 * n1 + bl2 * n2 + bl3 * n3;
        const G bp[4] = { b0 - bn * n0, b1 - bn * n1, b2_ - bn * n2, b3 - bn * n3 };
        G kbr, kbi;
        walker_penrose<G>(a, r, s, c, kup, bp, kbr, kbi);
        const G k0r = G(k0r_d), k0i = G(k0i_d);
        const G zr = k0r * kbr + k0i * kbi;
        const G zi = k0i * kbr - k0r * kbi;
        const G zn = zr * zr + zi * zi;
        G c2x = G(1), s2x = G(0);
        if (zn > G(0)) {
            const G izn = frcp(zn);
            c2x = (zr * zr - zi * zi) * izn;
            s2x = G(2) * zr * zi * izn;
        }
        R jI, jQ, jV, aI, aQ, aV, rQ, rV;
        thermal_coefs<R>(ne, Th, Bm, R(P.freq) * R(ku), R(cth), jI, jQ, jV, aI, aQ, aV, rQ, rV);
        const R fJ = R(P.L_cm) * R(iku) * R(iku), fK = R(P.L_cm) * R(ku);
        const R c2 = R(c2x), s2r = R(s2x);
        C.jI = fJ * jI; C.jQ = fJ * jQ * c2; C.jU = fJ * jQ * s2r; C.jV = fJ * jV;
        C.aI = fK * aI; C.aQ = fK * aQ * c2; C.aU = fK * aQ * s2r; C.aV = fK * aV;
        C.rQ = fK * rQ * c2; C.rU = fK * rQ * s2r; C.rV = fK * rV;
        return true;
    }
}

// ---------------------------------------------------------- transfer maths
// Polynomial parts (u, v < 1) of sinh(u)/u, sin(v)/v, (sinh(u)/u - 1)/u^2 and
// (1 - sin(v)/v)/v^2: Taylor series to the 1/15! term in Horner form (one FMA
// per term).
template <typename R>
__device__ __forceinline__ R shc_poly(R u2)
{
    return R(1) + u2 * (R(1.0 / 6.0) + u2 * (R(1.0 / 120.0) + u2 * (R(1.0 / 5040.0) + u2 * (R(1.0 / 362880.0)
           + u2 * (R(1.0 / 39916800.0) + u2 * R(1.0 / 6227020800.0))))));
}
template <typename R>
__device__ __forceinline__ R sinc_poly(R v2)
{
    return R(1) + v2 * (R(-1.0 / 6.0) + v2 * (R(1.0 / 120.0) + v2 * (R(-1.0 / 5040.0) + v2 * (R(1.0 / 362880.0)
           + v2 * (R(-1.0 / 39916800.0) + v2 * R(1.0 / 6227020800.0))))));
}
template <typename R>
__device__ __forceinline__ R g_poly(R u2)
{
    return R(1.0 / 6.0) + u2 * (R(1.0 / 120.0) + u2 * (R(1.0 / 5040.0) + u2 * (R(1.0 / 362880.0)
           + u2 * (R(1.0 / 39916800.0) + u2 * (R(1.0 / 6227020800.0) + u2 * R(1.0 / 1307674368000.0))))));
}
template <typename R>
__device__ __forceinline__ R h_poly(R v2)
{
    return R(1.0 / 6.0) + v2 * (R(-1.0 / 120.0) + v2 * (R(1.0 / 5040.0) + v2 * (R(-1.0 / 362880.0)
           + v2 * (R(1.0 / 39916800.0) + v2 * (R(-1.0 / 6227020800.0) + v2 * R(1.0 / 1307674368000.0))))));
}
__device__ __forceinline__ void fsincos(double x, double* s, double* c) { ::sincos(x, s, c); }
__device__ __forceinline__ void fsincos(float x, float* s, float* c) { ::sincosf(x, s, c); }

// Invariants of A = [[0, a^T], [a, K]] (a = (aQ, aU, aV), K x = x × rho)
// shared by every exponential of one step: |a|^2, |rho|^2, a.rho and the
// eigenvalue parameters (the eigenvalues of A are +-L1, +-i L2 with
// L1^2 - L2^2 = |a|^2 - |rho|^2, L1 L2 = a.rho, D = L1^2 + L2^2).
template <typename R>
struct LorentzInv {
    R a2, r2, ad, D, iD, L1s, L2s, L1, L2;
};
template <typename R>
__device__ __forceinline__ LorentzInv<R> lorentz_inv(const R av[3], const R rv[3])
{
    LorentzInv<R> L;
    L.a2 = av[0] * av[0] + av[1] * av[1] + av[2] * av[2];
    L.r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    L.ad = av[0] * rv[0] + av[1] * rv[1] + av[2] * rv[2];
    const R dl = L.a2 - L.r2;
    L.D = fsqrt(dl * dl + R(4) * L.ad * L.ad);
    L.iD = L.D > R(0) ? frcp(L.D) : R(0);
    L.L1s = R(0.5) * (L.D + dl); L.L1s = L.L1s < R(0) ? R(0) : L.L1s;
    L.L2s = R(0.5) * (L.D - dl); L.L2s = L.L2s < R(0) ? R(0) : L.L2s;
    L.L1 = fsqrt(L.L1s);
    L.L2 = fsqrt(L.L2s);
    return L;
}

// Coefficients c0..c3 with exp(-aI x) exp(-A x) = c0 + c1 A + c2 A^2 + c3 A^3;
// with u = x L1, v = x L2, w = x aI (u <= w for physical coefficients):
//   c2 = x^2/2 (L1^2 e^-w shc(u/2)^2 + L2^2 e^-w sinc(v/2)^2) / D
//   c1 = -x (L2^2 e^-w shc(u) + L1^2 e^-w sinc(v)) / D
//   c3 = -x^3 (L1^2 e^-w g(u) + L2^2 e^-w h(v)) / D,   c0 = e^-w cosh u - L1^2 c2.
// The caller supplies w, ew = e^-w and ew2 = e^-w/2 (1, 1 for an undamped
// exponential, folded at compile time); e^u and square roots give the half
// arguments, sin/cos of v/2 give sin v and the half-argument sinc.
template <typename R>
__device__ __forceinline__ void lorentz_coeffs(const LorentzInv<R>& L, R x, R w, R ew, R ew2,
                                               R& c0, R& c1, R& c2, R& c3)
{
    const R L1s = L.L1s, L2s = L.L2s;
    const R u = x * L.L1, v = x * L.L2;
    // hyperbolic parts, damped by e^-w
    R ch, shc, sh2, gu;
    const R u2 = u * u;
    if (u < R(1)) {
        const R p2 = shc_poly(R(0.25) * u2);   // sinh(u/2)/(u/2)
        ch = ew * (R(1) + R(0.5) * u2 * p2 * p2);   // cosh u = 1 + 2 sinh^2(u/2)
        shc = ew * shc_poly(u2);
        sh2 = ew2 * p2;
        gu = ew * g_poly(u2);
    } else {
        R ep, em;                              // e^(u-w), e^(-u-w)
        if (u < R(60)) {
            const R eu = fexp(u);
            ep = eu * ew;
            em = ew * frcp(eu);
        } else {
            ep = fexp(u - w);
            em = fexp(-u - w);
        }
        ch = R(0.5) * (ep + em);
        const R iu = frcp(u);
        shc = R(0.5) * (ep - em) * iu;
        sh2 = (fsqrt(ep) - fsqrt(em)) * iu;
        gu = (shc - ew) * (iu * iu);
    }
    // trigonometric parts
    R snc, sn2, hv;
    const R v2 = v * v;
    if (v < R(1)) {
        snc = sinc_poly(v2);
        sn2 = sinc_poly(R(0.25) * v2);
        hv = h_poly(v2);
    } else {
        R sh, chh;
        fsincos(R(0.5) * v, &sh, &chh);
        const R iv = frcp(v);
        const R sv = R(2) * sh * chh;
        snc = sv * iv;
        sn2 = R(2) * sh * iv;
        hv = (R(1) - snc) * (iv * iv);
    }
    if (L.D > R(0)) {
        const R iD = L.iD;
        c2 = R(0.5) * x * x * (L1s * sh2 * sh2 + L2s * ew * sn2 * sn2) * iD;
        c1 = -x * (L2s * shc + L1s * ew * snc) * iD;
        c3 = -x * x * x * (L1s * gu + L2s * ew * hv) * iD;
    } else {
        c2 = R(0.5) * x * x * ew;
        c1 = -x * ew;
        c3 = -x * x * x * ew * R(1.0 * (1.0 / 6.0));
    }
    c0 = ch - L1s * c2;
}

// Step functions of the optical depth w = aI h, from ew = e^-w (computed
// once per step): phi1(w) = (1 - e^-w)/w, the weight of the step's emission,
// and the mean depth m(w) = 1/w - 1/(e^w - 1) = 1/w + 1 + 1/(e^-w - 1) at
// which the emission integral's exponential is evaluated (series below the
// cancellation thresholds).
template <typename R>
__device__ __forceinline__ void depth_fns(R w, R ew, R& phi1, R& mdepth)
{
    const R em1 = w < R(1e-4) ? R(0) : fexpm1_u(-w, ew);
    const R iw = w < R(1e-4) ? R(0) : frcp(w);
    phi1 = w < R(1e-4) ? R(1) + w * (R(-1.0 / 2.0) + w * (R(1.0 / 6.0) + w * R(-1.0 / 24.0))) : -em1 * iw;
    if (w < R(0.1)) {
        const R w2 = w * w;
        mdepth = R(0.5) + w * (R(-1.0 / 12.0) + w2 * (R(1.0 / 720.0) + w2 * R(-1.0 / 30240.0)));
    } else {
        mdepth = (iw + R(1)) + frcp(em1);
    }
}
template <typename R>
__device__ __forceinline__ R phi1_(R w, R ew)
{
    if (w < R(1e-4)) return R(1) + w * (R(-1.0 / 2.0) + w * (R(1.0 / 6.0) + w * R(-1.0 / 24.0)));
    return -fexpm1_u(-w, ew) * frcp(w);
}

// y = A x for A = [[0,aQ,aU,aV],[aQ,0,rV,-rU],[aU,-rV,0,rQ],[aV,rU,-rQ,0]]
template <typename R>
__device__ __forceinline__ void applyA(const Coef<R>& K, const R x[4], R y[4])
{
    y[0] = K.aQ * x[1] + K.aU * x[2] + K.aV * x[3];
    y[1] = K.aQ * x[0] + K.rV * x[2] - K.rU * x[3];
    y[2] = K.aU * x[0] - K.rV * x[1] + K.rQ * x[3];
    y[3] = K.aV * x[0] + K.rU * x[1] - K.rQ * x[2];
}
// M = c0 + c1 A + c2 A^2 + c3 A^3 written out from the block structure of A:
// first row and column a = (aQ, aU, aV), lower block K with K x = x × rho
// (rho = (rQ, rU, rV)).  With w = a × rho, sa = |a|^2, sr = |rho|^2 and
// p = a . rho (K a = w, K rho = 0, K^2 = rho rho^T - sr):
//   A^2 = [[sa, -w^T], [w, a a^T + rho rho^T - sr]],
//   A^3 = [[0, u^T], [u, w a^T - a w^T - sr K]],   u = (sa - sr) a + p rho.
// 60-odd operations, then O M in 64 against 208 for three row products per
// row of O.
template <typename R>
__device__ __forceinline__ void lorentz_matrix(const Coef<R>& K, const LorentzInv<R>& L, R c0, R c1, R c2, R c3,
                                               R M[16])
{
    const R a[3] = { K.aQ, K.aU, K.aV };
    const R q[3] = { K.rQ, K.rU, K.rV };
    const R w[3] = { a[1] * q[2] - a[2] * q[1], a[2] * q[0] - a[0] * q[2], a[0] * q[1] - a[1] * q[0] };
    const R sa = L.a2, sr = L.r2, p = L.ad;
    const R e = c1 + c3 * (sa - sr), f = c3 * p;      // c1 a + c3 u = e a + f rho
    M[0] = c0 + c2 * sa;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const R uj = e * a[j] + f * q[j];
        M[1 + j] = uj - c2 * w[j];
        M[4 * (1 + j)] = uj + c2 * w[j];
        M[5 * (1 + j)] = c0 + c2 * (a[j] * a[j] + q[j] * q[j] - sr);
    }
    // off-diagonal pairs (i, j), i < j: M_ij = sym + anti, M_ji = sym - anti with
    // sym = c2 (a_i a_j + rho_i rho_j), anti = (c1 - c3 sr) K_ij + c3 (w_i a_j - a_i w_j);
    // K_QU = rV, K_QV = -rU, K_UV = rQ
    const R g = c1 - c3 * sr;
    const int pi[3] = { 0, 0, 1 }, pj[3] = { 1, 2, 2 };
    const R kij[3] = { q[2], -q[1], q[0] };
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int i = pi[t], j = pj[t];
        const R sym = c2 * (a[i] * a[j] + q[i] * q[j]);
        const R anti = g * kij[t] + c3 * (w[i] * a[j] - a[i] * w[j]);
        M[4 * (1 + i) + 1 + j] = sym + anti;
        M[4 * (1 + j) + 1 + i] = sym - anti;
    }
}

// One constant-coefficient polarised step of affine length h:
//   S += O * h phi1(aI h) exp(-A sbar) J,   O <- O exp(-aI h) exp(-A h),
// sbar = h m(aI h); both exponentials share the invariants of A and e^-aI h.
template <typename R, typename RS>
__device__ __forceinline__ void transfer_step4(RS S[4], R O[16], const Coef<R>& K, R h)
{
    const R av[3] = { K.aQ, K.aU, K.aV };
    const R rv[3] = { K.rQ, K.rU, K.rV };
    const LorentzInv<R> L = lorentz_inv<R>(av, rv);
    const R w = K.aI * h;
    const R ew = fexp(-w);
    R ph1, md;
    depth_fns<R>(w, ew, ph1, md);
    const R sbar = h * md;
    R g0, g1, g2, g3;
    lorentz_coeffs<R>(L, sbar, R(0), R(1), R(1), g0, g1, g2, g3);
    const R J[4] = { K.jI, K.jQ, K.jU, K.jV };
    R AJ[4], A2J[4], A3J[4];
    applyA(K, J, AJ);
    applyA(K, AJ, A2J);
    applyA(K, A2J, A3J);
    const R sc = h * ph1;
    R d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = sc * (g0 * J[i] + g1 * AJ[i] + g2 * A2J[i] + g3 * A3J[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        S[i] += RS(O[i * 4 + 0] * d[0] + O[i * 4 + 1] * d[1] + O[i * 4 + 2] * d[2] + O[i * 4 + 3] * d[3]);
    R c0, c1, c2, c3;
    lorentz_coeffs<R>(L, h, w, ew, fsqrt(ew), c0, c1, c2, c3);
    R M[16];
    lorentz_matrix<R>(K, L, c0, c1, c2, c3, M);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const R x[4] = { O[i * 4 + 0], O[i * 4 + 1], O[i * 4 + 2], O[i * 4 + 3] };
#pragma unroll
        for (int j = 0; j < 4; ++j) O[i * 4 + j] = x[0] * M[j] + x[1] * M[4 + j] + x[2] * M[8 + j] + x[3] * M[12 + j];
    }
}

// Closed-form screen intensities (refinement tests without ray tracing).
__device__ __forceinline__ void screen_fn(const Params& P, double al, double be, double S[4])
{
    double I;
    if (P.model == MODEL_SCREEN_RING) {
        const double rho = ::sqrt(al * al + be * be);
        const double d = (rho - P.mp[0]) / P.mp[1];
        I = ::exp(-0.5 * d * d) * (1.0 + 0.5 * al / (rho + 1.0))
            + P.mp[2] * ::exp(-rho * rho / (2.0 * P.mp[3] * P.mp[3]));
    } else {
        I = P.mp[0] + P.mp[1] * al + P.mp[2] * be + P.mp[3] * al * al + P.mp[4] * al * be
            + P.mp[5] * be * be;
    }
    S[0] = I;
    S[1] = 0.5 * I * ::cos(0.3 * al);
    S[2] = 0.5 * I * ::sin(0.3 * be);
    S[3] = 0.1 * I;
}

}  // namespace art
