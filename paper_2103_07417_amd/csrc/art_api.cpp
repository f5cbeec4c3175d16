// art_api.cpp -- C ABI of the adaptive ray tracer (see include/art.h).
//
// Host orchestration of one adaptive render (Sec. 3.2): base-grid trace,
// Ibar_int / max reduction, then per level the estimator + compaction kernel
// followed by the persistent tracer.  All counts stay on the device, so the
// level loop needs no host synchronisation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/art.h"
#include "art_internal.hpp"

using namespace art;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ART_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// Library-owned scratch, one per device, grown on demand.
struct Workspace {
    uint32_t* list = nullptr;
    size_t list_cap = 0;
    Counters* ctr = nullptr;
    double* partial = nullptr;     // metrics: 1024 blocks x 4 + 4
    int cus = 0;
    hipEvent_t ev[2 * 34] = {};    // start/stop around each tracing launch
    int nev = 0;                   // launches recorded in the current call
};

// Record an event pair around a tracing launch when timing is requested.
struct TraceTimer {
    Workspace* w;
    hipStream_t s;
    bool on;
    hipError_t begin()
    {
        if (!on || w->nev >= 34) return hipSuccess;
        if (!w->ev[2 * w->nev]) {
            hipError_t e = hipEventCreate(&w->ev[2 * w->nev]);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&w->ev[2 * w->nev + 1]);
            if (e != hipSuccess) return e;
        }
        return hipEventRecord(w->ev[2 * w->nev], s);
    }
    hipError_t end()
    {
        if (!on || w->nev >= 34) return hipSuccess;
        hipError_t e = hipEventRecord(w->ev[2 * w->nev + 1], s);
        w->nev++;
        return e;
    }
};

constexpr int kMaxDev = 64;
Workspace g_ws[kMaxDev];
std::mutex g_mu;

int get_ws(Workspace** out, size_t list_need)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(ART_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace& w = g_ws[dev];
    if (!w.ctr) {
        if (hipMalloc(&w.ctr, sizeof(Counters)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(counters) failed");
        if (hipMalloc(&w.partial, sizeof(double) * (1024 * 4 + 4)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(partials) failed");
        HIP_TRY(hipDeviceGetAttribute(&w.cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    if (list_need > w.list_cap) {
        if (w.list) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(w.list));
            w.list = nullptr;
            w.list_cap = 0;
        }
        if (hipMalloc(&w.list, list_need * sizeof(uint32_t)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(trace list, %zu entries) failed", list_need);
        w.list_cap = list_need;
    }
    *out = &w;
    return ART_OK;
}

long long grid_n(int n0, int levels) { return (1LL << levels) * (long long)(n0 - 1) + 1; }

int env_int(const char* name, int dflt)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

LaunchCfg launch_cfg(const Workspace& w, int precision, int model, int nstokes)
{
    LaunchCfg L;
    L.trace_threads = 256;
    const int occ = trace_occupancy_blocks(precision, model, nstokes, L.trace_threads);
    L.trace_blocks = env_int("ART_TRACE_BLOCKS", w.cus * occ);
    if (L.trace_blocks < 1) L.trace_blocks = 1;
    L.refill = env_int("ART_REFILL", 1);
    if (L.refill < 1) L.refill = 1;
    if (L.refill > 64) L.refill = 64;
    return L;
}

int validate(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
             const art_transfer* tr)
{
    if (!sp || !cam || !em || !tr) return fail(ART_EINVAL, "null parameter block");
    const double a = sp->a_spin;
    if (!(std::fabs(a) < 1.0)) return fail(ART_EINVAL, "spin |a| must be < 1 (got %g)", a);
    const double rh = 1.0 + std::sqrt(1.0 - a * a);
    if (!(cam->r_cam > 1.01 * rh)) return fail(ART_EINVAL, "camera radius %g inside the horizon", cam->r_cam);
    if (!(cam->inc_deg > 0.0 && cam->inc_deg < 180.0))
        return fail(ART_EINVAL, "inclination must be in (0, 180) deg");
    if (!(cam->fov_M > 0.0)) return fail(ART_EINVAL, "field of view must be > 0");
    if (tr->nstokes != 1 && tr->nstokes != 4) return fail(ART_EINVAL, "nstokes must be 1 or 4");
    if (tr->precision != ART_PREC_FP64 && tr->precision != ART_PREC_MIXED)
        return fail(ART_EINVAL, "unknown precision %d", tr->precision);
    if (!(tr->eps > 0.0 && tr->eps <= 0.5)) return fail(ART_EINVAL, "eps must be in (0, 0.5]");
    if (tr->max_steps <= 0) return fail(ART_EINVAL, "max_steps must be > 0");
    const int k = em->kind;
    if (k != ART_EMIS_TOY_DISK && k != ART_EMIS_THERMAL && k != ART_EMIS_SCREEN_RING &&
        k != ART_EMIS_SCREEN_POLY)
        return fail(ART_EINVAL, "unknown emission kind %d", k);
    if (k == ART_EMIS_THERMAL && !(em->freq_hz > 0.0 && em->mass_msun > 0.0))
        return fail(ART_EINVAL, "thermal model needs freq_hz > 0 and mass_msun > 0");
    if (k == ART_EMIS_THERMAL && !(em->params[1] > 0.0 && em->params[2] > 0.0 && em->params[3] > 0.0))
        return fail(ART_EINVAL, "thermal model needs Theta0, beta_ref, r_ref > 0");
    if (k == ART_EMIS_TOY_DISK && !(em->params[1] > 0.0))
        return fail(ART_EINVAL, "toy disk needs h/r > 0");
    if (k == ART_EMIS_SCREEN_RING && !(em->params[1] > 0.0 && em->params[3] > 0.0))
        return fail(ART_EINVAL, "screen ring needs width > 0 and diffuse scale > 0");
    return ART_OK;
}

void circ_EL(double a, double r, double* E, double* L)
{
    const double sr = std::sqrt(r), r34 = std::pow(r, 0.75);
    const double den = r34 * std::sqrt(r * sr - 3.0 * sr + 2.0 * a);
    *E = (r * sr - 2.0 * sr + a) / den;
    *L = (r * r - 2.0 * a * sr + a * a) / den;
}

double r_isco(double a)
{
    const double z1 = 1.0 + std::cbrt(1.0 - a * a) * (std::cbrt(1.0 + a) + std::cbrt(1.0 - a));
    const double z2 = std::sqrt(3.0 * a * a + z1 * z1);
    const double sg = a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0);
    return 3.0 + z2 - sg * std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

// Fill the kernel parameter block (nx, ny = final grid; 0 for point tracing).
void make_params(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                 const art_transfer* tr, int nx, int ny, Params& P)
{
    std::memset(&P, 0, sizeof(P));
    const double a = sp->a_spin;
    P.a = a;
    P.rh = 1.0 + std::sqrt(1.0 - a * a);
    P.rstop = 1.01 * P.rh;
    P.r_cam = cam->r_cam;
    P.th_cam = cam->inc_deg * (M_PI / 180.0);
    P.r_out = cam->r_out > 0.0 ? cam->r_out : cam->r_cam;
    P.eps = tr->eps;
    P.nx = nx;
    P.ny = ny;
    if (nx > 1) {
        P.dx = cam->fov_M / (double)(nx - 1);
        P.x0 = -0.5 * cam->fov_M;
        P.y0 = -0.5 * P.dx * (double)(ny - 1);
    }
    // ZAMO frame and BL metric at the camera
    const double r = P.r_cam, th = P.th_cam;
    const double s = std::sin(th), c = std::cos(th);
    const double Sig = r * r + a * a * c * c, Del = r * r - 2.0 * r + a * a;
    const double A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s * s;
    P.c_al = std::sqrt(Sig * Del / A);
    P.c_om = 2.0 * a * r / A;
    P.c_er = std::sqrt(Del / Sig);
    P.c_eh = 1.0 / std::sqrt(Sig);
    P.c_ep = 1.0 / (std::sqrt(A / Sig) * s);
    P.c_gtt = -(1.0 - 2.0 * r / Sig);
    P.c_gtp = -2.0 * a * r * s * s / Sig;
    P.c_grr = Sig / Del;
    P.c_ghh = Sig;
    P.c_gpp = (r * r + a * a + 2.0 * a * a * r * s * s / Sig) * s * s;
    P.c_del = Del;
    P.risco = r_isco(a);
    circ_EL(a, P.risco, &P.Eis, &P.Lis);
    P.model = em->kind;
    P.nstokes = tr->nstokes;
    P.max_steps = tr->max_steps;
    P.freq = em->freq_hz;
    const double G = 6.67430e-8, C = 2.99792458e10, MSUN = 1.98847e33;
    P.L_cm = G * em->mass_msun * MSUN / (C * C);
    for (int i = 0; i < 16; ++i) P.mp[i] = em->params[i];
    if (em->kind == ART_EMIS_THERMAL) {
        const double n0 = em->params[0], Th0 = em->params[1], beta = em->params[2];
        const double rref = em->params[3];
        const double ne_ref = n0 * std::pow(rref, -em->params[6]);
        const double th_ref = Th0 * std::pow(rref, -em->params[7]);
        const double me = 9.1093837015e-28;
        P.Bref = std::sqrt(8.0 * M_PI * ne_ref * me * C * C * th_ref / beta);
        P.r_ref = rref;
        P.psi_c = std::cos(em->params[4]);
        P.psi_s = std::sin(em->params[4]);
    }
}

int check_image(const art_image* out, long long nx, long long ny, bool need_level)
{
    if (!out || !out->image_dev) return fail(ART_EINVAL, "output image is NULL");
    if (need_level && !out->level_dev) return fail(ART_EINVAL, "level map is NULL");
    if (out->nx != nx || out->ny != ny)
        return fail(ART_EINVAL, "image is %dx%d, camera grid is %lldx%lld", out->nx, out->ny, nx, ny);
    return ART_OK;
}

int finish_stats(Workspace* w, hipStream_t s, int levels, long long npix, bool adaptive, art_stats* st,
                 int nx0 = 0, int ny0 = 0)
{
    Counters h;
    HIP_TRY(hipMemcpyAsync(&h, w->ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memset(st, 0, sizeof(*st));
    st->levels = levels;
    long long traced = 0;
    for (int l = 0; l <= levels && l < 32; ++l) {
        st->traced[l] = h.count[l];
        traced += h.count[l];
    }
    st->rays_traced = traced;
    if (adaptive) {
        st->candidates[0] = (int64_t)nx0 * ny0;
        for (int l = 0; l < levels && l < 31; ++l)
            st->candidates[l + 1] = grid_n(nx0, l + 1) * grid_n(ny0, l + 1) - grid_n(nx0, l) * grid_n(ny0, l);
    } else {
        st->candidates[0] = npix;
    }
    st->steps_total = (int64_t)h.steps;
    for (int k = 0; k < 8; ++k) st->status_hist[k] = (int64_t)h.status[k];
    st->interp_frac = adaptive ? (double)(npix - traced) / (double)npix : 0.0;
    st->steps_emit = (int64_t)h.steps_emit;
    double tms = 0.0;
    for (int k = 0; k < w->nev; ++k) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, w->ev[2 * k], w->ev[2 * k + 1]));
        tms += ms;
    }
    st->t_trace_ms = tms;
    st->trace_launches = w->nev;
    st->ibar_int = h.scal[0];
    st->imax0 = h.scal[1];
    st->n_abs = h.scal[2];
    if (h.status[RAY_NAN] > 0)
        return fail(ART_ENUMERIC, "%llu rays produced NaN", (unsigned long long)h.status[RAY_NAN]);
    return ART_OK;
}

}  // namespace

extern "C" {

const char* art_last_error(void) { return g_err.c_str(); }

int art_image_size(const art_camera* cam, int32_t nstokes, int32_t* nx, int32_t* ny,
                   size_t* image_bytes)
{
    if (!cam) return fail(ART_EINVAL, "camera is NULL");
    if (cam->nx0 < 2 || cam->ny0 < 2) return fail(ART_EINVAL, "base grid must be at least 2x2");
    if (cam->levels < 0 || cam->levels > 20) return fail(ART_EINVAL, "levels must be in 0..20");
    if (nstokes != 1 && nstokes != 4) return fail(ART_EINVAL, "nstokes must be 1 or 4");
    const long long X = grid_n(cam->nx0, cam->levels), Y = grid_n(cam->ny0, cam->levels);
    if (X * Y >= (1LL << 32) || X > (1LL << 30) || Y > (1LL << 30))
        return fail(ART_EINVAL, "final grid %lldx%lld exceeds 2^32 pixels", X, Y);
    if (nx) *nx = (int32_t)X;
    if (ny) *ny = (int32_t)Y;
    if (image_bytes) *image_bytes = (size_t)(X * Y) * (size_t)nstokes * sizeof(double);
    return ART_OK;
}

int art_render(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
               const art_refine* rf, const art_transfer* tr, art_image* out, art_stats* st,
               void* stream)
{
    int rc = validate(sp, cam, em, tr);
    if (rc) return rc;
    if (!rf) return fail(ART_EINVAL, "refinement block is NULL");
    if (rf->abs_norm != ART_NORM_MEAN && rf->abs_norm != ART_NORM_MAX)
        return fail(ART_EINVAL, "unknown abs_norm %d", rf->abs_norm);
    if (std::isnan(rf->r_rel) || std::isnan(rf->r_abs)) return fail(ART_EINVAL, "NaN tolerance");
    int32_t nx, ny;
    rc = art_image_size(cam, tr->nstokes, &nx, &ny, nullptr);
    if (rc) return rc;
    rc = check_image(out, nx, ny, true);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long npix = (long long)nx * ny;
    Workspace* w = nullptr;
    rc = get_ws(&w, (size_t)npix);
    if (rc) return rc;
    Params P;
    make_params(sp, cam, em, tr, nx, ny, P);
    const LaunchCfg L = launch_cfg(*w, tr->precision, em->kind, tr->nstokes);
    const int levels = cam->levels;
    const int st0 = 1 << levels;

    HIP_TRY(launch_fill_u32((uint32_t*)w->ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_base_list(w->list, &w->ctr->count[0], cam->nx0, cam->ny0, st0, nx,
                             out->level_dev, s));
    TraceJob J;
    std::memset(&J, 0, sizeof(J));
    J.src = SRC_LIST;
    J.list = w->list;
    J.out = out->image_dev;
    J.plane = npix;
    J.feat = (RayFeat*)out->feat_dev;
    J.ctr = w->ctr;
    J.refill = L.refill;
    J.count = &w->ctr->count[0];
    J.cursor = &w->ctr->cursor[0];
    TraceTimer tt{w, s, st != nullptr};
    w->nev = 0;
    HIP_TRY(tt.begin());
    HIP_TRY(launch_trace(P, tr->precision, J, L, s));
    HIP_TRY(tt.end());
    HIP_TRY(launch_reduce_base(out->image_dev, nx, cam->nx0, cam->ny0, st0, rf->abs_norm, w->ctr, s));
    for (int l = 0; l < levels; ++l) {
        HIP_TRY(launch_estimate(out->image_dev, tr->nstokes, npix, nx, cam->nx0, cam->ny0, levels, l,
                                rf->r_rel, rf->r_abs, w->ctr, w->list, out->level_dev, s));
        J.count = &w->ctr->count[l + 1];
        J.cursor = &w->ctr->cursor[l + 1];
        HIP_TRY(tt.begin());
        HIP_TRY(launch_trace(P, tr->precision, J, L, s));
        HIP_TRY(tt.end());
    }
    if (st) return finish_stats(w, s, levels, npix, true, st, cam->nx0, cam->ny0);
    return ART_OK;
}

int art_render_uniform(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_transfer* tr, art_image* out, art_stats* st, void* stream)
{
    int rc = validate(sp, cam, em, tr);
    if (rc) return rc;
    int32_t nx, ny;
    rc = art_image_size(cam, tr->nstokes, &nx, &ny, nullptr);
    if (rc) return rc;
    rc = check_image(out, nx, ny, false);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long long npix = (long long)nx * ny;
    Workspace* w = nullptr;
    rc = get_ws(&w, 0);
    if (rc) return rc;
    Params P;
    make_params(sp, cam, em, tr, nx, ny, P);
    const LaunchCfg L = launch_cfg(*w, tr->precision, em->kind, tr->nstokes);
    HIP_TRY(launch_fill_u32((uint32_t*)w->ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_fill_u32(&w->ctr->count[0], 1, (uint32_t)npix, s));
    if (out->level_dev) HIP_TRY(launch_fill_i8(out->level_dev, npix, 0, s));
    TraceJob J;
    std::memset(&J, 0, sizeof(J));
    J.src = SRC_IDENTITY;
    J.out = out->image_dev;
    J.plane = npix;
    J.feat = (RayFeat*)out->feat_dev;
    J.ctr = w->ctr;
    J.refill = L.refill;
    J.count = &w->ctr->count[0];
    J.cursor = &w->ctr->cursor[0];
    TraceTimer tt{w, s, st != nullptr};
    w->nev = 0;
    HIP_TRY(tt.begin());
    HIP_TRY(launch_trace(P, tr->precision, J, L, s));
    HIP_TRY(tt.end());
    if (st) return finish_stats(w, s, 0, npix, false, st);
    return ART_OK;
}

int art_trace_points(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                     const art_transfer* tr, int64_t n, const double* alpha_dev,
                     const double* beta_dev, double* stokes_dev, void* feat_dev, void* stream)
{
    int rc = validate(sp, cam, em, tr);
    if (rc) return rc;
    if (n < 0 || n >= (1LL << 32)) return fail(ART_EINVAL, "point count %lld out of range", (long long)n);
    if (n == 0) return ART_OK;
    if (!alpha_dev || !beta_dev || !stokes_dev) return fail(ART_EINVAL, "NULL point buffer");
    hipStream_t s = (hipStream_t)stream;
    Workspace* w = nullptr;
    rc = get_ws(&w, 0);
    if (rc) return rc;
    Params P;
    make_params(sp, cam, em, tr, 0, 0, P);
    const LaunchCfg L = launch_cfg(*w, tr->precision, em->kind, tr->nstokes);
    HIP_TRY(launch_fill_u32((uint32_t*)w->ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_fill_u32(&w->ctr->count[0], 1, (uint32_t)n, s));
    TraceJob J;
    std::memset(&J, 0, sizeof(J));
    J.src = SRC_POINTS;
    J.alpha = alpha_dev;
    J.beta = beta_dev;
    J.out = stokes_dev;
    J.feat = (RayFeat*)feat_dev;
    J.ctr = w->ctr;
    J.refill = L.refill;
    J.count = &w->ctr->count[0];
    J.cursor = &w->ctr->cursor[0];
    HIP_TRY(launch_trace(P, tr->precision, J, L, s));
    return ART_OK;
}

int art_metrics(const double* truth_dev, const double* approx_dev, int64_t n, double* flux_error,
                double* mse, void* stream)
{
    if (!truth_dev || !approx_dev) return fail(ART_EINVAL, "NULL image");
    if (n <= 0) return fail(ART_EINVAL, "empty image");
    hipStream_t s = (hipStream_t)stream;
    Workspace* w = nullptr;
    int rc = get_ws(&w, 0);
    if (rc) return rc;
    const int nb = 1024;
    HIP_TRY(launch_metrics(truth_dev, approx_dev, n, w->partial, nb, s));
    double h[4];
    HIP_TRY(hipMemcpyAsync(h, w->partial + nb * 4, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flux_error) *flux_error = std::fabs(h[0] - h[1]) / std::fabs(h[0]);
    if (mse) *mse = h[2] / h[3];
    return ART_OK;
}

int art_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    for (int d = 0; d < kMaxDev; ++d) {
        Workspace& w = g_ws[d];
        if (!w.ctr && !w.list) continue;
        HIP_TRY(hipSetDevice(d));
        HIP_TRY(hipDeviceSynchronize());
        if (w.list) HIP_TRY(hipFree(w.list));
        if (w.ctr) HIP_TRY(hipFree(w.ctr));
        if (w.partial) HIP_TRY(hipFree(w.partial));
        for (int k = 0; k < 2 * 34; ++k)
            if (w.ev[k]) HIP_TRY(hipEventDestroy(w.ev[k]));
        w = Workspace();
    }
    HIP_TRY(hipSetDevice(cur));
    return ART_OK;
}

}  // extern "C"
