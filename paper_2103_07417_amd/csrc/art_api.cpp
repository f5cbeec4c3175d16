// art_api.cpp -- C ABI of the adaptive ray tracer (see include/art.h).
//
// Host orchestration of adaptive renders (Sec. 3.2).  A render is a batch of
// 1..64 images: base-grid lists for every image, one persistent tracing
// launch for all base rays, the per-image Ibar_int / max reduction, then per
// level one estimator + compaction launch over all images followed by one
// tracing launch over every image's new rays.  All counts stay on the device,
// so the level loop needs no host synchronisation and can be captured once in
// a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/art.h"
#include "art_cnn.hpp"
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

}  // namespace

namespace art {
int api_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace art

namespace {

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ART_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

long long grid_n(int n0, int levels) { return (1LL << levels) * (long long)(n0 - 1) + 1; }

int env_int(const char* name, int dflt)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

art_launch g_launch = { 0, 0, 0, 0, 0, 0 };   // user override (0 = default)
size_t g_list_limit = 0;                // bytes a trace list + cost map may take (0: no limit)
std::mutex g_mu;

constexpr int kMaxEv = 64;   // timed tracing launches per group and render

}  // namespace

// A batch: device descriptors, trace list, counters, timing events, graph.
// Its images are split into groups of consecutive images; every group runs
// its own level loop (own counters, trace-list slice and stream), so the
// long-ray tail of one group's pass overlaps the other groups' work.  Group 0
// runs on the caller's stream; the others fork from it and join back.
constexpr int kMaxGroups = 8;

struct BatchGroup {
    int i0 = 0, n = 0;             // images [i0, i0 + n)
    int lmax = 0, max_base = 0;    // deepest level, largest base grid of the group
    int nx0m = 0, ny0m = 0;        // largest base grid sizes (estimator launch shape)
    size_t list_off = 0;           // the group's slice of the trace list
    size_t list_len = 0;
    hipEvent_t ev[2 * kMaxEv] = {};
    int nev = 0;                   // timed tracing launches of the last eager render
    CnnWork ws;                    // network workspace (learned renders)
    // learned renders: the group-local images the network runs on at level l
    // are imap[imap_off[l] .. imap_off[l] + nnet[l]) (device)
    int* imap = nullptr;
    int imap_off[kMaxLevels + 1] = {};
    int nnet[kMaxLevels + 1] = {};
    // the group-local images that have a level l+1 are emap(g, l)[0 .. nest[l])
    int nest[kMaxLevels + 1] = {};
};

struct art_batch {
    int dev = 0;
    int n = 0;
    int model = 0, nstokes = 1, precision = 0, nsub = 0;
    bool uniform = false;
    bool spectral = false;         // spectral cube render in progress (one group)
    std::vector<Params> hP;
    std::vector<ImageDesc> hD;
    Params* dP = nullptr;
    ImageDesc* dD = nullptr;
    unsigned long long* list = nullptr;
    uint16_t* cost = nullptr;      // per pixel: steps of the traced ray (queue ordering)
    size_t list_cap = 0;
    Counters* ctr = nullptr;       // one block of counters per group
    double* dTh = nullptr;         // gridded model: theta table of the batch's snapshot
    double hTh[kMaxThetaCells] = {};
    int ngroups = 1;
    int req_groups = 0;            // requested group count (0: default)
    BatchGroup grp[kMaxGroups];
    hipStream_t gs[kMaxGroups] = {};     // streams of groups 1.. (created on demand)
    hipEvent_t ev_fork = nullptr, ev_join[kMaxGroups] = {};
    hipEvent_t ev_render[2] = {};  // whole eager render on the caller's stream
    bool render_timed = false;
    int ntrace = 0;                // tracing launches per render (eager or captured)
    int graph_ntrace = 0;          // tracing launches in the captured graph
    bool timing = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    LaunchCfg L{};
    int cus = 0;
    art_cnn* net = nullptr;        // learned renders when set
    art_learned lopt{};
    int* emap = nullptr;           // device [group][level][image]: images an estimator pass concerns
    int hemap[kMaxGroups][kMaxLevels + 1][kMaxBatch] = {};
    bool fixed_mem = false;        // buffers live in the library's static scratch: never (re)allocated
    Counters* hstat = nullptr;     // host buffer for statistics (no per-call allocation), or null
    int cube_n0 = 0;               // axis-sampled cube (cube_levels >= 0): base images
    int cube_levels = -1;          // refinements along the axis (-1: not a cube)
    std::vector<int> cube_perm;    // internal index -> axis index
    std::vector<int> cube_inv;     // axis index -> internal index
};

namespace {

int validate(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
             const art_transfer* tr)
{
    if (!sp || !cam || !em || !tr) return fail(ART_EINVAL, "null parameter block");
    const double a = sp->a_spin;
    if (!(std::fabs(a) < 1.0)) return fail(ART_EINVAL, "spin |a| must be < 1 (got %g)", a);
    const double rh = 1.0 + std::sqrt(1.0 - a * a);
    if (!(cam->r_cam > 1.01 * rh)) return fail(ART_EINVAL, "camera radius %g inside the horizon", cam->r_cam);
    if (!std::isfinite(cam->phi_deg)) return fail(ART_EINVAL, "camera azimuth must be finite");
    if (!(cam->inc_deg > 0.0 && cam->inc_deg < 180.0))
        return fail(ART_EINVAL, "inclination must be in (0, 180) deg");
    if (!(cam->fov_M > 0.0)) return fail(ART_EINVAL, "field of view must be > 0");
    if (tr->nstokes != 1 && tr->nstokes != 4) return fail(ART_EINVAL, "nstokes must be 1 or 4");
    if (tr->precision != ART_PREC_FP64 && tr->precision != ART_PREC_MIXED && tr->precision != ART_PREC_MIXED_GEO)
        return fail(ART_EINVAL, "unknown precision %d", tr->precision);
    if (std::isnan(tr->fp64_radius) || std::isnan(tr->fp64_ktheta))
        return fail(ART_EINVAL, "NaN precision-policy threshold");
    if (tr->subrings < 0 || tr->subrings > kMaxSub) return fail(ART_EINVAL, "subrings must be in 0..%d", kMaxSub);
    if (tr->subrings > 0 && tr->precision == ART_PREC_MIXED_GEO)
        return fail(ART_EINVAL, "subrings need precision FP64 or MIXED");
    if (!(tr->eps > 0.0 && tr->eps <= 0.5)) return fail(ART_EINVAL, "eps must be in (0, 0.5]");
    if (tr->max_steps <= 0) return fail(ART_EINVAL, "max_steps must be > 0");
    const int k = em->kind;
    if (k != ART_EMIS_TOY_DISK && k != ART_EMIS_THERMAL && k != ART_EMIS_GRID &&
        k != ART_EMIS_SCREEN_RING && k != ART_EMIS_SCREEN_POLY)
        return fail(ART_EINVAL, "unknown emission kind %d", k);
    if (k == ART_EMIS_GRID) {
        const double* mp = em->params;
        const long long n1 = (long long)mp[9], n2 = (long long)mp[10], n3 = (long long)mp[11];
        if (!em->grid_dev) return fail(ART_EINVAL, "gridded model needs grid_dev");
        if (n1 < 2 || n2 < 2 || n3 < 1 || n2 > kMaxThetaCells || (double)n1 != mp[9] ||
            (double)n2 != mp[10] || (double)n3 != mp[11])
            return fail(ART_EINVAL, "grid dimensions must be integers, n1, n2 >= 2, n3 >= 1, n2 <= %d",
                        kMaxThetaCells);
        if (em->grid_len != n1 * n2 * n3 * 8)
            return fail(ART_EINVAL, "grid_len %lld != n1 n2 n3 8 = %lld", (long long)em->grid_len,
                        n1 * n2 * n3 * 8);
        if (!(mp[0] > 0.0 && mp[3] > 1.0 && mp[7] > 0.0 && mp[8] >= 0.0 && mp[8] <= 1.0))
            return fail(ART_EINVAL, "gridded model needs n_unit > 0, gamma > 1, dx1 > 0, 0 <= h <= 1");
        if (((uintptr_t)em->grid_dev) % 16 != 0) return fail(ART_EINVAL, "grid_dev must be 16-byte aligned");
    }
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

int grid_size(const art_camera* cam, int nstokes, int32_t* nx, int32_t* ny)
{
    if (!cam) return fail(ART_EINVAL, "camera is NULL");
    if (cam->nx0 < 2 || cam->ny0 < 2) return fail(ART_EINVAL, "base grid must be at least 2x2");
    if (cam->levels < 0 || cam->levels > 20) return fail(ART_EINVAL, "levels must be in 0..20");
    if (nstokes != 1 && nstokes != 4) return fail(ART_EINVAL, "nstokes must be 1 or 4");
    const long long X = grid_n(cam->nx0, cam->levels), Y = grid_n(cam->ny0, cam->levels);
    if (X * Y >= (1LL << 32) || X > 65535LL * 256 || Y > 65535)
        return fail(ART_EINVAL, "final grid %lldx%lld too large (< 2^32 pixels, <= 65535 rows)", X, Y);
    *nx = (int32_t)X;
    *ny = (int32_t)Y;
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

// Kernel parameter block of one image (nx, ny = final grid; 0 for points).
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
    P.phi_cam = cam->phi_deg * (M_PI / 180.0);
    P.r_out = cam->r_out > 0.0 ? cam->r_out : cam->r_cam;
    P.eps = tr->eps;
    P.r64 = tr->fp64_radius > 0.0 ? tr->fp64_radius : 6.0;
    P.kth64 = tr->fp64_ktheta >= 0.0 ? tr->fp64_ktheta : 0.05;
    P.nx = nx;
    P.ny = ny;
    if (nx > 1) {
        P.dx = cam->fov_M / (double)(nx - 1);
        P.x0 = -0.5 * cam->fov_M;
        P.y0 = -0.5 * P.dx * (double)(ny - 1);
    }
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
    P.s_cam = s;
    P.c_cam = c;
    P.ic_al = 1.0 / P.c_al;
    P.ic_del = 1.0 / Del;
    P.ic_ep = std::sqrt(A / Sig) * s;
    P.risco = r_isco(a);
    circ_EL(a, P.risco, &P.Eis, &P.Lis);
    P.model = em->kind;
    P.nstokes = tr->nstokes;
    P.nsub = tr->subrings;
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
        P.lnr_ref = std::log(rref);
        P.psi_c = std::cos(em->params[4]);
        P.psi_s = std::sin(em->params[4]);
    }
    if (em->kind == ART_EMIS_GRID) {
        const double mp_g = 1.67262192369e-24;
        P.grid = em->grid_dev;
        P.g_n1 = (int32_t)em->params[9];
        P.g_n2 = (int32_t)em->params[10];
        P.g_n3 = (int32_t)em->params[11];
        P.B_unit = C * std::sqrt(4.0 * M_PI * em->params[0] * mp_g);
    }
}

// Cell-centre angles theta(x2_j) = pi x2 + (1-h)/2 sin(2 pi x2), x2_j = (j + 1/2)/n2.
void theta_table(double h, int n2, double* out)
{
    for (int j = 0; j < n2; ++j) {
        const double x2 = (j + 0.5) / n2;
        out[j] = M_PI * x2 + 0.5 * (1.0 - h) * std::sin(2.0 * M_PI * x2);
    }
}

LaunchCfg launch_cfg(int cus, int precision, int model, int nstokes, bool sub = false)
{
    LaunchCfg L;
    art_launch u;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        u = g_launch;
    }
    L.trace_threads = u.trace_threads > 0 ? u.trace_threads : env_int("ART_TRACE_THREADS", 256);
    if (L.trace_threads != 64 && L.trace_threads != 128 && L.trace_threads != 256) L.trace_threads = 256;
    const int occ = trace_occupancy_blocks(precision, model, nstokes, sub, L.trace_threads);
    L.trace_blocks = u.trace_blocks > 0 ? u.trace_blocks : env_int("ART_TRACE_BLOCKS", cus * occ);
    if (L.trace_blocks < 1) L.trace_blocks = 1;
    L.refine_blocks = u.refine_blocks > 0 ? u.refine_blocks : L.trace_blocks;
    L.refill = u.refill > 0 ? u.refill : env_int("ART_REFILL", 1);
    if (L.refill < 1) L.refill = 1;
    if (L.refill > 64) L.refill = 64;
    L.long_steps = u.long_steps > 0 ? u.long_steps : env_int("ART_LONG_STEPS", 800);
    return L;
}

int check_image(const art_image* out, long long nx, long long ny, bool need_level)
{
    if (!out || !out->image_dev) return fail(ART_EINVAL, "output image is NULL");
    if (need_level && !out->level_dev) return fail(ART_EINVAL, "level map is NULL");
    if (out->nx != nx || out->ny != ny)
        return fail(ART_EINVAL, "image is %dx%d, camera grid is %lldx%lld", out->nx, out->ny, nx, ny);
    return ART_OK;
}

void free_batch_mem(art_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    for (int g = 0; g < kMaxGroups; ++g) {
        BatchGroup& G = b->grp[g];
        for (int k = 0; k < 2 * kMaxEv; ++k) {
            if (G.ev[k]) (void)hipEventDestroy(G.ev[k]);
            G.ev[k] = nullptr;
        }
        cnn_work_free(&G.ws);
        if (G.imap) (void)hipFree(G.imap);
        G.imap = nullptr;
        if (b->gs[g]) (void)hipStreamDestroy(b->gs[g]);
        b->gs[g] = nullptr;
        if (b->ev_join[g]) (void)hipEventDestroy(b->ev_join[g]);
        b->ev_join[g] = nullptr;
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    b->ev_fork = nullptr;
    for (int k = 0; k < 2; ++k) {
        if (b->ev_render[k]) (void)hipEventDestroy(b->ev_render[k]);
        b->ev_render[k] = nullptr;
    }
    if (b->emap) (void)hipFree(b->emap);
    b->emap = nullptr;
    if (b->list) (void)hipFree(b->list);
    if (b->cost) (void)hipFree(b->cost);
    b->cost = nullptr;
    if (b->ctr) (void)hipFree(b->ctr);
    if (b->dP) (void)hipFree(b->dP);
    if (b->dD) (void)hipFree(b->dD);
    if (b->dTh) (void)hipFree(b->dTh);
    b->net = nullptr;
    b->list = nullptr; b->ctr = nullptr; b->dP = nullptr; b->dD = nullptr; b->dTh = nullptr;
    b->list_cap = 0;
}

// Grow-only device buffers of a batch.
int ensure_mem(art_batch* b, size_t list_need)
{
    if (b->fixed_mem)
        return list_need > b->list_cap ? fail(ART_EINVAL, "%zu pixels exceed the static scratch (%zu pixels)",
                                              list_need, b->list_cap)
                                       : ART_OK;
    if (!b->ctr) {
        if (hipMalloc(&b->ctr, sizeof(Counters) * kMaxGroups) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(counters) failed");
        if (hipMalloc(&b->dP, sizeof(Params) * kMaxBatch) != hipSuccess) return fail(ART_ENOMEM, "hipMalloc(params) failed");
        if (hipMalloc(&b->dD, sizeof(ImageDesc) * kMaxBatch) != hipSuccess) return fail(ART_ENOMEM, "hipMalloc(descs) failed");
        if (hipMalloc(&b->dTh, sizeof(double) * kMaxThetaCells) != hipSuccess) return fail(ART_ENOMEM, "hipMalloc(theta table) failed");
        if (hipMalloc(&b->emap, sizeof(b->hemap)) != hipSuccess) return fail(ART_ENOMEM, "hipMalloc(image maps) failed");
        for (int g = 0; g < kMaxGroups; ++g)
            for (int k = 0; k < 2 * kMaxEv; ++k) HIP_TRY(hipEventCreate(&b->grp[g].ev[k]));
        HIP_TRY(hipEventCreate(&b->ev_render[0]));
        HIP_TRY(hipEventCreate(&b->ev_render[1]));
        HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        for (int g = 0; g < kMaxGroups; ++g) HIP_TRY(hipEventCreateWithFlags(&b->ev_join[g], hipEventDisableTiming));
        HIP_TRY(hipGetDevice(&b->dev));
        HIP_TRY(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->dev));
    }
    if (list_need > b->list_cap) {
        size_t limit;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            limit = g_list_limit;
        }
        const size_t bytes = list_need * (sizeof(unsigned long long) + sizeof(uint16_t));
        if (limit && bytes > limit)
            return fail(ART_ENOMEM, "trace list and cost map of %zu pixels need %zu bytes (allocation limit %zu)",
                        list_need, bytes, limit);
        if (b->list || b->cost) {
            HIP_TRY(hipDeviceSynchronize());
            if (b->list) HIP_TRY(hipFree(b->list));
            if (b->cost) HIP_TRY(hipFree(b->cost));
            b->list = nullptr;
            b->cost = nullptr;
            b->list_cap = 0;
        }
        if (hipMalloc(&b->list, list_need * sizeof(unsigned long long)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(trace list, %zu entries) failed", list_need);
        if (hipMalloc(&b->cost, list_need * sizeof(uint16_t)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(cost map, %zu entries) failed", list_need);
        b->list_cap = list_need;
    }
    return ART_OK;
}

// Default group count: two groups from 16 images on (measured best for the
// 64-image batches; more concurrent groups than hardware queues serialise).
int default_groups(int n)
{
    return n >= 16 ? 2 : 1;
}

// Split the images into groups, set each image's base-list offset inside its
// group's slice of the trace list and upload the descriptors.
int layout(art_batch* b, hipStream_t s)
{
    int G = (b->uniform || b->spectral || b->fixed_mem) ? 1
                                                        : (b->req_groups > 0 ? b->req_groups : default_groups(b->n));
    if (G > b->n) G = b->n;
    if (G > kMaxGroups) G = kMaxGroups;
    b->ngroups = G;
    size_t off = 0;
    for (int g = 0; g < G; ++g) {
        BatchGroup& Gr = b->grp[g];
        Gr.i0 = (int)((long long)g * b->n / G);
        Gr.n = (int)((long long)(g + 1) * b->n / G) - Gr.i0;
        Gr.lmax = 0;
        Gr.max_base = 0;
        Gr.nx0m = Gr.ny0m = 0;
        Gr.list_off = off;
        const size_t off0 = off;
        for (int k = 0; k < Gr.n; ++k) {
            ImageDesc& D = b->hD[Gr.i0 + k];
            Gr.lmax = D.levels > Gr.lmax ? D.levels : Gr.lmax;
            Gr.max_base = D.nx0 * D.ny0 > Gr.max_base ? D.nx0 * D.ny0 : Gr.max_base;
            Gr.nx0m = D.nx0 > Gr.nx0m ? D.nx0 : Gr.nx0m;
            Gr.ny0m = D.ny0 > Gr.ny0m ? D.ny0 : Gr.ny0m;
            D.cost = b->uniform ? nullptr : b->cost + off;   // same offsets as the list slices
            off += (size_t)D.plane;
        }
        Gr.list_len = off - off0;
        for (int l = 0; l <= kMaxLevels; ++l) {
            Gr.nest[l] = 0;
            for (int k = 0; k < Gr.n; ++k)
                if (b->hD[Gr.i0 + k].levels > l) b->hemap[g][l][Gr.nest[l]++] = k;
        }
    }
    if (b->emap)
        HIP_TRY(hipMemcpyAsync(b->emap, b->hemap, sizeof(int) * kMaxBatch * (kMaxLevels + 1) * G,
                               hipMemcpyHostToDevice, s));
    for (int g = 1; g < G; ++g)
        if (!b->gs[g]) HIP_TRY(hipStreamCreateWithFlags(&b->gs[g], hipStreamNonBlocking));
    HIP_TRY(hipMemcpyAsync(b->dD, b->hD.data(), sizeof(ImageDesc) * b->n, hipMemcpyHostToDevice, s));
    return ART_OK;
}

// Validate jobs, fill host descriptors, grow buffers and upload descriptors.
int prepare(art_batch* b, int n, const art_job* jobs, const art_image* images, bool uniform,
            hipStream_t s)
{
    if (n < 1 || n > kMaxBatch) return fail(ART_EINVAL, "batch size %d outside 1..%d", n, kMaxBatch);
    if (!jobs || !images) return fail(ART_EINVAL, "NULL jobs or images");
    if (uniform && n != 1) return fail(ART_EINVAL, "uniform renders take one image");
    b->n = n;
    b->uniform = uniform;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        b->req_groups = g_launch.groups;
    }
    b->hP.resize(n);
    b->hD.resize(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const art_job& J = jobs[i];
        int rc = validate(&J.sp, &J.cam, &J.em, &J.tr);
        if (rc) return rc;
        if (!uniform) {
            if (J.rf.abs_norm != ART_NORM_MEAN && J.rf.abs_norm != ART_NORM_MAX)
                return fail(ART_EINVAL, "image %d: unknown abs_norm %d", i, J.rf.abs_norm);
            if (std::isnan(J.rf.r_rel) || std::isnan(J.rf.r_abs))
                return fail(ART_EINVAL, "image %d: NaN tolerance", i);
            if (J.rf.interp != ART_INTERP_LINEAR && J.rf.interp != ART_INTERP_NEAREST)
                return fail(ART_EINVAL, "image %d: unknown interpolation %d", i, J.rf.interp);
            if (J.rf.all_planes < 0 || J.rf.all_planes > 2)
                return fail(ART_EINVAL, "image %d: all_planes must be 0, 1 or 2", i);
            if (J.rf.all_planes == 2 && J.rf.interp != ART_INTERP_LINEAR)
                return fail(ART_EINVAL, "image %d: per-plane normalisation needs the linear branch", i);
        }
        if (i == 0) {
            b->model = J.em.kind;
            b->nstokes = J.tr.nstokes;
            b->precision = J.tr.precision;
            b->nsub = J.tr.subrings;
        } else if (J.em.kind != b->model || J.tr.nstokes != b->nstokes || J.tr.precision != b->precision ||
                   J.tr.subrings != b->nsub) {
            return fail(ART_EINVAL, "image %d: a batch needs one emission kind, nstokes, precision and subring count", i);
        } else if (J.em.kind == ART_EMIS_GRID &&
                   (J.em.params[8] != jobs[0].em.params[8] || J.em.params[10] != jobs[0].em.params[10])) {
            return fail(ART_EINVAL, "image %d: all snapshots of a batch need the same theta grid (h, n2)", i);
        }
        int32_t nx, ny;
        rc = grid_size(&J.cam, J.tr.nstokes, &nx, &ny);
        if (rc) return rc;
        rc = check_image(&images[i], nx, ny, !uniform);
        if (rc) return rc;
        make_params(&J.sp, &J.cam, &J.em, &J.tr, nx, ny, b->hP[i]);
        ImageDesc& D = b->hD[i];
        D.img = images[i].image_dev;
        D.level = images[i].level_dev;
        D.feat = (RayFeat*)images[i].feat_dev;
        D.plane = (long long)nx * ny;
        D.nx = nx; D.ny = ny;
        D.nx0 = J.cam.nx0; D.ny0 = J.cam.ny0;
        D.levels = uniform ? 0 : J.cam.levels;
        D.nstokes = J.tr.nstokes;
        D.nplanes = J.tr.nstokes + J.tr.subrings;
        D.flags = uniform ? 0 : ((J.rf.interp == ART_INTERP_NEAREST ? kRefineNearest : 0) |
                                 (J.rf.all_planes ? kRefineAllPlanes : 0) |
                                 (J.rf.all_planes == 2 ? kRefineOwnNorm : 0));
        D.abs_norm = J.rf.abs_norm;
        D.pad0 = 0;
        D.r_rel = J.rf.r_rel;
        D.r_abs = J.rf.r_abs;
        D.sa = D.sb = D.sc = D.sd = -1;
        D.sr_rel = D.sr_abs = 0.0;
        total += (size_t)D.plane;
    }
    if (total >= (1ULL << 31)) return fail(ART_EINVAL, "batch has %zu pixels (limit 2^31)", total);
    int rc = ensure_mem(b, uniform ? 0 : total);
    if (rc) return rc;
    b->L = launch_cfg(b->cus, b->precision, b->model, b->nstokes, b->nsub > 0);
    if (b->model == ART_EMIS_GRID) {
        const int n2 = (int)jobs[0].em.params[10];
        theta_table(jobs[0].em.params[8], n2, b->hTh);
        HIP_TRY(hipMemcpyAsync(b->dTh, b->hTh, sizeof(double) * n2, hipMemcpyHostToDevice, s));
        for (int i = 0; i < n; ++i) b->hP[i].theta_tab = b->dTh;
    }
    HIP_TRY(hipMemcpyAsync(b->dP, b->hP.data(), sizeof(Params) * n, hipMemcpyHostToDevice, s));
    return layout(b, s);
}

// Images of group g that have level l+1 (device map) and their number; a
// batch without maps (static scratch) launches over all its images.
const int* est_map(const art_batch* b, int g, int l, int& n)
{
    const BatchGroup& G = b->grp[g];
    if (!b->emap) {
        n = G.n;
        return nullptr;
    }
    n = G.nest[l];
    return b->emap + ((size_t)g * (kMaxLevels + 1) + l) * kMaxBatch;
}

TraceJob base_job(const art_batch* b, int g, int level)
{
    const BatchGroup& G = b->grp[g];
    Counters* ctr = b->ctr + g;
    TraceJob J;
    std::memset(&J, 0, sizeof(J));
    J.src = SRC_LIST;
    J.nimg = G.n;
    J.params = b->dP + G.i0;
    J.desc = b->dD + G.i0;
    J.list = b->list + G.list_off;
    J.cap = (long long)G.list_len;
    J.count = &ctr->count[level];
    J.count_back = &ctr->count_back[level];
    J.cursor = &ctr->cursor[level];
    J.ctr = ctr;
    J.refill = b->L.refill;
    return J;
}

hipError_t ev_begin(art_batch* b, int g, hipStream_t s)
{
    b->ntrace++;
    BatchGroup& G = b->grp[g];
    if (!b->timing || G.nev >= kMaxEv) return hipSuccess;
    return hipEventRecord(G.ev[2 * G.nev], s);
}
hipError_t ev_end(art_batch* b, int g, hipStream_t s)
{
    BatchGroup& G = b->grp[g];
    if (!b->timing || G.nev >= kMaxEv) return hipSuccess;
    hipError_t e = hipEventRecord(G.ev[2 * G.nev + 1], s);
    G.nev++;
    return e;
}

int trace_pass(art_batch* b, int g, int level, hipStream_t s)
{
    TraceJob J = base_job(b, g, level);
    LaunchCfg L = b->L;
    if (level > 0) L.trace_blocks = b->L.refine_blocks;
    HIP_TRY(ev_begin(b, g, s));
    HIP_TRY(launch_trace(b->precision, b->model, b->nstokes, b->nsub > 0, J, L, s));
    HIP_TRY(ev_end(b, g, s));
    return ART_OK;
}

// Base grid of group g: clear its counters, list and trace the base points,
// then the per-image level-0 reductions.
int enqueue_base(art_batch* b, int g, hipStream_t s)
{
    const BatchGroup& G = b->grp[g];
    Counters* ctr = b->ctr + g;
    HIP_TRY(launch_fill_u32((uint32_t*)ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_base_list(b->dD + G.i0, b->dP + G.i0, G.n, G.max_base, b->list + G.list_off,
                             (long long)G.list_len, ctr, 0, s));
    int rc = trace_pass(b, g, 0, s);
    if (rc) return rc;
    HIP_TRY(launch_reduce_base(b->dD + G.i0, G.n, ctr, s));
    return ART_OK;
}

// The adaptive level loop of group g (Sec. 3.2).
int enqueue_adaptive(art_batch* b, int g, hipStream_t s)
{
    const BatchGroup& G = b->grp[g];
    int rc = enqueue_base(b, g, s);
    if (rc) return rc;
    for (int l = 0; l < G.lmax; ++l) {
        const int nxl = (int)grid_n(G.nx0m, l + 1), nyl = (int)grid_n(G.ny0m, l + 1);
        int ne;
        const int* em = est_map(b, g, l, ne);
        HIP_TRY(launch_estimate(b->dD + G.i0, ne, nxl, nyl, l, b->ctr + g, b->list + G.list_off,
                                (long long)G.list_len, b->L.long_steps, s, 0, 1, 0, -1, em));
        rc = trace_pass(b, g, l + 1, s);
        if (rc) return rc;
    }
    return ART_OK;
}

// Learned level loop of group g: where the network can look two levels ahead
// it runs on the level-l grid of every image, its level-(l+2) proposals are
// traced in pass l+1 together with the level-(l+1) points (proposed or flagged
// by the criterion and not suppressed), and the criterion then judges level
// l+2 and traces what the look-ahead missed (fallback) or only counts it.
// Images may have different level counts (one base grid): at level l an image
// with levels >= l+2 takes the look-ahead, one with l+1 levels its last level
// by the criterion alone (the network too with all_levels), and one with fewer
// is finished; every kernel skips the images a level does not concern.
// Interpolated points get feature records only up to the last level the
// network reads (traced points always get theirs).
int enqueue_learned(art_batch* b, int g, hipStream_t s)
{
    BatchGroup& G = b->grp[g];
    const ImageDesc& D0 = b->hD[G.i0];
    const int N = G.lmax;
    const ImageDesc* dD = b->dD + G.i0;
    Counters* ctr = b->ctr + g;
    unsigned long long* list = b->list + G.list_off;
    const long long cap = (long long)G.list_len;
    int rc = enqueue_base(b, g, s);
    if (rc) return rc;
    const art_learned& o = b->lopt;
    auto any_with = [&](int lo) {             // an image of the group with >= lo levels
        for (int i = G.i0; i < G.i0 + G.n; ++i)
            if (b->hD[i].levels >= lo) return true;
        return false;
    };
    // the last level the network reads: interpolated points of deeper levels
    // need no feature records (the same walk over the levels as below)
    int last_net = -1;
    for (int l = 0; l < N;) {
        if (G.nnet[l] > 0) {
            last_net = l;
            l += any_with(l + 2) ? 2 : 1;
        } else {
            l += 1;
        }
    }
    int l = 0;
    while (l < N) {
        const bool ahead = any_with(l + 2);
        const bool net_here = G.nnet[l] > 0;
        const int nxl = (int)grid_n(D0.nx0, l + 1), nyl = (int)grid_n(D0.ny0, l + 1);
        if (!net_here) {
            int ne;
            const int* em = est_map(b, g, l, ne);
            HIP_TRY(launch_estimate(dD, ne, nxl, nyl, l, ctr, list, cap, b->L.long_steps, s, 0, 1, 0, -1, em,
                                    l + 1 <= last_net));
            rc = trace_pass(b, g, l + 1, s);
            if (rc) return rc;
            l += 1;
            continue;
        }
        // the network only on the images it decides for at this level
        const int W = (int)grid_n(D0.nx0, l), H = (int)grid_n(D0.ny0, l);
        const int* im = G.imap + G.imap_off[l];
        HIP_TRY(cnn_features_batch(dD, ctr, G.nnet[l], l, H, W, nullptr, G.ws.x, s, im));
        HIP_TRY(cnn_net_forward(&b->net->net, &G.ws, nullptr, G.nnet[l], H, W, G.ws.logits, s));
        HIP_TRY(cnn_propose(G.ws.logits, dD, G.nnet[l], l, H, W, o.z_propose, o.z_suppress, o.all_levels, list,
                            cap, b->L.long_steps, ctr, s, im));
        // mode 1: images the network decided for read its marks; the others
        // (one level left, no all_levels) take the plain criterion
        int ne;
        const int* em = est_map(b, g, l, ne);
        HIP_TRY(launch_estimate(dD, ne, nxl, nyl, l, ctr, list, cap, b->L.long_steps, s, 1, o.all_levels ? 1 : 0, 0,
                                -1, em, l + 1 <= last_net));
        rc = trace_pass(b, g, l + 1, s);
        if (rc) return rc;
        if (ahead) {
            const int nx2 = (int)grid_n(D0.nx0, l + 2), ny2 = (int)grid_n(D0.ny0, l + 2);
            int ne2;
            const int* em2 = est_map(b, g, l + 1, ne2);
            HIP_TRY(launch_estimate(dD, ne2, nx2, ny2, l + 1, ctr, list, cap, b->L.long_steps, s, 2,
                                    o.fallback ? 1 : 0, 0, -1, em2, l + 2 <= last_net));
            if (o.fallback) {
                rc = trace_pass(b, g, l + 2, s);
                if (rc) return rc;
            }
            l += 2;
        } else {
            l += 1;
        }
    }
    return ART_OK;
}

// One render of the whole batch on stream s: every group's level loop on its
// own stream, forked from and joined back into s (capturable).
int enqueue_spectral(art_batch* b, int n0, int slevels, hipStream_t s);

int enqueue_render(art_batch* b, hipStream_t s)
{
    if (b->cube_levels >= 0) return enqueue_spectral(b, b->cube_n0, b->cube_levels, s);
    b->ntrace = 0;
    for (int g = 0; g < b->ngroups; ++g) b->grp[g].nev = 0;
    b->render_timed = b->timing;
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[0], s));
    if (b->ngroups > 1) HIP_TRY(hipEventRecord(b->ev_fork, s));
    for (int g = 0; g < b->ngroups; ++g) {
        hipStream_t sg = g == 0 ? s : b->gs[g];
        if (g > 0) HIP_TRY(hipStreamWaitEvent(sg, b->ev_fork, 0));
        int rc = b->net ? enqueue_learned(b, g, sg) : enqueue_adaptive(b, g, sg);
        if (rc) return rc;
        if (g > 0) {
            HIP_TRY(hipEventRecord(b->ev_join[g], sg));
            HIP_TRY(hipStreamWaitEvent(s, b->ev_join[g], 0));
        }
    }
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[1], s));
    return ART_OK;
}

// Spectral cube (one group; images in internal order: the n0 base
// frequencies, then each spectral level's images).  Step (s, l) decides the
// level-l points of the spectral-level-s images: for s = 0 the plain
// criterion (base list at l = 0), for s > 0 the spectral base pass (l = 0)
// or the criterion with the spectral alternative (mode 3).  It needs the
// image's own level l-1 and the spectral neighbours' level l, so the steps
// run as a wavefront: pass t decides and traces every (s, l) with s + l = t
// (N + L + 1 passes instead of (N + 1)(L + 1)), each pass in its own list
// slot; the level-0 reduction of level-s images follows pass s.
int enqueue_spectral(art_batch* b, int n0, int slevels, hipStream_t s)
{
    b->ntrace = 0;
    BatchGroup& G = b->grp[0];
    G.nev = 0;
    b->render_timed = b->timing;
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[0], s));
    Counters* ctr = b->ctr;
    unsigned long long* list = b->list + G.list_off;
    const long long cap = (long long)G.list_len;
    const ImageDesc& D0 = b->hD[0];
    const int N = D0.levels;
    const int nb = D0.nx0 * D0.ny0;
    int off[8], m[8];
    off[0] = 0;
    m[0] = n0;
    for (int sl = 1; sl <= slevels; ++sl) {
        off[sl] = off[sl - 1] + m[sl - 1];
        m[sl] = (n0 - 1) << (sl - 1);
    }
    HIP_TRY(launch_fill_u32((uint32_t*)ctr, sizeof(Counters) / 4, 0u, s));
    for (int t = 0; t <= N + slevels; ++t) {
        for (int sl = 0; sl <= slevels; ++sl) {
            const int l = t - sl;
            if (l < 0 || l > N) continue;
            if (l == 0) {
                if (sl == 0)
                    HIP_TRY(launch_base_list(b->dD, b->dP, n0, nb, list, cap, ctr, t, s));
                else
                    HIP_TRY(launch_spectral_base(b->dD, off[sl], m[sl], nb, ctr, list, cap, b->L.long_steps, t, s));
            } else {
                const int nxl = (int)grid_n(D0.nx0, l), nyl = (int)grid_n(D0.ny0, l);
                HIP_TRY(launch_estimate(b->dD, m[sl], nxl, nyl, l - 1, ctr, list, cap, b->L.long_steps, s,
                                        sl == 0 ? 0 : 3, 1, off[sl], t));
            }
        }
        int rc = trace_pass(b, 0, t, s);
        if (rc) return rc;
        if (t <= slevels) HIP_TRY(launch_reduce_base(b->dD, m[t], ctr, s, off[t]));
    }
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[1], s));
    return ART_OK;
}

// Check that a prepared batch can run learned renders and size its workspaces.
int setup_learned(art_batch* b, art_cnn* net, const art_learned* opt)
{
    if (!net) {
        b->net = nullptr;
        return ART_OK;
    }
    if (!opt) return fail(ART_EINVAL, "NULL learned-render options");
    if (std::isnan(opt->z_propose) || std::isnan(opt->z_suppress) || !(opt->z_suppress <= opt->z_propose))
        return fail(ART_EINVAL, "need z_suppress <= z_propose (no NaN)");
    if (opt->level_cap < 0) return fail(ART_EINVAL, "level_cap must be >= 0");
    if (b->uniform) return fail(ART_EINVAL, "uniform renders have no refinement");
    const ImageDesc& D0 = b->hD[0];
    int nmax = 0;
    for (int i = 0; i < b->n; ++i) {
        const ImageDesc& D = b->hD[i];
        if (D.nx0 != D0.nx0 || D.ny0 != D0.ny0)
            return fail(ART_EINVAL, "learned renders need one base grid for the whole batch");
        if (!D.feat) return fail(ART_EINVAL, "image %d: learned renders need a feature buffer", i);
        nmax = D.levels > nmax ? D.levels : nmax;
    }
    // per group and level, the images the network decides for: those that
    // can look two levels ahead (levels >= l + 2), with all_levels also those
    // with one level left, at levels below level_cap if it is set; the
    // workspace holds the largest such set's grids
    for (int g = 0; g < b->ngroups; ++g) {
        BatchGroup& G = b->grp[g];
        std::vector<int> h;
        long long P = 0;
        for (int l = 0; l <= kMaxLevels; ++l) {
            G.imap_off[l] = (int)h.size();
            G.nnet[l] = 0;
            for (int i = 0; i < G.n; ++i) {
                const int Li = b->hD[G.i0 + i].levels;
                const bool capped = opt->level_cap > 0 && l >= opt->level_cap;
                if (!capped && (Li >= l + 2 || (opt->all_levels && Li >= l + 1))) {
                    h.push_back(i);
                    G.nnet[l]++;
                }
            }
            if (G.nnet[l]) {
                const long long Pl = (long long)G.nnet[l] * grid_n(D0.nx0, l) * grid_n(D0.ny0, l);
                P = Pl > P ? Pl : P;
            }
        }
        if (P > (1LL << 28)) return fail(ART_EINVAL, "network grid of %lld positions too large", P);
        if (P > 0) {
            int rc = cnn_work_reserve(&G.ws, P);
            if (rc) return rc;
        }
        if (G.imap) (void)hipFree(G.imap);
        G.imap = nullptr;
        if (!h.empty()) {
            if (hipMalloc((void**)&G.imap, sizeof(int) * h.size()) != hipSuccess)
                return fail(ART_ENOMEM, "hipMalloc(network image map) failed");
            HIP_TRY(hipMemcpy(G.imap, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice));
        }
    }
    b->net = net;
    b->lopt = *opt;
    return ART_OK;
}

int enqueue_uniform(art_batch* b, hipStream_t s)
{
    b->ntrace = 0;
    b->grp[0].nev = 0;
    b->render_timed = b->timing;
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[0], s));
    const ImageDesc& D = b->hD[0];
    HIP_TRY(launch_fill_u32((uint32_t*)b->ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_fill_u32(&b->ctr->count[0], 1, (uint32_t)D.plane, s));
    if (D.level) HIP_TRY(launch_fill_i8(D.level, D.plane, 0, s));
    TraceJob J = base_job(b, 0, 0);
    J.list = nullptr;    // implicit list: item k = pixel k of image 0
    HIP_TRY(ev_begin(b, 0, s));
    HIP_TRY(launch_trace(b->precision, b->model, b->nstokes, b->nsub > 0, J, b->L, s));
    HIP_TRY(ev_end(b, 0, s));
    if (b->timing) HIP_TRY(hipEventRecord(b->ev_render[1], s));
    return ART_OK;
}

// Statistics of image i (i < 0: whole batch).  Synchronises the stream.
// Step counts and the status histogram are batch-wide.
int batch_stats(art_batch* b, int i, art_stats* st, hipStream_t s)
{
    std::vector<Counters> hv;
    Counters* h = b->hstat;
    if (!h) {
        hv.resize(b->ngroups);
        h = hv.data();
    }
    HIP_TRY(hipMemcpyAsync(h, b->ctr, sizeof(Counters) * b->ngroups, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memset(st, 0, sizeof(*st));
    long long npix = 0, traced = 0;
    int lv = 0;
    for (int g = 0; g < b->ngroups; ++g) {
        const BatchGroup& G = b->grp[g];
        const Counters& c = h[g];
        for (int q = 0; q < G.n; ++q) {
            const int k = G.i0 + q;
            if (i >= 0 && k != i) continue;
            const ImageDesc& D = b->hD[k];
            npix += D.plane;
            lv = D.levels > lv ? D.levels : lv;
            for (int l = 0; l <= D.levels && l < 32; ++l) {
                const long long t = b->uniform ? (long long)D.plane : (long long)c.img_traced[q][l];
                st->traced[l] += t;
                traced += t;
                if (l == 0)
                    st->candidates[0] += b->uniform ? D.plane : (long long)D.nx0 * D.ny0;
                else
                    st->candidates[l] += grid_n(D.nx0, l) * grid_n(D.ny0, l) -
                                         grid_n(D.nx0, l - 1) * grid_n(D.ny0, l - 1);
            }
            for (int j = 0; j < 5; ++j) st->learned[j] += (int64_t)c.judge[q][j];
            st->spectral += (int64_t)c.judge[q][5];
            if (k == (i >= 0 ? i : 0)) {
                st->ibar_int = c.scal[q][0];
                st->imax0 = c.scal[q][1];
                st->n_abs = c.scal[q][2];
            }
        }
        st->steps_total += (int64_t)c.steps;
        st->steps_emit += (int64_t)c.steps_emit;
        for (int k = 0; k < 8; ++k) st->status_hist[k] += (int64_t)c.status[k];
    }
    st->levels = lv;
    st->rays_traced = traced;
    st->interp_frac = b->uniform ? 0.0 : (double)(npix - traced) / (double)npix;
    double tms = 0.0;
    for (int g = 0; g < b->ngroups; ++g) {
        const BatchGroup& G = b->grp[g];
        for (int k = 0; k < G.nev; ++k) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, G.ev[2 * k], G.ev[2 * k + 1]));
            tms += ms;
        }
    }
    st->t_trace_ms = tms;
    st->trace_launches = b->ntrace;
    if (b->render_timed) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev_render[0], b->ev_render[1]));
        st->t_render_ms = ms;
    }
    if (st->status_hist[RAY_NAN] > 0)
        return fail(ART_ENUMERIC, "%lld rays produced NaN", (long long)st->status_hist[RAY_NAN]);
    return ART_OK;
}

// One reusable batch per device for the single-image entry points.
art_batch g_single[64];
std::mutex g_single_mu;

// ---------------------------------------------------------------- scratch
// Static device scratch of art_render_noalloc: counters, parameter block,
// image descriptor and theta table of one image group, then the trace list
// (8 B per pixel) and the cost map (2 B per pixel) of an image of at most
// kNoAllocPixels pixels (2049^2: the largest image of the batched workload).
// Each device holds its own copy from module load to process exit.
constexpr size_t kNoAllocPixels = 2049ull * 2049ull;
constexpr size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaCtr = 0;
constexpr size_t kNaPar = kNaCtr + round256(sizeof(Counters));
constexpr size_t kNaDesc = kNaPar + round256(sizeof(Params));
constexpr size_t kNaTheta = kNaDesc + round256(sizeof(ImageDesc));
constexpr size_t kNaList = kNaTheta + round256(sizeof(double) * kMaxThetaCells);
constexpr size_t kNaCost = kNaList + round256(sizeof(unsigned long long) * kNoAllocPixels);
constexpr size_t kNoAllocBytes = kNaCost + round256(sizeof(uint16_t) * kNoAllocPixels);

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocState {
    bool ready = false;
    unsigned char* ptr = nullptr;  // device address of this device's scratch
    art_batch b;
    Counters hstat;
};
NoAllocState g_noalloc[64];
std::mutex g_noalloc_mu;

// Set-up on the first call on a device (that device current): the scratch's
// device address, the batch's fixed buffers, host vectors reserved.
int noalloc_setup(NoAllocState& N, int dev)
{
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(ART_EDEVICE, "no address for the static scratch on device %d", dev);
    N.ptr = (unsigned char*)ptr;
    art_batch& b = N.b;
    b.dev = dev;
    HIP_TRY(hipDeviceGetAttribute(&b.cus, hipDeviceAttributeMultiprocessorCount, dev));
    b.ctr = (Counters*)(N.ptr + kNaCtr);
    b.dP = (Params*)(N.ptr + kNaPar);
    b.dD = (ImageDesc*)(N.ptr + kNaDesc);
    b.dTh = (double*)(N.ptr + kNaTheta);
    b.list = (unsigned long long*)(N.ptr + kNaList);
    b.cost = (uint16_t*)(N.ptr + kNaCost);
    b.list_cap = kNoAllocPixels;
    b.fixed_mem = true;
    b.hstat = &N.hstat;
    b.hP.reserve(1);
    b.hD.reserve(1);
    N.ready = true;
    return ART_OK;
}

art_batch* single_batch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    return &g_single[dev];
}

art_job make_job(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                 const art_refine* rf, const art_transfer* tr)
{
    art_job j;
    std::memset(&j, 0, sizeof(j));
    j.sp = *sp;
    j.cam = *cam;
    j.em = *em;
    if (rf) j.rf = *rf;
    j.tr = *tr;
    return j;
}

}  // namespace

extern "C" {

const char* art_last_error(void) { return g_err.c_str(); }

int art_image_size(const art_camera* cam, int32_t nstokes, int32_t* nx, int32_t* ny,
                   size_t* image_bytes)
{
    int32_t X, Y;
    int rc = grid_size(cam, nstokes, &X, &Y);
    if (rc) return rc;
    if (nx) *nx = X;
    if (ny) *ny = Y;
    if (image_bytes) *image_bytes = (size_t)X * (size_t)Y * (size_t)nstokes * sizeof(double);
    return ART_OK;
}

int art_render(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
               const art_refine* rf, const art_transfer* tr, art_image* out, art_stats* st,
               void* stream)
{
    if (!sp || !cam || !em || !rf || !tr || !out) return fail(ART_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_single_mu);
    art_batch* b = single_batch();
    if (!b) return fail(ART_EDEVICE, "no current device");
    hipStream_t s = (hipStream_t)stream;
    const art_job j = make_job(sp, cam, em, rf, tr);
    int rc = prepare(b, 1, &j, out, false, s);
    if (rc) return rc;
    b->timing = st != nullptr;
    b->net = nullptr;
    rc = enqueue_render(b, s);
    if (rc) return rc;
    if (st) return batch_stats(b, 0, st, s);
    return ART_OK;
}

int art_render_noalloc(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_refine* rf, const art_transfer* tr, art_image* out, art_stats* st,
                       void* stream)
{
    if (!sp || !cam || !em || !rf || !tr || !out) return fail(ART_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(ART_EDEVICE, "no current device");
    NoAllocState& N = g_noalloc[dev];
    if (!N.ready) {
        int rc = noalloc_setup(N, dev);
        if (rc) return rc;
    }
    int32_t nx, ny;
    int rc = grid_size(cam, tr->nstokes, &nx, &ny);
    if (rc) return rc;
    if ((size_t)nx * (size_t)ny > kNoAllocPixels)
        return fail(ART_EINVAL, "%d x %d image exceeds the no-allocation limit of %zu pixels", nx, ny,
                    kNoAllocPixels);
    hipStream_t s = (hipStream_t)stream;
    const art_job j = make_job(sp, cam, em, rf, tr);
    rc = prepare(&N.b, 1, &j, out, false, s);
    if (rc) return rc;
    N.b.timing = false;
    N.b.net = nullptr;
    rc = enqueue_render(&N.b, s);
    if (rc) return rc;
    if (st) return batch_stats(&N.b, 0, st, s);
    return ART_OK;
}

int art_render_learned(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_refine* rf, const art_transfer* tr, art_cnn* net, const art_learned* opt,
                       art_image* out, art_stats* st, void* stream)
{
    if (!sp || !cam || !em || !rf || !tr || !out || !net || !opt) return fail(ART_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_single_mu);
    art_batch* b = single_batch();
    if (!b) return fail(ART_EDEVICE, "no current device");
    hipStream_t s = (hipStream_t)stream;
    const art_job j = make_job(sp, cam, em, rf, tr);
    int rc = prepare(b, 1, &j, out, false, s);
    if (rc) return rc;
    rc = setup_learned(b, net, opt);
    if (rc) return rc;
    b->timing = st != nullptr;
    rc = enqueue_render(b, s);
    b->net = nullptr;             // the single-image batch keeps no network
    if (rc) return rc;
    if (st) return batch_stats(b, 0, st, s);
    return ART_OK;
}

namespace {

// Set up batch b as an axis-sampled cube: jobs and images in axis order are
// stored in the internal order (the n0 base images, then each axis level's
// images), every non-base image gets its axis neighbours a, b, c, d (-1
// outside the cube) and the axis tolerances; descriptors are uploaded on s.
int check_cube(int32_t n, const art_job* jobs, int32_t n0, int32_t L, double r_rel, double r_abs,
               const art_image* out)
{
    if (!jobs || !out) return fail(ART_EINVAL, "null argument");
    if (n0 < 2 || L < 0 || L > 6) return fail(ART_EINVAL, "a cube needs n0 >= 2 and 0 <= levels <= 6");
    if ((long long)n != ((long long)(n0 - 1) << L) + 1)
        return fail(ART_EINVAL, "a cube of n0 = %d and %d levels has %lld images, not %d", n0, L,
                    ((long long)(n0 - 1) << L) + 1, n);
    if (n > kMaxBatch) return fail(ART_EINVAL, "cube of %d images (limit %d)", n, kMaxBatch);
    if (std::isnan(r_rel) || std::isnan(r_abs)) return fail(ART_EINVAL, "NaN cube tolerance");
    for (int i = 1; i < n; ++i)
        if (jobs[i].cam.nx0 != jobs[0].cam.nx0 || jobs[i].cam.ny0 != jobs[0].cam.ny0 ||
            jobs[i].cam.levels != jobs[0].cam.levels)
            return fail(ART_EINVAL, "cube image %d: every image needs the same base grid and levels", i);
    if (jobs[0].cam.levels + L > kMaxLevels)
        return fail(ART_EINVAL, "cube of %d + %d levels (limit %d)", jobs[0].cam.levels, L, kMaxLevels);
    return ART_OK;
}

int setup_cube(art_batch* b, int32_t n, const art_job* jobs, int32_t n0, int32_t L, double r_rel, double r_abs,
               const art_image* out, hipStream_t s)
{
    int rc = check_cube(n, jobs, n0, L, r_rel, r_abs, out);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
        if (jobs[i].rf.all_planes == 2)
            return fail(ART_EINVAL, "image %d: axis-sampled cubes take all_planes 0 or 1", i);
    std::vector<int> perm, inv(n, -1);
    for (int k = 0; k < n0; ++k) perm.push_back(k << L);
    for (int sl = 1; sl <= L; ++sl) {
        const int h = 1 << (L - sl);
        for (int i = h; i < n; i += 2 * h) perm.push_back(i);
    }
    for (int k = 0; k < n; ++k) inv[perm[k]] = k;
    std::vector<art_job> J((size_t)n);
    std::vector<art_image> imgs((size_t)n);
    for (int k = 0; k < n; ++k) {
        J[k] = jobs[perm[k]];
        imgs[k] = out[perm[k]];
    }
    b->spectral = true;
    rc = prepare(b, n, J.data(), imgs.data(), false, s);
    if (rc) {
        b->spectral = false;
        return rc;
    }
    for (int k = n0; k < n; ++k) {
        const int i = perm[k];
        int lvl = L;
        for (int q = i; q % 2 == 0; q /= 2) --lvl;
        const int h = 1 << (L - lvl);
        ImageDesc& D = b->hD[k];
        D.sb = inv[i - h];
        D.sc = inv[i + h];
        D.sa = i - 3 * h >= 0 ? inv[i - 3 * h] : -1;
        D.sd = i + 3 * h < n ? inv[i + 3 * h] : -1;
        D.sr_rel = r_rel;
        D.sr_abs = r_abs;
    }
    hipError_t e = hipMemcpyAsync(b->dD, b->hD.data(), sizeof(ImageDesc) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        b->spectral = false;
        return fail(ART_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
    }
    b->net = nullptr;
    b->cube_n0 = n0;
    b->cube_levels = L;
    b->cube_perm = perm;
    b->cube_inv = inv;
    return ART_OK;
}

void clear_cube(art_batch* b)
{
    b->spectral = false;
    b->cube_levels = -1;
    b->cube_n0 = 0;
    b->cube_perm.clear();
    b->cube_inv.clear();
}

}  // namespace

int art_render_cube(int32_t n, const art_job* jobs, int32_t n0, int32_t levels, double r_rel, double r_abs,
                    art_image* out, art_stats* st, void* stream)
{
    int rc = check_cube(n, jobs, n0, levels, r_rel, r_abs, out);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_single_mu);
    art_batch* b = single_batch();
    if (!b) return fail(ART_EDEVICE, "no current device");
    hipStream_t s = (hipStream_t)stream;
    rc = setup_cube(b, n, jobs, n0, levels, r_rel, r_abs, out, s);
    if (rc) {
        clear_cube(b);
        return rc;
    }
    b->timing = st != nullptr;
    rc = enqueue_spectral(b, n0, levels, s);
    if (rc == ART_OK && st) {
        for (int k = 0; k < n && rc == ART_OK; ++k) rc = batch_stats(b, k, &st[b->cube_perm[k]], s);
    }
    clear_cube(b);
    return rc;
}

int art_cube_create(int32_t n, const art_job* jobs, int32_t n0, int32_t levels, double r_rel, double r_abs,
                    const art_image* images, art_batch** out)
{
    if (!out) return fail(ART_EINVAL, "NULL output handle");
    *out = nullptr;
    int rc = check_cube(n, jobs, n0, levels, r_rel, r_abs, images);
    if (rc) return rc;
    art_batch* b = new (std::nothrow) art_batch();
    if (!b) return fail(ART_ENOMEM, "out of host memory");
    rc = setup_cube(b, n, jobs, n0, levels, r_rel, r_abs, images, nullptr);
    if (rc == ART_OK && hipStreamSynchronize(nullptr) != hipSuccess) rc = fail(ART_EDEVICE, "upload failed");
    if (rc) {
        free_batch_mem(b);
        delete b;
        return rc;
    }
    *out = b;
    return ART_OK;
}

int art_render_spectral(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                        const art_refine* rf, const art_transfer* tr, const art_spectral* spec, art_image* out,
                        art_stats* st, void* stream)
{
    if (!sp || !cam || !em || !rf || !tr || !spec || !out) return fail(ART_EINVAL, "null argument");
    const int n0 = spec->n0, L = spec->levels;
    if (n0 < 2 || L < 0 || L > 6) return fail(ART_EINVAL, "spectral cube needs n0 >= 2 and 0 <= levels <= 6");
    const long long n = ((long long)(n0 - 1) << L) + 1;
    if (n > kMaxBatch) return fail(ART_EINVAL, "spectral cube of %lld images (limit %d)", n, kMaxBatch);
    if (!(spec->nu_min_hz > 0.0) || !(spec->nu_max_hz > spec->nu_min_hz) || !std::isfinite(spec->nu_max_hz))
        return fail(ART_EINVAL, "spectral cube needs 0 < nu_min < nu_max (finite)");
    std::vector<art_job> jobs((size_t)n);
    for (int i = 0; i < (int)n; ++i) {
        art_emission e = *em;
        e.freq_hz = spec->nu_min_hz * std::pow(spec->nu_max_hz / spec->nu_min_hz, (double)i / (double)(n - 1));
        jobs[i] = make_job(sp, cam, &e, rf, tr);
    }
    return art_render_cube((int32_t)n, jobs.data(), n0, L, spec->r_rel, spec->r_abs, out, st, stream);
}

int art_render_uniform(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_transfer* tr, art_image* out, art_stats* st, void* stream)
{
    if (!sp || !cam || !em || !tr || !out) return fail(ART_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_single_mu);
    art_batch* b = single_batch();
    if (!b) return fail(ART_EDEVICE, "no current device");
    hipStream_t s = (hipStream_t)stream;
    const art_job j = make_job(sp, cam, em, nullptr, tr);
    int rc = prepare(b, 1, &j, out, true, s);
    if (rc) return rc;
    b->timing = st != nullptr;
    rc = enqueue_uniform(b, s);
    if (rc) return rc;
    if (st) return batch_stats(b, 0, st, s);
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
    std::lock_guard<std::mutex> lk(g_single_mu);
    art_batch* b = single_batch();
    if (!b) return fail(ART_EDEVICE, "no current device");
    hipStream_t s = (hipStream_t)stream;
    rc = ensure_mem(b, 0);
    if (rc) return rc;
    b->n = 1;
    b->ngroups = 1;
    b->grp[0].i0 = 0;
    b->grp[0].n = 1;
    b->grp[0].list_off = 0;
    b->hP.resize(1);
    make_params(sp, cam, em, tr, 0, 0, b->hP[0]);
    b->L = launch_cfg(b->cus, tr->precision, em->kind, tr->nstokes, tr->subrings > 0);
    if (em->kind == ART_EMIS_GRID) {
        const int n2 = (int)em->params[10];
        theta_table(em->params[8], n2, b->hTh);
        HIP_TRY(hipMemcpyAsync(b->dTh, b->hTh, sizeof(double) * n2, hipMemcpyHostToDevice, s));
        b->hP[0].theta_tab = b->dTh;
    }
    HIP_TRY(hipMemcpyAsync(b->dP, b->hP.data(), sizeof(Params), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u32((uint32_t*)b->ctr, sizeof(Counters) / 4, 0u, s));
    HIP_TRY(launch_fill_u32(&b->ctr->count[0], 1, (uint32_t)n, s));
    TraceJob J = base_job(b, 0, 0);
    J.src = SRC_POINTS;
    J.list = nullptr;
    J.alpha = alpha_dev;
    J.beta = beta_dev;
    J.out = stokes_dev;
    J.feat = (RayFeat*)feat_dev;
    HIP_TRY(launch_trace(tr->precision, em->kind, tr->nstokes, tr->subrings > 0, J, b->L, s));
    return ART_OK;
}

int art_batch_create(int32_t n, const art_job* jobs, const art_image* images, art_batch** out)
{
    if (!out) return fail(ART_EINVAL, "NULL output handle");
    *out = nullptr;
    art_batch* b = new (std::nothrow) art_batch();
    if (!b) return fail(ART_ENOMEM, "out of host memory");
    int rc = prepare(b, n, jobs, images, false, nullptr);
    if (rc == ART_OK && hipStreamSynchronize(nullptr) != hipSuccess) rc = fail(ART_EDEVICE, "upload failed");
    if (rc) {
        free_batch_mem(b);
        delete b;
        return rc;
    }
    *out = b;
    return ART_OK;
}

int art_batch_render(art_batch* b, void* stream)
{
    if (!b) return fail(ART_EINVAL, "NULL batch");
    b->timing = true;
    return enqueue_render(b, (hipStream_t)stream);
}

int art_batch_capture(art_batch* b, void* stream)
{
    if (!b) return fail(ART_EINVAL, "NULL batch");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(ART_EINVAL, "graph capture needs a non-default stream");
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->timing = false;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_render(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(ART_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_ntrace = b->ntrace;
    return ART_OK;
}

int art_batch_launch(art_batch* b, void* stream)
{
    if (!b) return fail(ART_EINVAL, "NULL batch");
    if (!b->gexec) return fail(ART_EINVAL, "batch has no captured graph (call art_batch_capture)");
    for (int g = 0; g < b->ngroups; ++g) b->grp[g].nev = 0;
    b->render_timed = false;
    b->ntrace = b->graph_ntrace;
    HIP_TRY(hipGraphLaunch(b->gexec, (hipStream_t)stream));
    return ART_OK;
}

int art_batch_set_learned(art_batch* b, art_cnn* net, const art_learned* opt)
{
    if (!b) return fail(ART_EINVAL, "NULL batch");
    if (net && b->cube_levels >= 0) return fail(ART_EINVAL, "axis-sampled cubes render with the criterion only");
    return setup_learned(b, net, opt);
}

int art_batch_stats(art_batch* b, int32_t i, art_stats* st, void* stream)
{
    if (!b || !st) return fail(ART_EINVAL, "NULL argument");
    if (i >= b->n) return fail(ART_EINVAL, "image index %d outside batch of %d", i, b->n);
    const int k = (i >= 0 && b->cube_levels >= 0) ? b->cube_inv[i] : i;   // cubes: axis order
    return batch_stats(b, k, st, (hipStream_t)stream);
}

int art_batch_destroy(art_batch* b)
{
    if (!b) return ART_OK;
    (void)hipDeviceSynchronize();
    free_batch_mem(b);
    delete b;
    return ART_OK;
}

int art_set_alloc_limit(size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_list_limit = bytes;
    return ART_OK;
}

int art_set_launch(const art_launch* L)
{
    if (!L) return fail(ART_EINVAL, "NULL launch configuration");
    if (L->trace_threads != 0 && L->trace_threads != 64 && L->trace_threads != 128 && L->trace_threads != 256)
        return fail(ART_EINVAL, "trace_threads must be 0, 64, 128 or 256");
    if (L->trace_blocks < 0 || L->refine_blocks < 0 || L->refill < 0 || L->refill > 64)
        return fail(ART_EINVAL, "trace_blocks >= 0, refine_blocks >= 0 and 0 <= refill <= 64 required");
    if (L->long_steps < 0 || L->long_steps > 65535) return fail(ART_EINVAL, "long_steps must be in 0..65535");
    if (L->groups < 0 || L->groups > kMaxGroups) return fail(ART_EINVAL, "groups must be in 0..%d", kMaxGroups);
    std::lock_guard<std::mutex> lk(g_mu);
    g_launch = *L;
    return ART_OK;
}

int art_batch_set_launch(art_batch* b, const art_launch* L)
{
    if (!b || !L) return fail(ART_EINVAL, "NULL argument");
    if (L->trace_threads != 0 && L->trace_threads != 64 && L->trace_threads != 128 && L->trace_threads != 256)
        return fail(ART_EINVAL, "trace_threads must be 0, 64, 128 or 256");
    if (L->trace_blocks < 0 || L->refine_blocks < 0 || L->refill < 0 || L->refill > 64)
        return fail(ART_EINVAL, "trace_blocks >= 0, refine_blocks >= 0 and 0 <= refill <= 64 required");
    if (L->long_steps < 0 || L->long_steps > 65535) return fail(ART_EINVAL, "long_steps must be in 0..65535");
    if (L->groups < 0 || L->groups > kMaxGroups) return fail(ART_EINVAL, "groups must be in 0..%d", kMaxGroups);
    const LaunchCfg d = launch_cfg(b->cus, b->precision, b->model, b->nstokes, b->nsub > 0);
    b->L.trace_threads = L->trace_threads ? L->trace_threads : d.trace_threads;
    b->L.trace_blocks = L->trace_blocks ? L->trace_blocks : d.trace_blocks;
    b->L.refine_blocks = L->refine_blocks ? L->refine_blocks : b->L.trace_blocks;
    b->L.refill = L->refill ? L->refill : d.refill;
    b->L.long_steps = L->long_steps ? L->long_steps : d.long_steps;
    if (L->groups != b->req_groups) {
        // a new split of the images: new descriptors, and a captured graph is stale
        HIP_TRY(hipDeviceSynchronize());
        if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        b->req_groups = L->groups;
        int rc = layout(b, nullptr);
        if (rc) return rc;
        if (b->net) {
            const art_learned o = b->lopt;
            rc = setup_learned(b, b->net, &o);
            if (rc) return rc;
        }
        HIP_TRY(hipStreamSynchronize(nullptr));
    }
    return ART_OK;
}

int art_batch_get_launch(const art_batch* b, art_launch* L)
{
    if (!b || !L) return fail(ART_EINVAL, "NULL argument");
    L->trace_blocks = b->L.trace_blocks;
    L->refine_blocks = b->L.refine_blocks;
    L->long_steps = b->L.long_steps;
    L->trace_threads = b->L.trace_threads;
    L->refill = b->L.refill;
    L->groups = b->ngroups;
    return ART_OK;
}

int art_get_launch(int32_t precision, int32_t kind, int32_t nstokes, art_launch* L)
{
    if (!L) return fail(ART_EINVAL, "NULL launch configuration");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const LaunchCfg c = launch_cfg(cus, precision, kind, nstokes);
    L->trace_blocks = c.trace_blocks;
    L->refine_blocks = c.refine_blocks;
    L->long_steps = c.long_steps;
    L->trace_threads = c.trace_threads;
    L->refill = c.refill;
    L->groups = 0;
    return ART_OK;
}

int art_metrics(const double* truth_dev, const double* approx_dev, int64_t n, double* flux_error,
                double* mse, void* stream)
{
    if (!truth_dev || !approx_dev) return fail(ART_EINVAL, "NULL image");
    if (n <= 0) return fail(ART_EINVAL, "empty image");
    hipStream_t s = (hipStream_t)stream;
    static double* partial[64] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(ART_EDEVICE, "device index out of range");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!partial[dev] && hipMalloc(&partial[dev], sizeof(double) * (1024 * 4 + 4)) != hipSuccess)
            return fail(ART_ENOMEM, "hipMalloc(partials) failed");
    }
    const int nb = 1024;
    HIP_TRY(launch_metrics(truth_dev, approx_dev, n, partial[dev], nb, s));
    double h[4];
    HIP_TRY(hipMemcpyAsync(h, partial[dev] + nb * 4, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flux_error) *flux_error = std::fabs(h[0] - h[1]) / std::fabs(h[0]);
    if (mse) *mse = h[2] / h[3];
    return ART_OK;
}

int art_stream_create(void** stream)
{
    if (!stream) return fail(ART_EINVAL, "NULL stream pointer");
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *stream = (void*)s;
    return ART_OK;
}

int art_stream_destroy(void* stream)
{
    if (!stream) return fail(ART_EINVAL, "NULL stream");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipStreamDestroy((hipStream_t)stream));
    return ART_OK;
}

int art_release(void)
{
    std::lock_guard<std::mutex> lk(g_single_mu);
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    for (int d = 0; d < 64; ++d) {
        art_batch& b = g_single[d];
        if (!b.ctr && !b.list) continue;
        HIP_TRY(hipSetDevice(d));
        HIP_TRY(hipDeviceSynchronize());
        free_batch_mem(&b);
    }
    HIP_TRY(hipSetDevice(cur));
    return ART_OK;
}

}  // extern "C"
