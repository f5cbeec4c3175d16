// art_vis.hip -- visibilities of screen images (Sec. 4.3): the Fourier pixel
// sum over a rectangle of baselines, evaluated as two real contractions on the
// FP64 matrix cores, plus the C ABI of the operation.
//
// V(u_m, v_l) = dx^2 sum_j sum_i g(x_i) g(y_j) I[j][i] exp(-2 pi i (u_m x_i + v_l y_j))
//
// is separable: one stage sums along one image axis for every frequency of that
// axis (a real matrix product of the image with a generated cosine/sine
// matrix), the next stage sums the intermediate along the other axis, and a
// small kernel combines the real products into complex visibilities.  The
// twiddle operand is never stored: each workgroup generates its (k, frequency)
// tile in LDS from the pixel coordinate and the frequency, with the Gaussian
// taper folded in.  The order of the two stages is chosen so the long stage
// runs over the shorter frequency list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/art.h"

namespace art {
int api_fail(int code, const char* fmt, ...);
}

namespace art {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64;          // rows per workgroup tile
constexpr int kTN = 64;          // real columns per tile (32 frequencies x {cos, -sin})
constexpr int kResync = 32;      // chunks between exact twiddle evaluations
constexpr int kKC = 16;          // sum-axis chunk staged in LDS (a multiple of 16)
constexpr int kThreads = 256;    // 4 waves, each a 32 x 32 block of the tile
constexpr int kNumXcd = 8;       // accelerator dies sharing the dispatch round robin
constexpr int kMaxFreq = 1 << 20;
constexpr int kMaxAxis = 1 << 24;

// One stage: D(z, row, 2m + s) = sum_k A(z, row, k) B(k, 2m + s) with
// B(k, 2m) = g_k cos(2 pi f_m t_k), B(k, 2m + 1) = -g_k sin(2 pi f_m t_k),
// t_k = (k - (K - 1) / 2) dx and the taper g_k = exp(-4 ln 2 t_k^2 / FWHM^2).
struct VisStage {
    const double* A;
    long long a_rs, a_ks, a_zs;   // A(z, row, k) = A[z a_zs + row a_rs + k a_ks]
    int M, K, nf;                 // rows, sum length, frequencies (2 nf columns)
    const double* f;              // frequencies, cycles per unit of the sum axis
    double dx;                    // sum-axis pixel size
    const double* g;              // taper factors g_k of the sum axis [K]
    double* D;
    long long ldd, d_zs;          // D(z, row, col) = D[z d_zs + row ldd + col]
    int gx;                       // column tiles (the grid is gx x row tiles, flattened)
};

// Workgroup tile order: consecutive tiles of one row band go to the same die
// so its L2 serves the band's image rows to every column tile.
__device__ __forceinline__ void tile_of_block(int gx, int& rt, int& ct)
{
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int q = nb / kNumXcd, r = nb % kNumXcd;
    const int x = b % kNumXcd, loc = b / kNumXcd;
    const int lb = x * q + (x < r ? x : r) + loc;
    ct = lb % gx;
    rt = lb / gx;
}

template <bool KCONT, int TN>
__global__ __launch_bounds__(kThreads) void k_vis_stage(VisStage p)
{
    constexpr int NF = TN / 2;          // frequencies per tile
    constexpr int NE = NF / 16;         // twiddle columns per thread
    constexpr int WB = TN / 32;         // 16-wide column blocks per wave
    __shared__ double As[2][kKC][kTM + 1];
    __shared__ double Bs[2][kKC][TN];
    int rt, ct;
    tile_of_block(p.gx, rt, ct);
    const int row0 = rt * kTM, col0 = ct * TN, m0 = col0 >> 1;
    const double* A = p.A + (long long)blockIdx.z * p.a_zs;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int N = 2 * p.nf;
    const double kc = 0.5 * (double)(p.K - 1);

    // staging roles: A elements (kk_a + 16 h, row_a + 16 i), twiddles (kk_b + 16 h, m_b + 16 e)
    constexpr int KH = kKC / 16;
    const int kk_a = KCONT ? (t & 15) : (t >> 4);
    const int row_a = KCONT ? (t >> 4) : (t & 15);
    const int kk_b = t >> 4, m_b = t & 15;
    // twiddle of (k, m) as a phasor exp(-2 pi i f_m t_k) advanced one chunk at
    // a time by the rotation exp(-2 pi i f_m KC dx), recomputed exactly every
    // kResync chunks so rounding cannot accumulate
    double fb[NE], rr[NE], ri[NE], pr[KH][NE], pim[KH][NE];
    for (int e = 0; e < NE; ++e) {
        const int m = m0 + m_b + 16 * e;
        fb[e] = m < p.nf ? p.f[m] : 0.0;
        double a = fb[e] * (kKC * p.dx);
        a -= rint(a);
        double sn, cs;
        sincospi(2.0 * a, &sn, &cs);
        rr[e] = cs;
        ri[e] = -sn;
        for (int h = 0; h < KH; ++h) {
            pr[h][e] = 1.0;
            pim[h][e] = 0.0;
        }
    }
    double ra[KH][4], rb[KH][2 * NE];

    auto load = [&](int c) {
        for (int h = 0; h < KH; ++h) {
            const int k = c * kKC + 16 * h + kk_a;
            for (int i = 0; i < 4; ++i) {
                const int row = row0 + row_a + 16 * i;
                ra[h][i] = (row < p.M && k < p.K) ? A[(long long)row * p.a_rs + (long long)k * p.a_ks] : 0.0;
            }
        }
        for (int h = 0; h < KH; ++h) {
            const int kb = c * kKC + 16 * h + kk_b;
            const double g = kb < p.K ? p.g[kb] : 0.0;
            if (c % kResync == 0) {
                const double tk = ((double)kb - kc) * p.dx;
                for (int e = 0; e < NE; ++e) {
                    double a = fb[e] * tk;      // phase in cycles, reduced to [-1/2, 1/2]
                    a -= rint(a);
                    double sn, cs;
                    sincospi(2.0 * a, &sn, &cs);
                    pr[h][e] = cs;
                    pim[h][e] = -sn;
                }
            } else {
                for (int e = 0; e < NE; ++e) {
                    const double x = pr[h][e] * rr[e] - pim[h][e] * ri[e];
                    pim[h][e] = pr[h][e] * ri[e] + pim[h][e] * rr[e];
                    pr[h][e] = x;
                }
            }
            for (int e = 0; e < NE; ++e) {
                const bool ok = m0 + m_b + 16 * e < p.nf;
                rb[h][2 * e] = ok ? g * pr[h][e] : 0.0;
                rb[h][2 * e + 1] = ok ? g * pim[h][e] : 0.0;
            }
        }
    };
    auto store = [&](int buf) {
        for (int h = 0; h < KH; ++h) {
            for (int i = 0; i < 4; ++i) As[buf][16 * h + kk_a][row_a + 16 * i] = ra[h][i];
            for (int e = 0; e < NE; ++e) {
                Bs[buf][16 * h + kk_b][2 * (m_b + 16 * e)] = rb[h][2 * e];
                Bs[buf][16 * h + kk_b][2 * (m_b + 16 * e) + 1] = rb[h][2 * e + 1];
            }
        }
    };

    d4 acc[2][WB];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < WB; ++b) acc[a][b] = d4{ 0.0, 0.0, 0.0, 0.0 };
    const int wr = (w >> 1) * 32, wc = (w & 1) * (TN / 2);
    const int nchunk = (p.K + kKC - 1) / kKC;
    if (nchunk > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) load(c + 1);
        for (int ks = 0; ks < kKC / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            const double a0 = As[buf][kr][wr + (lane & 15)];
            const double a1 = As[buf][kr][wr + 16 + (lane & 15)];
            for (int b = 0; b < WB; ++b) {
                const double bv = Bs[buf][kr][wc + 16 * b + (lane & 15)];
                acc[0][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc[0][b], 0, 0, 0);
                acc[1][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc[1][b], 0, 0, 0);
            }
        }
        if (c + 1 < nchunk) store(buf ^ 1);
        __syncthreads();
    }
    // accumulator element j of lane l: row l / 16 + 4 j, column l % 16 of its 16 x 16 block
    double* D = p.D + (long long)blockIdx.z * p.d_zs;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < WB; ++b) {
            const int col = col0 + wc + 16 * b + (lane & 15);
            if (col >= N) continue;
            for (int j = 0; j < 4; ++j) {
                const int row = row0 + wr + 16 * a + (lane >> 4) + 4 * j;
                if (row < p.M) D[(long long)row * p.ldd + col] = acc[a][b][j];
            }
        }
}

// Taper factors g_k = exp(-tc t_k^2) of one image axis (1 without a taper).
__global__ void k_vis_taper(double* g, int n, double dx, double tc)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double t = ((double)k - 0.5 * (double)(n - 1)) * dx;
    g[k] = tc > 0.0 ? exp(-tc * t * t) : 1.0;
}

// V from the second stage's products R(c, col), c = 2 a + s over the first
// stage's frequencies a and col = 2 b + s' over the second's b:
//   Re V = R(2a, 2b) - R(2a+1, 2b+1),  Im V = R(2a+1, 2b) + R(2a, 2b+1).
// Output V[z][l][m] = (Re, Im) with l over v and m over u.
__global__ void k_vis_combine(const double* R, long long z_r, int nA, int nB, int a_is_u, double scale,
                              double* V, int nu, int nv, int P)
{
    const long long n = (long long)P * nA * nB;
    const long long ld = 2LL * nB;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(idx / ((long long)nA * nB));
        const long long rem = idx % ((long long)nA * nB);
        const int a = (int)(rem / nB), b = (int)(rem % nB);
        const double* r = R + z * z_r;
        const double re = r[(2LL * a) * ld + 2 * b] - r[(2LL * a + 1) * ld + 2 * b + 1];
        const double im = r[(2LL * a + 1) * ld + 2 * b] + r[(2LL * a) * ld + 2 * b + 1];
        const int l = a_is_u ? b : a, m = a_is_u ? a : b;
        double* o = V + 2 * (((long long)z * nv + l) * nu + m);
        o[0] = scale * re;
        o[1] = scale * im;
    }
}

bool rows_first(long long nx, long long ny, long long nu, long long nv)
{
    const double cost_rows = (double)ny * nx * nu + (double)nu * ny * nv;
    const double cost_cols = (double)nx * ny * nv + (double)nv * nx * nu;
    return cost_rows <= cost_cols;
}

size_t workspace_doubles(long long P, long long nx, long long ny, long long nu, long long nv)
{
    const long long tapers = nx + ny;
    if (rows_first(nx, ny, nu, nv)) return (size_t)(P * (ny * 2 * nu + 4 * nu * nv) + tapers);
    return (size_t)(P * (nx * 2 * nv + 4 * nv * nu) + tapers);
}

// Tile width: 32 frequencies per tile.  Wider tiles (64) halve the re-reads
// of the image rows but need 172 VGPRs, and the lower occupancy costs more
// than the reads save (28.6 vs 24.8 ms for the 16385^2 window on one MI355X).
int tile_cols(int) { return kTN; }

long long stage_tiles(int M, int nf)
{
    const int tn = tile_cols(nf);
    return (long long)((2LL * nf + tn - 1) / tn) * ((M + kTM - 1) / kTM);
}

hipError_t launch_stage(VisStage p, int P, hipStream_t s)
{
    if (p.M <= 0 || p.nf <= 0 || P <= 0) return hipSuccess;
    const int tn = tile_cols(p.nf);
    p.gx = (2 * p.nf + tn - 1) / tn;
    const dim3 grid((unsigned)stage_tiles(p.M, p.nf), 1, P);
    if (p.a_ks == 1)
        k_vis_stage<true, kTN><<<grid, kThreads, 0, s>>>(p);
    else
        k_vis_stage<false, kTN><<<grid, kThreads, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace
}  // namespace art

using namespace art;

extern "C" {

size_t art_vis_workspace_bytes(int32_t nplanes, int32_t nx, int32_t ny, int32_t nu, int32_t nv)
{
    if (nplanes <= 0 || nx < 0 || ny < 0 || nu <= 0 || nv <= 0) return 0;
    return sizeof(double) * workspace_doubles(nplanes, nx, ny, nu, nv);
}

int art_visibility(const double* img_dev, int64_t plane_stride, int32_t nplanes, int32_t nx, int32_t ny,
                   double dx, double fwhm, const double* u_dev, int32_t nu, const double* v_dev, int32_t nv,
                   double* vis_dev, void* work_dev, size_t work_bytes, void* stream)
{
    if (nplanes < 0 || nx < 0 || ny < 0 || nu < 0 || nv < 0)
        return api_fail(ART_EINVAL, "negative size (planes %d, image %d x %d, baselines %d x %d)", nplanes, nx,
                        ny, nu, nv);
    if (nx > kMaxAxis || ny > kMaxAxis || nu > kMaxFreq || nv > kMaxFreq || nplanes > 65535)
        return api_fail(ART_EINVAL, "size out of range (image axes <= 2^24, baselines <= 2^20 per axis, "
                                    "planes <= 65535)");
    if (!(dx > 0.0) || !std::isfinite(dx)) return api_fail(ART_EINVAL, "pixel size must be finite and > 0");
    if (!std::isfinite(fwhm)) return api_fail(ART_EINVAL, "taper FWHM must be finite (<= 0: no taper)");
    if (nplanes == 0 || nu == 0 || nv == 0) return ART_OK;
    if (!vis_dev || !u_dev || !v_dev) return api_fail(ART_EINVAL, "NULL baseline or output pointer");
    const long long npix = (long long)nx * ny;
    if (npix > 0 && !img_dev) return api_fail(ART_EINVAL, "NULL image pointer");
    if (nplanes > 1 && plane_stride < npix)
        return api_fail(ART_EINVAL, "plane stride %lld smaller than nx * ny = %lld", (long long)plane_stride,
                        npix);
    const size_t need = art_vis_workspace_bytes(nplanes, nx, ny, nu, nv);
    if (!work_dev || work_bytes < need)
        return api_fail(ART_EINVAL, "workspace of %zu bytes too small (need %zu)", work_bytes, need);

    hipStream_t s = (hipStream_t)stream;
    const double tc = fwhm > 0.0 ? 4.0 * std::log(2.0) / (fwhm * fwhm) : 0.0;
    double* ws = (double*)work_dev;
    const bool rf = rows_first(nx, ny, nu, nv);
    // first stage: along x for u (rows first) or along y for v (columns first)
    const int nA = rf ? nu : nv, nB = rf ? nv : nu;
    const int M1 = rf ? ny : nx;
    if (stage_tiles(M1, nA) >= (1LL << 31) || stage_tiles(2 * nA, nB) >= (1LL << 31))
        return api_fail(ART_EINVAL, "too many tiles for one launch (image axis x baselines too large)");
    double* T = ws;
    double* R = ws + (size_t)nplanes * M1 * 2 * nA;
    double* gx = R + (size_t)nplanes * 4 * nA * nB;     // taper factors along x, then y
    double* gy = gx + nx;
    VisStage a{};
    a.A = img_dev;
    a.a_rs = rf ? nx : 1;
    a.a_ks = rf ? 1 : nx;
    a.a_zs = plane_stride;
    a.M = M1;
    a.K = rf ? nx : ny;
    a.nf = nA;
    a.f = rf ? u_dev : v_dev;
    a.dx = dx;
    a.g = rf ? gx : gy;
    a.D = T;
    a.ldd = 2LL * nA;
    a.d_zs = (long long)M1 * 2 * nA;
    VisStage b{};
    b.A = T;
    b.a_rs = 1;
    b.a_ks = 2LL * nA;
    b.a_zs = (long long)M1 * 2 * nA;
    b.M = 2 * nA;
    b.K = M1;
    b.nf = nB;
    b.f = rf ? v_dev : u_dev;
    b.dx = dx;
    b.g = rf ? gy : gx;
    b.D = R;
    b.ldd = 2LL * nB;
    b.d_zs = 4LL * nA * nB;
    hipError_t e = hipSuccess;
    if (nx > 0) {
        k_vis_taper<<<(nx + 255) / 256, 256, 0, s>>>(gx, nx, dx, tc);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ny > 0) {
        k_vis_taper<<<(ny + 255) / 256, 256, 0, s>>>(gy, ny, dx, tc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_stage(a, nplanes, s);
    if (e == hipSuccess) e = launch_stage(b, nplanes, s);
    if (e == hipSuccess) {
        const long long n = (long long)nplanes * nA * nB;
        const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
        k_vis_combine<<<blocks, 256, 0, s>>>(R, b.d_zs, nA, nB, rf ? 1 : 0, dx * dx, vis_dev, nu, nv, nplanes);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return api_fail(ART_EDEVICE, "visibility launch failed: %s", hipGetErrorString(e));
    return ART_OK;
}

}  // extern "C"
