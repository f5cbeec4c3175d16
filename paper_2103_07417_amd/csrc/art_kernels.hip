// art_kernels.hip -- gfx950 kernels of the adaptive ray tracer.
//
//   (the persistent tracer k_trace lives in art_trace.hip)
//   k_base_list  the level-0 work items of every image.
//   k_estimate   one refinement level (Sec. 3.2): category from index parity,
//                neighbour/continuation sums, the linear-branch estimates of
//                Eqs. 5-6 evaluated without division, interpolation, and
//                wavefront-ballot compaction of the points to trace.
//   k_reduce_base  trapezoid mean and maximum of the level-0 image (Ibar_int,
//                Sec. 3.2 after Eq. 6), one block, fixed summation order.
//   k_spectral_base  base points of the time / frequency axis levels of a
//                cube (Sec. 6 extension of the one-axis rule of Sec. 3.2).
//   k_metrics_*  flux error and normalised MSE (Sec. 4.1, Eqs. 8-9),
//                deterministic two-pass reduction.
#include "art_internal.hpp"
#include "art_cnn.hpp"

namespace art {

// ---------------------------------------------------------------- fill kernels
__global__ void k_fill_u32(uint32_t* p, long long n, uint32_t v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i8(int8_t* p, long long n, int8_t v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_blocks(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i8(int8_t* p, long long n, int8_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i8, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------ base-grid list
// grid (x: base points, y: image).  Base points within kFrontRadius (in M) of
// the screen centre, where the critical curve of every Kerr spin and view
// lies, are queued at the front of the list, the others from its back: the
// photon-ring rays, the longest of the pass, start first instead of wherever
// their image falls in the batch, so the pass does not end on a late one.
// The order changes no result.  List slots are reserved once per block.
constexpr double kFrontRadius = 8.0;
constexpr int kBaseThreads = 256;

__global__ __launch_bounds__(kBaseThreads) void k_base_list(const ImageDesc* desc, const Params* params,
                                                            unsigned long long* list, long long cap,
                                                            Counters* ctr, int slot)
{
    constexpr int kWaves = kBaseThreads / 64;
    __shared__ unsigned s_cnt[2][kWaves];
    __shared__ unsigned s_base[2];
    const int img = blockIdx.y;
    const ImageDesc D = desc[img];
    const double x0 = params[img].x0, y0 = params[img].y0, dx = params[img].dx;
    const int n = D.nx0 * D.ny0;
    const int st0 = 1 << D.levels;
    const int wave = threadIdx.x >> 6;
    // block-uniform trip count: every lane takes part in the ballots and barriers
    for (int t0 = blockIdx.x * kBaseThreads; t0 < n; t0 += gridDim.x * kBaseThreads) {
        const int t = t0 + threadIdx.x;
        const bool valid = t < n;
        bool front = false;
        uint32_t pix = 0;
        if (valid) {
            const int i = t % D.nx0, j = t / D.nx0;
            pix = (uint32_t)(j * st0) * (uint32_t)D.nx + (uint32_t)(i * st0);
            const double al = x0 + (double)(i * st0) * dx, be = y0 + (double)(j * st0) * dx;
            front = al * al + be * be <= kFrontRadius * kFrontRadius;
            if (D.level) D.level[pix] = 0;
        }
        const unsigned long long mf = __ballot(valid && front), mb = __ballot(valid && !front);
        if (__lane_id() == 0) {
            s_cnt[0][wave] = (unsigned)__popcll(mf);
            s_cnt[1][wave] = (unsigned)__popcll(mb);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned nf = 0, nb = 0;
            for (int w = 0; w < kWaves; ++w) { nf += s_cnt[0][w]; nb += s_cnt[1][w]; }
            s_base[0] = nf ? atomicAdd(&ctr->count[slot], nf) : 0u;
            s_base[1] = nb ? atomicAdd(&ctr->count_back[slot], nb) : 0u;
        }
        __syncthreads();
        unsigned of = s_base[0], ob = s_base[1];
        for (int w = 0; w < wave; ++w) { of += s_cnt[0][w]; ob += s_cnt[1][w]; }
        const unsigned long long item = make_item((uint32_t)img, pix);
        if (valid && front) list[of + lane_prefix(mf)] = item;
        if (valid && !front) list[cap - 1 - (long long)(ob + lane_prefix(mb))] = item;
        __syncthreads();                       // s_cnt and s_base are reused
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->img_traced[img][0] = (uint32_t)n;
}

hipError_t launch_base_list(const ImageDesc* desc, const Params* params, int nimg, int max_base,
                            unsigned long long* list, long long cap, Counters* ctr, int slot, hipStream_t s)
{
    if (nimg <= 0) return hipSuccess;
    int bx = (max_base + kBaseThreads - 1) / kBaseThreads;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_base_list, dim3(bx, nimg), dim3(kBaseThreads), 0, s, desc, params, list, cap, ctr,
                       slot);
    return hipGetLastError();
}

// ------------------------------------------------------ level-0 reduction
// One block per image: trapezoid-weighted mean and maximum of the base grid
// (Stokes I; with kRefineOwnNorm also of |plane| for every further plane, each
// plane's own N_abs).  Four waves per block (not sixteen), so that a batch's
// reduction fits into the wave slots the tracing launches of other batches in
// flight leave free.
__global__ __launch_bounds__(256) void k_reduce_base(const ImageDesc* desc, Counters* ctr, int img_off)
{
    __shared__ double ssum[256];
    __shared__ double smax[256];
    const int img = img_off + blockIdx.x;
    const ImageDesc D = desc[img];
    const int t = threadIdx.x;
    const int st0 = 1 << D.levels;
    const int n = D.nx0 * D.ny0;
    const int nplanes = (D.flags & kRefineOwnNorm) ? D.nplanes : 1;      // uniform over the block
    for (int pl = 0; pl < nplanes; ++pl) {
        const double* P = D.img + (long long)pl * D.plane;
        double sum = 0.0, mx = -HUGE_VAL;
        for (int k = t; k < n; k += 256) {
            const int i = k % D.nx0, j = k / D.nx0;
            const double v0 = P[(long long)(j * st0) * D.nx + (long long)(i * st0)];
            const double v = pl == 0 ? v0 : ::fabs(v0);
            const double wx = (i == 0 || i == D.nx0 - 1) ? 0.5 : 1.0;
            const double wy = (j == 0 || j == D.ny0 - 1) ? 0.5 : 1.0;
            sum += (wy * wx) * v;
            mx = v > mx ? v : mx;
        }
        ssum[t] = sum;
        smax[t] = mx;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (t < off) {
                ssum[t] += ssum[t + off];
                smax[t] = smax[t + off] > smax[t] ? smax[t + off] : smax[t];
            }
            __syncthreads();
        }
        if (t == 0) {
            const double mean = ssum[0] / ((double)(D.nx0 - 1) * (double)(D.ny0 - 1));
            const double na = D.abs_norm == 0 ? mean : smax[0];
            if (pl == 0) {
                ctr->scal[img][0] = mean;
                ctr->scal[img][1] = smax[0];
                ctr->scal[img][2] = na;
            }
            ctr->nabs_plane[img][pl] = na;
        }
        __syncthreads();                      // the shared sums are reused by the next plane
    }
}

hipError_t launch_reduce_base(const ImageDesc* desc, int nimg, Counters* ctr, hipStream_t s, int img_off)
{
    hipLaunchKernelGGL(k_reduce_base, dim3(nimg), dim3(256), 0, s, desc, ctr, img_off);
    return hipGetLastError();
}

// ------------------------------------------------------ spectral cube
// The one-axis rule of Sec. 3.2 along ln nu at pixel pix of a spectral-level
// image: with the bracketing images b, c and the continuations a, d (finished
// coarser levels), D = (a + d) - (b + c), twice the one-sided second
// difference if one continuation is outside the cube, no estimate (trace) if
// both are; the spectral value (b + c)/2 is accepted unless |D| > 8 R_abs N_abs
// and |D| > 4 R_rel |b + c|, N_abs the mean of b's and c's own N_abs (every
// plane with the per-plane option).
__device__ bool spectral_ok(const ImageDesc* desc, const ImageDesc& D, long long pix, const Counters* ctr)
{
    if (D.sa < 0 && D.sd < 0) return false;
    const double* Ib = desc[D.sb].img;
    const double* Ic = desc[D.sc].img;
    const double* Ia = D.sa >= 0 ? desc[D.sa].img : nullptr;
    const double* Id = D.sd >= 0 ? desc[D.sd].img : nullptr;
    const double nabs = 0.5 * (ctr->scal[D.sb][2] + ctr->scal[D.sc][2]);
    const double thrA = 8.0 * D.sr_abs * nabs;
    const double crel = 4.0 * D.sr_rel;
    const double S0 = Ib[pix] + Ic[pix];
    if (!(S0 == S0)) return false;
    const double aS = ::fabs(S0);
    const int np = (D.flags & kRefineAllPlanes) ? D.nplanes : 1;
    for (int st = 0; st < np; ++st) {
        const long long o = st * D.plane + pix;
        const double b = Ib[o], c = Ic[o];
        double Dv;
        if (Ia && Id)
            Dv = (Ia[o] + Id[o]) - (b + c);
        else if (Id)
            Dv = 2.0 * ((Id[o] - 2.0 * c) + b);
        else
            Dv = 2.0 * ((Ia[o] - 2.0 * b) + c);
        const double aD = ::fabs(Dv);
        if (!(Dv == Dv) || (aD > thrA && aD > crel * aS)) return false;
    }
    return true;
}

// Spectral value at pix: (b + c)/2 on every plane; features from b and c
// (smallest radius, largest crossing count); the costlier neighbour's cost.
__device__ void spectral_write(const ImageDesc* desc, const ImageDesc& D, long long pix)
{
    const ImageDesc& B = desc[D.sb];
    const ImageDesc& C = desc[D.sc];
    for (int st = 0; st < D.nplanes; ++st) {
        const long long o = st * D.plane + pix;
        D.img[o] = (B.img[o] + C.img[o]) * 0.5;
    }
    D.level[pix] = kMarkSpectral;
    if (D.feat && B.feat && C.feat) {
        RayFeat f = B.feat[pix];
        const RayFeat g = C.feat[pix];
        f.rmin = g.rmin < f.rmin ? g.rmin : f.rmin;
        f.ncross = g.ncross > f.ncross ? g.ncross : f.ncross;
        f.steps = 0;
        f.status = RAY_OK;
        D.feat[pix] = f;
    }
    if (D.cost) {
        const uint16_t cb = B.cost[pix], cc = C.cost[pix];
        D.cost[pix] = cb > cc ? cb : cc;
    }
}

// grid (x: base points, y: image).  Base points of spectral-level images.
__global__ __launch_bounds__(256) void k_spectral_base(const ImageDesc* desc, int img_off, Counters* ctr,
                                                       unsigned long long* list, long long cap, int long_steps,
                                                       int slot)
{
    const int img = img_off + blockIdx.y;
    const ImageDesc D = desc[img];
    const int n = D.nx0 * D.ny0;
    const int st0 = 1 << D.levels;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    bool trace = false, longr = false, spec = false;
    long long pix = 0;
    if (t < n) {
        const int i = t % D.nx0, j = t / D.nx0;
        pix = (long long)(j * st0) * D.nx + (long long)(i * st0);
        if (spectral_ok(desc, D, pix, ctr)) {
            spectral_write(desc, D, pix);
            spec = true;
        } else {
            trace = true;
            D.level[pix] = 0;
            if (D.cost) {
                const uint16_t cb = desc[D.sb].cost[pix], cc = desc[D.sc].cost[pix];
                longr = (int)(cb > cc ? cb : cc) >= long_steps;
            }
        }
    }
    const int lane = __lane_id();
    const unsigned long long ms = __ballot(spec);
    if (ms && lane == __ffsll((long long)ms) - 1) atomicAdd(&ctr->judge[img][5], (unsigned long long)__popcll(ms));
    const unsigned long long mlong = __ballot(trace && longr);
    const unsigned long long mshort = __ballot(trace && !longr);
    if (mlong | mshort) {
        const int leader = __ffsll((long long)(mlong | mshort)) - 1;
        unsigned bl = 0, bs = 0;
        if (lane == leader) {
            if (mlong) bl = atomicAdd(&ctr->count[slot], (unsigned)__popcll(mlong));
            if (mshort) bs = atomicAdd(&ctr->count_back[slot], (unsigned)__popcll(mshort));
            atomicAdd(&ctr->img_traced[img][0], (unsigned)__popcll(mlong | mshort));
        }
        bl = __shfl(bl, leader);
        bs = __shfl(bs, leader);
        const unsigned long long item = make_item((uint32_t)img, (uint32_t)pix);
        if (trace && longr) list[bl + lane_prefix(mlong)] = item;
        if (trace && !longr) list[cap - 1 - (long long)(bs + lane_prefix(mshort))] = item;
    }
}

hipError_t launch_spectral_base(const ImageDesc* desc, int img_off, int nimg, int max_base, Counters* ctr,
                                unsigned long long* list, long long cap, int long_steps, int slot, hipStream_t s)
{
    dim3 grid((max_base + 255) / 256, nimg);
    hipLaunchKernelGGL(k_spectral_base, grid, dim3(256), 0, s, desc, img_off, ctr, list, cap, long_steps, slot);
    return hipGetLastError();
}

// ------------------------------------------------------ refinement level
// Per axis with in-points lo, hi and continuations at -3, +3 (level-(l+1)
// units): D = (out_lo + out_hi) - (lo + hi); one continuation outside the
// image: twice the one-sided second difference; both outside: unavailable.
__device__ __forceinline__ bool axis_D(const double* I, long long nx, int s, int nxl, int nyl,
                                       int p, int q, int dx, int dy, double lo, double hi, double& D)
{
    const int pl = p - 3 * dx, ql = q - 3 * dy, ph = p + 3 * dx, qh = q + 3 * dy;
    const bool has_lo = pl >= 0 && pl < nxl && ql >= 0 && ql < nyl;
    const bool has_hi = ph >= 0 && ph < nxl && qh >= 0 && qh < nyl;
    const double olo = has_lo ? I[(long long)(ql * s) * nx + (long long)(pl * s)] : 0.0;
    const double ohi = has_hi ? I[(long long)(qh * s) * nx + (long long)(ph * s)] : 0.0;
    if (has_lo && has_hi) { D = (olo + ohi) - (lo + hi); return true; }
    if (has_hi) { D = 2.0 * ((ohi - 2.0 * hi) + lo); return true; }
    if (has_lo) { D = 2.0 * ((olo - 2.0 * lo) + hi); return true; }
    D = 0.0;
    return false;
}

// Blocks of a launch are placed on the eight XCDs round robin (block b on
// XCD b mod 8).  The estimator maps hardware block b to a logical block so
// that each XCD gets one contiguous range of logical blocks, i.e. runs of
// consecutive rows of an image: the neighbour and continuation rows a block
// reads (q -+ 1, q -+ 3) were fetched into that XCD's L2 by its neighbours.
// A bijection on [0, nb) for any nb.
__device__ __forceinline__ unsigned long long xcd_contiguous(unsigned long long b, unsigned long long nb)
{
    const unsigned long long q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// grid (x: 256-wide strips of the new points of an image, z: image), remapped
// per XCD as above.  One thread per new point of the level-(l+1) grid, taken
// row pair by row pair: the (nxl - 1) / 2 odd columns of an even row, then
// all nxl columns of the next odd row (the old points, even row and column,
// get no thread); new points are classified by index parity (categories 2-4).
__host__ __device__ __forceinline__ long long estimate_points(int nxl, int nyl)
{
    return (long long)((nyl - 1) >> 1) * (((nxl - 1) >> 1) + nxl) + ((nxl - 1) >> 1);
}

__global__ __launch_bounds__(256) void k_estimate(const ImageDesc* desc, int l, Counters* ctr,
                                                  unsigned long long* list, long long cap, int long_steps,
                                                  int mode, int fallback, int img_off, int slot,
                                                  const int* __restrict__ imap, int feat)
{
    const unsigned long long gx = gridDim.x, gy = gridDim.y;
    const unsigned long long lb = xcd_contiguous(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z),
                                                 gx * gy * gridDim.z);
    const int bx = (int)(lb % gx), by = (int)((lb / gx) % gy), bz = (int)(lb / (gx * gy));
    const int img = imap ? imap[bz] : img_off + bz;
    const ImageDesc D = desc[img];
    if (l >= D.levels) return;                     // uniform over the block
    const int nxl = (1 << (l + 1)) * (D.nx0 - 1) + 1;
    const int nyl = (1 << (l + 1)) * (D.ny0 - 1) + 1;
    const int s = 1 << (D.levels - l - 1);
    (void)by;
    const int m0 = (nxl - 1) >> 1;                 // new points of an even row
    const long long t = (long long)bx * blockDim.x + threadIdx.x;
    const bool isnew = t < estimate_points(nxl, nyl);
    int p = 0, q = 0;
    if (isnew) {
        const long long k = t / (m0 + nxl);
        const int r = (int)(t - k * (m0 + nxl));
        q = (int)(2 * k) + (r < m0 ? 0 : 1);
        p = r < m0 ? 2 * r + 1 : r - m0;
    }
    bool trace = false;
    bool longr = false;                      // expected to be a long ray: queue at the front
    bool spec = false;                       // value taken from the spectral neighbours
    bool jd[4] = { false, false, false, false };
    long long pix = 0;
    if (isnew) {
        const double* I = D.img;
        const long long NX = D.nx;
        pix = (long long)(q * s) * NX + (long long)(p * s);
        const bool c4 = (p & 1) && (q & 1);
        double Ssum, D2;
        bool avail;
        double m;
        long long o[4];
        int nnb;
        if (c4) {
            // diagonal x': I1 (-1,-1) -> I4 (+1,+1), continuations I5, I8 at -+3;
            // diagonal y': I2 (+1,-1) -> I3 (-1,+1), continuations I6 (+3,-3), I7 (-3,+3)
            o[0] = (long long)((q - 1) * s) * NX + (long long)((p - 1) * s);
            o[1] = (long long)((q + 1) * s) * NX + (long long)((p + 1) * s);
            o[2] = (long long)((q - 1) * s) * NX + (long long)((p + 1) * s);
            o[3] = (long long)((q + 1) * s) * NX + (long long)((p - 1) * s);
            nnb = 4;
            const double i1 = I[o[0]], i4 = I[o[1]], i2 = I[o[2]], i3 = I[o[3]];
            Ssum = (i1 + i4) + (i2 + i3);
            double Dx, Dy;
            const bool ax = axis_D(I, NX, s, nxl, nyl, p, q, 1, 1, i1, i4, Dx);
            const bool ay = axis_D(I, NX, s, nxl, nyl, p, q, -1, 1, i2, i3, Dy);
            D2 = ax ? (ay ? Dx + Dy : 2.0 * Dx) : 2.0 * Dy;
            avail = ax || ay;
            m = 4.0;
        } else {
            const int dx = (p & 1) ? 1 : 0, dy = (p & 1) ? 0 : 1;
            o[0] = (long long)((q - dy) * s) * NX + (long long)((p - dx) * s);
            o[1] = (long long)((q + dy) * s) * NX + (long long)((p + dx) * s);
            o[2] = o[3] = 0;
            nnb = 2;
            const double lo = I[o[0]], hi = I[o[1]];
            Ssum = lo + hi;
            avail = axis_D(I, NX, s, nxl, nyl, p, q, dx, dy, lo, hi, D2);
            m = 2.0;
        }
        const double nabs = ctr->scal[img][2];
        const bool nearest = (D.flags & kRefineNearest) != 0;
        const bool allp = (D.flags & kRefineAllPlanes) != 0;
        bool crit;
        if (nearest) {
            // nearest branch of Eqs. 5-6: G = |c - b|/2 (1D) or
            // sqrt(((I4 - I1)/2)^2 + ((I3 - I2)/2)^2) (2D), against N_abs and |I_nn|
            const double thrA = D.r_abs * nabs;
            const double inn = ::fabs(I[o[0]]);
            crit = !(I[o[0]] == I[o[0]]);
            for (int st = 0; st < (allp ? D.nplanes : 1); ++st) {
                const double* Is = I + st * D.plane;
                double G;
                if (nnb == 4) {
                    const double gx = 0.5 * (Is[o[1]] - Is[o[0]]), gy = 0.5 * (Is[o[3]] - Is[o[2]]);
                    G = ::sqrt(gx * gx + gy * gy);
                } else {
                    G = 0.5 * ::fabs(Is[o[1]] - Is[o[0]]);
                }
                crit = crit || !(G == G) || (G > thrA && G > D.r_rel * inn);
            }
        } else {
            const double thrA = (4.0 * m * D.r_abs) * nabs;
            const double crel = 4.0 * D.r_rel;
            const double aS = ::fabs(Ssum);
            const double aD = ::fabs(D2);
            crit = !avail || !(D2 == D2) || !(Ssum == Ssum) || (aD > thrA && aD > crel * aS);
            if (allp) {
                // the same estimate on every further plane (Q, U, V, subrings),
                // against Stokes I's N_abs and |S|, or (kRefineOwnNorm) against
                // the plane's own N_abs and neighbour sum
                const bool own = (D.flags & kRefineOwnNorm) != 0;
                for (int st = 1; st < D.nplanes; ++st) {
                    const double* Is = I + st * D.plane;
                    double Dp;
                    if (c4) {
                        double Dx, Dy;
                        const bool ax = axis_D(Is, NX, s, nxl, nyl, p, q, 1, 1, Is[o[0]], Is[o[1]], Dx);
                        const bool ay = axis_D(Is, NX, s, nxl, nyl, p, q, -1, 1, Is[o[2]], Is[o[3]], Dy);
                        Dp = ax ? (ay ? Dx + Dy : 2.0 * Dx) : 2.0 * Dy;
                    } else {
                        const int dx = (p & 1) ? 1 : 0, dy = (p & 1) ? 0 : 1;
                        axis_D(Is, NX, s, nxl, nyl, p, q, dx, dy, Is[o[0]], Is[o[1]], Dp);
                    }
                    double thrP = thrA, aSp = aS;
                    if (own) {
                        thrP = (4.0 * m * D.r_abs) * ctr->nabs_plane[img][st];
                        aSp = ::fabs(nnb == 4 ? (Is[o[0]] + Is[o[1]]) + (Is[o[2]] + Is[o[3]]) : Is[o[0]] + Is[o[1]]);
                    }
                    const double aDp = ::fabs(Dp);
                    crit = crit || !(Dp == Dp) || (aDp > thrP && aDp > crel * aSp);
                }
            }
        }
        bool keep = false;               // point already traced by a look-ahead pass
        if (mode == 0) {
            trace = crit;
        } else if (mode == 3) {
            spec = crit && spectral_ok(desc, D, pix, ctr);
            trace = crit && !spec;
        } else {
            // mode 1: the network marked the images that can look ahead
            // (levels >= l + 2), with all_levels (fallback = 1 here) also those
            // with one level left; the others take the plain criterion
            const bool marked = mode != 1 || D.levels >= l + 2 || fallback;
            const int8_t mk = marked ? D.level[pix] : kMarkUnset;
            const bool sup = mk == kMarkSuppress;
            if (mode == 1) {
                const bool prop = mk == kMarkPropose;
                trace = prop || (crit && !sup);
                jd[0] = prop && !crit;
                jd[1] = crit && sup;
            } else {
                keep = mk == (int8_t)(l + 1);
                const bool want = crit && !sup && !keep;
                trace = want && fallback;
                jd[1] = crit && sup && !keep;
                jd[2] = want && fallback;
                jd[3] = want && !fallback;
            }
        }
        if (spec) {
            spectral_write(desc, D, pix);
        } else if (D.cost && (trace || !keep)) {
            // expected cost: the most expensive neighbour
            uint16_t c = D.cost[o[0]];
            for (int q2 = 1; q2 < nnb; ++q2) {
                const uint16_t c2 = D.cost[o[q2]];
                c = c2 > c ? c2 : c;
            }
            longr = trace && (int)c >= long_steps;
            if (!trace) D.cost[pix] = c;
        }
        if (trace) {
            D.level[pix] = (int8_t)(l + 1);
        } else if (!keep && !spec) {
            D.level[pix] = (int8_t)-1;
            if (D.flags & kRefineNearest) {
                // nearest neighbour: I1 (2D) or the lower neighbour b (1D)
                for (int st = 0; st < D.nplanes; ++st) D.img[st * D.plane + pix] = I[st * D.plane + o[0]];
            } else {
                const double w = 1.0 / m;
                D.img[pix] = Ssum * w;
                for (int st = 1; st < D.nplanes; ++st) {
                    const double* Is = I + st * D.plane;
                    const double S = nnb == 4 ? (Is[o[0]] + Is[o[1]]) + (Is[o[2]] + Is[o[3]]) : Is[o[0]] + Is[o[1]];
                    D.img[st * D.plane + pix] = S * w;
                }
            }
            if (D.feat && feat) {
                // interpolated points inherit the smallest radius and the largest
                // crossing count of their neighbours
                RayFeat f = D.feat[o[0]];
                for (int q2 = 1; q2 < nnb; ++q2) {
                    const RayFeat g = D.feat[o[q2]];
                    f.rmin = g.rmin < f.rmin ? g.rmin : f.rmin;
                    f.ncross = g.ncross > f.ncross ? g.ncross : f.ncross;
                }
                f.steps = 0;
                f.status = RAY_OK;
                D.feat[pix] = f;
            }
        }
    }
    if (mode == 3) {
        const unsigned long long mk = __ballot(spec);
        if (mk && __lane_id() == __ffsll((long long)mk) - 1)
            atomicAdd(&ctr->judge[img][5], (unsigned long long)__popcll(mk));
    } else if (mode != 0) {
        // judge counters: one atomic per wave and counter
        const int lane = __lane_id();
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            const unsigned long long mk = __ballot(jd[q2]);
            if (mk && lane == __ffsll((long long)mk) - 1) atomicAdd(&ctr->judge[img][q2], (unsigned long long)__popcll(mk));
        }
    }
    // wavefront-ballot compaction of the points to trace: expected long rays
    // to the front of the list, the others from the back
    const unsigned long long mlong = __ballot(trace && longr);
    const unsigned long long mshort = __ballot(trace && !longr);
    if (mlong | mshort) {
        const int lane = __lane_id();
        const int leader = __ffsll((long long)(mlong | mshort)) - 1;
        unsigned bl = 0, bs = 0;
        if (lane == leader) {
            if (mlong) bl = atomicAdd(&ctr->count[slot], (unsigned)__popcll(mlong));
            if (mshort) bs = atomicAdd(&ctr->count_back[slot], (unsigned)__popcll(mshort));
            atomicAdd(&ctr->img_traced[img][l + 1], (unsigned)__popcll(mlong | mshort));
        }
        bl = __shfl(bl, leader);
        bs = __shfl(bs, leader);
        const unsigned long long item = make_item((uint32_t)img, (uint32_t)pix);
        if (trace && longr) list[bl + lane_prefix(mlong)] = item;
        if (trace && !longr) list[cap - 1 - (long long)(bs + lane_prefix(mshort))] = item;
    }
}

hipError_t launch_estimate(const ImageDesc* desc, int nimg, int nxl_max, int nyl_max, int l,
                           Counters* ctr, unsigned long long* list, long long cap, int long_steps,
                           hipStream_t s, int mode, int fallback, int img_off, int slot, const int* imap,
                           int feat)
{
    if (nimg <= 0) return hipSuccess;
    const long long pts = estimate_points(nxl_max, nyl_max);
    if ((pts + 255) / 256 >= (1LL << 31)) return hipErrorInvalidValue;
    dim3 grid((unsigned)((pts + 255) / 256), 1, nimg);
    hipLaunchKernelGGL(k_estimate, grid, dim3(256), 0, s, desc, l, ctr, list, cap, long_steps, mode, fallback,
                       img_off, slot < 0 ? l + 1 : slot, imap, feat);
    return hipGetLastError();
}

// ---------------------------------------------------------------- metrics
// partial[b*4 + {0,1,2,3}] = sum t, sum a, sum (t-a)^2, sum t^2 over block b.
__global__ __launch_bounds__(256) void k_metrics_partial(const double* t, const double* a, long long n,
                                                         double* partial)
{
    __shared__ double sh[4][256];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double x = t[i], y = a[i], d = x - y;
        s0 += x; s1 += y; s2 += d * d; s3 += x * x;
    }
    const int k = threadIdx.x;
    sh[0][k] = s0; sh[1][k] = s1; sh[2][k] = s2; sh[3][k] = s3;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (k < off) {
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[c][k] += sh[c][k + off];
        }
        __syncthreads();
    }
    if (k < 4) partial[blockIdx.x * 4 + k] = sh[k][0];
}

__global__ __launch_bounds__(256) void k_metrics_final(double* partial, int nb)
{
    __shared__ double sh[4][256];
    const int k = threadIdx.x;
    double s[4] = { 0.0, 0.0, 0.0, 0.0 };
    for (int b = k; b < nb; b += 256)
        for (int c = 0; c < 4; ++c) s[c] += partial[b * 4 + c];
    for (int c = 0; c < 4; ++c) sh[c][k] = s[c];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (k < off)
            for (int c = 0; c < 4; ++c) sh[c][k] += sh[c][k + off];
        __syncthreads();
    }
    if (k < 4) partial[(long long)nb * 4 + k] = sh[k][0];
}

hipError_t launch_metrics(const double* t, const double* a, long long n, double* partial,
                          int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_metrics_partial, dim3(nblocks), dim3(256), 0, s, t, a, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(256), 0, s, partial, nblocks);
    return hipGetLastError();
}

}  // namespace art
