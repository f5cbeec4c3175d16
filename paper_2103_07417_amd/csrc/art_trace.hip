// art_trace.hip -- the persistent work-queue ray tracer of the adaptive
// renderer (gfx950).
//
//   k_trace      one lane per ray; lanes refill from a global atomic cursor at
//                wave-uniform points, so rays of very uneven step counts
//                (photon-ring rays wind many times, Sec. 4.2 last paragraphs)
//                keep every lane busy.  Per step: the FP64 Kerr-Schild
//                geodesic (RK4), the plasma sample and the polarised transfer
//                at the step midpoint, the ray features and the subring index.
#include "art_internal.hpp"

namespace art {

// ------------------------------------------------------------- ray tracing
template <typename R, int MODEL, int NS, int SUB = 0>
struct RayState {
    double y[5];
    double sth, cth;               // sin, cos of y[1]
    double kt, kph, k0r, k0i;
    double cprev, rmin;
    R S[NS];
    R O[NS == 4 ? 16 : 1];
    R Ssub[SUB > 0 ? SUB : 1];     // subring planes of I
    int ncross, nstep, nturn;
    uint32_t pix;
    int img;
};

template <typename R, int MODEL, int NS, int SUB>
__device__ __forceinline__ void ray_init(const Params& P, RayState<R, MODEL, NS, SUB>& st, double al, double be)
{
    RayStart rs;
    camera_start(P, al, be, rs);
#pragma unroll
    for (int i = 0; i < 5; ++i) st.y[i] = rs.y[i];
    st.kt = rs.kt; st.kph = rs.kph; st.k0r = rs.k0r; st.k0i = rs.k0i;
    st.sth = P.s_cam;                  // the ray starts at the camera's theta
    st.cth = P.c_cam;
    st.cprev = st.cth;
    st.rmin = rs.y[0];
#pragma unroll
    for (int i = 0; i < NS; ++i) st.S[i] = R(0);
    if constexpr (NS == 4) {
#pragma unroll
        for (int i = 0; i < 16; ++i) st.O[i] = (i % 5 == 0) ? R(1) : R(0);
    } else {
        st.O[0] = R(1);
    }
    st.ncross = 0;
    st.nstep = 0;
    st.nturn = 0;
#pragma unroll
    for (int q = 0; q < (SUB > 0 ? SUB : 1); ++q) st.Ssub[q] = R(0);
}

// Advance one ray by one step.  Returns a RAY_* status (RAY_OK = continue).
// sin/cos of theta are evaluated once per ray and carried in the state: the
// RK stages, the midpoint and the step's end rotate them by their (small)
// theta increments (angle addition, error ~1e-16 per step).
// G32 (precision policy): the four right-hand sides of the step are evaluated
// in FP32 when the ray is outside every sensitive zone (r < r64: photon shell
// and horizon; |k_theta| < kth64: theta turning points; |sin theta| < 0.1:
// the polar barrier); the state, the RK4 sums and the step rule stay FP64.
// The decision is the ray's own (per lane), so a ray's result does not depend
// on which rays share its wave: batches, launch shapes and queue orders give
// the same bits.
template <typename R, int MODEL, int NS, bool G32, int SUB>
__device__ __forceinline__ int ray_step(const Params& P, const double* tht, RayState<R, MODEL, NS, SUB>& st,
                                        unsigned& emit)
{
    const double a = P.a;
    double k1[5], acc[5], yt[5], kk[5];
    const double s0 = st.sth, c0 = st.cth;
    bool fast = false;
    if constexpr (G32)
        fast = !(st.y[0] < P.r64 || ::fabs(st.y[4]) < P.kth64 || ::fabs(s0) < 0.1);
    auto rhs = [&](const double* y, double s, double c, double* d) {
        if (G32 && fast) geo_rhs32(a, st.kt, st.kph, y, s, c, d);
        else geo_rhs(a, st.kt, st.kph, y, s, c, d);
    };
    rhs(st.y, s0, c0, k1);
    if (st.cprev * c0 < 0.0) st.ncross++;
    st.cprev = c0;
    if (st.y[0] < st.rmin) st.rmin = st.y[0];
    // termination, first matching test wins (escape, capture, step cap,
    // optically thick, NaN); one status select per test and a single exit, so
    // the ray state is not copied once per test
    int status = RAY_OK;
    status = (!(st.y[0] == st.y[0]) || !(st.y[3] == st.y[3])) ? RAY_NAN : status;
    status = st.O[0] < R(1e-12) ? RAY_THICK : status;
    status = st.nstep >= P.max_steps ? RAY_STEPCAP : status;
    status = st.y[0] < P.rstop ? RAY_CAPTURED : status;
    status = (st.y[0] > P.r_out && k1[0] > 0.0) ? RAY_ESCAPED : status;
    if (status != RAY_OK) return status;
    double rate = ::fabs(k1[0]) * frcp(st.y[0]) + ::fabs(k1[1]) + ::fabs(k1[2]);
    // pole control: within |sin theta| < 0.1 of a pole (k_phi != 0: centrifugal
    // barrier) the theta step is limited to a fraction of the distance to the
    // pole, floored at half the barrier's sin theta ~ |k_phi| / |k_theta|
    if (st.kph != 0.0) {
        double se = ::fabs(s0);
        const double ka = ::fabs(st.y[4]);
        if (0.5 * ::fabs(st.kph) > se * ka) se = 0.5 * ::fabs(st.kph) / ka;
        if (se < 0.1) rate += ::fabs(k1[1]) * (frcp(se) - 10.0);
    }
    double far = st.y[0] * (1.0 / 20.0);
    far = far < 1.0 ? 1.0 : (far > 4.0 ? 4.0 : far);
    double h = P.eps * far * frcp(rate);
    if (k1[0] < 0.0) {
        const double hh = 0.5 * (st.y[0] - P.rh) * frcp(-k1[0]);
        h = hh < h ? hh : h;
    }
    const double h2 = 0.5 * h;
    double s, c;
#pragma unroll
    for (int i = 0; i < 5; ++i) { yt[i] = st.y[i] + h2 * k1[i]; acc[i] = k1[i]; }
    rotate_sc(s0, c0, h2 * k1[1], s, c);
    rhs(yt, s, c, kk);
#pragma unroll
    for (int i = 0; i < 5; ++i) { yt[i] = st.y[i] + h2 * kk[i]; acc[i] += 2.0 * kk[i]; }
    rotate_sc(s0, c0, h2 * kk[1], s, c);
    rhs(yt, s, c, kk);
#pragma unroll
    for (int i = 0; i < 5; ++i) { yt[i] = st.y[i] + h * kk[i]; acc[i] += 2.0 * kk[i]; }
    rotate_sc(s0, c0, h * kk[1], s, c);
    rhs(yt, s, c, kk);
    const double h6 = h * (1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 5; ++i) yt[i] = st.y[i] + h6 * (acc[i] + kk[i]);
    // transfer at the step midpoint
    const double rm = 0.5 * (st.y[0] + yt[0]), thm = 0.5 * (st.y[1] + yt[1]);
    const double phm = 0.5 * (st.y[2] + yt[2]);
    const double krm = 0.5 * (st.y[3] + yt[3]), kthm = 0.5 * (st.y[4] + yt[4]);
    rotate_sc(s0, c0, 0.5 * (yt[1] - st.y[1]), s, c);
    Coef<R> C;
    if (plasma_point<R, MODEL>(P, tht, rm, thm, s, c, phm, st.kt, st.kph, krm, kthm, st.k0r, st.k0i, C)) {
        ++emit;
        const R I0 = st.S[0];
        if constexpr (NS == 4) {
            transfer_step4<R, R>(st.S, st.O, C, R(h));
        } else {
            const R w = C.aI * R(h);
            const R ew = fexp(-w);
            st.S[0] += st.O[0] * R(h) * phi1_(w, ew) * C.jI;
            st.O[0] *= ew;
        }
        if constexpr (SUB > 0) {
            // subring decomposition (Sec. 5.1): the step's increment of I goes
            // to the plane of the half-orbits passed so far
            const int n = st.nturn < P.nsub - 1 ? st.nturn : P.nsub - 1;
            const R dI = st.S[0] - I0;
#pragma unroll
            for (int q = 0; q < SUB; ++q)
                if (q == n) st.Ssub[q] += dI;
        }
    }
    if constexpr (SUB > 0) {
        if (st.y[4] * yt[4] < 0.0) st.nturn++;      // theta turning point
    }
    rotate_sc(s0, c0, yt[1] - st.y[1], st.sth, st.cth);
#pragma unroll
    for (int i = 0; i < 5; ++i) st.y[i] = yt[i];
    st.nstep++;
    return RAY_OK;
}

// Persistent work-queue tracer.  Every wave loops: idle lanes are counted by
// a ballot, one lane claims that many items with a single atomic, the items
// are handed out by lane prefix; then every busy lane advances its ray by one
// step.  The per-image parameter blocks are staged in LDS once per block.
template <typename R, int MODEL, int NS, bool G32, int SUB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_trace(TraceJob J)
{
    __shared__ Params sP[kMaxBatch];
    {
        static_assert(sizeof(Params) % 8 == 0, "Params must be a whole number of doubles");
        const int nw = J.nimg * (int)(sizeof(Params) / 8);
        const double* src = reinterpret_cast<const double*>(J.params);
        double* dst = reinterpret_cast<double*>(sP);
        for (int k = threadIdx.x; k < nw; k += blockDim.x) dst[k] = src[k];
    }
    // gridded model: cell-centre angles of the snapshot shared by the batch
    __shared__ double sTh[MODEL == MODEL_GRID ? kMaxThetaCells : 1];
    if constexpr (MODEL == MODEL_GRID) {
        const double* tab = J.params[0].theta_tab;
        const int n2 = J.params[0].g_n2;
        for (int k = threadIdx.x; k < n2; k += blockDim.x) sTh[k] = tab[k];
    }
    __syncthreads();
    const int lane = __lane_id();
    RayState<R, MODEL, NS, SUB> st;
    bool active = false, drained = false;
    unsigned long long my_steps = 0;
    unsigned my_emit = 0;
    unsigned hist[6] = { 0, 0, 0, 0, 0, 0 };
    const uint32_t cnt_front = *J.count;
    const uint32_t cnt = cnt_front + (J.count_back ? *J.count_back : 0u);

    for (;;) {
        if (!drained) {
            const unsigned long long need = __ballot(!active);
            const int nidle = __popcll(need);
            if (nidle >= J.refill && nidle > 0) {
                const int leader = __ffsll((long long)need) - 1;
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(J.cursor, (unsigned)nidle);
                base = __shfl(base, leader);
                if ((unsigned long long)base + (unsigned)nidle >= cnt) drained = true;
                if (!active) {
                    const unsigned my = base + lane_prefix(need);
                    if (my < cnt) {
                        double al = 0.0, be = 0.0;
                        int img = 0;
                        uint32_t pix = my;
                        bool ok = true;
                        if (J.src == SRC_POINTS) {
                            al = J.alpha[my];
                            be = J.beta[my];
                        } else {
                            if (J.list) {
                                const long long at = my < cnt_front ? (long long)my
                                                                    : J.cap - 1 - (long long)(my - cnt_front);
                                const unsigned long long it = J.list[at];
                                img = (int)(it >> 32);
                                pix = (uint32_t)it;
                            }
                            // a malformed item is dropped rather than written out of bounds
                            ok = img < J.nimg && (long long)pix < J.desc[img].plane;
                            if (ok) {
                                const Params& Pi = sP[img];
                                const uint32_t i = pix % (uint32_t)Pi.nx, j = pix / (uint32_t)Pi.nx;
                                al = Pi.x0 + (double)i * Pi.dx;
                                be = Pi.y0 + (double)j * Pi.dx;
                            }
                        }
                        if (ok) {
                            st.img = img;
                            st.pix = pix;
                            const Params& P = sP[img];
                            if (P.model >= MODEL_SCREEN_RING) {
                                double S4[4];
                                screen_fn(P, al, be, S4);
                                RayFeat f; f.rmin = (float)P.r_cam; f.ncross = 0; f.steps = 0; f.status = RAY_OK;
                                // a screen function has no rays: all of I in subring plane 0
                                if (J.src == SRC_POINTS) {
                                    const int np = P.nstokes + P.nsub;
                                    for (int s = 0; s < P.nstokes; ++s) J.out[(long long)pix * np + s] = S4[s];
                                    for (int q = 0; q < P.nsub; ++q)
                                        J.out[(long long)pix * np + P.nstokes + q] = q == 0 ? S4[0] : 0.0;
                                    if (J.feat) J.feat[pix] = f;
                                } else {
                                    const ImageDesc& D = J.desc[img];
                                    for (int s = 0; s < D.nstokes; ++s) D.img[s * D.plane + pix] = S4[s];
                                    for (int q = D.nstokes; q < D.nplanes; ++q)
                                        D.img[q * D.plane + pix] = q == D.nstokes ? S4[0] : 0.0;
                                    if (D.feat) D.feat[pix] = f;
                                }
                                hist[RAY_OK]++;
                            } else {
                                ray_init<R, MODEL, NS, SUB>(P, st, al, be);
                                active = true;
                            }
                        }
                    }
                }
            }
        }
        if (!__any(active)) {
            if (drained) break;
            continue;
        }
        if (active) {
            const Params& P = sP[st.img];
            // step until a ray of the wave terminates: the state stays in the
            // same registers across steps (the refill path above merges into
            // it once per termination, not once per step); every ray ends by
            // the step cap at the latest, so the loop is bounded
            int status;
            do {
                status = ray_step<R, MODEL, NS, G32, SUB>(P, sTh, st, my_emit);
            } while (!__any(status != RAY_OK));
            if (status != RAY_OK) {
                double Sd[4] = { 0.0, 0.0, 0.0, 0.0 };
#pragma unroll
                for (int s = 0; s < NS; ++s) Sd[s] = (double)st.S[s];
                int stt = status;
                if (!(Sd[0] == Sd[0])) stt = RAY_NAN;
                RayFeat f;
                f.rmin = (float)st.rmin; f.ncross = st.ncross; f.steps = st.nstep; f.status = stt;
                if (J.src == SRC_POINTS) {
                    const int np = P.nstokes + P.nsub;
                    for (int s = 0; s < P.nstokes; ++s) J.out[(long long)st.pix * np + s] = Sd[s];
                    if constexpr (SUB > 0) {
#pragma unroll
                        for (int q = 0; q < SUB; ++q)
                            if (q < P.nsub) J.out[(long long)st.pix * np + P.nstokes + q] = (double)st.Ssub[q];
                    }
                    if (J.feat) J.feat[st.pix] = f;
                } else {
                    const ImageDesc& D = J.desc[st.img];
                    for (int s = 0; s < D.nstokes; ++s) D.img[s * D.plane + st.pix] = Sd[s];
                    if constexpr (SUB > 0) {
#pragma unroll
                        for (int q = 0; q < SUB; ++q)
                            if (D.nstokes + q < D.nplanes) D.img[(D.nstokes + q) * D.plane + st.pix] = (double)st.Ssub[q];
                    }
                    if (D.feat) D.feat[st.pix] = f;
                    if (D.cost) D.cost[st.pix] = (uint16_t)(st.nstep < 65535 ? st.nstep : 65535);
                }
                my_steps += (unsigned long long)st.nstep;
                hist[stt]++;
                active = false;
            }
        }
    }
    // wave-level statistics: one atomic per counter per wave
    unsigned long long my_emit64 = my_emit;
    for (int off = 32; off > 0; off >>= 1) my_steps += __shfl_xor(my_steps, off);
    for (int off = 32; off > 0; off >>= 1) my_emit64 += __shfl_xor(my_emit64, off);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off > 0; off >>= 1) hist[k] += __shfl_xor(hist[k], off);
    if (lane == 0 && J.ctr) {
        if (my_steps) atomicAdd(&J.ctr->steps, my_steps);
        if (my_emit64) atomicAdd(&J.ctr->steps_emit, my_emit64);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (hist[k]) atomicAdd(&J.ctr->status[k], (unsigned long long)hist[k]);
    }
}

// Kernel instantiation for (precision, model, nstokes, subrings): the screen
// test functions run through the toy-disk instantiation (they never
// integrate).  precision 0: FP64 throughout; 1: FP64 geodesic, FP32 plasma
// and transfer; 2: as 1 with FP32 geodesic right-hand sides outside the
// sensitive zones (no subring variant).
template <typename F>
static hipError_t dispatch(int precision, int model, int nstokes, bool sub, F&& f)
{
    const bool pol = nstokes == 4;
    if (sub) {
        if (precision == 0) {
            if (model == MODEL_THERMAL) return pol ? f((k_trace<double, MODEL_THERMAL, 4, false, kMaxSub>)) : f((k_trace<double, MODEL_THERMAL, 1, false, kMaxSub>));
            if (model == MODEL_GRID) return pol ? f((k_trace<double, MODEL_GRID, 4, false, kMaxSub>)) : f((k_trace<double, MODEL_GRID, 1, false, kMaxSub>));
            return f((k_trace<double, MODEL_TOY, 1, false, kMaxSub>));
        }
        if (model == MODEL_THERMAL) return pol ? f((k_trace<float, MODEL_THERMAL, 4, false, kMaxSub>)) : f((k_trace<float, MODEL_THERMAL, 1, false, kMaxSub>));
        if (model == MODEL_GRID) return pol ? f((k_trace<float, MODEL_GRID, 4, false, kMaxSub>)) : f((k_trace<float, MODEL_GRID, 1, false, kMaxSub>));
        return f((k_trace<float, MODEL_TOY, 1, false, kMaxSub>));
    }
    if (precision == 0) {
        if (model == MODEL_THERMAL) return pol ? f((k_trace<double, MODEL_THERMAL, 4, false, 0>)) : f((k_trace<double, MODEL_THERMAL, 1, false, 0>));
        if (model == MODEL_GRID) return pol ? f((k_trace<double, MODEL_GRID, 4, false, 0>)) : f((k_trace<double, MODEL_GRID, 1, false, 0>));
        return f((k_trace<double, MODEL_TOY, 1, false, 0>));
    }
    if (precision == 1) {
        if (model == MODEL_THERMAL) return pol ? f((k_trace<float, MODEL_THERMAL, 4, false, 0>)) : f((k_trace<float, MODEL_THERMAL, 1, false, 0>));
        if (model == MODEL_GRID) return pol ? f((k_trace<float, MODEL_GRID, 4, false, 0>)) : f((k_trace<float, MODEL_GRID, 1, false, 0>));
        return f((k_trace<float, MODEL_TOY, 1, false, 0>));
    }
    if (model == MODEL_THERMAL) return pol ? f((k_trace<float, MODEL_THERMAL, 4, true, 0>)) : f((k_trace<float, MODEL_THERMAL, 1, true, 0>));
    if (model == MODEL_GRID) return pol ? f((k_trace<float, MODEL_GRID, 4, true, 0>)) : f((k_trace<float, MODEL_GRID, 1, true, 0>));
    return f((k_trace<float, MODEL_TOY, 1, true, 0>));
}

hipError_t launch_trace(int precision, int model, int nstokes, bool subrings, const TraceJob& J,
                        const LaunchCfg& L, hipStream_t s)
{
    return dispatch(precision, model, nstokes, subrings, [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(L.trace_blocks), dim3(L.trace_threads), 0, s, J);
        return hipGetLastError();
    });
}

int trace_occupancy_blocks(int precision, int model, int nstokes, bool subrings, int threads)
{
    int nb = 0;
    hipError_t e = dispatch(precision, model, nstokes, subrings, [&](auto kern) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, 0);
    });
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace art
