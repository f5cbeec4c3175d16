// art_internal.hpp -- host/kernel declarations shared by the kernels and the
// C ABI implementation (not part of the public interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "art_device.hpp"

namespace art {

constexpr int kMaxBatch = 64;     // images per launch (their Params are staged in LDS)
constexpr int kMaxLevels = 21;

// Device counters of one batch, zeroed by a fill kernel at the start.
struct Counters {
    uint32_t count[kMaxLevels + 1];       // per level: work items at the front of the trace list
    uint32_t count_back[kMaxLevels + 1];  // per level: work items filled from the back
    uint32_t cursor[kMaxLevels + 1];      // per level: work-queue cursor
    unsigned long long steps;             // geodesic steps
    unsigned long long steps_emit;        // steps that evaluated the plasma/transfer
    unsigned long long status[8];
    uint32_t img_traced[kMaxBatch][kMaxLevels + 1];   // per image and level
    double scal[kMaxBatch][4];            // per image: ibar_int, imax0, n_abs, spare
    double nabs_plane[kMaxBatch][12];     // per image and plane (kRefineOwnNorm): the plane's own N_abs
    // learned proposals, per image: [0] proposed points the criterion would
    // not trace, [1] criterion-flagged points the network rejected, [2] points
    // traced by the criterion as fallback after a look-ahead pass, [3]
    // criterion-flagged points left interpolated (judge-only mode), [4]
    // look-ahead proposals; [5] points taken from the spectral neighbours
    unsigned long long judge[kMaxBatch][8];
};

// Per-image description (device memory).
struct ImageDesc {
    double* img;          // [nstokes][ny][nx]
    int8_t* level;        // [ny][nx]
    RayFeat* feat;        // optional
    uint16_t* cost;       // steps of each traced ray, neighbours' maximum for interpolated points
    long long plane;      // nx * ny
    int32_t nx, ny, nx0, ny0, levels, nstokes, abs_norm, pad0;
    int32_t nplanes;       // image planes: nstokes + subring planes
    int32_t flags;         // kRefine* bits
    double r_rel, r_abs;
    // spectral cube renders: the one-axis stencil along ln nu (indices of the
    // images a, b, c, d in the same descriptor array; sb < 0: not a spectral
    // image, sa or sd < 0: that continuation is outside the cube) and its
    // tolerances
    int32_t sa, sb, sc, sd;
    double sr_rel, sr_abs;
};

constexpr int32_t kRefineNearest = 1;     // nearest branch of Eqs. 5-6 and nearest interpolation
constexpr int32_t kRefineAllPlanes = 2;   // criterion ORed over every image plane
constexpr int32_t kRefineOwnNorm = 4;     // ... each plane against its own N_abs and neighbour sum

constexpr int kMaxSub = 8;        // subring planes a ray accumulates
static_assert(4 + kMaxSub <= 12, "Counters::nabs_plane holds every image plane");
constexpr int8_t kMarkSpectral = -3;   // level map: value taken from the spectral neighbours

enum TraceSrc : int { SRC_LIST = 0, SRC_POINTS = 1 };

// Number of set bits of mask below the calling lane (wave-wide prefix).
__device__ __forceinline__ unsigned lane_prefix(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Work item of the pixel queue: image index in the high 32 bits.
__host__ __device__ inline unsigned long long make_item(uint32_t img, uint32_t pix)
{
    return ((unsigned long long)img << 32) | pix;
}

struct TraceJob {
    int src;                      // TraceSrc
    int nimg;                     // images in the batch (Params staged in LDS)
    const Params* params;         // [nimg]
    const ImageDesc* desc;        // [nimg] (pixel sources)
    const unsigned long long* list;   // SRC_LIST: items; front items in order, then the
                                  // back-filled items from list[cap - 1] downwards
    long long cap;                // list capacity (back-filled items)
    long long identity_n;         // > 0: the list is implicit, item = pixel of image 0
    const double* alpha;          // SRC_POINTS
    const double* beta;
    double* out;                  // SRC_POINTS: n x nstokes
    RayFeat* feat;                // SRC_POINTS features (optional)
    uint32_t* count;              // device count of front work items
    uint32_t* count_back;         // device count of back-filled work items (or NULL)
    uint32_t* cursor;             // device queue cursor (zeroed)
    Counters* ctr;                // statistics
    int refill;                   // refill when at least this many lanes idle
};

struct LaunchCfg {
    int trace_blocks;             // persistent grid size of the base pass
    int refine_blocks;            // persistent grid size of the refinement passes
    int trace_threads;            // 64, 128 or 256
    int refill;                   // refill threshold (1..64)
    int long_steps;               // expected steps from which a point is queued first
};

hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_fill_i8(int8_t* p, long long n, int8_t v, hipStream_t s);
hipError_t launch_base_list(const ImageDesc* desc, const Params* params, int nimg, int max_base,
                            unsigned long long* list, long long cap, Counters* ctr, int level_slot, hipStream_t s);
hipError_t launch_trace(int precision, int model, int nstokes, bool subrings, const TraceJob& J,
                        const LaunchCfg& L, hipStream_t s);
hipError_t launch_reduce_base(const ImageDesc* desc, int nimg, Counters* ctr, hipStream_t s, int img_off = 0);
// Base points of the spectral-level images [img_off, img_off + nimg): the
// spectral value where the one-axis rule along ln nu accepts it, else the
// point is queued for tracing in list slot `slot` (front: expected long rays).
hipError_t launch_spectral_base(const ImageDesc* desc, int img_off, int nimg, int max_base, Counters* ctr,
                                unsigned long long* list, long long cap, int long_steps, int slot,
                                hipStream_t s);
// Images [img_off, img_off + nimg) of desc; work items go to list slot
// `slot` (< 0: l + 1, the level's own slot).
// mode 0: plain criterion.  mode 3: spectral images: a point the criterion
// flags takes the spectral value where the rule along ln nu accepts it and is
// traced otherwise.  mode 1: learned, level l -> l+1 (points marked
// proposed are traced, points marked suppressed are interpolated, the
// criterion decides the rest; `fallback` here means all_levels: without it
// images with one level left carry no marks and take the criterion).  mode 2: learned, after a look-ahead pass
// (points already traced are kept, suppressed points are interpolated, the
// criterion decides the rest and its points are traced only if `fallback`).
// Points whose neighbours needed at least `long_steps` geodesic steps are
// queued at the front of the list (traced first), the others from the back
// (list capacity `cap`).
// imap: if given, block z of the launch takes image imap[z] (nimg of them),
// else image img_off + z.  feat: interpolated points inherit feature records
// (images with a feature buffer); 0 where no later network run reads this
// level.
hipError_t launch_estimate(const ImageDesc* desc, int nimg, int nxl_max, int nyl_max, int l,
                           Counters* ctr, unsigned long long* list, long long cap, int long_steps,
                           hipStream_t s, int mode = 0, int fallback = 1, int img_off = 0, int slot = -1,
                           const int* imap = nullptr, int feat = 1);
hipError_t launch_metrics(const double* t, const double* a, long long n, double* partial,
                          int nblocks, hipStream_t s);
int trace_occupancy_blocks(int precision, int model, int nstokes, bool subrings, int threads);

}  // namespace art
