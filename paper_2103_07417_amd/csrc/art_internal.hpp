// art_internal.hpp -- host-side declarations shared by the kernels and the
// C ABI implementation (not part of the public interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "art_device.hpp"

namespace art {

// Device counters of one render, zeroed by a fill kernel at the start.
struct Counters {
    uint32_t count[33];        // per level: points in the trace list
    uint32_t cursor[33];       // per level: work-queue cursor
    unsigned long long steps;  // geodesic steps
    unsigned long long steps_emit;  // steps that evaluated the plasma/transfer
    unsigned long long status[8];
    double scal[4];            // ibar_int, imax0, n_abs, spare
};

enum TraceSrc : int { SRC_LIST = 0, SRC_IDENTITY = 1, SRC_POINTS = 2 };

struct TraceJob {
    int src;                   // TraceSrc
    const uint32_t* list;      // SRC_LIST: pixel indices
    const double* alpha;       // SRC_POINTS
    const double* beta;
    uint32_t* count;           // device count of work items
    uint32_t* cursor;          // device queue cursor (zeroed)
    double* out;               // image planes (pixel sources) or n x nstokes (points)
    long long plane;           // stride between Stokes planes (pixel sources)
    RayFeat* feat;             // optional
    Counters* ctr;             // statistics (steps, status histogram)
    int refill;                // refill when at least this many lanes idle
};

struct LaunchCfg {
    int trace_blocks;          // persistent grid size
    int trace_threads;         // 64..1024, multiple of 64
    int refill;                // refill threshold
};

hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, long long n, double v, hipStream_t s);
hipError_t launch_fill_i8(int8_t* p, long long n, int8_t v, hipStream_t s);
hipError_t launch_base_list(uint32_t* list, uint32_t* count, int nx0, int ny0, int st0,
                            int nx, int8_t* level, hipStream_t s);
hipError_t launch_trace(const Params& P, int precision, const TraceJob& J, const LaunchCfg& L,
                        hipStream_t s);
hipError_t launch_reduce_base(const double* img, int nx, int nx0, int ny0, int st0, int norm,
                              Counters* ctr, hipStream_t s);
hipError_t launch_estimate(double* img, int nstokes, long long plane, int nx, int nx0, int ny0,
                           int levels, int l, double r_rel, double r_abs, Counters* ctr,
                           uint32_t* list, int8_t* level, hipStream_t s);
hipError_t launch_metrics(const double* t, const double* a, long long n, double* partial,
                          int nblocks, hipStream_t s);
int trace_occupancy_blocks(int precision, int model, int nstokes, int threads);

}  // namespace art
