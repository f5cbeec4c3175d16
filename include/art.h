/*
 * art.h -- C ABI of the adaptive black-hole ray tracer for MI355X (gfx950).
 *
 * Method: Gelles, Prather, Palumbo, Johnson, Wong & Georgiev (2021), "The Role
 * of Adaptive Ray Tracing in Analyzing Black Hole Structure", arXiv:2103.07417.
 *
 * The library samples the screen intensity I(x) of a Kerr black hole by
 * backward ray tracing (Sec. 3, opening paragraph) and builds the image by the
 * level-by-level recursive subdivision of Sec. 3.2: an n0x x n0y vertex grid is
 * traced, then each level doubles the resolution, (n) -> (2n - 1) points per
 * axis, and a new point is traced only when both estimated interpolation
 * errors exceed their tolerances (eps_abs > R_abs and eps_rel > R_rel,
 * Eqs. 5-6 linear branch); otherwise it is linearly interpolated.  After N
 * levels n_x = 2^N (n0x - 1) + 1.
 *
 * Conventions (all entry points):
 *  - Units G = c = M = 1; screen coordinates (alpha, beta) are in M at the
 *    hole's distance; x = -fov/2 + i fov/(nx-1), square cells, y centred.
 *  - Buffers named *_dev are device pointers owned by the caller (the
 *    library never frees them).  Images are planar FP64:
 *    image[s][y][x], s = 0..nstokes-1 (I, Q, U, V), followed by the subring
 *    planes of I when art_transfer.subrings > 0.  The level map is int8
 *    [y][x]: -1 interpolated, l >= 0 traced at refinement level l.  The
 *    feature buffer is art_ray_feat[y][x]: traced pixels get their ray's
 *    values; an interpolated pixel gets the smallest r_min and the largest
 *    n_cross of the points it is interpolated from, steps = 0.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Work is enqueued asynchronously; a call that fills an art_stats
 *    synchronises the stream before returning.
 *  - Every call returns ART_OK (0) or a negative error code; the message of
 *    the last failure on the calling thread is art_last_error().
 *  - Scratch memory (trace lists, counters, partial sums) is owned by the
 *    library, grown on demand and kept per device until art_release().
 */
#ifndef ART_H
#define ART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ART_OK        0
#define ART_EINVAL   -1   /* invalid argument (|a| >= 1, n0 < 2, fov <= 0, ...) */
#define ART_ENOMEM   -2   /* device allocation failed, or above the allocation limit */
#define ART_EDEVICE  -3   /* HIP runtime error */
#define ART_ENUMERIC -4   /* a NaN reached the image (rays flagged in features) */

/* emission models */
#define ART_EMIS_TOY_DISK     1   /* j = r^-2 exp(-z^2/(2(h r)^2)), r > r_in, no absorption */
#define ART_EMIS_THERMAL      2   /* power-law thermal plasma, polarised synchrotron */
#define ART_EMIS_GRID         3   /* gridded snapshot (MKS cells), polarised synchrotron */
#define ART_EMIS_SCREEN_RING 10   /* closed-form screen intensity (no ray tracing) */
#define ART_EMIS_SCREEN_POLY 11   /* quadratic screen intensity (no ray tracing) */

/* absolute-error normalisation N_abs */
#define ART_NORM_MEAN 0   /* Ibar_int: mean of the level-0 interpolant (Sec. 3.2) */
#define ART_NORM_MAX  1   /* maximum of the level-0 image */

/* per-ray status */
#define ART_RAY_OK       0
#define ART_RAY_CAPTURED 1
#define ART_RAY_ESCAPED  2
#define ART_RAY_STEPCAP  3
#define ART_RAY_THICK    4
#define ART_RAY_NAN      5

/* transfer precision */
#define ART_PREC_FP64  0  /* geodesic, coefficients and transfer in FP64 */
#define ART_PREC_MIXED 1  /* FP64 geodesic, FP32 plasma/coefficients/transfer */
#define ART_PREC_MIXED_GEO 2  /* as MIXED, and the geodesic right-hand sides in FP32 for
                                 every wave whose rays are all outside the sensitive zones
                                 (art_transfer.fp64_radius / fp64_ktheta); the state,
                                 the RK4 sums and the step rule stay FP64 */

typedef struct {
    double a_spin;                 /* dimensionless spin, |a| < 1 */
} art_spacetime;

typedef struct {
    double r_cam;                  /* camera radius [M], > horizon */
    double inc_deg;                /* inclination [deg], 0 < inc < 180 */
    double fov_M;                  /* screen width [M] at the hole's distance */
    double r_out;                  /* escape radius [M] (<= 0: r_cam) */
    int32_t nx0, ny0;              /* base vertex grid, >= 2 each */
    int32_t levels;                /* refinement levels N, 0..20 */
    int32_t pad;
    double phi_deg;                /* camera azimuth [deg] (matters only for non-axisymmetric
                                      models: the gridded snapshot) */
} art_camera;

typedef struct {
    int32_t kind;                  /* ART_EMIS_* */
    int32_t pad;
    double freq_hz;                /* observing frequency */
    double mass_msun;              /* black-hole mass (sets the length unit GM/c^2) */
    double params[16];             /* model constants, by kind:
        TOY_DISK:    [0] r_in [M], [1] h/r
        THERMAL:     [0] n0 [cm^-3], [1] Theta0, [2] plasma beta at r_ref,
                     [3] r_ref [M], [4] field phase psi0 [rad], [5] outer
                     emission radius [M], [6..8] power-law indices of n_e,
                     Theta_e and |B| (n_e = n0 r^-[6], Theta_e = Theta0 r^-[7],
                     |B| ~ r^-[8]; electron pressure n_e m c^2 Theta_e sets
                     |B| at r_ref from beta)
        GRID:        [0] n_e per code density [cm^-3], [1] R_high, [2] R_low,
                     [3] adiabatic index, [4] sigma cut (no emission where
                     |B|^2/rho exceeds it), [5] outer emission radius [M],
                     [6] x1 = ln r of the first cell edge, [7] dx1,
                     [8] h of theta = pi x2 + (1-h)/2 sin(2 pi x2), [9..11]
                     n1, n2 (<= 256), n3; T_i/T_e = (R_high b^2 + R_low)/(1 + b^2)
                     with b the plasma beta
        SCREEN_RING: [0] radius, [1] width, [2] diffuse amplitude, [3] diffuse scale
        SCREEN_POLY: I = [0] + [1] x + [2] y + [3] x^2 + [4] x y + [5] y^2  */
    const float* grid_dev;         /* GRID: device array [n3][n2][n1][8] of cell-centre
                                      rho, u, v_r, v_th, v_ph (ZAMO frame), B_r, B_th,
                                      B_ph (ZAMO frame, code units); caller-owned */
    int64_t grid_len;              /* GRID: number of floats, n1 n2 n3 8 */
} art_emission;

/* interpolation and error estimate (Eqs. 5-6) */
#define ART_INTERP_LINEAR  0   /* linear branch: neighbour mean, second differences */
#define ART_INTERP_NEAREST 1   /* nearest branch: the nearest neighbour's value (I1 in 2D,
                                  the lower/left neighbour in 1D), gradient estimate */

typedef struct {
    double r_rel;                  /* R_rel (Sec. 3.2); < 0 traces every point */
    double r_abs;                  /* R_abs (Sec. 3.2) */
    int32_t abs_norm;              /* ART_NORM_MEAN or ART_NORM_MAX */
    int32_t interp;                /* ART_INTERP_* */
    int32_t all_planes;            /* 0: the criterion on Stokes I; 1: traced if the criterion
                                      holds on any image plane (Q, U, V, subrings), each
                                      plane's estimate compared with N_abs and |Stokes I|;
                                      2 (linear branch only): the same OR with every plane
                                      compared with its own normalisation (abs_norm applied
                                      to |plane| on the base grid) and its own neighbour
                                      sum, so faint planes are refined on their own
                                      structure (Sec. 6's per-Stokes rule, Sec. 5.1) */
    int32_t pad;
} art_refine;

typedef struct {
    int32_t nstokes;               /* 1 (I) or 4 (I, Q, U, V) */
    int32_t precision;             /* ART_PREC_* (subrings: FP64 or MIXED) */
    int32_t max_steps;             /* geodesic step cap (> 0) */
    int32_t subrings;              /* 0..8: subring decomposition of Stokes I (Sec. 5.1).  The
                                      image then has nstokes + subrings planes; plane
                                      nstokes + n holds the I emitted on the ray's n-th
                                      half-orbit, n = the number of theta turning points (sign
                                      changes of k_theta) the backward ray passed before the
                                      emission point; the last plane collects n >= subrings-1.
                                      The planes sum to I.  Refinement decisions use I; the
                                      planes are interpolated like Q, U, V. */
    double eps;                    /* step-rule accuracy, 0 < eps <= 0.5 */
    double fp64_radius;            /* ART_PREC_MIXED_GEO: FP64 steps where r < this [M]
                                      (photon shell, horizon); <= 0 selects 6 M */
    double fp64_ktheta;            /* ART_PREC_MIXED_GEO: FP64 steps where |k_theta| < this
                                      (theta turning points); < 0 selects 0.05 */
} art_transfer;

typedef struct {
    double* image_dev;             /* [nstokes][ny][nx] FP64, required */
    int8_t* level_dev;             /* [ny][nx], required by art_render */
    void* feat_dev;                /* art_ray_feat[ny][nx] or NULL */
    int32_t nx, ny;                /* must equal the camera's final grid */
} art_image;

typedef struct {
    float rmin;                    /* minimum Boyer-Lindquist radius reached */
    int32_t ncross;                /* equatorial crossings (sign changes of cos theta) */
    int32_t steps;                 /* geodesic steps taken */
    int32_t status;                /* ART_RAY_* */
} art_ray_feat;

typedef struct {
    int64_t rays_traced;           /* base + refined rays */
    int64_t candidates[32];        /* per level: points examined (level 0: base) */
    int64_t traced[32];            /* per level: points ray traced */
    int64_t steps_total;           /* geodesic steps over all traced rays */
    int64_t status_hist[8];        /* rays per ART_RAY_* status */
    double interp_frac;            /* Sec. 4.1, Eq. 7 */
    double ibar_int;               /* trapezoid mean of the level-0 image */
    double imax0;                  /* maximum of the level-0 image */
    double n_abs;                  /* normalisation used for eps_abs */
    int64_t steps_emit;            /* steps that evaluated emission and transfer */
    double t_trace_ms;             /* summed duration of the tracing kernels (HIP events;
                                      the launches of concurrent groups overlap) */
    int32_t trace_launches;        /* number of tracing-kernel launches */
    int32_t levels;
    int64_t learned[5];            /* learned renders (else 0): [0] proposed points the
                                      criterion would not trace, [1] criterion-flagged
                                      points the network suppressed, [2] points the
                                      criterion traced as fallback after a look-ahead
                                      pass, [3] criterion-flagged points left
                                      interpolated (fallback off), [4] look-ahead rays */
    double t_render_ms;            /* wall time of the whole render on the caller's stream
                                      (HIP events; eager renders, else 0) */
    int64_t spectral;              /* spectral cube renders: points that took the spectral
                                      neighbours' value instead of a ray (else 0) */
} art_stats;

/* Final grid size n = 2^N (n0 - 1) + 1 per axis (Sec. 3.2) and the image size
 * in bytes for nstokes planes.  No device work. */
int art_image_size(const art_camera* cam, int32_t nstokes,
                   int32_t* nx, int32_t* ny, size_t* image_bytes);

/* Adaptive render (Sec. 3.2): trace the base grid, then for each level
 * estimate, interpolate, compact the points to trace (wavefront ballot) and
 * trace them with the persistent work-queue kernel.  The level loop runs on
 * the device without host synchronisation.  If st != NULL the stream is
 * synchronised and the statistics are filled; then ART_ENUMERIC is returned
 * if any traced ray produced a NaN. */
int art_render(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
               const art_refine* rf, const art_transfer* tr, art_image* out,
               art_stats* st, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * adaptive render as art_render, with the trace list, cost map, counters,
 * parameter block, descriptor and theta table in a static device array of
 * the library (about 42 MB, held by each device the library runs on until
 * the process ends) instead of library allocations.  Images of at most
 * 2049 x 2049 pixels (any base grid and level count reaching at most that);
 * larger ones return ART_EINVAL before any device work.  Calls no hipMalloc,
 * hipFree, stream or event creation; the first call on a device looks up its
 * array's address.  The caller still owns and passes the image, level-map
 * and feature buffers.  Every call on one device shares that device's array
 * and leaves its contents behind (the counters are cleared at the start of
 * each render): calls that overlap on one device, on any streams, race.
 * Statistics as art_render, except that t_trace_ms, t_render_ms and
 * trace-launch timing are not recorded (0). */
int art_render_noalloc(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_refine* rf, const art_transfer* tr, art_image* out,
                       art_stats* st, void* stream);

/* Uniform render: one ray per vertex of the camera's final grid (the "truth"
 * image of Sec. 4.1).  The level map, if given, is set to 0 everywhere. */
int art_render_uniform(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_transfer* tr, art_image* out, art_stats* st, void* stream);

/* Trace n arbitrary screen points (alpha_dev[i], beta_dev[i]) [M]; writes
 * stokes_dev[i*(nstokes+subrings) + s] (FP64: Stokes, then the subring
 * planes of I) and, if feat_dev != NULL, art_ray_feat[i].
 * The camera's grid fields are ignored. */
int art_trace_points(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                     const art_transfer* tr, int64_t n, const double* alpha_dev,
                     const double* beta_dev, double* stokes_dev, void* feat_dev,
                     void* stream);

/* ------------------------------------------------------------------ batches
 * Many images (different spin, inclination, frequency, tolerances and number
 * of levels) rendered together: every level's new rays of every image go into
 * one work queue of the persistent tracer, so long photon-ring rays of one
 * image overlap with the work of the others.  All images of a batch use the
 * same emission kind, nstokes, precision and subring count, and gridded-model
 * images the same theta grid (h and n2; the snapshots themselves may differ);
 * at most 64 images. */
typedef struct {
    art_spacetime sp;
    art_camera cam;
    art_emission em;
    art_refine rf;
    art_transfer tr;
} art_job;

typedef struct art_batch art_batch;   /* opaque */

/* Validate n jobs and their caller-owned output images (image_dev and
 * level_dev required, nx/ny equal to each camera's final grid), allocate the
 * batch's device scratch (trace list of sum nx*ny 8-byte items, counters,
 * descriptors) and upload the descriptors.  Synchronises the null stream. */
int art_batch_create(int32_t n, const art_job* jobs, const art_image* images, art_batch** out);

/* Enqueue one adaptive render of every image of the batch on `stream`
 * (asynchronous; the tracing launches are timed with HIP events). */
int art_batch_render(art_batch* b, void* stream);

/* Capture the batch's whole level loop (clears, base lists, tracing,
 * reductions, estimators) into a hipGraph on a non-default `stream`; the
 * graph contains kernel nodes only.  Replaces a previous capture. */
int art_batch_capture(art_batch* b, void* stream);

/* Replay the captured graph on `stream` (asynchronous). */
int art_batch_launch(art_batch* b, void* stream);

/* Statistics of image i of the last render or replay (i = -1: all images
 * summed; ibar_int/imax0/n_abs then refer to image 0).  Synchronises. */
int art_batch_stats(art_batch* b, int32_t i, art_stats* st, void* stream);

/* Free the batch (after synchronising the device). */
int art_batch_destroy(art_batch* b);

/* Upper bound on the device memory one render or batch may allocate for its
 * trace list and cost map (10 bytes per pixel of the batch; 0 = no bound, the
 * default).  A render or batch set-up that would need more returns ART_ENOMEM
 * and leaves earlier buffers in place; buffers already allocated are kept.
 * Process-wide, applies to later calls. */
int art_set_alloc_limit(size_t bytes);

/* ------------------------------------------------------- launch configuration
 * Persistent-tracer launch shape: grid size, threads per block (64, 128 or
 * 256) and the refill threshold (a wave claims new rays when at least this
 * many of its lanes are idle).  Zero fields select the defaults (one block per
 * CU per resident block of the kernel's occupancy, 256 threads, refill 1).
 * art_set_launch applies to renders issued afterwards (process-wide). */
typedef struct {
    int32_t trace_blocks;
    int32_t trace_threads;
    int32_t refill;
    int32_t groups;                /* batches: images are split into this many groups of
                                      consecutive images, each running its level loop on its
                                      own stream (forked from and joined back into the
                                      caller's stream) so that one group's long-ray tail
                                      overlaps the others' work; 0 = two groups from 16
                                      images on, else one; at most 8 */
    int32_t refine_blocks;         /* grid size of the refinement passes (every pass after a
                                      batch's base grid, and a cube's passes after its first);
                                      0 = trace_blocks */
    int32_t long_steps;            /* refinement queues: a new point whose neighbours' largest
                                      step count reaches this is queued at the front of its pass
                                      (started first), the others at the back; 0 = 800; at most
                                      65535 */
} art_launch;

int art_set_launch(const art_launch* launch);
int art_get_launch(int32_t precision, int32_t kind, int32_t nstokes, art_launch* launch);

/* Launch shape of one batch (used by its next render or capture; a captured
 * graph keeps the shape it was captured with, except that a new group count
 * discards the captured graph).  Synchronises the device when the group
 * count changes. */
int art_batch_set_launch(art_batch* b, const art_launch* launch);
int art_batch_get_launch(const art_batch* b, art_launch* launch);

/* ----------------------------------------------- learned refinement proposal
 * A small convolutional network (4 layers of 3x3 convolutions, channels
 * 3 -> 32 -> 32 -> 32 -> 15, ReLU between layers; 23,727 FP32 master
 * parameters, BF16 MFMA arithmetic with FP32 accumulation) reads the level-l
 * vertex grid of an adaptive render and predicts, for each level-l vertex,
 * whether each of the 15 new points of its cell (3 at level l+1, 12 at level
 * l+2) is traced by the refinement criterion of Sec. 3.2.  It is trained on
 * level maps of plain renders.  In a learned render the network looks ahead:
 * level-(l+2) points it proposes are traced in the same pass as level l+1, and
 * the criterion of Eqs. 5-6 stays the judge (every point it flags is counted)
 * and the fallback (flagged points the look-ahead missed are traced).
 *
 * Tensors (device, caller-owned):
 *   features  x[B][3][H][W] FP32: ln(max(I,0)/N_abs + 1e-4), min(r_min, 20)/10,
 *             min(n_cross, 4)/4 at the level-l vertices (H = 2^l (n0y-1) + 1,
 *             W = 2^l (n0x-1) + 1)
 *   logits    z[B][15][H][W] FP32
 *   labels, valid  [B][15][H][W] uint8 (valid = the point exists)
 * Output k of vertex (i, j): k = 0..2 the level-(l+1) points (2i+1, 2j),
 * (2i, 2j+1), (2i+1, 2j+1); k = 3..14 the level-(l+2) points (4i+dx, 4j+dy)
 * with (dx, dy) in row-major order over the 4x4 block, both even excluded.
 * Parameter order: W0, b0, W1, b1, W2, b2, W3, b3, W[l] as [c_out][c_in][3][3].
 * The forward/gradient/training calls of one network share its workspace:
 * issue them on one stream at a time. */
typedef struct art_cnn art_cnn;       /* opaque */

/* Number of FP32 parameters (23,727). */
int art_cnn_num_params(void);

/* Create a network with seeded He-normal weights and zero biases. */
int art_cnn_create(uint64_t seed, art_cnn** out);
int art_cnn_destroy(art_cnn* net);

/* Copy n FP32 parameters from / to host memory; set also resets the Adam
 * state.  Both synchronise the device. */
int art_cnn_set_params(art_cnn* net, const float* host, int64_t n);
int art_cnn_get_params(art_cnn* net, float* host, int64_t n);

/* Logits of B feature grids (B H W <= 2^28).  Asynchronous on `stream`. */
int art_cnn_forward(art_cnn* net, const float* x_dev, int32_t B, int32_t H, int32_t W,
                    float* logits_dev, void* stream);

/* Loss L = mean over valid outputs of the positive-weighted binary cross-
 * entropy -[w y ln s(z) + (1-y) ln(1-s(z))], and its gradient w.r.t. every
 * parameter (copied to grad_host[num_params] if non-NULL; the loss to
 * *loss_out if non-NULL).  Synchronises when either output is requested. */
int art_cnn_gradients(art_cnn* net, const float* x_dev, const uint8_t* labels_dev,
                      const uint8_t* valid_dev, int32_t B, int32_t H, int32_t W,
                      float pos_weight, float* grad_host, float* loss_out, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of the loss above; the loss before the step goes to *loss_out if
 * non-NULL (then synchronises). */
int art_cnn_train_step(art_cnn* net, const float* x_dev, const uint8_t* labels_dev,
                       const uint8_t* valid_dev, int32_t B, int32_t H, int32_t W, float lr,
                       float pos_weight, float* loss_out, void* stream);

/* Features of level `level` of one rendered image (image plane 0 and the
 * art_ray_feat buffer, NULL = zeros for r_min and n_cross) into x_dev[3][H][W]. */
int art_cnn_features(const double* image_dev, const void* feat_dev, int32_t nx, int32_t ny,
                     int32_t nx0, int32_t ny0, int32_t levels, int32_t level, double n_abs,
                     float* x_dev, void* stream);

/* Training labels of level `level` (< levels) from a plain render's level map:
 * label = 1 if the point was traced at its own level. */
int art_cnn_labels(const int8_t* level_dev, int32_t nx, int32_t ny, int32_t nx0, int32_t ny0,
                   int32_t levels, int32_t level, uint8_t* labels_dev, uint8_t* valid_dev,
                   void* stream);

typedef struct {
    float z_propose;               /* logit above which a point is traced without waiting
                                      for the criterion */
    float z_suppress;              /* logit below which a flagged point is interpolated
                                      (-INFINITY: never) */
    int32_t fallback;              /* 1: after a look-ahead pass the criterion traces the
                                      points it flags that were not traced; 0: it only
                                      counts them (art_stats.learned[3]) */
    int32_t all_levels;            /* 0: the network runs only at levels l with l + 2 <= N
                                      (look-ahead); 1: also at l = N - 1 */
    int32_t level_cap;             /* 0: the network runs at every such level; k > 0: only at
                                      levels l < k, deeper levels take the criterion alone */
    int32_t pad;
} art_learned;

/* Switch a batch to learned renders with `net` (NULL: back to plain).  All
 * images need the same base grid and feature buffers (art_image.feat_dev);
 * their level counts may differ.  In a learned render the feature records of
 * interpolated points are written only on the levels up to the last one the
 * network reads (traced points always get theirs); elsewhere the buffer keeps
 * what it held.  Allocates the batch's own network workspace; later
 * art_batch_render / art_batch_capture use the network (a captured graph
 * reads the parameters at replay, so training in between is seen).  `net`
 * must outlive the batch's use of it. */
int art_batch_set_learned(art_batch* b, art_cnn* net, const art_learned* opt);

/* Single-image learned render (like art_render, plus the network). */
int art_render_learned(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                       const art_refine* rf, const art_transfer* tr, art_cnn* net,
                       const art_learned* opt, art_image* out, art_stats* st, void* stream);

/* Adaptive sampling along frequency (the extension to the frequency domain
 * that Sec. 6 proposes, built from the one-axis rule of Sec. 3.2).  The cube
 * has n = 2^levels (n0 - 1) + 1 images (n <= 64) at frequencies equally spaced
 * in ln nu from nu_min_hz to nu_max_hz (em->freq_hz is ignored); out[i] is
 * image i in frequency order, each with the camera's final grid and a level
 * map, and st (if non-NULL) receives n per-image statistics (step counts,
 * status histogram and timings are cube-wide).  Images at indices k 2^levels
 * are the base frequencies: plain adaptive renders (Sec. 3.2).  Spectral
 * level s adds the odd multiples of h = 2^(levels - s).  In those images every
 * base point and every point the spatial criterion flags first tries the
 * spectral value (b + c)/2 of the finished images b, c at indices i -+ h,
 * accepted unless, with the continuations a, d at i -+ 3h,
 *   |D| > 8 r_abs N_abs  and  |D| > 4 r_rel |b + c|,   D = (a + d) - (b + c)
 * (twice the one-sided second difference if a or d is outside the cube, never
 * accepted if both are; N_abs the mean of b's and c's own N_abs; every plane
 * with rf->all_planes, which must be 0 or 1 here); points it rejects are traced.  Level map: l = traced at
 * spatial level l, -1 spatially interpolated, -3 spectral value.  Eager (for
 * capture and replay see art_cube_create); camera levels + spectral levels
 * <= 21.  The decisions of
 * spectral level s at spatial level l need only the coarser levels, so they
 * run as a wavefront: camera levels + levels + 1 tracing passes. */
typedef struct {
    double nu_min_hz, nu_max_hz;   /* first and last frequency, 0 < nu_min < nu_max */
    int32_t n0;                    /* base frequencies, >= 2 */
    int32_t levels;                /* refinements along ln nu, 0..6 */
    double r_rel, r_abs;           /* tolerances of the spectral rule (< 0: never accepted) */
} art_spectral;

int art_render_spectral(const art_spacetime* sp, const art_camera* cam, const art_emission* em,
                        const art_refine* rf, const art_transfer* tr, const art_spectral* spec,
                        art_image* out, art_stats* st, void* stream);

/* The same adaptive sampling along any sequence axis (time, frequency, ...):
 * jobs[n] in axis order, taken as equally spaced along it (snapshots of a
 * movie at a fixed cadence, frequencies equally spaced in ln nu, ...), with
 * n = 2^levels (n0 - 1) + 1 <= 64 and one base grid and level count; the
 * rule above with tolerances r_rel, r_abs decides between the axis
 * neighbours' mean and a ray.  Gridded-model images may use different
 * snapshots of one theta grid (same h and n2).  Sec. 6 names time sampling
 * for movies as the other target of the extension. */
int art_render_cube(int32_t n, const art_job* jobs, int32_t n0, int32_t levels, double r_rel, double r_abs,
                    art_image* out, art_stats* st, void* stream);

/* The cube of art_render_cube as a batch object, set up once: jobs and the
 * caller-owned images (as for art_batch_create) in axis order.  It takes
 * art_batch_render (eager, timed), art_batch_capture / art_batch_launch (one
 * hipGraph of the whole wavefront), art_batch_stats (image index in axis
 * order, -1 for the whole cube), art_batch_set_launch (tracing grid and
 * refill; always one image group) and art_batch_destroy; art_batch_set_learned
 * rejects a network (the cube renders with the criterion).  Cubes on
 * different streams can be in flight together.  Synchronises the null
 * stream. */
int art_cube_create(int32_t n, const art_job* jobs, int32_t n0, int32_t levels, double r_rel, double r_abs,
                    const art_image* images, art_batch** out);

/* Image metrics of Sec. 4.1 on n FP64 values (one Stokes plane), computed on
 * the device with a deterministic two-pass reduction; synchronises:
 *   flux error = |sum t - sum a| / |sum t|   (Eq. 8)
 *   MSE        = sum (t - a)^2 / sum t^2     (Eq. 9)                      */
int art_metrics(const double* truth_dev, const double* approx_dev, int64_t n,
                double* flux_error, double* mse, void* stream);

/* Visibilities of screen images (Sec. 4.3): complex Fourier components on a
 * rectangle of baselines, u_dev[nu] x v_dev[nv] in cycles per unit of screen
 * coordinate,
 *   V(u_m, v_l) = dx^2 sum_j sum_i g(x_i) g(y_j) I[j][i] exp(-2 pi i (u_m x_i + v_l y_j)),
 * pixel (j, i) at x_i = (i - (nx-1)/2) dx, y_j = (j - (ny-1)/2) dx (square
 * pixels, image centre on the origin), for each of `nplanes` FP64 planes
 * I = img_dev + z * plane_stride (row-major ny x nx, device).  The Gaussian
 * taper g(x) = exp(-4 ln 2 x^2 / fwhm^2) is the paper's guard against power
 * from the field edge (fwhm <= 0: none).  Output vis_dev[nplanes][nv][nu][2]
 * (re, im) FP64, device; the residual visibilities of Sec. 4.3 are those of
 * the residual image.  Computed in FP64 (matrix cores) as two separable
 * stages through the caller's device workspace of art_vis_workspace_bytes()
 * bytes; asynchronous on `stream`, no allocation.  Empty images give V = 0;
 * nplanes, nu or nv = 0 is a no-op.  ART_EINVAL for negative or oversized
 * sizes, dx <= 0, a non-finite fwhm, NULL pointers or a short workspace. */
size_t art_vis_workspace_bytes(int32_t nplanes, int32_t nx, int32_t ny, int32_t nu, int32_t nv);
int art_visibility(const double* img_dev, int64_t plane_stride, int32_t nplanes, int32_t nx, int32_t ny,
                   double dx, double fwhm, const double* u_dev, int32_t nu, const double* v_dev, int32_t nv,
                   double* vis_dev, void* work_dev, size_t work_bytes, void* stream);

/* A non-blocking HIP stream created by the library for the current device
 * (the runtime gives each new stream its least-used hardware queue).  Batches
 * replayed on distinct such streams run concurrently: with two batches in
 * flight one batch's latency-bound refinement passes overlap the other's
 * base pass.  Streams taken from a framework's pool can share one hardware
 * queue and then serialise.  Destroy with art_stream_destroy (synchronises). */
int art_stream_create(void** stream);
int art_stream_destroy(void* stream);

/* Last error message of the calling thread ("" if none). */
const char* art_last_error(void);

/* Free the library's scratch memory on every device (after synchronising). */
int art_release(void);

#ifdef __cplusplus
}
#endif
#endif /* ART_H */
