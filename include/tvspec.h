/*
 * tvspec -- spectral total-variation decomposition on one AMD MI355X (gfx950).
 *
 * The method is that of Grossmann, Korolev, Gilboa, Schoenlieb, "Deeply
 * Learned Spectral Total Variation Decomposition" (arXiv 2006.10004):
 *
 *   TV flow, Sec. 2.1 Eq. (1):      u_t = -p, p in dJ(u), u(0) = f, with J the
 *                                   isotropic TV of Eq. (2);
 *   implicit Euler, Sec. 2.2 Eq. (8): u_{s+1} = argmin_v 0.5||u_s - v||^2
 *                                   + dt J(v), one ROF problem per step, solved
 *                                   by Chambolle's dual projection iteration
 *                                   (the solver Sec. 4.3 names);
 *   TV transform, Eq. (3):          phi(t) = t u_tt(t), on t_k = k dt by the
 *                                   central second difference;
 *   spectrum (display after Eq. (3)): S(t_k) = ||phi(t_k)||_1;
 *   bands, Eq. (7):                 b_j = integral of phi over (t_{e_{j-1}}, t_{e_j}];
 *   residual, Eq. (5):              f_r(T) = u(T) - T u_t(T), T = K dt,
 *                                   so that f = sum_j b_j + f_r.
 *
 * Discretisation (the paper only says "finite differences"): forward
 * differences with Neumann boundary for the gradient, the negative adjoint
 * for the divergence, isotropic pointwise norm; Chambolle's semi-implicit
 * update  p <- (p + tau grad w) / (1 + tau |grad w|),  w = div p - g/dt,
 * v = g - dt div p.  Every ROF solve starts from p = 0 by default (cold
 * start; see warm_start below).  K counts spectral samples phi_1..phi_K, which takes K+1
 * ROF solves (u_1..u_{K+1}).  Band edges are step indices
 * 0 = e_0 < e_1 < ... < e_B = K; band j holds the samples e_{j-1} < k <= e_j.
 * The residual is returned on its own (the paper adds it to the last band).
 *
 * Layouts (row-major, column index fastest):
 *   f         [C][H][W]  float32
 *   bands     [n_bands][C][H][W]  float64
 *   S         [C][K]     float64,  S[c][k-1] = S_c(t_k)
 *   residual  [C][H][W]  float64
 * Channels are independent decompositions.
 *
 * Precision: the inner Chambolle iterations run in one of the modes
 * TVSPEC_PRECISION_* below.  The flow state u, its step differences, phi,
 * the bands, S and the reconstruction check are always float64.
 *
 * Threading and streams: the decomposition entry points (tvspec_decompose,
 * _ex, _dev, _pdhg_dev, _batch_dev) may be called from any host thread and
 * on any streams.  Calls of one precision mode on one device share that
 * device's scratch memory; each call's device work is ordered after the
 * previous call's on the device (its stream waits for an event the previous
 * call recorded on its own stream), so calls on different streams run one
 * after the other and never mix their state.  The host is not blocked by
 * this ordering.  The server (tvspec_server_*) has memory of its own.
 */
#ifndef TVSPEC_H
#define TVSPEC_H

#include <stddef.h>

/* Symbols of the C ABI (the library is built with hidden visibility). */
#if defined(__GNUC__) || defined(__clang__)
#define TVSPEC_API __attribute__((visibility("default")))
#else
#define TVSPEC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define TVSPEC_OK 0
#define TVSPEC_EINVAL (-1)   /* invalid argument; nothing was done on the device */
#define TVSPEC_ENUMERIC (-2) /* non-finite input value (host buffers, or tvspec_decompose_ex with a report) */
#define TVSPEC_ENOMEM (-3)   /* device or host allocation failed */
#define TVSPEC_EDEVICE (-4)  /* HIP runtime error; tvspec_last_error() has the text */
#define TVSPEC_EBUSY (-5)    /* request can never fit the server's memory budget */
#define TVSPEC_PENDING 1     /* tvspec_poll: the request is not complete yet */

/* Precision of the inner Chambolle iteration:
 *   F32    float32 dual field and arithmetic (fastest; on long flows its
 *          rounding moves the bands by more than 2e-4, e.g. ~4.5e-4 on a
 *          512x512 image with dt = 0.002, K = 200, 300 iterations)
 *   F64    IEEE float64 dual field and arithmetic
 *   MIXED  float64 dual field and arithmetic; |grad w| and the reciprocal
 *          from float32 hardware estimates refined by one float64 Newton
 *          step.  Float64-level results
 *          (~3e-6 on the workload above) at less cost than F64.  Default. */
#define TVSPEC_PRECISION_F32 0
#define TVSPEC_PRECISION_F64 1
#define TVSPEC_PRECISION_MIXED 2
#define TVSPEC_DEFAULT_PRECISION TVSPEC_PRECISION_MIXED

#define TVSPEC_DEFAULT_TAU 0.248
/* Default primal and dual steps of the primal-dual solver: 1/sqrt(8), so
 * that tau sigma ||grad||^2 <= 1 (||grad||^2 <= 8). */
#define TVSPEC_PDHG_DEFAULT_STEP 0.35355339059327373

/* Number of doubles tvspec_decompose_dev writes to its stats buffer. */
#define TVSPEC_NSTATS 4

/*
 * Host entry point: decompose a C x H x W float32 image held in host memory.
 * Synchronous.  The caller owns and allocates every buffer (sizes above);
 * the library keeps no pointer after return.  Defaults: tau = 0.248, cold
 * start, TVSPEC_DEFAULT_PRECISION, automatic temporal blocking.
 *
 *   dt           time step of the flow (> 0, finite)
 *   K            number of spectral samples (>= 1); K+1 ROF solves are run
 *   inner_iters  Chambolle iterations per ROF solve (>= 1)
 *   band_edges   n_bands+1 step indices, 0 = e_0 < ... < e_B = K
 *
 * Errors: TVSPEC_EINVAL for H < 2, W < 2, C < 1, C > 65535, H*W > 2^30,
 * C*H*W > 2^40, bad dt, K, inner_iters, n_bands, edges or a null pointer;
 * TVSPEC_ENUMERIC if f holds a NaN or infinity (checked on the host before
 * any device work); TVSPEC_ENOMEM; TVSPEC_EDEVICE.  Outputs are unspecified
 * on error.
 */
TVSPEC_API int tvspec_decompose(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                     const int *band_edges, int n_bands, double *bands, double *S,
                     double *residual);

/*
 * Entry point with an options struct and a per-call report (the device work
 * and wall time of the call, and the checks of the decomposition).
 *
 * args:  the image and the outputs, layouts as above.  f, bands, S, residual
 *        and stats are host pointers with device_ptrs = 0 (stats may then be
 *        NULL) and device pointers with device_ptrs = 1 (stats required,
 *        TVSPEC_NSTATS doubles, filled as by tvspec_decompose_dev);
 *        band_edges is always a host array.
 * opt:   NULL = the defaults tvspec_default_options() fills (as
 *        tvspec_decompose: Chambolle, tau 0.248, cold start, MIXED,
 *        automatic blocking, host buffers).
 *          solver            TVSPEC_SOLVER_CHAMBOLLE or TVSPEC_SOLVER_PDHG
 *          tau, sigma        Chambolle step (0 = 0.248; sigma unused), or
 *                            the primal-dual steps (both 0 = 1/sqrt(8) each)
 *          warm_start, precision, iters_per_launch
 *                            as tvspec_decompose_dev
 *          device_ptrs       0: host buffers, the call is synchronous;
 *                            1: device buffers, work enqueued on `stream`
 *          stream            hipStream_t for device_ptrs = 1 (NULL = null stream)
 *          tile_shape        output pixels per workgroup of the Chambolle
 *                            tile kernel: TVSPEC_TILE_SQUARE (32 x 32 on
 *                            1024 threads, the default) or TVSPEC_TILE_NARROW
 *                            (32 x 16 on 512 threads: twice the workgroups
 *                            for images too small to fill the device;
 *                            iters_per_launch <= 8, Chambolle only).  Results
 *                            do not depend on the shape.
 * rep:   NULL = no report.  Otherwise the call waits until its work is
 *        complete (also with device_ptrs = 1) and fills
 *          recon_err   max |f - sum of bands - residual|
 *          mean_err    max over channels of |mean(u_{K+1}) - mean(f_c)|
 *          nonfinite   number of non-finite values in f
 *          device_ms   device time from the first to the last kernel of the
 *                      decomposition (hipEvents on its stream; excludes the
 *                      host-buffer copies)
 *          total_ms    host wall time of the whole call
 *
 * Errors: as tvspec_decompose_dev, TVSPEC_EINVAL for a bad solver,
 * device_ptrs, tile_shape or step, and TVSPEC_ENUMERIC for non-finite input: with host
 * buffers before any device work; with device buffers when a report is
 * requested (after the work: the outputs are then meaningless; without a
 * report the count is only in stats[2]).
 */
#define TVSPEC_SOLVER_CHAMBOLLE 0
#define TVSPEC_SOLVER_PDHG 1
#define TVSPEC_TILE_SQUARE 0
#define TVSPEC_TILE_NARROW 1

typedef struct tvspec_args {
    const float *f;
    int H, W, C;
    double dt;
    int K;
    int inner_iters;
    const int *band_edges;
    int n_bands;
    double *bands;
    double *S;
    double *residual;
    double *stats;
} tvspec_args;

typedef struct tvspec_options {
    int solver;
    double tau;
    double sigma;
    int warm_start;
    int precision;
    int iters_per_launch;
    int device_ptrs;
    void *stream;
    int tile_shape;
} tvspec_options;

typedef struct tvspec_report {
    double recon_err;
    double mean_err;
    double nonfinite;
    double device_ms;
    double total_ms;
} tvspec_report;

TVSPEC_API void tvspec_default_options(tvspec_options *opt);
TVSPEC_API int tvspec_decompose_ex(const tvspec_args *args, const tvspec_options *opt, tvspec_report *rep);

/*
 * Device entry point with all options.  f, bands, S, residual and stats are
 * DEVICE pointers (e.g. torch tensors' data_ptr()); band_edges is a HOST
 * array.  The work is enqueued on `stream` (a hipStream_t; NULL = the null
 * stream) and the call returns without waiting; the caller keeps every
 * buffer alive until the stream has completed it.
 *
 *   tau               Chambolle step, 0 < tau <= 0.25 (Chambolle's theorem
 *                     asks tau <= 1/8; up to 1/4 converges in practice)
 *   warm_start        0 (default of tvspec_decompose): every ROF solve
 *                     starts its dual field from zero; 1: the dual field
 *                     carries over from the previous solve.  The paper does
 *                     not say which.  Warm starting converges each solve
 *                     further for the same inner_iters, but the dual field
 *                     is not unique and drifts from solve to solve: over
 *                     long flows (200 steps of 300 iterations on 512x512)
 *                     the result then changes by ~1e-3 under a one-ulp
 *                     change of one input pixel, against ~3e-7 cold.
 *   precision         TVSPEC_PRECISION_F32, _F64 or _MIXED
 *   iters_per_launch  temporal blocking factor: Chambolle iterations done per
 *                     kernel launch on an LDS-resident tile (1..16 for F32,
 *                     1..8 for F64 and MIXED; 0 = automatic: 8 for F32, 5 for
 *                     F64, and for MIXED 5 when a launch has at least two
 *                     workgroups per compute unit (several images or
 *                     channels, or planes above ~512x512) and planes larger
 *                     than 64x64, else 8).  Results
 *                     do not depend on it: every variant applies the same
 *                     per-pixel arithmetic in the same order.
 *   stats             TVSPEC_NSTATS doubles (device): [0] max |f - sum of
 *                     bands - residual|, [1] max over channels of
 *                     |mean(u_{K+1}) - mean(f_c)|, [2] number of non-finite
 *                     values found in f (the outputs are then meaningless),
 *                     [3] reserved (0).
 *
 * Errors: as tvspec_decompose, except that non-finite input is reported in
 * stats[2] instead of a return code.  Argument validation happens before any
 * device work.
 */
TVSPEC_API int tvspec_decompose_dev(const float *f, int H, int W, int C, double dt, int K,
                         int inner_iters, const int *band_edges, int n_bands, double *bands,
                         double *S, double *residual, double *stats, double tau, int warm_start,
                         int precision, int iters_per_launch, void *stream);

/*
 * Allocation-free variant of tvspec_decompose_dev, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (bit for bit),
 * layouts, ownership, ordering and errors as tvspec_decompose_dev.  The call
 * allocates nothing (no hipMalloc, no pinned staging, no memset: one setup
 * kernel writes the slot table from arguments passed by value); its scratch
 * is a fixed 64 MiB device array inside the library, one per device, held
 * until the process ends.
 *
 * Limits: the decomposition's scratch must fit in 64 MiB, about
 * C*H*W*(2*4*s + 2*g + 24) + 8*C*K*ceil(H*W/256) bytes + 4*K (s, g as for the
 * server's working state: 512x512x1 at K = 200 in MIXED needs ~16 MB,
 * 1024x1024x1 does not fit), and n_bands <= 64; larger calls return
 * TVSPEC_EINVAL with the size in the message, before any device work.
 *
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (everything a call reads is written by the call first):
 * calls that overlap on one device -- different streams or threads --
 * race.  Serialise them.  Calls of the other entry points do not share it.
 */
TVSPEC_API int tvspec_decompose_noalloc_dev(const float *f, int H, int W, int C, double dt, int K,
                                            int inner_iters, const int *band_edges, int n_bands,
                                            double *bands, double *S, double *residual, double *stats,
                                            double tau, int warm_start, int precision,
                                            int iters_per_launch, void *stream);

/*
 * Device entry point with the primal-dual ROF solver in place of Chambolle's
 * dual fixed point: every implicit Euler step (Sec. 2.2, Eq. (8)) is solved by
 * inner_iters iterations of Chambolle and Pock's first-order primal-dual
 * algorithm (2011, Algorithm 1; the paper's GPU baseline is a primal-dual
 * solver, Sec. 4.3) with operator grad, F = dt ||.||_{2,1}, G = 0.5 ||. - u_k||^2:
 *     y    <- proj_{|y| <= dt}(y + sigma grad xbar)
 *     x'   <- (x + tau div y + tau u_k) / (1 + tau)
 *     xbar <- 2 x' - x,   x <- x'
 * from x = xbar = u_k; u_{k+1} = x after the last iteration.  The spectral
 * transform, bands, S, residual and report are those of
 * tvspec_decompose_dev, computed from this flow.
 *
 *   tau, sigma  primal and dual steps, tau > 0, sigma > 0, 8 tau sigma <= 1;
 *               tau = sigma = 0 selects TVSPEC_PDHG_DEFAULT_STEP for both
 *   warm_start  0: every solve starts with y = 0; 1: y carries over from the
 *               previous solve (x and xbar always start at u_k)
 *   other arguments, layouts, ownership and ordering as
 *   tvspec_decompose_dev (iters_per_launch: the same ranges and automatic
 *   choice, for this solver's tile kernel).
 *
 * Errors: TVSPEC_EINVAL for bad steps and as tvspec_decompose_dev.
 */
TVSPEC_API int tvspec_decompose_pdhg_dev(const float *f, int H, int W, int C, double dt, int K,
                                         int inner_iters, const int *band_edges, int n_bands,
                                         double *bands, double *S, double *residual, double *stats,
                                         double tau, double sigma, int warm_start, int precision,
                                         int iters_per_launch, void *stream);

/*
 * Batched device entry point: B images of the same size (H, W, C) and the
 * same number of Chambolle iterations, each with its own dt, K and band
 * edges, decomposed in one sequence of launches (every kernel covers all
 * B*C channel planes; an image whose flow is complete is skipped by later
 * launches).  Results are those of B separate tvspec_decompose_dev calls
 * with the same options, bit for bit.
 *
 *   f          device, [B][C][H][W] float32
 *   dt, K      host arrays [B]
 *   band_edges host, image b's n_bands[b]+1 edges, concatenated in image order
 *   n_bands    host array [B]
 *   bands      device, image b's [n_bands[b]][C][H][W] float64 blocks
 *              concatenated in image order
 *   S          device, image b's [C][K[b]] float64 blocks concatenated
 *   residual   device, [B][C][H][W] float64
 *   stats      device, [B][TVSPEC_NSTATS] float64 (as tvspec_decompose_dev)
 *   other arguments as tvspec_decompose_dev.
 *
 * Ownership and ordering as tvspec_decompose_dev.  Errors: TVSPEC_EINVAL for
 * B < 1, B*C > 65535, B*C*H*W > 2^40, or any image's invalid dt, K, n_bands
 * or edges (the message names the image), and as tvspec_decompose_dev
 * otherwise.
 */
TVSPEC_API int tvspec_decompose_batch_dev(const float *f, int B, int H, int W, int C, int inner_iters,
                               const double *dt, const int *K, const int *band_edges,
                               const int *n_bands, double *bands, double *S, double *residual,
                               double *stats, double tau, int warm_start, int precision,
                               int iters_per_launch, void *stream);

/*
 * Decomposition server: continuous batching of requests of mixed sizes on
 * one device (the spectral transform of Sec. 2.1 over the flow of Sec. 2.2,
 * as tvspec_decompose_dev, for a stream of images).
 *
 * A server owns a worker thread, one pool of device memory of budget_bytes
 * for the requests' working state, and one stream per size bucket (requests
 * with equal H, W, C and inner_iters).  A submitted request waits in a FIFO
 * queue until its working state fits in the pool and its bucket runs fewer
 * than its cap of requests -- as many as fill the device on their own
 * (16 workgroups per compute unit, one per 32 x 32 tile and channel): two
 * for 3 x 1024 x 1024, 86 for 3 x 128 x 128; more would only share the
 * device and each finish later.  A request held back by its bucket's cap
 * does not hold back requests of other buckets; a request that does not fit
 * in memory holds back everything after it.  Once admitted it joins at the
 * bucket's next step boundary and advances one ROF solve per bucket step
 * alongside the bucket's other requests.
 * Buckets step concurrently on their streams; requests leave as they
 * complete, which frees their memory and slot for the next admission.
 * Every request's results equal those of tvspec_decompose_dev with the
 * server's options, bit for bit, whatever else is in flight.
 *
 * Working state per request (what admission charges against the budget):
 * about C*H*W*(2*4*s + 2*g + 24) bytes + C*K*8*ceil(H*W/256) for the
 * partial sums of S, with s = 4 (F32) or 8 bytes per dual-field element and
 * g = 4 (F32) or 0 (MIXED, F64: they read the data term from the flow state)
 * per stored data-term element.
 *
 *   budget_bytes      size of the pool (allocated at creation)
 *   tau, warm_start, precision
 *                     as tvspec_decompose_dev, for every request
 *   iters_per_launch  as tvspec_decompose_dev; 0 = picked per bucket by the
 *                     server's autotuner, which times the bucket's first
 *                     steps with each candidate temporal blocking factor
 *                     (results do not depend on the choice)
 *   use_graphs        1: each bucket's step (its tile-kernel launches, the
 *                     fused outer step and the slot advance) is captured
 *                     once in a hipGraph and replayed; 0: launched directly
 *
 * The server is bound to the device current at creation.  Errors:
 * TVSPEC_EINVAL (bad option, budget_bytes < 1 MiB, out NULL), TVSPEC_ENOMEM,
 * TVSPEC_EDEVICE.
 */
typedef struct tvspec_server tvspec_server;

typedef struct tvspec_request {
    const float *f;         /* device [C][H][W]; must hold its values when submitted */
    int H, W, C;
    double dt;
    int K;
    int inner_iters;
    const int *band_edges;  /* host, n_bands + 1 entries; copied by tvspec_submit */
    int n_bands;
    double *bands;          /* device outputs, layouts as tvspec_decompose_dev */
    double *S;
    double *residual;
    double *stats;          /* device, TVSPEC_NSTATS doubles */
} tvspec_request;

typedef struct tvspec_result {
    double queue_ms;        /* submission to admission */
    double latency_ms;      /* submission to completion of every output */
} tvspec_result;

typedef struct tvspec_server_stats {
    unsigned long long submitted, admitted, completed;
    unsigned long long steps;        /* bucket steps enqueued */
    unsigned long long replays;      /* step runs enqueued (one graph replay each; up to 4 steps) */
    unsigned long long graph_builds; /* step graphs captured */
    int buckets;
    int max_in_flight;               /* most requests admitted at once */
    size_t budget_bytes, used_bytes, peak_bytes;
} tvspec_server_stats;

TVSPEC_API int tvspec_server_create(size_t budget_bytes, double tau, int warm_start, int precision,
                                    int iters_per_launch, int use_graphs, tvspec_server **out);

/*
 * Queue one request.  The request's device buffers are the caller's and must
 * stay allocated, f unchanged and the outputs unread, until tvspec_poll or
 * tvspec_wait reports the ticket complete.  *ticket identifies it.
 * Errors: TVSPEC_EINVAL (as tvspec_decompose_dev), TVSPEC_EBUSY (its
 * working state exceeds the budget, or B*C would exceed the grid limit of a
 * slot table), or the server's own failure code once it has failed.
 */
TVSPEC_API int tvspec_submit(tvspec_server *srv, const tvspec_request *req, unsigned long long *ticket);

/*
 * TVSPEC_PENDING while the request is queued or running; TVSPEC_OK once its
 * outputs are complete on the device (the ticket is then retired and *res,
 * if not NULL, holds its timings); a negative code if the server failed
 * (tvspec_last_error() has the text) or the ticket is unknown (EINVAL).
 */
TVSPEC_API int tvspec_poll(tvspec_server *srv, unsigned long long ticket, tvspec_result *res);

/* As tvspec_poll, but blocks until the request is complete or has failed. */
TVSPEC_API int tvspec_wait(tvspec_server *srv, unsigned long long ticket, tvspec_result *res);

/* Counters of the server so far. */
TVSPEC_API int tvspec_server_info(tvspec_server *srv, tvspec_server_stats *info);

/*
 * Stop the worker, wait for the device work it enqueued, free the pool and
 * the server.  Requests not yet complete are abandoned (their outputs are
 * unspecified).  srv may be NULL.
 */
TVSPEC_API int tvspec_server_destroy(tvspec_server *srv);

/*
 * Dyadic band edges (the paper groups unit-step bands dyadically, Sec. 4.1):
 * edges = {0, 1, 2, 4, ..., 2^(B-2), K} for B = n_bands >= 2, {0, K} for
 * B = 1.  `edges` has room for n_bands+1 ints (host memory).
 * Errors: TVSPEC_EINVAL if K < 1, n_bands < 1, edges is NULL, or
 * 2^(B-2) >= K.
 */
TVSPEC_API int tvspec_dyadic_edges(int K, int n_bands, int *edges);

/*
 * Kernel timing for benchmarks.  While enabled (on = 1), the back-to-back
 * launches of the Chambolle iteration kernel of every ROF solve are
 * bracketed by one pair of hipEvents recorded on their stream.
 * tvspec_timing_read() waits for the recorded events, returns the summed
 * time (ms), the number of launches and the number of pixel-iterations
 * (pixels x Chambolle iterations) they performed, and clears the record.
 * Any pointer may be NULL.  Leave it off for throughput runs.
 * Errors: TVSPEC_EDEVICE (event creation, query or timing failed).
 */
TVSPEC_API int tvspec_timing_enable(int on);
TVSPEC_API int tvspec_timing_read(double *kernel_ms, long long *launches, long long *pixel_iters);

/* Text of the last error on the calling thread ("" if none). */
TVSPEC_API const char *tvspec_last_error(void);

/* Library version string. */
TVSPEC_API const char *tvspec_version(void);

/* Free every device buffer the library caches.  Must not overlap a call in
 * flight on any stream. */
TVSPEC_API void tvspec_release(void);

#ifdef __cplusplus
}
#endif

#endif /* TVSPEC_H */
