// tvspec C ABI: argument validation, device scratch, and the decomposition
// of one image or of a batch of equal-size images through the slot engine
// (engine.h).
//
// A call lays its images out as slots in a per-device scratch arena, uploads
// the slot table through pinned staging, initialises every slot, runs
// max K + 1 engine steps (a slot with a smaller K falls out once its flow is
// complete) and finalises every slot.  All device work is ordered on the
// caller's stream; the device entry points return once it is enqueued.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "engine.h"

#define TVSPEC_VERSION_STRING "tvspec 0.3.0 (gfx950)"

// Scratch of the allocation-free entry point (tvspec_decompose_noalloc_dev):
// slot table | band rows | non-finite counter | slot buffers, carved as the
// arena of the other entry points.  Every device the library runs on holds
// its own copy until the process ends.  Host code never takes this name as
// an address: the device address of each copy is looked up once per device
// (noalloc_scratch below) and passed to the kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxBands = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace tvspec {
namespace {

// ---------------------------------------------------------------------------
// per-device state, guarded by g_mu

// One scratch arena per (device, precision).  `done` is recorded on the
// stream of the last call that used the arena, after its last use; the next
// call makes its own stream wait for it before touching the arena, so calls
// on different streams (or threads) are ordered on the device without a host
// synchronisation.
struct Arena {
    size_t bytes = 0;
    char *base = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
};

// Pinned host staging of a slot table and its band rows, and an event marking
// the upload that last read it (the next call waits for it before rewriting).
struct Staging {
    size_t bytes = 0;
    char *host = nullptr;
    hipEvent_t uploaded = nullptr;
    bool pending = false;
};

// Device copies of the host entry point's inputs and outputs.
struct HostIO {
    size_t f_n = 0, bands_n = 0, s_n = 0, r_n = 0;
    float *f = nullptr;
    double *bands = nullptr, *S = nullptr, *res = nullptr, *stats = nullptr;
    hipStream_t stream = nullptr;
};

constexpr int kMaxDevices = 64;
constexpr int kModes = 3;
std::mutex g_mu;
Arena g_arena[kMaxDevices][kModes];
Staging g_staging[kMaxDevices];
HostIO g_hostio[kMaxDevices];

template <typename T> void free_dev(T *&p)
{
    if (p)
        (void)hipFree((void *)p);
    p = nullptr;
}

// Order `st` after the previous user of the arena (device-side wait).
int arena_acquire(Arena &a, hipStream_t st)
{
    if (!a.done)
        HIP_TRY(hipEventCreateWithFlags(&a.done, hipEventDisableTiming));
    if (a.used)
        HIP_TRY(hipStreamWaitEvent(st, a.done, 0));
    return TVSPEC_OK;
}

// Mark the end of this call's use of the arena on `st`.
int arena_release(Arena &a, hipStream_t st)
{
    HIP_TRY(hipEventRecord(a.done, st));
    a.used = true;
    return TVSPEC_OK;
}

// Releases the arena when the call leaves, also on its error paths (work it
// enqueued before failing is then still ordered before the next call).
struct ArenaUse {
    Arena &a;
    hipStream_t st;
    ~ArenaUse() { (void)arena_release(a, st); }
};

int ensure_arena(Arena &a, size_t bytes)
{
    if (a.base && a.bytes >= bytes)
        return TVSPEC_OK;
    // the old arena may still be in use by work enqueued earlier
    HIP_TRY(hipDeviceSynchronize());
    free_dev(a.base);
    a.bytes = 0;
    HIP_TRY(hipMalloc((void **)&a.base, bytes));
    a.bytes = bytes;
    return TVSPEC_OK;
}

int ensure_staging(Staging &s, size_t bytes)
{
    if (s.pending) {
        HIP_TRY(hipEventSynchronize(s.uploaded));
        s.pending = false;
    }
    if (!s.uploaded)
        HIP_TRY(hipEventCreateWithFlags(&s.uploaded, hipEventDisableTiming));
    if (s.host && s.bytes >= bytes)
        return TVSPEC_OK;
    if (s.host)
        HIP_TRY(hipHostFree(s.host));
    s.host = nullptr;
    s.bytes = 0;
    HIP_TRY(hipHostMalloc((void **)&s.host, bytes, hipHostMallocDefault));
    s.bytes = bytes;
    return TVSPEC_OK;
}

template <typename T> int grow(T *&p, size_t &cap, size_t n)
{
    if (p && cap >= n)
        return TVSPEC_OK;
    free_dev(p);
    cap = 0;
    HIP_TRY(hipMalloc((void **)&p, n * sizeof(T)));
    cap = n;
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// a batch through the engine, enqueued on a stream

struct Batch {
    const float *f; // device [B][C][H][W]
    int B, H, W, C, iters;
    const double *dt; // host [B]
    const int *K;     // host [B]
    const int *edges; // host, n_bands[b] + 1 entries per image, concatenated
    const int *nb;    // host [B]
    double *bands, *S, *res, *stats;
    double tau;
    int warm, ipl, precision;
    hipStream_t st;
    int solver = kSolverChambolle;
    double sigma = 0.0;
    int tile = kTileShapeSquare;
};

// The slot descriptor and band edges of an allocation-free call, passed by
// value (no host staging, nothing to capture but a kernel launch).
struct NoAllocSetup {
    SlotDesc slot;
    int edges[kNoAllocMaxBands + 1];
};

// Writes the slot table entry, the band row of every sample k = 0..K
// (sample k belongs to band j when e_j < k <= e_{j+1}; sample 0 carries no
// phi) and clears the non-finite counter.  One block.
__global__ __launch_bounds__(256) void k_noalloc_setup(NoAllocSetup a, SlotDesc *table, int *rows,
                                                       unsigned int *nf)
{
    for (int k = threadIdx.x; k <= a.slot.K; k += blockDim.x) {
        int r = 0;
        for (int j = 0; j < a.slot.nbands; ++j)
            if (k > a.edges[j] && k <= a.edges[j + 1])
                r = j;
        rows[k] = r;
    }
    if (threadIdx.x == 0) {
        *table = a.slot;
        *nf = 0u;
    }
}

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, with that device current).
char *g_noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch(int dev, char **out)
{
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr)
            return fail(TVSPEC_EDEVICE, "no device address for the allocation-free scratch");
        g_noalloc_ptr[dev] = (char *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return TVSPEC_OK;
}

int run_batch(const Batch &a)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    const size_t n = (size_t)a.C * a.H * a.W;

    // arena: slot table | band rows | non-finite counters | slot buffers
    int Kmax = 0;
    size_t rows_n = 0, slots_bytes = 0;
    for (int b = 0; b < a.B; ++b) {
        Kmax = a.K[b] > Kmax ? a.K[b] : Kmax;
        rows_n += (size_t)a.K[b] + 1;
        slots_bytes += slot_scratch_bytes(a.precision, a.solver, a.H, a.W, a.C, a.K[b]);
    }
    const size_t table_bytes = align256((size_t)a.B * sizeof(SlotDesc));
    const size_t rows_bytes = align256(rows_n * sizeof(int));
    const size_t nf_bytes = align256((size_t)a.B * sizeof(unsigned int));
    Arena &ar = g_arena[dev][a.precision];
    TVSPEC_TRY(ensure_arena(ar, table_bytes + rows_bytes + nf_bytes + slots_bytes));
    TVSPEC_TRY(arena_acquire(ar, a.st));
    ArenaUse use{ar, a.st};
    SlotDesc *d_table = (SlotDesc *)ar.base;
    int *d_rows = (int *)(ar.base + table_bytes);
    unsigned int *d_nf = (unsigned int *)(ar.base + table_bytes + rows_bytes);
    char *slot_base = ar.base + table_bytes + rows_bytes + nf_bytes;

    Staging &sg = g_staging[dev];
    TVSPEC_TRY(ensure_staging(sg, table_bytes + rows_bytes));
    SlotDesc *h_table = (SlotDesc *)sg.host;
    int *h_rows = (int *)(sg.host + table_bytes);
    size_t row0 = 0, band_off = 0, s_off = 0;
    for (int b = 0, e0 = 0; b < a.B; ++b) {
        SlotDesc d;
        std::memset(&d, 0, sizeof(d));
        slot_carve(d, slot_base, a.precision, a.solver, a.H, a.W, a.C, a.K[b]);
        slot_base += slot_scratch_bytes(a.precision, a.solver, a.H, a.W, a.C, a.K[b]);
        band_rows_of(a.edges + e0, a.nb[b], h_rows + row0);
        d.band_rows = d_rows + row0;
        d.nonfinite = d_nf + b;
        d.f = a.f + (size_t)b * n;
        d.bands = a.bands + band_off;
        d.S = a.S + s_off;
        d.res = a.res + (size_t)b * n;
        d.stats = a.stats + (size_t)b * TVSPEC_NSTATS;
        d.dt = a.dt[b];
        d.nbands = a.nb[b];
        h_table[b] = d;
        row0 += (size_t)a.K[b] + 1;
        band_off += (size_t)a.nb[b] * n;
        s_off += (size_t)a.C * a.K[b];
        e0 += a.nb[b] + 1;
    }
    HIP_TRY(hipMemcpyAsync(d_table, h_table, (size_t)a.B * sizeof(SlotDesc), hipMemcpyHostToDevice, a.st));
    HIP_TRY(hipMemcpyAsync(d_rows, h_rows, rows_n * sizeof(int), hipMemcpyHostToDevice, a.st));
    HIP_TRY(hipEventRecord(sg.uploaded, a.st));
    sg.pending = true;
    HIP_TRY(hipMemsetAsync(d_nf, 0, (size_t)a.B * sizeof(unsigned int), a.st));

    StepConfig cfg{a.H, a.W, a.C, a.iters, a.tau, a.warm, a.ipl, a.precision};
    cfg.solver = a.solver;
    cfg.sigma = a.sigma;
    cfg.tile = a.tile;
    TVSPEC_TRY(engine_init(cfg, d_table, 0, a.B, a.st));
    int parity = 0;
    for (int s = 0; s <= Kmax; ++s) {
        long long live = 0;
        for (int b = 0; b < a.B; ++b)
            live += (s <= a.K[b]) ? a.C : 0;
        TVSPEC_TRY(engine_step(cfg, d_table, a.B, &parity, a.st, live));
    }
    return engine_finalize(cfg, d_table, 0, a.B, Kmax, a.st);
}

} // namespace

// ---------------------------------------------------------------------------
// argument validation (host only, before any device call)

} // namespace tvspec

using namespace tvspec;

// ---------------------------------------------------------------------------
// C ABI

extern "C" int tvspec_decompose_batch_dev(const float *f, int B, int H, int W, int C, int inner_iters,
                                          const double *dt, const int *K, const int *band_edges, const int *n_bands,
                                          double *bands, double *S, double *residual, double *stats, double tau,
                                          int warm_start, int precision, int iters_per_launch, void *stream)
{
    g_last_error.clear();
    if (!f || !dt || !K || !band_edges || !n_bands || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(validate_shape(B, H, W, C, inner_iters));
    for (int b = 0, e0 = 0; b < B; ++b) {
        if (K[b] < 1 || n_bands[b] < 1 || n_bands[b] > K[b])
            return fail(TVSPEC_EINVAL, "image " + std::to_string(b) + ": need K >= 1 and 1 <= n_bands <= K");
        if (validate_image(dt[b], K[b], band_edges + e0, n_bands[b]) != TVSPEC_OK)
            return fail(TVSPEC_EINVAL, "image " + std::to_string(b) + ": " + g_last_error);
        e0 += n_bands[b] + 1;
    }
    TVSPEC_TRY(validate_opts(tau, warm_start, precision, iters_per_launch));
    std::lock_guard<std::mutex> lock(g_mu);
    Batch a;
    a.f = f;
    a.B = B;
    a.H = H;
    a.W = W;
    a.C = C;
    a.iters = inner_iters;
    a.dt = dt;
    a.K = K;
    a.edges = band_edges;
    a.nb = n_bands;
    a.bands = bands;
    a.S = S;
    a.res = residual;
    a.stats = stats;
    a.tau = tau;
    a.warm = warm_start;
    a.ipl = iters_per_launch;
    a.precision = precision;
    a.st = (hipStream_t)stream;
    return run_batch(a);
}

extern "C" int tvspec_decompose_dev(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                    const int *band_edges, int n_bands, double *bands, double *S, double *residual,
                                    double *stats, double tau, int warm_start, int precision, int iters_per_launch,
                                    void *stream)
{
    g_last_error.clear();
    if (!f || !band_edges || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(validate_shape(1, H, W, C, inner_iters));
    TVSPEC_TRY(validate_image(dt, K, band_edges, n_bands));
    TVSPEC_TRY(validate_opts(tau, warm_start, precision, iters_per_launch));
    std::lock_guard<std::mutex> lock(g_mu);
    Batch a;
    a.f = f;
    a.B = 1;
    a.H = H;
    a.W = W;
    a.C = C;
    a.iters = inner_iters;
    a.dt = &dt;
    a.K = &K;
    a.edges = band_edges;
    a.nb = &n_bands;
    a.bands = bands;
    a.S = S;
    a.res = residual;
    a.stats = stats;
    a.tau = tau;
    a.warm = warm_start;
    a.ipl = iters_per_launch;
    a.precision = precision;
    a.st = (hipStream_t)stream;
    return run_batch(a);
}

extern "C" int tvspec_decompose_pdhg_dev(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                         const int *band_edges, int n_bands, double *bands, double *S,
                                         double *residual, double *stats, double tau, double sigma, int warm_start,
                                         int precision, int iters_per_launch, void *stream)
{
    g_last_error.clear();
    if (!f || !band_edges || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (tau == 0.0 && sigma == 0.0)
        tau = sigma = TVSPEC_PDHG_DEFAULT_STEP;
    if (!std::isfinite(tau) || !std::isfinite(sigma) || !(tau > 0.0) || !(sigma > 0.0) ||
        tau * sigma * 8.0 > 1.0 + 1e-12)
        return fail(TVSPEC_EINVAL, "PDHG steps need tau > 0, sigma > 0 and 8 tau sigma <= 1");
    TVSPEC_TRY(validate_shape(1, H, W, C, inner_iters));
    TVSPEC_TRY(validate_image(dt, K, band_edges, n_bands));
    TVSPEC_TRY(validate_opts(TVSPEC_DEFAULT_TAU, warm_start, precision, iters_per_launch));
    std::lock_guard<std::mutex> lock(g_mu);
    Batch a;
    a.f = f;
    a.B = 1;
    a.H = H;
    a.W = W;
    a.C = C;
    a.iters = inner_iters;
    a.dt = &dt;
    a.K = &K;
    a.edges = band_edges;
    a.nb = &n_bands;
    a.bands = bands;
    a.S = S;
    a.res = residual;
    a.stats = stats;
    a.tau = tau;
    a.warm = warm_start;
    a.ipl = iters_per_launch;
    a.precision = precision;
    a.st = (hipStream_t)stream;
    a.solver = kSolverPDHG;
    a.sigma = sigma;
    return run_batch(a);
}

extern "C" void tvspec_default_options(tvspec_options *o)
{
    if (!o)
        return;
    o->solver = TVSPEC_SOLVER_CHAMBOLLE;
    o->tau = 0.0;
    o->sigma = 0.0;
    o->warm_start = 0;
    o->precision = TVSPEC_DEFAULT_PRECISION;
    o->iters_per_launch = 0;
    o->device_ptrs = 0;
    o->stream = nullptr;
    o->tile_shape = TVSPEC_TILE_SQUARE;
}

namespace {

// Events around the device work of one call (report timing); destroyed on
// every exit path.
struct CallEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~CallEvents()
    {
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    }
};

} // namespace

extern "C" int tvspec_decompose_ex(const tvspec_args *args, const tvspec_options *opt, tvspec_report *rep)
{
    const auto t_start = std::chrono::steady_clock::now();
    g_last_error.clear();
    if (!args)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    tvspec_options o;
    tvspec_default_options(&o);
    if (opt)
        o = *opt;
    const tvspec_args &x = *args;
    if (o.device_ptrs != 0 && o.device_ptrs != 1)
        return fail(TVSPEC_EINVAL, "device_ptrs must be 0 or 1");
    if (!x.f || !x.band_edges || !x.bands || !x.S || !x.residual || (o.device_ptrs && !x.stats))
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(validate_shape(1, x.H, x.W, x.C, x.inner_iters));
    TVSPEC_TRY(validate_image(x.dt, x.K, x.band_edges, x.n_bands));
    double tau = o.tau, sigma = o.sigma;
    int solver = kSolverChambolle;
    if (o.solver == TVSPEC_SOLVER_PDHG) {
        solver = kSolverPDHG;
        if (tau == 0.0 && sigma == 0.0)
            tau = sigma = TVSPEC_PDHG_DEFAULT_STEP;
        if (!std::isfinite(tau) || !std::isfinite(sigma) || !(tau > 0.0) || !(sigma > 0.0) ||
            tau * sigma * 8.0 > 1.0 + 1e-12)
            return fail(TVSPEC_EINVAL, "PDHG steps need tau > 0, sigma > 0 and 8 tau sigma <= 1");
        TVSPEC_TRY(validate_opts(TVSPEC_DEFAULT_TAU, o.warm_start, o.precision, o.iters_per_launch));
    } else if (o.solver == TVSPEC_SOLVER_CHAMBOLLE) {
        if (tau == 0.0)
            tau = TVSPEC_DEFAULT_TAU;
        TVSPEC_TRY(validate_opts(tau, o.warm_start, o.precision, o.iters_per_launch));
    } else {
        return fail(TVSPEC_EINVAL, "solver must be TVSPEC_SOLVER_CHAMBOLLE or TVSPEC_SOLVER_PDHG");
    }
    TVSPEC_TRY(validate_tile_shape(o.tile_shape, o.solver, o.iters_per_launch));
    const size_t n_all = (size_t)x.H * x.W * x.C;
    if (!o.device_ptrs)
        for (size_t q = 0; q < n_all; ++q)
            if (!std::isfinite(x.f[q]))
                return fail(TVSPEC_ENUMERIC, "input holds a NaN or infinity");

    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    const size_t nb_n = (size_t)x.n_bands * n_all;
    const size_t s_n = (size_t)x.C * x.K;
    int K = x.K, nb = x.n_bands;
    double dt = x.dt;
    Batch a;
    a.B = 1;
    a.H = x.H;
    a.W = x.W;
    a.C = x.C;
    a.iters = x.inner_iters;
    a.dt = &dt;
    a.K = &K;
    a.edges = x.band_edges;
    a.nb = &nb;
    a.tau = tau;
    a.warm = o.warm_start;
    a.ipl = o.iters_per_launch;
    a.precision = o.precision;
    a.solver = solver;
    a.sigma = solver == kSolverPDHG ? sigma : 0.0;
    a.tile = o.tile_shape == TVSPEC_TILE_NARROW ? kTileShapeNarrow : kTileShapeSquare;
    HostIO &h = g_hostio[dev];
    if (o.device_ptrs) {
        a.f = x.f;
        a.bands = x.bands;
        a.S = x.S;
        a.res = x.residual;
        a.stats = x.stats;
        a.st = (hipStream_t)o.stream;
    } else {
        if (!h.stream)
            HIP_TRY(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
        TVSPEC_TRY(grow(h.f, h.f_n, n_all));
        TVSPEC_TRY(grow(h.bands, h.bands_n, nb_n));
        TVSPEC_TRY(grow(h.S, h.s_n, s_n));
        TVSPEC_TRY(grow(h.res, h.r_n, n_all));
        if (!h.stats)
            HIP_TRY(hipMalloc((void **)&h.stats, TVSPEC_NSTATS * sizeof(double)));
        a.f = h.f;
        a.bands = h.bands;
        a.S = h.S;
        a.res = h.res;
        a.stats = h.stats;
        a.st = h.stream;
        HIP_TRY(hipMemcpyAsync(h.f, x.f, n_all * sizeof(float), hipMemcpyHostToDevice, a.st));
    }
    CallEvents ev;
    if (rep) {
        HIP_TRY(hipEventCreate(&ev.e0));
        HIP_TRY(hipEventCreate(&ev.e1));
        HIP_TRY(hipEventRecord(ev.e0, a.st));
    }
    TVSPEC_TRY(run_batch(a));
    if (rep)
        HIP_TRY(hipEventRecord(ev.e1, a.st));
    double st_h[TVSPEC_NSTATS] = {0.0, 0.0, 0.0, 0.0};
    if (!o.device_ptrs) {
        HIP_TRY(hipMemcpyAsync(x.bands, h.bands, nb_n * sizeof(double), hipMemcpyDeviceToHost, a.st));
        HIP_TRY(hipMemcpyAsync(x.S, h.S, s_n * sizeof(double), hipMemcpyDeviceToHost, a.st));
        HIP_TRY(hipMemcpyAsync(x.residual, h.res, n_all * sizeof(double), hipMemcpyDeviceToHost, a.st));
    }
    if (rep || !o.device_ptrs) {
        if (rep || x.stats)
            HIP_TRY(hipMemcpyAsync(st_h, a.stats, sizeof(st_h), hipMemcpyDeviceToHost, a.st));
        HIP_TRY(hipStreamSynchronize(a.st));
        if (!o.device_ptrs && x.stats)
            std::memcpy(x.stats, st_h, sizeof(st_h));
    }
    if (rep) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        rep->recon_err = st_h[0];
        rep->mean_err = st_h[1];
        rep->nonfinite = st_h[2];
        rep->device_ms = (double)ms;
        rep->total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        if (st_h[2] > 0.0)
            return fail(TVSPEC_ENUMERIC, "input holds a NaN or infinity (outputs are meaningless)");
    }
    return TVSPEC_OK;
}

extern "C" int tvspec_decompose(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                const int *band_edges, int n_bands, double *bands, double *S, double *residual)
{
    tvspec_args x;
    x.f = f;
    x.H = H;
    x.W = W;
    x.C = C;
    x.dt = dt;
    x.K = K;
    x.inner_iters = inner_iters;
    x.band_edges = band_edges;
    x.n_bands = n_bands;
    x.bands = bands;
    x.S = S;
    x.residual = residual;
    x.stats = nullptr;
    return tvspec_decompose_ex(&x, nullptr, nullptr);
}

extern "C" int tvspec_decompose_noalloc_dev(const float *f, int H, int W, int C, double dt, int K,
                                            int inner_iters, const int *band_edges, int n_bands, double *bands,
                                            double *S, double *residual, double *stats, double tau,
                                            int warm_start, int precision, int iters_per_launch, void *stream)
{
    g_last_error.clear();
    if (!f || !band_edges || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(validate_shape(1, H, W, C, inner_iters));
    TVSPEC_TRY(validate_image(dt, K, band_edges, n_bands));
    TVSPEC_TRY(validate_opts(tau, warm_start, precision, iters_per_launch));
    if (n_bands > kNoAllocMaxBands)
        return fail(TVSPEC_EINVAL, "the allocation-free entry point takes at most 64 bands");
    const size_t table_bytes = align256(sizeof(SlotDesc));
    const size_t rows_bytes = align256(((size_t)K + 1) * sizeof(int));
    const size_t nf_bytes = align256(sizeof(unsigned int));
    const size_t need = table_bytes + rows_bytes + nf_bytes +
                        slot_scratch_bytes(precision, kSolverChambolle, H, W, C, K);
    if (need > kNoAllocScratchBytes)
        return fail(TVSPEC_EINVAL, "the decomposition needs " + std::to_string(need) +
                                       " bytes of scratch; the allocation-free entry point has " +
                                       std::to_string(kNoAllocScratchBytes));

    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    char *base = nullptr;
    TVSPEC_TRY(noalloc_scratch(dev, &base));
    SlotDesc *d_table = (SlotDesc *)base;
    int *d_rows = (int *)(base + table_bytes);
    unsigned int *d_nf = (unsigned int *)(base + table_bytes + rows_bytes);
    char *slot_base = base + table_bytes + rows_bytes + nf_bytes;

    NoAllocSetup su;
    std::memset(&su, 0, sizeof(su));
    SlotDesc &d = su.slot;
    slot_carve(d, slot_base, precision, kSolverChambolle, H, W, C, K);
    d.band_rows = d_rows;
    d.nonfinite = d_nf;
    d.f = f;
    d.bands = bands;
    d.S = S;
    d.res = residual;
    d.stats = stats;
    d.dt = dt;
    d.nbands = n_bands;
    for (int j = 0; j <= n_bands; ++j)
        su.edges[j] = band_edges[j];
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, st, su, d_table, d_rows, d_nf);
    HIP_TRY(hipGetLastError());

    StepConfig cfg{H, W, C, inner_iters, tau, warm_start, iters_per_launch, precision};
    cfg.timed = 0;
    TVSPEC_TRY(engine_init(cfg, d_table, 0, 1, st));
    int parity = 0;
    for (int s = 0; s <= K; ++s)
        TVSPEC_TRY(engine_step(cfg, d_table, 1, &parity, st, C));
    return engine_finalize(cfg, d_table, 0, 1, K, st);
}

extern "C" int tvspec_dyadic_edges(int K, int n_bands, int *edges)
{
    g_last_error.clear();
    if (!edges || K < 1 || n_bands < 1)
        return fail(TVSPEC_EINVAL, "need K >= 1, n_bands >= 1 and an output array");
    edges[0] = 0;
    if (n_bands == 1) {
        edges[1] = K;
        return TVSPEC_OK;
    }
    if (n_bands - 2 >= 30 || (1 << (n_bands - 2)) >= K)
        return fail(TVSPEC_EINVAL, "2^(n_bands-2) must be < K");
    for (int j = 1; j < n_bands; ++j)
        edges[j] = 1 << (j - 1);
    edges[n_bands] = K;
    return TVSPEC_OK;
}

extern "C" int tvspec_timing_enable(int on)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> lock(g_mu);
    return timing_enable(on);
}

extern "C" int tvspec_timing_read(double *kernel_ms, long long *launches, long long *pixel_iters)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> lock(g_mu);
    return timing_read(kernel_ms, launches, pixel_iters);
}

extern "C" const char *tvspec_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *tvspec_version(void) { return TVSPEC_VERSION_STRING; }

extern "C" void tvspec_release(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess)
        return;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess)
        return;
    for (int d = 0; d < ndev && d < kMaxDevices; ++d) {
        bool any = g_hostio[d].stream || g_hostio[d].f || g_hostio[d].stats || g_staging[d].host;
        for (int m = 0; m < kModes; ++m)
            any = any || g_arena[d][m].base;
        if (!any)
            continue;
        if (hipSetDevice(d) != hipSuccess)
            continue;
        (void)hipDeviceSynchronize();
        for (int m = 0; m < kModes; ++m) {
            free_dev(g_arena[d][m].base);
            if (g_arena[d][m].done)
                (void)hipEventDestroy(g_arena[d][m].done);
            g_arena[d][m] = Arena();
        }
        HostIO &h = g_hostio[d];
        free_dev(h.f);
        free_dev(h.bands);
        free_dev(h.S);
        free_dev(h.res);
        free_dev(h.stats);
        h.f_n = h.bands_n = h.s_n = h.r_n = 0;
        if (h.stream) {
            (void)hipStreamDestroy(h.stream);
            h.stream = nullptr;
        }
        Staging &s = g_staging[d];
        if (s.host)
            (void)hipHostFree(s.host);
        if (s.uploaded)
            (void)hipEventDestroy(s.uploaded);
        s = Staging();
    }
    (void)hipSetDevice(cur);
}
