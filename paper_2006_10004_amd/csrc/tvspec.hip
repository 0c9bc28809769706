// tvspec: spectral total-variation decomposition on one MI355X (gfx950).
//
// Method: Grossmann, Korolev, Gilboa, Schoenlieb, arXiv 2006.10004.
//   Sec. 2.2 Eq. (8)   one implicit Euler step of the TV flow Eq. (1) is a ROF
//                      problem; it is solved here by Chambolle's dual
//                      projection iteration (the solver Sec. 4.3 names);
//   Sec. 2.1 Eq. (3)   phi(t_k) = t_k u_tt(t_k) by the central second
//                      difference, S(t_k) = ||phi(t_k)||_1, band integrals of
//                      Eq. (7) and the residual of Eq. (5).
//
// Device work per decomposition (one C x H x W image, channels independent):
//   k_init           u_0 = f (float64), g/dt for the first solve, p = 0,
//                    bands = 0, count of non-finite inputs;
//   k_chambolle_tile the hot loop.  Each launch runs `iters` (<= TB) Jacobi
//                    iterations of Chambolle's fixed point on a 32x32 output
//                    tile whose (32+2TB)^2 neighbourhood is staged once in LDS;
//                    the dual field stays in registers, only the neighbour
//                    values cross lanes through LDS.  Tiles are mapped to
//                    workgroups so that each XCD works on one horizontal band
//                    of the image (neighbouring halos then hit the same L2);
//   k_flow_step      one launch per ROF solve, fused: div p, u_{s+1} =
//                    u_s - dt div p, D_s = dt div p, phi_s dt = s (D_{s-1} -
//                    D_s) added to its band, a per-block partial of sum |D_{s-1}
//                    - D_s| for S(t_s), the residual at s = K, and g/dt of the
//                    next solve.  u_{s-1}, u_s, u_{s+1} never exist as planes;
//   k_check          per-block partials of the reconstruction error and of
//                    the mean of u_{K+1} and f;
//   k_reduce         one block: S(t_k) and the report, in a fixed order
//                    (results are bit-reproducible run to run).
//
// Arithmetic contract: every kernel variant (any temporal blocking factor)
// applies the same per-pixel operations in the same order, so results do not
// depend on the launch configuration.  Build with -ffp-contract=off; fused
// multiply-adds are written explicitly.

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tvspec.h"

#define TVSPEC_VERSION_STRING "tvspec 0.1.0 (gfx950)"

namespace {

// ---------------------------------------------------------------------------
// error reporting

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? TVSPEC_ENOMEM : TVSPEC_EDEVICE,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

// ---------------------------------------------------------------------------
// per-precision scalar operations of the Chambolle update

template <typename R> struct Arith;

template <> struct Arith<float> {
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    // p / d as p * (1/d): one reciprocal shared by both components
    static __device__ __forceinline__ float inv_(float d) { return __builtin_amdgcn_rcpf(d); }
};

template <> struct Arith<double> {
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
    static __device__ __forceinline__ double inv_(double d) { return 1.0 / d; }
};

// One Chambolle update of a pixel's dual vector (px, py) from the gradient
// (ax, ay) of w = div p - g/dt:  p <- (p + tau a) / (1 + tau |a|).
template <typename R>
__device__ __forceinline__ void chambolle_update(R &px, R &py, R ax, R ay, R tau)
{
    using A = Arith<R>;
    R nrm = A::sqrt_(A::fma_(ax, ax, ay * ay));
    R r = A::inv_(A::fma_(tau, nrm, R(1)));
    px = A::fma_(tau, ax, px) * r;
    py = A::fma_(tau, ay, py) * r;
}

// ---------------------------------------------------------------------------
// reductions (wave64, fixed order)

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block of 256 threads (4 waves).  Every thread returns the block sum.
__device__ __forceinline__ double block_sum256(double v, double *sh)
{
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[wid] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__device__ __forceinline__ double block_max256(double v, double *sh)
{
    v = wave_max(v);
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[wid] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// kernels

// u = f, gl = f/dt, p = 0 (buffer A), bands = 0; counts non-finite inputs.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_init(const float *__restrict__ f, double *__restrict__ u,
                                                   R *__restrict__ gl, R *__restrict__ px, R *__restrict__ py,
                                                   double *__restrict__ bands, size_t n_all, int nbands,
                                                   double dt, unsigned int *__restrict__ nonfinite)
{
    __shared__ double sh[4];
    double bad = 0.0;
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n_all; q += stride) {
        const float v = f[q];
        if (!isfinite(v))
            bad += 1.0;
        u[q] = (double)v;
        gl[q] = (R)((double)v / dt);
        px[q] = R(0);
        py[q] = R(0);
        for (int j = 0; j < nbands; ++j)
            bands[(size_t)j * n_all + q] = 0.0;
    }
    bad = block_sum256(bad, sh);
    if (threadIdx.x == 0 && bad > 0.0)
        atomicAdd(nonfinite, (unsigned int)bad);
}

__global__ __launch_bounds__(kThreads) void k_zero2(float *__restrict__ a, float *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += stride) {
        a[q] = 0.f;
        b[q] = 0.f;
    }
}

__global__ __launch_bounds__(kThreads) void k_zero2d(double *__restrict__ a, double *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += stride) {
        a[q] = 0.0;
        b[q] = 0.0;
    }
}

// Temporally blocked Chambolle iterations.
//
// Grid: (number of BX x BY output tiles, C).  The workgroup stages the
// (BX+2TB) x (BY+2TB) region around its tile: the dual field (px, py) and
// g/dt of every region pixel live in registers of the thread that owns the
// pixel for all `iters` iterations; LDS only carries the values a neighbour
// needs (px of the left pixel and py of the upper one for w, w of the right
// and lower pixels for grad w).  One iteration on every region pixel:
//     w   = ((px - px_left) + (py - py_up)) - g/dt        (div p - g/dt)
//     a   = (w_right - w, w_down - w), zero on the last column / row
//     p  <- (p + tau a) / (1 + tau |a|)
// Pixels outside the image hold p = 0 and are never updated, which realises
// the Neumann divergence (p_x = 0 on the last column and p_y = 0 on the last
// row is preserved by the update because a_x, a_y vanish there).  A region
// pixel at distance d from the region edge is exact for d >= iteration count,
// so after iters <= TB iterations the BX x BY centre is exact and is written.
template <typename R, int BX, int BY, int TB>
__global__ __launch_bounds__(kThreads) void k_chambolle_tile(
    const R *__restrict__ pxi, const R *__restrict__ pyi, const R *__restrict__ gl, R *__restrict__ pxo,
    R *__restrict__ pyo, int H, int W, int ntx, int ntiles, R tau, int iters)
{
    constexpr int RX = BX + 2 * TB;
    constexpr int RY = BY + 2 * TB;
    constexpr int RN = RX * RY;
    constexpr int PPT = (RN + kThreads - 1) / kThreads;
    static_assert(PPT <= 32, "pixel masks are 32-bit");
    __shared__ R s_px[RN];
    __shared__ R s_py[RN];
    __shared__ R s_w[RN];

    const size_t plane = (size_t)H * (size_t)W;
    const size_t coff = (size_t)blockIdx.y * plane;
    pxi += coff;
    pyi += coff;
    gl += coff;
    pxo += coff;
    pyo += coff;

    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs,
    // so give XCD x the x-th contiguous run of row-major tiles.
    const int b = blockIdx.x;
    const int L = ((ntiles & 7) == 0) ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
    const int ty = L / ntx;
    const int tx = L - ty * ntx;
    const int oy = ty * BY - TB;
    const int ox = tx * BX - TB;

    R px[PPT], py[PPT], g[PPT], w[PPT];
    unsigned live = 0, xin = 0, yin = 0, outm = 0, hasl = 0, hasu = 0, hasr = 0, hasd = 0;
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * kThreads;
        R vx = R(0), vy = R(0), vg = R(0);
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            if (rj > 0) hasl |= 1u << m;
            if (ri > 0) hasu |= 1u << m;
            if (rj < RX - 1) hasr |= 1u << m;
            if (ri < RY - 1) hasd |= 1u << m;
            if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                vx = pxi[q];
                vy = pyi[q];
                vg = gl[q];
                live |= 1u << m;
                if (gj < W - 1) xin |= 1u << m;
                if (gi < H - 1) yin |= 1u << m;
                if (ri >= TB && ri < TB + BY && rj >= TB && rj < TB + BX) outm |= 1u << m;
            }
            s_px[idx] = vx;
            s_py[idx] = vy;
        }
        px[m] = vx;
        py[m] = vy;
        g[m] = vg;
        w[m] = R(0);
    }
    __syncthreads();

    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int idx = threadIdx.x + m * kThreads;
            if (idx < RN) {
                const R pxl = ((hasl >> m) & 1u) ? s_px[idx - 1] : R(0);
                const R pyu = ((hasu >> m) & 1u) ? s_py[idx - RX] : R(0);
                const R wv = ((px[m] - pxl) + (py[m] - pyu)) - g[m];
                w[m] = wv;
                s_w[idx] = wv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            const int idx = threadIdx.x + m * kThreads;
            if ((live >> m) & 1u) {
                const R wr = ((hasr >> m) & 1u) ? s_w[idx + 1] : w[m];
                const R wd = ((hasd >> m) & 1u) ? s_w[idx + RX] : w[m];
                const R ax = ((xin >> m) & 1u) ? wr - w[m] : R(0);
                const R ay = ((yin >> m) & 1u) ? wd - w[m] : R(0);
                chambolle_update<R>(px[m], py[m], ax, ay, tau);
                s_px[idx] = px[m];
                s_py[idx] = py[m];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        if ((outm >> m) & 1u) {
            const int idx = threadIdx.x + m * kThreads;
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const size_t q = (size_t)(oy + ri) * W + (ox + rj);
            pxo[q] = px[m];
            pyo[q] = py[m];
        }
    }
}

// Outer step s of the flow, fused with the spectral transform.
// Grid: (nblk, C), nblk fixed per image size so partial sums are reproducible.
//   D_s     = dt div p                     (u_s - u_{s+1})
//   u_{s+1} = u_s - D_s
//   s >= 1: phi_s dt = s (D_{s-1} - D_s)   added to the band holding s
//           spart  <- block sum of |D_{s-1} - D_s|   (S(t_s) = s/dt * total)
//   s == K: residual = u_K + K D_K          (u(T) - T u_t(T), forward u_t)
//   gl      = u_{s+1} / dt                  (data term of the next solve)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_flow_step(const R *__restrict__ px, const R *__restrict__ py,
                                                        double *__restrict__ u, double *__restrict__ dprev,
                                                        R *__restrict__ gl, double *__restrict__ band,
                                                        double *__restrict__ resid, double *__restrict__ spart,
                                                        int H, int W, int C, int k, int K, double dt)
{
    __shared__ double sh[4];
    const int c = blockIdx.y;
    const int plane = H * W;
    const size_t coff = (size_t)c * (size_t)plane;
    px += coff;
    py += coff;
    u += coff;
    dprev += coff;
    gl += coff;
    const double kd = (double)k;
    double acc = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        const int i = q / W;
        const int j = q - i * W;
        const double pxc = (double)px[q];
        const double pyc = (double)py[q];
        const double pxl = (j > 0) ? (double)px[q - 1] : 0.0;
        const double pyu = (i > 0) ? (double)py[q - W] : 0.0;
        const double divp = (pxc - pxl) + (pyc - pyu);
        const double D = dt * divp;
        const double uo = u[q];
        const double un = uo - D;
        if (k >= 1) {
            const double dl = dprev[q] - D;
            band[coff + q] += kd * dl;
            acc += fabs(dl);
        }
        if (k == K)
            resid[coff + q] = uo + (double)K * D;
        u[q] = un;
        dprev[q] = D;
        gl[q] = (R)(un / dt);
    }
    if (k >= 1) {
        acc = block_sum256(acc, sh);
        if (threadIdx.x == 0)
            spart[((size_t)(k - 1) * C + c) * gridDim.x + blockIdx.x] = acc;
    }
}

// Per-block partials of: max |f - sum_j b_j - r|, sum u_{K+1}, sum f.
__global__ __launch_bounds__(kThreads) void k_check(const float *__restrict__ f, const double *__restrict__ bands,
                                                    const double *__restrict__ resid, const double *__restrict__ u,
                                                    int plane, int C, int nbands, double *__restrict__ rpart)
{
    __shared__ double sh[4];
    const int c = blockIdx.y;
    const size_t coff = (size_t)c * (size_t)plane;
    const size_t n_all = (size_t)C * (size_t)plane;
    double emax = 0.0, su = 0.0, sf = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        const size_t g = coff + q;
        double acc = 0.0;
        for (int j = 0; j < nbands; ++j)
            acc += bands[(size_t)j * n_all + g];
        const double fv = (double)f[g];
        emax = fmax(emax, fabs(fv - acc - resid[g]));
        su += u[g];
        sf += fv;
    }
    emax = block_max256(emax, sh);
    su = block_sum256(su, sh);
    sf = block_sum256(sf, sh);
    if (threadIdx.x == 0) {
        double *o = rpart + ((size_t)c * gridDim.x + blockIdx.x) * 3;
        o[0] = emax;
        o[1] = su;
        o[2] = sf;
    }
}

// One block: S[c][k-1] = k/dt * sum of the step partials; the report.
__global__ __launch_bounds__(kThreads) void k_reduce(const double *__restrict__ spart, const double *__restrict__ rpart,
                                                     int C, int K, int nblk_step, int nblk_chk, int plane, double dt,
                                                     double *__restrict__ S, double *__restrict__ stats,
                                                     unsigned int *__restrict__ nonfinite)
{
    for (int t = threadIdx.x; t < C * K; t += kThreads) {
        const int c = t / K;
        const int k = t - c * K + 1;
        const double *p = spart + ((size_t)(k - 1) * C + c) * nblk_step;
        double s = 0.0;
        for (int b = 0; b < nblk_step; ++b)
            s += p[b];
        S[t] = s * ((double)k / dt);
    }
    if (threadIdx.x == 0) {
        double emax = 0.0, drift = 0.0;
        for (int c = 0; c < C; ++c) {
            double su = 0.0, sf = 0.0;
            for (int b = 0; b < nblk_chk; ++b) {
                const double *o = rpart + ((size_t)c * nblk_chk + b) * 3;
                emax = fmax(emax, o[0]);
                su += o[1];
                sf += o[2];
            }
            drift = fmax(drift, fabs(su / (double)plane - sf / (double)plane));
        }
        stats[0] = emax;
        stats[1] = drift;
        stats[2] = (double)(*nonfinite);
        stats[3] = 0.0;
        *nonfinite = 0u;
    }
}

// ---------------------------------------------------------------------------
// launch configuration

constexpr int kTileX = 32;
constexpr int kTileY = 32;

int blocks_for(size_t n, int cap)
{
    size_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

// Workgroups per channel plane of the per-pixel kernels: fixed per plane
// size so that partial sums (and hence S) are reproducible.
int plane_blocks(int plane) { return blocks_for((size_t)plane, 1024); }

template <typename R>
using TileKernel = void (*)(const R *, const R *, const R *, R *, R *, int, int, int, int, R, int);

template <typename R> int max_tb();
template <> int max_tb<float>() { return 16; }
template <> int max_tb<double>() { return 8; }

// Smallest compiled halo width >= t.
template <typename R> TileKernel<R> tile_kernel(int t, int *tb);

template <> TileKernel<float> tile_kernel<float>(int t, int *tb)
{
    if (t <= 1) { *tb = 1; return k_chambolle_tile<float, kTileX, kTileY, 1>; }
    if (t <= 2) { *tb = 2; return k_chambolle_tile<float, kTileX, kTileY, 2>; }
    if (t <= 4) { *tb = 4; return k_chambolle_tile<float, kTileX, kTileY, 4>; }
    if (t <= 8) { *tb = 8; return k_chambolle_tile<float, kTileX, kTileY, 8>; }
    *tb = 16;
    return k_chambolle_tile<float, kTileX, kTileY, 16>;
}

template <> TileKernel<double> tile_kernel<double>(int t, int *tb)
{
    if (t <= 1) { *tb = 1; return k_chambolle_tile<double, kTileX, kTileY, 1>; }
    if (t <= 2) { *tb = 2; return k_chambolle_tile<double, kTileX, kTileY, 2>; }
    if (t <= 4) { *tb = 4; return k_chambolle_tile<double, kTileX, kTileY, 4>; }
    *tb = 8;
    return k_chambolle_tile<double, kTileX, kTileY, 8>;
}

// ---------------------------------------------------------------------------
// device scratch, cached per (device, precision) and grown on demand

struct Scratch {
    size_t n_all = 0;      // C*H*W the plane buffers hold
    size_t spart_n = 0;    // doubles in spart
    size_t rpart_n = 0;    // doubles in rpart
    size_t elem = 0;       // sizeof(R)
    void *pa[2] = {nullptr, nullptr}; // dual field buffer A: px, py
    void *pb[2] = {nullptr, nullptr}; // dual field buffer B: px, py
    void *gl = nullptr;
    double *u = nullptr;
    double *dprev = nullptr;
    double *spart = nullptr;
    double *rpart = nullptr;
    unsigned int *nonfinite = nullptr;
};

struct HostStage {
    size_t f_n = 0, bands_n = 0, s_n = 0, r_n = 0;
    float *f = nullptr;
    double *bands = nullptr, *S = nullptr, *res = nullptr, *stats = nullptr;
    hipStream_t stream = nullptr;
};

constexpr int kMaxDevices = 64;
std::mutex g_mu;
Scratch g_scratch[kMaxDevices][2];
HostStage g_stage[kMaxDevices];

// Benchmark timing of the Chambolle kernel: event pairs around each launch.
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev; // start, stop, start, stop, ...
    size_t used = 0;            // pairs recorded and not yet read
    double ms = 0.0;            // time of pairs already read
    long long launches = 0;
    long long pixel_iters = 0;
};
Timing g_timing;
constexpr size_t kMaxTimingPairs = 1 << 15;

// Fold the recorded pairs into g_timing.ms (waits for them).
int timing_drain()
{
    for (size_t i = 0; i < g_timing.used; ++i) {
        HIP_TRY(hipEventSynchronize(g_timing.ev[2 * i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]));
        g_timing.ms += ms;
    }
    g_timing.used = 0;
    return TVSPEC_OK;
}

// Event pair for the next launch (created on demand, recycled after a drain).
int timing_pair(hipEvent_t *a, hipEvent_t *b)
{
    if (g_timing.used == kMaxTimingPairs) {
        int rc = timing_drain();
        if (rc != TVSPEC_OK)
            return rc;
    }
    while (g_timing.ev.size() < 2 * (g_timing.used + 1)) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        g_timing.ev.push_back(e);
    }
    *a = g_timing.ev[2 * g_timing.used];
    *b = g_timing.ev[2 * g_timing.used + 1];
    ++g_timing.used;
    return TVSPEC_OK;
}

void free_ptr(void *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_scratch(Scratch &s)
{
    free_ptr(s.pa[0]);
    free_ptr(s.pa[1]);
    free_ptr(s.pb[0]);
    free_ptr(s.pb[1]);
    free_ptr(s.gl);
    void *p;
    p = s.u; free_ptr(p); s.u = nullptr;
    p = s.dprev; free_ptr(p); s.dprev = nullptr;
    p = s.spart; free_ptr(p); s.spart = nullptr;
    p = s.rpart; free_ptr(p); s.rpart = nullptr;
    p = s.nonfinite; free_ptr(p); s.nonfinite = nullptr;
    s.n_all = s.spart_n = s.rpart_n = 0;
}

void free_stage(HostStage &h)
{
    void *p;
    p = h.f; free_ptr(p); h.f = nullptr;
    p = h.bands; free_ptr(p); h.bands = nullptr;
    p = h.S; free_ptr(p); h.S = nullptr;
    p = h.res; free_ptr(p); h.res = nullptr;
    p = h.stats; free_ptr(p); h.stats = nullptr;
    h.f_n = h.bands_n = h.s_n = h.r_n = 0;
}

int ensure_scratch(Scratch &s, size_t elem, size_t n_all, size_t spart_n, size_t rpart_n)
{
    if (s.elem == elem && s.n_all >= n_all && s.spart_n >= spart_n && s.rpart_n >= rpart_n && s.u)
        return TVSPEC_OK;
    // buffers may still be in use by earlier enqueued work
    HIP_TRY(hipDeviceSynchronize());
    free_scratch(s);
    s.elem = elem;
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipMalloc(&s.pa[i], n_all * elem));
        HIP_TRY(hipMalloc(&s.pb[i], n_all * elem));
    }
    HIP_TRY(hipMalloc(&s.gl, n_all * elem));
    HIP_TRY(hipMalloc((void **)&s.u, n_all * sizeof(double)));
    HIP_TRY(hipMalloc((void **)&s.dprev, n_all * sizeof(double)));
    HIP_TRY(hipMalloc((void **)&s.spart, spart_n * sizeof(double)));
    HIP_TRY(hipMalloc((void **)&s.rpart, rpart_n * sizeof(double)));
    HIP_TRY(hipMalloc((void **)&s.nonfinite, sizeof(unsigned int)));
    HIP_TRY(hipMemset(s.nonfinite, 0, sizeof(unsigned int)));
    HIP_TRY(hipDeviceSynchronize());
    s.n_all = n_all;
    s.spart_n = spart_n;
    s.rpart_n = rpart_n;
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// argument validation (host only, before any device call)

int validate(const void *f, int H, int W, int C, double dt, int K, int iters, const int *edges, int nb,
             const void *bands, const void *S, const void *res)
{
    if (!f || !bands || !S || !res || !edges)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (H < 2 || W < 2)
        return fail(TVSPEC_EINVAL, "H and W must be >= 2");
    if (C < 1)
        return fail(TVSPEC_EINVAL, "C must be >= 1");
    if ((long long)H * (long long)W > (1LL << 30))
        return fail(TVSPEC_EINVAL, "H*W must be <= 2^30");
    if ((long long)H * W * C > (1LL << 40))
        return fail(TVSPEC_EINVAL, "C*H*W too large");
    if (!std::isfinite(dt) || !(dt > 0.0))
        return fail(TVSPEC_EINVAL, "dt must be finite and > 0");
    if (K < 1)
        return fail(TVSPEC_EINVAL, "K must be >= 1");
    if (iters < 1)
        return fail(TVSPEC_EINVAL, "inner_iters must be >= 1");
    if (nb < 1 || nb > K)
        return fail(TVSPEC_EINVAL, "n_bands must be in [1, K]");
    if (edges[0] != 0 || edges[nb] != K)
        return fail(TVSPEC_EINVAL, "band edges must start at 0 and end at K");
    for (int j = 1; j <= nb; ++j)
        if (edges[j] <= edges[j - 1])
            return fail(TVSPEC_EINVAL, "band edges must be strictly increasing");
    return TVSPEC_OK;
}

int validate_opts(double tau, int warm, int precision, int ipl)
{
    if (!std::isfinite(tau) || !(tau > 0.0) || tau > 0.25)
        return fail(TVSPEC_EINVAL, "tau must be in (0, 0.25]");
    if (warm != 0 && warm != 1)
        return fail(TVSPEC_EINVAL, "warm_start must be 0 or 1");
    if (precision != TVSPEC_PRECISION_F32 && precision != TVSPEC_PRECISION_F64)
        return fail(TVSPEC_EINVAL, "precision must be TVSPEC_PRECISION_F32 or _F64");
    const int maxt = precision == TVSPEC_PRECISION_F32 ? 16 : 8;
    if (ipl < 0 || ipl > maxt)
        return fail(TVSPEC_EINVAL, "iters_per_launch out of range");
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// the decomposition, enqueued on a stream

template <typename R>
int enqueue(const float *f, int H, int W, int C, double dt, int K, int iters, const int *edges, int nb,
            double *bands, double *S, double *res, double *stats, double tau, int warm, int ipl,
            hipStream_t st, Scratch &sc)
{
    const int plane = H * W;
    const size_t n_all = (size_t)plane * (size_t)C;
    const int nblk = plane_blocks(plane);
    const size_t spart_n = (size_t)K * C * nblk;
    const size_t rpart_n = (size_t)C * nblk * 3;
    int rc = ensure_scratch(sc, sizeof(R), n_all, spart_n, rpart_n);
    if (rc != TVSPEC_OK)
        return rc;

    R *pbuf[2][2] = {{(R *)sc.pa[0], (R *)sc.pa[1]}, {(R *)sc.pb[0], (R *)sc.pb[1]}};
    R *gl = (R *)sc.gl;

    int tb = 0;
    const int want = ipl > 0 ? ipl : 8;
    TileKernel<R> kt = tile_kernel<R>(want < max_tb<R>() ? want : max_tb<R>(), &tb);
    const int ntx = (W + kTileX - 1) / kTileX;
    const int nty = (H + kTileY - 1) / kTileY;
    const int ntiles = ntx * nty;
    const int per_launch = ipl > 0 ? ipl : tb;

    // band index of every sample k = 1..K
    std::vector<int> band_of(K + 1, 0);
    for (int j = 0; j < nb; ++j)
        for (int k = edges[j] + 1; k <= edges[j + 1]; ++k)
            band_of[k] = j;

    const int gblk = blocks_for(n_all, 4096);
    hipLaunchKernelGGL(k_init<R>, dim3(gblk), dim3(kThreads), 0, st, f, sc.u, gl, pbuf[0][0], pbuf[0][1], bands,
                       n_all, nb, dt, sc.nonfinite);
    HIP_TRY(hipGetLastError());

    int cur = 0;
    for (int s = 0; s <= K; ++s) {
        if (!warm && s > 0) {
            if (sizeof(R) == 4)
                hipLaunchKernelGGL(k_zero2, dim3(gblk), dim3(kThreads), 0, st, (float *)pbuf[cur][0],
                                   (float *)pbuf[cur][1], n_all);
            else
                hipLaunchKernelGGL(k_zero2d, dim3(gblk), dim3(kThreads), 0, st, (double *)pbuf[cur][0],
                                   (double *)pbuf[cur][1], n_all);
        }
        for (int done = 0; done < iters;) {
            const int it = (iters - done) < per_launch ? (iters - done) : per_launch;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (g_timing.on) {
                if ((rc = timing_pair(&e0, &e1)) != TVSPEC_OK)
                    return rc;
                HIP_TRY(hipEventRecord(e0, st));
            }
            hipLaunchKernelGGL(kt, dim3(ntiles, C), dim3(kThreads), 0, st, pbuf[cur][0], pbuf[cur][1], gl,
                               pbuf[1 - cur][0], pbuf[1 - cur][1], H, W, ntx, ntiles, (R)tau, it);
            if (g_timing.on) {
                HIP_TRY(hipEventRecord(e1, st));
                ++g_timing.launches;
                g_timing.pixel_iters += (long long)n_all * it;
            }
            cur = 1 - cur;
            done += it;
        }
        double *band = s >= 1 ? bands + (size_t)band_of[s] * n_all : nullptr;
        hipLaunchKernelGGL(k_flow_step<R>, dim3(nblk, C), dim3(kThreads), 0, st, pbuf[cur][0], pbuf[cur][1],
                           sc.u, sc.dprev, gl, band, res, sc.spart, H, W, C, s, K, dt);
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_check, dim3(nblk, C), dim3(kThreads), 0, st, f, bands, res, sc.u, plane, C, nb, sc.rpart);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, st, sc.spart, sc.rpart, C, K, nblk, nblk, plane, dt, S,
                       stats, sc.nonfinite);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int decompose_on_device(const float *f, int H, int W, int C, double dt, int K, int iters, const int *edges, int nb,
                        double *bands, double *S, double *res, double *stats, double tau, int warm, int precision,
                        int ipl, hipStream_t st)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    if (precision == TVSPEC_PRECISION_F32)
        return enqueue<float>(f, H, W, C, dt, K, iters, edges, nb, bands, S, res, stats, tau, warm, ipl, st,
                              g_scratch[dev][0]);
    return enqueue<double>(f, H, W, C, dt, K, iters, edges, nb, bands, S, res, stats, tau, warm, ipl, st,
                           g_scratch[dev][1]);
}

template <typename T> int grow(T *&p, size_t &cap, size_t n)
{
    if (cap >= n && p)
        return TVSPEC_OK;
    void *v = p;
    free_ptr(v);
    p = nullptr;
    cap = 0;
    HIP_TRY(hipMalloc((void **)&p, n * sizeof(T)));
    cap = n;
    return TVSPEC_OK;
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" int tvspec_decompose_dev(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                    const int *band_edges, int n_bands, double *bands, double *S, double *residual,
                                    double *stats, double tau, int warm_start, int precision, int iters_per_launch,
                                    void *stream)
{
    g_last_error.clear();
    int rc = validate(f, H, W, C, dt, K, inner_iters, band_edges, n_bands, bands, S, residual);
    if (rc != TVSPEC_OK)
        return rc;
    if (!stats)
        return fail(TVSPEC_EINVAL, "null stats pointer");
    rc = validate_opts(tau, warm_start, precision, iters_per_launch);
    if (rc != TVSPEC_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    return decompose_on_device(f, H, W, C, dt, K, inner_iters, band_edges, n_bands, bands, S, residual, stats, tau,
                               warm_start, precision, iters_per_launch, (hipStream_t)stream);
}

extern "C" int tvspec_decompose(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                const int *band_edges, int n_bands, double *bands, double *S, double *residual)
{
    g_last_error.clear();
    int rc = validate(f, H, W, C, dt, K, inner_iters, band_edges, n_bands, bands, S, residual);
    if (rc != TVSPEC_OK)
        return rc;
    const size_t n_all = (size_t)H * W * C;
    for (size_t q = 0; q < n_all; ++q)
        if (!std::isfinite(f[q]))
            return fail(TVSPEC_ENUMERIC, "input holds a NaN or infinity");

    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    HostStage &h = g_stage[dev];
    if (!h.stream)
        HIP_TRY(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
    const size_t nb_n = (size_t)n_bands * n_all;
    const size_t s_n = (size_t)C * K;
    if ((rc = grow(h.f, h.f_n, n_all)) != TVSPEC_OK) return rc;
    if ((rc = grow(h.bands, h.bands_n, nb_n)) != TVSPEC_OK) return rc;
    if ((rc = grow(h.S, h.s_n, s_n)) != TVSPEC_OK) return rc;
    if ((rc = grow(h.res, h.r_n, n_all)) != TVSPEC_OK) return rc;
    if (!h.stats)
        HIP_TRY(hipMalloc((void **)&h.stats, TVSPEC_NSTATS * sizeof(double)));

    HIP_TRY(hipMemcpyAsync(h.f, f, n_all * sizeof(float), hipMemcpyHostToDevice, h.stream));
    rc = decompose_on_device(h.f, H, W, C, dt, K, inner_iters, band_edges, n_bands, h.bands, h.S, h.res, h.stats,
                             TVSPEC_DEFAULT_TAU, 1, TVSPEC_PRECISION_F32, 0, h.stream);
    if (rc != TVSPEC_OK)
        return rc;
    HIP_TRY(hipMemcpyAsync(bands, h.bands, nb_n * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    HIP_TRY(hipMemcpyAsync(S, h.S, s_n * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    HIP_TRY(hipMemcpyAsync(residual, h.res, n_all * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    HIP_TRY(hipStreamSynchronize(h.stream));
    return TVSPEC_OK;
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
    g_timing.on = on != 0;
    return TVSPEC_OK;
}

extern "C" int tvspec_timing_read(double *kernel_ms, long long *launches, long long *pixel_iters)
{
    g_last_error.clear();
    std::lock_guard<std::mutex> lock(g_mu);
    int rc = timing_drain();
    if (rc != TVSPEC_OK)
        return rc;
    if (kernel_ms) *kernel_ms = g_timing.ms;
    if (launches) *launches = g_timing.launches;
    if (pixel_iters) *pixel_iters = g_timing.pixel_iters;
    g_timing.ms = 0.0;
    g_timing.launches = 0;
    g_timing.pixel_iters = 0;
    return TVSPEC_OK;
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
        bool any = g_stage[d].stream || g_scratch[d][0].u || g_scratch[d][1].u || g_stage[d].f;
        if (!any)
            continue;
        if (hipSetDevice(d) != hipSuccess)
            continue;
        (void)hipDeviceSynchronize();
        free_scratch(g_scratch[d][0]);
        free_scratch(g_scratch[d][1]);
        free_stage(g_stage[d]);
        if (g_stage[d].stream) {
            (void)hipStreamDestroy(g_stage[d].stream);
            g_stage[d].stream = nullptr;
        }
    }
    (void)hipSetDevice(cur);
}
