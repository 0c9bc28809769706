// tvspec engine: kernels and launchers of the spectral TV decomposition on
// gfx950, over a table of image slots (see engine.h).
//
// Method: Grossmann, Korolev, Gilboa, Schoenlieb, arXiv 2006.10004.
//   Sec. 2.2 Eq. (8)   one implicit Euler step of the TV flow Eq. (1) is a ROF
//                      problem; it is solved here by Chambolle's dual
//                      projection iteration (the solver Sec. 4.3 names);
//   Sec. 2.1 Eq. (3)   phi(t_k) = t_k u_tt(t_k) by the central second
//                      difference, S(t_k) = ||phi(t_k)||_1, band integrals of
//                      Eq. (7) and the residual of Eq. (5).
//
// Device work per slot (one C x H x W image, channels independent):
//   k_init           u_0 = f (float64), p = 0, bands = 0, count of
//                    non-finite inputs (F32: G = grad(f)/dt of the first
//                    solve);
//   k_chambolle_tile the hot loop.  Each launch runs `iters` (<= TB) Jacobi
//                    iterations of Chambolle's fixed point on a 32x32 output
//                    tile whose (32+2TB)^2 neighbourhood is staged once; the
//                    dual field stays in registers, only neighbour values
//                    cross lanes through LDS.  Tiles are mapped to workgroups
//                    so that each XCD works on one horizontal band of the
//                    image (neighbouring halos then hit the same L2);
//   k_flow_step      one launch per ROF solve, fused: div p, u_{s+1} =
//                    u_s - dt div p, D_s = dt div p, phi_s dt = s (D_{s-1} -
//                    D_s) added to its band, a per-block partial of sum |D_{s-1}
//                    - D_s| for S(t_s), the residual at s = K, and grad(g)/dt
//                    of the next solve.  u_{s-1} and u_{s+1} never exist as
//                    planes beside u_s;
//   k_advance        moves every active slot to its next step;
//   k_check          per-block partials of the reconstruction error and of
//                    the mean of u_{K+1} and f;
//   k_reduce_s       S(t_k) from the step partials, one block per (k, c);
//   k_report         the report (reductions in a fixed order, so results are
//                    bit-reproducible run to run).
//
// Precision modes of the inner iteration.  S is the type of the dual field
// and of the update arithmetic; M selects how |a| and the reciprocal are
// formed (and, in F32, the type of the stored data-term gradient G):
//   F32    S = float,  M = float   (IEEE-rounded float32 except the
//          hardware square root and reciprocal estimates)
//   F64    S = double, M = double  (IEEE float64 throughout)
//   MIXED  S = double, M = float.  float64 arithmetic, but |a| and the
//          reciprocal come from the float32 hardware estimates refined by one
//          float64 Newton step.  On gfx950, with
//          packed float32 math off, float64 add and fma issue at the float32
//          rate; what makes float64 dear is its square root and division
//          sequences, which this avoids.  Float32 is not enough for long
//          flows: with dt = 0.002 and 200 steps the spectral sums weight
//          differences of the flow by up to 200, and the float32 rounding of
//          div p (a cancelling difference of O(1) values) and of the update's
//          nonlinear factor then moves the bands by ~4e-4.
// The flow state u, D, phi, the bands, S and the checks are float64 always.
//
// Arithmetic contract: every kernel variant (any temporal blocking factor)
// applies the same per-pixel operations in the same order, so results do not
// depend on the launch configuration or on which other slots share a table.
// Build with -ffp-contract=off; fused multiply-adds are written explicitly.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "engine.h"

namespace tvspec {

namespace {

#include "tile_kernels.h"

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

constexpr int kThreads = 256;

// Block of 256 threads (4 waves).  Every thread returns the block result.
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

// ---------------------------------------------------------------------------
// kernels

// u_0 = f, p = 0 (both buffers), bands = 0 (F32 Chambolle: G = grad f / dt),
// for slot first + blockIdx.y; counts non-finite inputs; starts the slot
// at step 0.  For PDHG p is its dual field y; its primal iterates are set at
// the start of every solve.
template <typename S, typename M, bool PD>
__global__ __launch_bounds__(kThreads) void k_init(SlotDesc *__restrict__ slots, int first, int H, int W, int C)
{
    SlotDesc &sd = slots[first + blockIdx.y];
    const int plane = H * W;
    const size_t n = (size_t)C * (size_t)plane;
    const double dt = sd.dt;
    const float *__restrict__ f = sd.f;
    S *__restrict__ p0 = (S *)sd.px[0];
    S *__restrict__ p1 = (S *)sd.px[1];
    S *__restrict__ p2 = (S *)sd.py[0];
    S *__restrict__ p3 = (S *)sd.py[1];
    M *__restrict__ gx = (M *)sd.gx;
    M *__restrict__ gy = (M *)sd.gy;
    double *__restrict__ u = sd.u[0];
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += stride) {
        const int qq = (int)(q % (size_t)plane);
        const int i = qq / W;
        const int j = qq - i * W;
        const float v = f[q];
        if (!isfinite(v))
            atomicAdd(sd.nonfinite, 1u);
        u[q] = (double)v;
        if constexpr (!PD && !std::is_same<S, double>::value) {
            gx[q] = (j < W - 1) ? (M)(((double)f[q + 1] - (double)v) / dt) : M(0);
            gy[q] = (i < H - 1) ? (M)(((double)f[q + W] - (double)v) / dt) : M(0);
        }
        p0[q] = S(0);
        p1[q] = S(0);
        p2[q] = S(0);
        p3[q] = S(0);
        for (int k = 0; k < sd.nbands; ++k)
            sd.bands[(size_t)k * n + q] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sd.k_cur = 0;
        sd.active = 1;
    }
}

// div p at pixel q = (i, j) of one channel plane, in float64 from the stored
// dual field (zero outside the image).
template <typename S>
__device__ __forceinline__ double div_p(const S *__restrict__ px, const S *__restrict__ py, int q, int i, int j,
                                        int W)
{
    const double pxl = (j > 0) ? (double)px[q - 1] : 0.0;
    const double pyu = (i > 0) ? (double)py[q - W] : 0.0;
    return ((double)px[q] - pxl) + ((double)py[q] - pyu);
}

// Outer step k = k_cur of every active slot, fused with the spectral
// transform.  Grid: (nblk, slots * C), nblk fixed per image size so partial
// sums are reproducible.  The final iterate of the solve is in buffer cur.
//   Chambolle (PD = false):
//     D_k     = dt div p                   (u_k - u_{k+1})
//     u_{k+1} = u_k - D_k                  (u[(k+1) % 2])
//   PDHG (PD = true):
//     u_{k+1} = x, the solve's primal iterate;  D_k = u_k - u_{k+1}
//   both:
//   k >= 1: phi_k dt = k (D_{k-1} - D_k)   added to the band holding k
//           spart  <- block sum of |D_{k-1} - D_k|   (S(t_k) = k/dt * total)
//   k == K: residual = u_K + K D_K          (u(T) - T u_t(T), forward u_t)
//   G       = grad(u_{k+1}) / dt           (F32 Chambolle only: data term of the
//             next solve; the right and lower neighbours' u_{k+1} are
//             recomputed here with the same operations their own threads
//             use, so they match bit for bit)
template <typename S, typename M, bool PD>
__global__ __launch_bounds__(kThreads) void k_flow_step(const SlotDesc *__restrict__ slots, int cur, int H, int W,
                                                        int C)
{
    __shared__ double sh[4];
    const int slot = blockIdx.y / C;
    const int c = blockIdx.y - slot * C;
    const SlotDesc &sd = slots[slot];
    if (!sd.active)
        return;
    const int k = sd.k_cur;
    const int K = sd.K;
    const double dt = sd.dt;
    const int plane = H * W;
    const size_t coff = (size_t)c * (size_t)plane;
    const S *__restrict__ px = (const S *)sd.px[cur] + coff;
    const S *__restrict__ py = (const S *)sd.py[cur] + coff;
    const double *__restrict__ uin = sd.u[k & 1] + coff;
    double *__restrict__ uout = sd.u[(k + 1) & 1] + coff;
    double *__restrict__ dprev = sd.dprev + coff;
    M *__restrict__ gx = (M *)sd.gx + coff;
    M *__restrict__ gy = (M *)sd.gy + coff;
    double *__restrict__ resid = sd.res + coff;
    double *__restrict__ band = nullptr;
    if (k >= 1)
        band = sd.bands + ((size_t)sd.band_rows[k] * C + c) * (size_t)plane;
    const double kd = (double)k;
    double acc = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        const int i = q / W;
        const int j = q - i * W;
        const double uo = uin[q];
        double D, un;
        if constexpr (PD) {
            un = (double)((const S *)sd.x[cur] + coff)[q]; // the solve's primal iterate
            D = uo - un;
        } else {
            D = dt * div_p(px, py, q, i, j, W);
            un = uo - D;
        }
        if (k >= 1) {
            const double dl = dprev[q] - D;
            band[q] += kd * dl;
            acc += fabs(dl);
        }
        if (k == K)
            resid[q] = uo + (double)K * D;
        uout[q] = un;
        dprev[q] = D;
        if constexpr (!PD && !std::is_same<S, double>::value) {
            if (j < W - 1) {
                const double unr = uin[q + 1] - dt * div_p(px, py, q + 1, i, j + 1, W);
                gx[q] = (M)((unr - un) / dt);
            } else {
                gx[q] = M(0);
            }
            if (i < H - 1) {
                const double und = uin[q + W] - dt * div_p(px, py, q + W, i + 1, j, W);
                gy[q] = (M)((und - un) / dt);
            } else {
                gy[q] = M(0);
            }
        }
    }
    if (k >= 1) {
        acc = block_sum256(acc, sh);
        if (threadIdx.x == 0)
            sd.spart[((size_t)(k - 1) * C + c) * gridDim.x + blockIdx.x] = acc;
    }
}

// Every active slot moves to its next step; a slot that has run step K
// becomes inactive (its k_cur ends at K + 1).
__global__ __launch_bounds__(kThreads) void k_advance(SlotDesc *__restrict__ slots, int nslots)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nslots || !slots[i].active)
        return;
    if (slots[i].k_cur == slots[i].K)
        slots[i].active = 0;
    slots[i].k_cur += 1;
}

// Per-block partials of: max |f - sum_j b_j - r|, sum u_{K+1}, sum f, for
// completed slots first, first + 1, ...  Grid: (nblk, count * C).  u_{K+1}
// is in u[(K + 1) % 2].
__global__ __launch_bounds__(kThreads) void k_check(const SlotDesc *__restrict__ slots, int first, int plane, int C)
{
    __shared__ double sh[4];
    const int rel = blockIdx.y / C;
    const SlotDesc &sd = slots[first + rel];
    const int c = blockIdx.y - rel * C;
    const size_t coff = (size_t)c * (size_t)plane;
    const double *__restrict__ u = sd.u[(sd.K + 1) & 1] + coff;
    const double *__restrict__ b0 = sd.bands + coff;
    const size_t bstride = (size_t)C * (size_t)plane;
    double emax = 0.0, su = 0.0, sf = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        double acc = 0.0;
        for (int j = 0; j < sd.nbands; ++j)
            acc += b0[(size_t)j * bstride + q];
        const double fv = (double)sd.f[coff + q];
        emax = fmax(emax, fabs(fv - acc - sd.res[coff + q]));
        su += u[q];
        sf += fv;
    }
    emax = block_max256(emax, sh);
    su = block_sum256(su, sh);
    sf = block_sum256(sf, sh);
    if (threadIdx.x == 0) {
        double *o = sd.rpart + ((size_t)c * gridDim.x + blockIdx.x) * 3;
        o[0] = emax;
        o[1] = su;
        o[2] = sf;
    }
}

// S of completed slots first, first + 1, ...: S[c][k-1] = k/dt * (sum of
// the step partials of sample k, channel c); one block per (k, slot, c), each
// thread summing a fixed stride of partials, then the block sum in a fixed
// order.  Grid: (max K, count * C); blocks beyond a slot's K exit.
__global__ __launch_bounds__(kThreads) void k_reduce_s(const SlotDesc *__restrict__ slots, int first, int C,
                                                       int nblk)
{
    __shared__ double sh[4];
    const int rel = blockIdx.y / C;
    const SlotDesc &sd = slots[first + rel];
    const int k = blockIdx.x + 1;
    const int c = blockIdx.y - rel * C;
    if (k > sd.K)
        return;
    const double *p = sd.spart + ((size_t)(k - 1) * C + c) * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
        s += p[b];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0)
        sd.S[(size_t)c * sd.K + (k - 1)] = s * ((double)k / sd.dt);
}

// The report of completed slot first + blockIdx.x from its check partials
// (fixed reduction order); clears the slot's non-finite counter.
__global__ __launch_bounds__(kThreads) void k_report(const SlotDesc *__restrict__ slots, int first, int C,
                                                     int nblk_chk, int plane)
{
    __shared__ double sh[4];
    const SlotDesc &sd = slots[first + blockIdx.x];
    double emax = 0.0, drift = 0.0;
    for (int c = 0; c < C; ++c) {
        double e = 0.0, su = 0.0, sf = 0.0;
        for (int b = threadIdx.x; b < nblk_chk; b += kThreads) {
            const double *o = sd.rpart + ((size_t)c * nblk_chk + b) * 3;
            e = fmax(e, o[0]);
            su += o[1];
            sf += o[2];
        }
        e = block_max256(e, sh);
        su = block_sum256(su, sh);
        sf = block_sum256(sf, sh);
        emax = fmax(emax, e);
        drift = fmax(drift, fabs(su / (double)plane - sf / (double)plane));
    }
    if (threadIdx.x == 0) {
        sd.stats[0] = emax;
        sd.stats[1] = drift;
        sd.stats[2] = (double)(*sd.nonfinite);
        sd.stats[3] = 0.0;
        *sd.nonfinite = 0u;
    }
}

// ---------------------------------------------------------------------------
// launch configuration

// Output tile of the Chambolle kernel and its workgroup size.
constexpr int kTileX = 32;
constexpr int kTileY = 32;
constexpr int kTileThreads = 1024;

int blocks_for(size_t n, int cap)
{
    size_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

template <typename S, typename M>
using TileKernel = void (*)(const SlotDesc *, int, int, int, int, int, int, S, int, int);

// Largest temporal blocking factor compiled for a mode (LDS and registers of
// the (32+2TB)^2 region, which are sized by the dual-field type S).
template <typename S> constexpr int max_tb() { return std::is_same<S, float>::value ? 16 : 8; }

template <typename S, typename M>
using PdhgKernel = void (*)(const SlotDesc *, int, int, int, int, int, int, S, S, S, int, int, int);

// Smallest compiled halo width >= t of the primal-dual kernel.
template <typename S, typename M> PdhgKernel<S, M> pdhg_kernel(int t, int *tb)
{
    if (t <= 1) { *tb = 1; return k_pdhg_tile<S, M, kTileX, kTileY, 1, kTileThreads>; }
    if (t <= 2) { *tb = 2; return k_pdhg_tile<S, M, kTileX, kTileY, 2, kTileThreads>; }
    if (t <= 4) { *tb = 4; return k_pdhg_tile<S, M, kTileX, kTileY, 4, kTileThreads>; }
    if (t <= 5) { *tb = 5; return k_pdhg_tile<S, M, kTileX, kTileY, 5, kTileThreads>; }
    if constexpr (max_tb<S>() >= 16) {
        if (t > 8) { *tb = 16; return k_pdhg_tile<S, M, kTileX, kTileY, 16, kTileThreads>; }
    }
    *tb = 8;
    return k_pdhg_tile<S, M, kTileX, kTileY, 8, kTileThreads>;
}

// The narrow tile shape (kTileShapeNarrow): 32 x 16 output pixels on 512
// threads, for launches that give the device too few 32 x 32 workgroups;
// compiled for TB = 4, 5 and 8.
constexpr int kNarrowY = 16;
constexpr int kNarrowThreads = 512;

template <typename S, typename M> TileKernel<S, M> narrow_tile_kernel(int t, int *tb)
{
    if (t <= 4) { *tb = 4; return k_chambolle_tile<S, M, kTileX, kNarrowY, 4, kNarrowThreads>; }
    if (t <= 5) { *tb = 5; return k_chambolle_tile<S, M, kTileX, kNarrowY, 5, kNarrowThreads>; }
    *tb = 8;
    return k_chambolle_tile<S, M, kTileX, kNarrowY, 8, kNarrowThreads>;
}

// The whole-plane form: a plane of at most kPlaneMax x kPlaneMax pixels is
// one tile whose region is the whole image (no halo, TB = 0), so one launch
// runs every iteration of a solve: nothing outside the region feeds it, and
// the region's pixels outside the image keep p = 0 as they do in the tiles.
// LDS: three (64 + 2)^2 planes of the state type, 104.5 KB in float64 (the
// 160 KB of a gfx950 CU); 4 pixels per thread.
constexpr int kPlaneMax = 64;

template <typename S, typename M> TileKernel<S, M> plane_kernel()
{
    return k_chambolle_tile<S, M, kPlaneMax, kPlaneMax, 0, kTileThreads>;
}

// Whether a step takes the whole-plane form: small planes, the Chambolle
// solver, automatic blocking and the square tile option.
bool whole_plane(const StepConfig &cfg)
{
    return cfg.solver != kSolverPDHG && cfg.iters_per_launch == 0 && cfg.tile == kTileShapeSquare &&
           cfg.H <= kPlaneMax && cfg.W <= kPlaneMax;
}

// Smallest compiled halo width >= t.
template <typename S, typename M> TileKernel<S, M> tile_kernel(int t, int *tb)
{
    if (t <= 1) { *tb = 1; return k_chambolle_tile<S, M, kTileX, kTileY, 1, kTileThreads>; }
    if (t <= 2) { *tb = 2; return k_chambolle_tile<S, M, kTileX, kTileY, 2, kTileThreads>; }
    if (t <= 4) { *tb = 4; return k_chambolle_tile<S, M, kTileX, kTileY, 4, kTileThreads>; }
    if (t <= 5) { *tb = 5; return k_chambolle_tile<S, M, kTileX, kTileY, 5, kTileThreads>; }
    if constexpr (max_tb<S>() >= 16) {
        if (t > 8) { *tb = 16; return k_chambolle_tile<S, M, kTileX, kTileY, 16, kTileThreads>; }
    }
    *tb = 8;
    return k_chambolle_tile<S, M, kTileX, kTileY, 8, kTileThreads>;
}

// Compute units of the current device (cached per device).
int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// Automatic temporal blocking factor.  The 32x32 tile with TB = 8 stages a
// 48x48 region (2.25 region pixels per output pixel, 62 VGPRs in MIXED); TB
// = 5 stages 42x42 (1.72 per output pixel, 48 VGPRs, 46 KB LDS) at 8/5 the
// launches.  Measured on MI355X (MIXED): with one workgroup per CU (a single
// 512x512 plane) TB = 8 is 7% faster (16.9 against 18.2 ms for 41 solves);
// where a launch gives every CU at least two workgroups, TB = 5 is 4-7%
// faster on planes of 256x256 and up (12 x 3 x 256^2: 36.5 against 38.1 ms;
// 3 x 1024^2: 41.4 against 44.6 ms), but planes of at most 64x64 (four
// tiles, half of every region outside the image) keep TB = 8 (256 x 64^2:
// 48.2 against 51.3 ms).  F64 favours TB = 5 in both regimes; F32 keeps
// TB = 8.
int auto_tb(int precision, long long workgroups, int H, int W)
{
    if (precision == TVSPEC_PRECISION_F32)
        return 8;
    if (precision == TVSPEC_PRECISION_F64)
        return 5;
    if (H <= 64 && W <= 64)
        return 8;
    return workgroups >= 2LL * device_cus() ? 5 : 8;
}

// ---------------------------------------------------------------------------
// benchmark timing of the tile kernel: one event pair per engine_step

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

int timing_pair(hipEvent_t *a, hipEvent_t *b)
{
    if (g_timing.used == kMaxTimingPairs)
        TVSPEC_TRY(timing_drain());
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

// ---------------------------------------------------------------------------
// launchers per mode

template <typename S, typename M> int init_impl(const StepConfig &cfg, SlotDesc *d_slots, int first, int count,
                                                hipStream_t st)
{
    const size_t n = (size_t)cfg.C * cfg.H * cfg.W;
    if (cfg.solver == kSolverPDHG)
        hipLaunchKernelGGL((k_init<S, M, true>), dim3(blocks_for(n, 1024), count), dim3(kThreads), 0, st, d_slots,
                           first, cfg.H, cfg.W, cfg.C);
    else
        hipLaunchKernelGGL((k_init<S, M, false>), dim3(blocks_for(n, 1024), count), dim3(kThreads), 0, st, d_slots,
                           first, cfg.H, cfg.W, cfg.C);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

template <typename S, typename M> int step_impl(const StepConfig &cfg, SlotDesc *d_slots, int nslots, int *parity,
                                                hipStream_t st, long long live_planes)
{
    const int plane = cfg.H * cfg.W;
    const bool pd = cfg.solver == kSolverPDHG;
    const bool whole = whole_plane(cfg);
    const bool narrow = !pd && cfg.tile == kTileShapeNarrow;
    const int tile_y = whole ? kPlaneMax : (narrow ? kNarrowY : kTileY);
    const int tile_x = whole ? kPlaneMax : kTileX;
    const int threads = narrow ? kNarrowThreads : kTileThreads;
    const int ntx = (cfg.W + tile_x - 1) / tile_x;
    const int nty = (cfg.H + tile_y - 1) / tile_y;
    const int ntiles = ntx * nty;
    int tb = 0;
    const int want = cfg.iters_per_launch > 0 ? cfg.iters_per_launch
                                              : auto_tb(cfg.precision, (long long)ntiles * nslots * cfg.C, cfg.H, cfg.W);
    TileKernel<S, M> kt = nullptr;
    PdhgKernel<S, M> kp = nullptr;
    if (pd)
        kp = pdhg_kernel<S, M>(want, &tb);
    else if (whole)
        kt = plane_kernel<S, M>();
    else if (narrow)
        kt = narrow_tile_kernel<S, M>(want, &tb);
    else
        kt = tile_kernel<S, M>(want, &tb);
    const int per_launch = whole ? cfg.iters : (cfg.iters_per_launch > 0 ? cfg.iters_per_launch : tb);
    int cur = *parity;

    // timing: one event pair around the back-to-back Chambolle launches of
    // this solve (events between launches would perturb them)
    const bool timed = cfg.timed && g_timing.on;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        TVSPEC_TRY(timing_pair(&e0, &e1));
        HIP_TRY(hipEventRecord(e0, st));
    }
    for (int done = 0; done < cfg.iters;) {
        // cold start: the first launch of a solve starts from p = 0
        const int zero_in = (!cfg.warm && done == 0) ? 1 : 0;
        const int it = (cfg.iters - done) < per_launch ? (cfg.iters - done) : per_launch;
        if (pd)
            hipLaunchKernelGGL(kp, dim3(ntiles, nslots * cfg.C), dim3(kTileThreads), 0, st, d_slots, cur, cfg.H,
                               cfg.W, cfg.C, ntx, ntiles, (S)cfg.tau, (S)cfg.sigma, (S)(1.0 / (1.0 + cfg.tau)), it,
                               done == 0 ? 1 : 0, zero_in);
        else
            hipLaunchKernelGGL(kt, dim3(ntiles, nslots * cfg.C), dim3(threads), 0, st, d_slots, cur, cfg.H,
                               cfg.W, cfg.C, ntx, ntiles, (S)cfg.tau, it, zero_in);
        if (timed) {
            ++g_timing.launches;
            g_timing.pixel_iters += live_planes * plane * it;
        }
        cur = 1 - cur;
        done += it;
    }
    if (timed)
        HIP_TRY(hipEventRecord(e1, st));
    if (pd)
        hipLaunchKernelGGL((k_flow_step<S, M, true>), dim3(plane_blocks(plane), nslots * cfg.C), dim3(kThreads), 0,
                           st, d_slots, cur, cfg.H, cfg.W, cfg.C);
    else
        hipLaunchKernelGGL((k_flow_step<S, M, false>), dim3(plane_blocks(plane), nslots * cfg.C), dim3(kThreads), 0,
                           st, d_slots, cur, cfg.H, cfg.W, cfg.C);
    hipLaunchKernelGGL(k_advance, dim3((nslots + kThreads - 1) / kThreads), dim3(kThreads), 0, st, d_slots, nslots);
    HIP_TRY(hipGetLastError());
    *parity = cur;
    return TVSPEC_OK;
}

} // namespace

size_t state_elem(int precision) { return precision == TVSPEC_PRECISION_F32 ? 4 : 8; }
size_t g_elem(int precision) { return precision == TVSPEC_PRECISION_F32 ? 4 : 0; }

int plane_blocks(int plane) { return blocks_for((size_t)plane, 1024); }

size_t slot_scratch_bytes(int precision, int solver, int H, int W, int C, int K)
{
    const size_t n = (size_t)C * H * W;
    const size_t nblk = (size_t)plane_blocks(H * W);
    const size_t solver_bytes = solver == kSolverPDHG ? 4 * align256(n * state_elem(precision)) // x[2], xb[2]
                                                      : 2 * align256(n * g_elem(precision));     // gx, gy (F32)
    return 4 * align256(n * state_elem(precision))     // px[2], py[2]
           + solver_bytes
           + 3 * align256(n * sizeof(double))           // u[2], dprev
           + align256((size_t)K * C * nblk * sizeof(double)) // spart
           + align256((size_t)C * nblk * 3 * sizeof(double)); // rpart
}

void slot_carve(SlotDesc &d, char *base, int precision, int solver, int H, int W, int C, int K)
{
    const size_t n = (size_t)C * H * W;
    const size_t nblk = (size_t)plane_blocks(H * W);
    char *p = base;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return r;
    };
    d.px[0] = take(n * state_elem(precision));
    d.px[1] = take(n * state_elem(precision));
    d.py[0] = take(n * state_elem(precision));
    d.py[1] = take(n * state_elem(precision));
    if (solver == kSolverPDHG) {
        d.gx = d.gy = nullptr;
        d.x[0] = take(n * state_elem(precision));
        d.x[1] = take(n * state_elem(precision));
        d.xb[0] = take(n * state_elem(precision));
        d.xb[1] = take(n * state_elem(precision));
    } else if (g_elem(precision) > 0) {
        d.gx = take(n * g_elem(precision));
        d.gy = take(n * g_elem(precision));
        d.x[0] = d.x[1] = d.xb[0] = d.xb[1] = nullptr;
    } else {
        // the float64 modes read the data term from u directly
        d.gx = d.gy = nullptr;
        d.x[0] = d.x[1] = d.xb[0] = d.xb[1] = nullptr;
    }
    d.u[0] = (double *)take(n * sizeof(double));
    d.u[1] = (double *)take(n * sizeof(double));
    d.dprev = (double *)take(n * sizeof(double));
    d.spart = (double *)take((size_t)K * C * nblk * sizeof(double));
    d.rpart = (double *)take((size_t)C * nblk * 3 * sizeof(double));
    d.K = K;
}


int tile_launches_per_step(const StepConfig &cfg, int nslots)
{
    if (whole_plane(cfg))
        return 1;
    const bool narrow = cfg.solver != kSolverPDHG && cfg.tile == kTileShapeNarrow;
    const int tile_y = narrow ? kNarrowY : kTileY;
    const int ntiles = ((cfg.W + kTileX - 1) / kTileX) * ((cfg.H + tile_y - 1) / tile_y);
    int tb = 0;
    const int want = cfg.iters_per_launch > 0 ? cfg.iters_per_launch
                                              : auto_tb(cfg.precision, (long long)ntiles * nslots * cfg.C, cfg.H, cfg.W);
    if (narrow && cfg.precision == TVSPEC_PRECISION_F32)
        (void)narrow_tile_kernel<float, float>(want, &tb);
    else if (narrow)
        (void)narrow_tile_kernel<double, double>(want, &tb);
    else if (cfg.precision == TVSPEC_PRECISION_F32)
        (void)tile_kernel<float, float>(want, &tb);
    else
        (void)tile_kernel<double, double>(want, &tb);
    const int per_launch = cfg.iters_per_launch > 0 ? cfg.iters_per_launch : tb;
    return (cfg.iters + per_launch - 1) / per_launch;
}

int engine_init(const StepConfig &cfg, SlotDesc *d_slots, int first, int count, hipStream_t st)
{
    switch (cfg.precision) {
    case TVSPEC_PRECISION_F32: return init_impl<float, float>(cfg, d_slots, first, count, st);
    case TVSPEC_PRECISION_F64: return init_impl<double, double>(cfg, d_slots, first, count, st);
    default: return init_impl<double, float>(cfg, d_slots, first, count, st);
    }
}

int engine_step(const StepConfig &cfg, SlotDesc *d_slots, int nslots, int *parity, hipStream_t st,
                long long live_planes)
{
    switch (cfg.precision) {
    case TVSPEC_PRECISION_F32: return step_impl<float, float>(cfg, d_slots, nslots, parity, st, live_planes);
    case TVSPEC_PRECISION_F64: return step_impl<double, double>(cfg, d_slots, nslots, parity, st, live_planes);
    default: return step_impl<double, float>(cfg, d_slots, nslots, parity, st, live_planes);
    }
}

int engine_finalize(const StepConfig &cfg, SlotDesc *d_slots, int first, int count, int Kmax, hipStream_t st)
{
    const int plane = cfg.H * cfg.W;
    const int nblk = plane_blocks(plane);
    hipLaunchKernelGGL(k_check, dim3(nblk, count * cfg.C), dim3(kThreads), 0, st, d_slots, first, plane, cfg.C);
    hipLaunchKernelGGL(k_reduce_s, dim3(Kmax, count * cfg.C), dim3(kThreads), 0, st, d_slots, first, cfg.C, nblk);
    hipLaunchKernelGGL(k_report, dim3(count), dim3(kThreads), 0, st, d_slots, first, cfg.C, nblk, plane);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int timing_enable(int on)
{
    g_timing.on = on != 0;
    return TVSPEC_OK;
}

int timing_read(double *kernel_ms, long long *launches, long long *pixel_iters)
{
    TVSPEC_TRY(timing_drain());
    if (kernel_ms) *kernel_ms = g_timing.ms;
    if (launches) *launches = g_timing.launches;
    if (pixel_iters) *pixel_iters = g_timing.pixel_iters;
    g_timing.ms = 0.0;
    g_timing.launches = 0;
    g_timing.pixel_iters = 0;
    return TVSPEC_OK;
}

} // namespace tvspec
