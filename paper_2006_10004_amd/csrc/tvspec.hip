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
//   k_init           u_0 = f (float64), G = grad(f)/dt for the first solve,
//                    p = 0, bands = 0, count of non-finite inputs;
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
//   k_check          per-block partials of the reconstruction error and of
//                    the mean of u_{K+1} and f;
//   k_reduce_s       S(t_k) from the step partials, one block per (k, c);
//   k_report         the report (reductions in a fixed order, so results are
//                    bit-reproducible run to run).
//
// Precision modes of the inner iteration.  S is the type of the dual field
// and of the update arithmetic, M the type G is stored in:
//   F32    S = float,  M = float   (IEEE-rounded float32 except the
//          hardware square root and reciprocal estimates)
//   F64    S = double, M = double  (IEEE float64 throughout)
//   MIXED  S = double, M = float.  float64 arithmetic, but |a| and the
//          reciprocal come from the float32 hardware estimates refined by one
//          float64 Newton step, and G is stored in float32.  On gfx950, with
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
#include <type_traits>
#include <vector>

#include "tvspec.h"

#define TVSPEC_VERSION_STRING "tvspec 0.2.0 (gfx950)"

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
// scalar operations of the Chambolle update

template <typename M> struct Arith;

template <> struct Arith<float> {
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    // one reciprocal shared by both components
    static __device__ __forceinline__ float inv_(float d) { return __builtin_amdgcn_rcpf(d); }
};

template <> struct Arith<double> {
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
    static __device__ __forceinline__ double inv_(double d) { return 1.0 / d; }
};

// One Chambolle update of a pixel's dual vector from the gradient a of
// div p - g/dt:  p <- (p + tau a) / (1 + tau |a|).
// |a| is formed as ax*ax + ay*ay (not a fused multiply-add) so that the
// update is symmetric in x and y, like the method.
template <typename S, typename M>
__device__ __forceinline__ void chambolle_update(S &px, S &py, S ax, S ay, S tau)
{
    if constexpr (std::is_same<S, M>::value) {
        using A = Arith<S>;
        const S nrm = A::sqrt_(ax * ax + ay * ay);
        const S r = A::inv_(A::fma_(tau, nrm, S(1)));
        px = A::fma_(tau, ax, px) * r;
        py = A::fma_(tau, ay, py) * r;
    } else {
        // float64 update in increment form, p += tau (a - |a| p) / (1 + tau |a|),
        // with |a| and the reciprocal from the float32 hardware estimates
        // (v_rsq_f32, v_rcp_f32) refined by one Newton step in float64
        // (relative error ~1e-14; the float64 square root and division
        // sequences cost several times more).  Below |a| = 1e-15 the
        // estimate's argument would leave the float32 normal range, and |a| is
        // taken as 0: the increment then differs by at most tau |a| |p|, far
        // below the rounding of p.
        const S x = ax * ax + ay * ay;
        S y = (S)__builtin_amdgcn_rsqf((float)x);
        y = __builtin_fma(S(0.5) * y, __builtin_fma(-(x * y), y, S(1)), y);
        const S nrm = x > S(1e-30) ? x * y : S(0);
        const S den = __builtin_fma(tau, nrm, S(1));
        S r = (S)__builtin_amdgcn_rcpf((float)den);
        r = __builtin_fma(r, __builtin_fma(-den, r, S(1)), r);
        const S tr = tau * r;
        px += tr * __builtin_fma(-nrm, px, ax);
        py += tr * __builtin_fma(-nrm, py, ay);
    }
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

// u = f, G = grad f / dt (data term of the first solve), p = 0 (buffer A),
// bands = 0; counts non-finite inputs.
template <typename S, typename M>
__global__ __launch_bounds__(kThreads) void k_init(const float *__restrict__ f, double *__restrict__ u,
                                                   M *__restrict__ gx, M *__restrict__ gy, S *__restrict__ px,
                                                   S *__restrict__ py, double *__restrict__ bands, int H, int W,
                                                   size_t n_all, int nbands, double dt,
                                                   unsigned int *__restrict__ nonfinite)
{
    __shared__ double sh[4];
    double bad = 0.0;
    const size_t plane = (size_t)H * (size_t)W;
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n_all; q += stride) {
        const int qq = (int)(q % plane);
        const int i = qq / W;
        const int j = qq - i * W;
        const float v = f[q];
        if (!isfinite(v))
            bad += 1.0;
        u[q] = (double)v;
        gx[q] = (j < W - 1) ? (M)(((double)f[q + 1] - (double)v) / dt) : M(0);
        gy[q] = (i < H - 1) ? (M)(((double)f[q + W] - (double)v) / dt) : M(0);
        px[q] = S(0);
        py[q] = S(0);
        for (int k = 0; k < nbands; ++k)
            bands[(size_t)k * n_all + q] = 0.0;
    }
    bad = block_sum256(bad, sh);
    if (threadIdx.x == 0 && bad > 0.0)
        atomicAdd(nonfinite, (unsigned int)bad);
}

// Temporally blocked Chambolle iterations.
//
// Chambolle's step needs a = grad(div p - g/dt).  It is evaluated as
//     a = grad(div p) - G,   G = grad(g)/dt,
// with G formed in float64 from the float64 flow state and stored in type M.
// This is the same quantity; the order matters in float32: g/dt is large
// (|g| <= 1, dt ~ 1e-3) and differencing two rounded values of it would bury
// the small gradients of flat regions, whereas G carries only the relative
// rounding of the gradient itself.
//
// Grid: (number of BX x BY output tiles, C); 1024 threads, so that every
// SIMD of the CU has four waves to interleave (the per-pixel chain of LDS
// reads, square root and reciprocal is long and a tile holds few pixels).
// The workgroup stages the (BX+2TB) x (BY+2TB) region around its tile: the
// dual field and G of every region pixel live in registers of the thread
// that owns the pixel for all `iters` iterations; LDS only carries the
// values a neighbour needs (px of the left pixel and py of the upper one for
// div p, div p of the right and lower pixels for its gradient).  The LDS
// planes carry a one-pixel ring that is never written, so neighbour reads
// need no tests.  One iteration on every region pixel:
//     d   = (px - px_left) + (py - py_up)                      (div p)
//     a   = ((d_right - d) - Gx, (d_down - d) - Gy), zero on the last
//           column / row and outside the image
//     p  <- (p + tau a) / (1 + tau |a|)
// Pixels outside the image start with p = 0 and a = 0, so they keep p = 0;
// that realises the Neumann divergence (p_x = 0 on the last column and
// p_y = 0 on the last row is preserved by the update because a_x, a_y vanish
// there).  With zero_in set (first launch of a cold-started solve) the
// incoming dual field is taken as zero instead of being read.  A region
// pixel at distance e from the region edge is exact while the iteration
// count is <= e, so after iters <= TB iterations the BX x BY centre is exact
// and is written.
constexpr int kTileThreads = 1024;

template <typename S, typename M, int BX, int BY, int TB>
__global__ __launch_bounds__(kTileThreads) void k_chambolle_tile(
    const S *__restrict__ pxi, const S *__restrict__ pyi, const M *__restrict__ gxi, const M *__restrict__ gyi,
    S *__restrict__ pxo, S *__restrict__ pyo, int H, int W, int ntx, int ntiles, S tau, int iters, int zero_in)
{
    constexpr int RX = BX + 2 * TB;
    constexpr int RY = BY + 2 * TB;
    constexpr int RN = RX * RY;
    constexpr int LX = RX + 2;            // LDS row pitch: region + zero ring
    constexpr int LN = LX * (RY + 2);
    constexpr int PPT = (RN + kTileThreads - 1) / kTileThreads;
    __shared__ S s_px[LN];
    __shared__ S s_py[LN];
    __shared__ S s_d[LN];

    const size_t plane = (size_t)H * (size_t)W;
    const size_t coff = (size_t)blockIdx.y * plane;
    pxi += coff;
    pyi += coff;
    gxi += coff;
    gyi += coff;
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

    // zero ring (read by the outermost region pixels only)
    for (int e = threadIdx.x; e < 2 * LX + 2 * RY; e += kTileThreads) {
        int li;
        if (e < LX)
            li = e;                              // top row
        else if (e < 2 * LX)
            li = (RY + 1) * LX + (e - LX);       // bottom row
        else if (e < 2 * LX + RY)
            li = (e - 2 * LX + 1) * LX;          // left column
        else
            li = (e - 2 * LX - RY + 1) * LX + LX - 1; // right column
        s_px[li] = S(0);
        s_py[li] = S(0);
        s_d[li] = S(0);
    }

    S px[PPT], py[PPT], d[PPT], gx[PPT], gy[PPT];
    int li[PPT];     // LDS index of the pixel
    S mx[PPT];       // 1 where a_x is live (inside the image, not its last column), else 0
    S my[PPT];       // 1 where a_y is live (inside the image, not its last row), else 0
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * kTileThreads;
        S vx = S(0), vy = S(0);
        M vgx = M(0), vgy = M(0);
        bool ax_live = false, ay_live = false;
        int l = 0;
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            l = (ri + 1) * LX + (rj + 1);
            if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                if (!zero_in) {
                    vx = pxi[q];
                    vy = pyi[q];
                }
                vgx = gxi[q];
                vgy = gyi[q];
                ax_live = gj < W - 1;
                ay_live = gi < H - 1;
            }
            s_px[l] = vx;
            s_py[l] = vy;
        }
        li[m] = l;
        px[m] = vx;
        py[m] = vy;
        gx[m] = (S)vgx;
        gy[m] = (S)vgy;
        d[m] = S(0);
        mx[m] = ax_live ? S(1) : S(0);
        my[m] = ay_live ? S(1) : S(0);
    }
    __syncthreads();

    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (m < PPT - 1 || threadIdx.x + m * kTileThreads < RN) {
                const int l = li[m];
                const S dv = (px[m] - s_px[l - 1]) + (py[m] - s_py[l - LX]);
                d[m] = dv;
                s_d[l] = dv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (m < PPT - 1 || threadIdx.x + m * kTileThreads < RN) {
                const int l = li[m];
                // unconditional LDS reads; the boundary masks multiply (a
                // select around the reads compiles to branches that expose
                // the LDS latency of every pixel)
                const S dr = s_d[l + 1];
                const S dd = s_d[l + LX];
                const S ax = ((dr - d[m]) - gx[m]) * mx[m];
                const S ay = ((dd - d[m]) - gy[m]) * my[m];
                chambolle_update<S, M>(px[m], py[m], ax, ay, tau);
                s_px[l] = px[m];
                s_py[l] = py[m];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * kTileThreads;
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            if (ri >= TB && ri < TB + BY && rj >= TB && rj < TB + BX && gi < H && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                pxo[q] = px[m];
                pyo[q] = py[m];
            }
        }
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

// Outer step s of the flow, fused with the spectral transform.
// Grid: (nblk, C), nblk fixed per image size so partial sums are reproducible.
//   D_s     = dt div p                     (u_s - u_{s+1})
//   u_{s+1} = u_s - D_s                    (written to the other u buffer)
//   s >= 1: phi_s dt = s (D_{s-1} - D_s)   added to the band holding s
//           spart  <- block sum of |D_{s-1} - D_s|   (S(t_s) = s/dt * total)
//   s == K: residual = u_K + K D_K          (u(T) - T u_t(T), forward u_t)
//   G       = grad(u_{s+1}) / dt           (data term of the next solve; the
//             right and lower neighbours' u_{s+1} are recomputed here with
//             the same operations their own threads use, so they match bit
//             for bit)
template <typename S, typename M>
__global__ __launch_bounds__(kThreads) void k_flow_step(const S *__restrict__ px, const S *__restrict__ py,
                                                        const double *__restrict__ uin, double *__restrict__ uout,
                                                        double *__restrict__ dprev, M *__restrict__ gx,
                                                        M *__restrict__ gy, double *__restrict__ band,
                                                        double *__restrict__ resid, double *__restrict__ spart,
                                                        int H, int W, int C, int k, int K, double dt)
{
    __shared__ double sh[4];
    const int c = blockIdx.y;
    const int plane = H * W;
    const size_t coff = (size_t)c * (size_t)plane;
    px += coff;
    py += coff;
    uin += coff;
    uout += coff;
    dprev += coff;
    gx += coff;
    gy += coff;
    const double kd = (double)k;
    double acc = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        const int i = q / W;
        const int j = q - i * W;
        const double D = dt * div_p(px, py, q, i, j, W);
        const double uo = uin[q];
        const double un = uo - D;
        if (k >= 1) {
            const double dl = dprev[q] - D;
            band[coff + q] += kd * dl;
            acc += fabs(dl);
        }
        if (k == K)
            resid[coff + q] = uo + (double)K * D;
        uout[q] = un;
        dprev[q] = D;
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

// S[c][k-1] = k/dt * (sum of the step partials of sample k, channel c):
// one block per (k, c), each thread summing a fixed stride of partials,
// then the block sum in a fixed order.
__global__ __launch_bounds__(kThreads) void k_reduce_s(const double *__restrict__ spart, int C, int K, int nblk,
                                                       double dt, double *__restrict__ S)
{
    __shared__ double sh[4];
    const int t = blockIdx.x;            // (k-1) * C + c
    const int k = t / C + 1;
    const int c = t - (k - 1) * C;
    const double *p = spart + (size_t)t * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
        s += p[b];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0)
        S[(size_t)c * K + (k - 1)] = s * ((double)k / dt);
}

// One block: the report from the check partials (fixed reduction order).
__global__ __launch_bounds__(kThreads) void k_report(const double *__restrict__ rpart, int C, int nblk_chk,
                                                     int plane, double *__restrict__ stats,
                                                     unsigned int *__restrict__ nonfinite)
{
    __shared__ double sh[4];
    double emax = 0.0, drift = 0.0;
    for (int c = 0; c < C; ++c) {
        double e = 0.0, su = 0.0, sf = 0.0;
        for (int b = threadIdx.x; b < nblk_chk; b += kThreads) {
            const double *o = rpart + ((size_t)c * nblk_chk + b) * 3;
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

template <typename S, typename M>
using TileKernel = void (*)(const S *, const S *, const M *, const M *, S *, S *, int, int, int, int, S, int, int);

// Largest temporal blocking factor compiled for a mode (LDS and registers of
// the (32+2TB)^2 region, which are sized by the dual-field type S).
template <typename S> constexpr int max_tb() { return std::is_same<S, float>::value ? 16 : 8; }

// Smallest compiled halo width >= t.
template <typename S, typename M> TileKernel<S, M> tile_kernel(int t, int *tb)
{
    if (t <= 1) { *tb = 1; return k_chambolle_tile<S, M, kTileX, kTileY, 1>; }
    if (t <= 2) { *tb = 2; return k_chambolle_tile<S, M, kTileX, kTileY, 2>; }
    if (t <= 4) { *tb = 4; return k_chambolle_tile<S, M, kTileX, kTileY, 4>; }
    if constexpr (max_tb<S>() >= 16) {
        if (t > 8) { *tb = 16; return k_chambolle_tile<S, M, kTileX, kTileY, 16>; }
    }
    *tb = 8;
    return k_chambolle_tile<S, M, kTileX, kTileY, 8>;
}

// ---------------------------------------------------------------------------
// device scratch, cached per (device, precision mode) and grown on demand

struct Scratch {
    size_t n_all = 0;                  // C*H*W the plane buffers hold
    size_t spart_n = 0;                // doubles in spart
    size_t rpart_n = 0;                // doubles in rpart
    void *pa[2] = {nullptr, nullptr};  // dual field buffer A: px, py (type S)
    void *pb[2] = {nullptr, nullptr};  // dual field buffer B: px, py (type S)
    void *g[2] = {nullptr, nullptr};   // G = grad(g)/dt: x and y planes (type M)
    double *u[2] = {nullptr, nullptr}; // flow state, double-buffered per step
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
constexpr int kModes = 3;
std::mutex g_mu;
Scratch g_scratch[kMaxDevices][kModes];
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

template <typename T> void free_typed(T *&p)
{
    void *v = p;
    free_ptr(v);
    p = nullptr;
}

void free_scratch(Scratch &s)
{
    for (int i = 0; i < 2; ++i) {
        free_ptr(s.pa[i]);
        free_ptr(s.pb[i]);
        free_ptr(s.g[i]);
        free_typed(s.u[i]);
    }
    free_typed(s.dprev);
    free_typed(s.spart);
    free_typed(s.rpart);
    free_typed(s.nonfinite);
    s.n_all = s.spart_n = s.rpart_n = 0;
}

void free_stage(HostStage &h)
{
    free_typed(h.f);
    free_typed(h.bands);
    free_typed(h.S);
    free_typed(h.res);
    free_typed(h.stats);
    h.f_n = h.bands_n = h.s_n = h.r_n = 0;
}

int ensure_scratch(Scratch &s, size_t elem_s, size_t elem_m, size_t n_all, size_t spart_n, size_t rpart_n)
{
    if (s.n_all >= n_all && s.spart_n >= spart_n && s.rpart_n >= rpart_n && s.u[0])
        return TVSPEC_OK;
    // buffers may still be in use by earlier enqueued work
    HIP_TRY(hipDeviceSynchronize());
    free_scratch(s);
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipMalloc(&s.pa[i], n_all * elem_s));
        HIP_TRY(hipMalloc(&s.pb[i], n_all * elem_s));
        HIP_TRY(hipMalloc(&s.g[i], n_all * elem_m));
        HIP_TRY(hipMalloc((void **)&s.u[i], n_all * sizeof(double)));
    }
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
    if (precision != TVSPEC_PRECISION_F32 && precision != TVSPEC_PRECISION_F64 &&
        precision != TVSPEC_PRECISION_MIXED)
        return fail(TVSPEC_EINVAL, "precision must be TVSPEC_PRECISION_F32, _F64 or _MIXED");
    const int maxt = precision == TVSPEC_PRECISION_F32 ? max_tb<float>() : max_tb<double>();
    if (ipl < 0 || ipl > maxt)
        return fail(TVSPEC_EINVAL, "iters_per_launch out of range");
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// the decomposition, enqueued on a stream

template <typename S, typename M>
int enqueue(const float *f, int H, int W, int C, double dt, int K, int iters, const int *edges, int nb,
            double *bands, double *Sout, double *res, double *stats, double tau, int warm, int ipl,
            hipStream_t st, Scratch &sc)
{
    const int plane = H * W;
    const size_t n_all = (size_t)plane * (size_t)C;
    const int nblk = plane_blocks(plane);
    const size_t spart_n = (size_t)K * C * nblk;
    const size_t rpart_n = (size_t)C * nblk * 3;
    int rc = ensure_scratch(sc, sizeof(S), sizeof(M), n_all, spart_n, rpart_n);
    if (rc != TVSPEC_OK)
        return rc;

    S *pbuf[2][2] = {{(S *)sc.pa[0], (S *)sc.pa[1]}, {(S *)sc.pb[0], (S *)sc.pb[1]}};
    M *gx = (M *)sc.g[0];
    M *gy = (M *)sc.g[1];

    int tb = 0;
    const int want = ipl > 0 ? ipl : 8;
    TileKernel<S, M> kt = tile_kernel<S, M>(want, &tb);
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
    hipLaunchKernelGGL((k_init<S, M>), dim3(gblk), dim3(kThreads), 0, st, f, sc.u[0], gx, gy, pbuf[0][0],
                       pbuf[0][1], bands, H, W, n_all, nb, dt, sc.nonfinite);
    HIP_TRY(hipGetLastError());

    int cur = 0;  // dual field buffer holding the current iterate
    int ucur = 0; // u buffer holding u_s
    for (int s = 0; s <= K; ++s) {
        // timing: one event pair around the back-to-back Chambolle launches
        // of this solve (events between launches would perturb them)
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (g_timing.on) {
            if ((rc = timing_pair(&e0, &e1)) != TVSPEC_OK)
                return rc;
            HIP_TRY(hipEventRecord(e0, st));
        }
        for (int done = 0; done < iters;) {
            // cold start: the first launch of a solve starts from p = 0
            const int zero_in = (!warm && done == 0) ? 1 : 0;
            const int it = (iters - done) < per_launch ? (iters - done) : per_launch;
            hipLaunchKernelGGL(kt, dim3(ntiles, C), dim3(kTileThreads), 0, st, pbuf[cur][0], pbuf[cur][1], gx, gy,
                               pbuf[1 - cur][0], pbuf[1 - cur][1], H, W, ntx, ntiles, (S)tau, it, zero_in);
            if (g_timing.on) {
                ++g_timing.launches;
                g_timing.pixel_iters += (long long)n_all * it;
            }
            cur = 1 - cur;
            done += it;
        }
        if (g_timing.on)
            HIP_TRY(hipEventRecord(e1, st));
        double *band = s >= 1 ? bands + (size_t)band_of[s] * n_all : nullptr;
        hipLaunchKernelGGL((k_flow_step<S, M>), dim3(nblk, C), dim3(kThreads), 0, st, pbuf[cur][0], pbuf[cur][1],
                           sc.u[ucur], sc.u[1 - ucur], sc.dprev, gx, gy, band, res, sc.spart, H, W, C, s, K, dt);
        ucur = 1 - ucur;
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_check, dim3(nblk, C), dim3(kThreads), 0, st, f, bands, res, sc.u[ucur], plane, C, nb,
                       sc.rpart);
    hipLaunchKernelGGL(k_reduce_s, dim3(K * C), dim3(kThreads), 0, st, sc.spart, C, K, nblk, dt, Sout);
    hipLaunchKernelGGL(k_report, dim3(1), dim3(kThreads), 0, st, sc.rpart, C, nblk, plane, stats, sc.nonfinite);
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
    Scratch &sc = g_scratch[dev][precision];
    switch (precision) {
    case TVSPEC_PRECISION_F32:
        return enqueue<float, float>(f, H, W, C, dt, K, iters, edges, nb, bands, S, res, stats, tau, warm, ipl, st,
                                     sc);
    case TVSPEC_PRECISION_F64:
        return enqueue<double, double>(f, H, W, C, dt, K, iters, edges, nb, bands, S, res, stats, tau, warm, ipl, st,
                                       sc);
    default:
        return enqueue<double, float>(f, H, W, C, dt, K, iters, edges, nb, bands, S, res, stats, tau, warm, ipl, st,
                                      sc);
    }
}

template <typename T> int grow(T *&p, size_t &cap, size_t n)
{
    if (cap >= n && p)
        return TVSPEC_OK;
    free_typed(p);
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
                             TVSPEC_DEFAULT_TAU, 0, TVSPEC_DEFAULT_PRECISION, 0, h.stream);
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
        bool any = g_stage[d].stream || g_stage[d].f;
        for (int m = 0; m < kModes; ++m)
            any = any || g_scratch[d][m].u[0];
        if (!any)
            continue;
        if (hipSetDevice(d) != hipSuccess)
            continue;
        (void)hipDeviceSynchronize();
        for (int m = 0; m < kModes; ++m)
            free_scratch(g_scratch[d][m]);
        free_stage(g_stage[d]);
        if (g_stage[d].stream) {
            (void)hipStreamDestroy(g_stage[d].stream);
            g_stage[d].stream = nullptr;
        }
    }
    (void)hipSetDevice(cur);
}
