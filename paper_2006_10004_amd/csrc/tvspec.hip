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

// Per-image parameters of a batch (device copy of the descriptor table).
struct ImageDesc {
    double dt;          // time step
    int K;              // spectral samples (K+1 ROF solves)
    int nbands;         // bands
    long long band_off; // element offset of the image's bands [nbands][C][H][W]
    long long s_off;    // element offset of the image's S [C][K]
    long long row_off;  // offset of the image's band-index row (K+1 ints)
};

// Zero a float64 buffer (the bands of every image of a batch).
__global__ __launch_bounds__(kThreads) void k_fill0(double *__restrict__ a, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += stride)
        a[q] = 0.0;
}

// u = f, G = grad f / dt (data term of the first solve), p = 0 (buffer A),
// every image active; counts non-finite inputs per image.  The buffers hold
// the B*C channel planes of the batch back to back.
template <typename S, typename M>
__global__ __launch_bounds__(kThreads) void k_init(const float *__restrict__ f, double *__restrict__ u,
                                                   M *__restrict__ gx, M *__restrict__ gy, S *__restrict__ px,
                                                   S *__restrict__ py, int H, int W, int C, size_t n_all,
                                                   const ImageDesc *__restrict__ desc,
                                                   unsigned int *__restrict__ nonfinite, int *__restrict__ active)
{
    const size_t plane = (size_t)H * (size_t)W;
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t q = (size_t)blockIdx.x * kThreads + threadIdx.x; q < n_all; q += stride) {
        const size_t ch = q / plane;
        const int qq = (int)(q - ch * plane);
        const int img = (int)(ch / (size_t)C);
        const int i = qq / W;
        const int j = qq - i * W;
        const double dt = desc[img].dt;
        const float v = f[q];
        if (!isfinite(v))
            atomicAdd(&nonfinite[img], 1u);
        if (qq == 0 && ch == (size_t)img * C)
            active[img] = 1;
        u[q] = (double)v;
        gx[q] = (j < W - 1) ? (M)(((double)f[q + 1] - (double)v) / dt) : M(0);
        gy[q] = (i < H - 1) ? (M)(((double)f[q + W] - (double)v) / dt) : M(0);
        px[q] = S(0);
        py[q] = S(0);
    }
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
// Grid: (number of BX x BY output tiles, B*C); 1024 threads, so that every
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
// incoming dual field is taken as zero instead of being read.  Channel planes
// of images whose flow is complete (active flag 0) are skipped.  A region
// pixel at distance e from the region edge is exact while the iteration
// count is <= e, so after iters <= TB iterations the BX x BY centre is exact
// and is written.
constexpr int kTileThreads = 1024;

template <typename S, typename M, int BX, int BY, int TB>
__global__ __launch_bounds__(kTileThreads) void k_chambolle_tile(
    const S *__restrict__ pxi, const S *__restrict__ pyi, const M *__restrict__ gxi, const M *__restrict__ gyi,
    S *__restrict__ pxo, S *__restrict__ pyo, int H, int W, int ntx, int ntiles, S tau, int iters, int zero_in,
    const int *__restrict__ active, int C)
{
    if (!active[blockIdx.y / C])
        return;
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
// Grid: (nblk, B*C), nblk fixed per image size so partial sums are
// reproducible; channel plane y belongs to image y / C.  Per image:
//   s > K:  nothing (the image's flow is complete)
//   D_s     = dt div p                     (u_s - u_{s+1})
//   u_{s+1} = u_s - D_s                    (written to the other u buffer)
//   s >= 1: phi_s dt = s (D_{s-1} - D_s)   added to the band holding s
//           spart  <- block sum of |D_{s-1} - D_s|   (S(t_s) = s/dt * total)
//   s == K: residual = u_K + K D_K          (u(T) - T u_t(T), forward u_t),
//           and the image is marked complete for the tile kernel
//   G       = grad(u_{s+1}) / dt           (data term of the next solve; the
//             right and lower neighbours' u_{s+1} are recomputed here with
//             the same operations their own threads use, so they match bit
//             for bit)
template <typename S, typename M>
__global__ __launch_bounds__(kThreads) void k_flow_step(const S *__restrict__ px, const S *__restrict__ py,
                                                        const double *__restrict__ uin, double *__restrict__ uout,
                                                        double *__restrict__ dprev, M *__restrict__ gx,
                                                        M *__restrict__ gy, double *__restrict__ bands,
                                                        double *__restrict__ resid, double *__restrict__ spart,
                                                        const ImageDesc *__restrict__ desc,
                                                        const int *__restrict__ band_rows, int *__restrict__ active,
                                                        int H, int W, int C, int BC, int k)
{
    __shared__ double sh[4];
    const int y = blockIdx.y;
    const int img = y / C;
    const int c = y - img * C;
    const ImageDesc dsc = desc[img];
    if (k > dsc.K)
        return;
    const double dt = dsc.dt;
    const int K = dsc.K;
    const int plane = H * W;
    const size_t coff = (size_t)y * (size_t)plane;
    px += coff;
    py += coff;
    uin += coff;
    uout += coff;
    dprev += coff;
    gx += coff;
    gy += coff;
    resid += coff;
    double *band = nullptr;
    if (k >= 1)
        band = bands + dsc.band_off + ((size_t)band_rows[dsc.row_off + k] * C + c) * (size_t)plane;
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
            band[q] += kd * dl;
            acc += fabs(dl);
        }
        if (k == K)
            resid[q] = uo + (double)K * D;
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
            spart[((size_t)(k - 1) * BC + y) * gridDim.x + blockIdx.x] = acc;
    }
    if (k == K && c == 0 && blockIdx.x == 0 && threadIdx.x == 0)
        active[img] = 0;
}

// Per-block partials of: max |f - sum_j b_j - r|, sum u_{K+1}, sum f.
// Grid: (nblk, B*C).
// u_{K+1} of an image is in u0 or u1 by the parity of K + 1 (step s writes
// u_{s+1} to buffer (s + 1) mod 2, and steps after the image's K are skipped).
__global__ __launch_bounds__(kThreads) void k_check(const float *__restrict__ f, const double *__restrict__ bands,
                                                    const double *__restrict__ resid, const double *__restrict__ u0,
                                                    const double *__restrict__ u1,
                                                    const ImageDesc *__restrict__ desc, int plane, int C,
                                                    double *__restrict__ rpart)
{
    __shared__ double sh[4];
    const int y = blockIdx.y;
    const int img = y / C;
    const int c = y - img * C;
    const ImageDesc dsc = desc[img];
    const double *u = ((dsc.K + 1) & 1) ? u1 : u0;
    const size_t coff = (size_t)y * (size_t)plane;
    const double *b0 = bands + dsc.band_off + (size_t)c * plane;
    const size_t bstride = (size_t)C * (size_t)plane;
    double emax = 0.0, su = 0.0, sf = 0.0;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < plane; q += gridDim.x * kThreads) {
        double acc = 0.0;
        for (int j = 0; j < dsc.nbands; ++j)
            acc += b0[(size_t)j * bstride + q];
        const double fv = (double)f[coff + q];
        emax = fmax(emax, fabs(fv - acc - resid[coff + q]));
        su += u[coff + q];
        sf += fv;
    }
    emax = block_max256(emax, sh);
    su = block_sum256(su, sh);
    sf = block_sum256(sf, sh);
    if (threadIdx.x == 0) {
        double *o = rpart + ((size_t)y * gridDim.x + blockIdx.x) * 3;
        o[0] = emax;
        o[1] = su;
        o[2] = sf;
    }
}

// S of image b, channel c, sample k: k/dt * (sum of the step partials),
// one block per (k, channel plane), each thread summing a fixed stride of
// partials, then the block sum in a fixed order.  Grid: (Kmax, B*C).
__global__ __launch_bounds__(kThreads) void k_reduce_s(const double *__restrict__ spart,
                                                       const ImageDesc *__restrict__ desc, int C, int BC, int nblk,
                                                       double *__restrict__ S)
{
    __shared__ double sh[4];
    const int k = blockIdx.x + 1;
    const int y = blockIdx.y;
    const int img = y / C;
    const int c = y - img * C;
    const ImageDesc dsc = desc[img];
    if (k > dsc.K)
        return;
    const double *p = spart + ((size_t)(k - 1) * BC + y) * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads)
        s += p[b];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0)
        S[dsc.s_off + (size_t)c * dsc.K + (k - 1)] = s * ((double)k / dsc.dt);
}

// The report of image blockIdx.x from the check partials (fixed reduction
// order); clears the image's non-finite counter.
__global__ __launch_bounds__(kThreads) void k_report(const double *__restrict__ rpart, int C, int nblk_chk,
                                                     int plane, double *__restrict__ stats,
                                                     unsigned int *__restrict__ nonfinite)
{
    __shared__ double sh[4];
    const int img = blockIdx.x;
    double emax = 0.0, drift = 0.0;
    for (int c = 0; c < C; ++c) {
        const int y = img * C + c;
        double e = 0.0, su = 0.0, sf = 0.0;
        for (int b = threadIdx.x; b < nblk_chk; b += kThreads) {
            const double *o = rpart + ((size_t)y * nblk_chk + b) * 3;
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
        double *st = stats + (size_t)img * TVSPEC_NSTATS;
        st[0] = emax;
        st[1] = drift;
        st[2] = (double)nonfinite[img];
        st[3] = 0.0;
        nonfinite[img] = 0u;
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
using TileKernel = void (*)(const S *, const S *, const M *, const M *, S *, S *, int, int, int, int, S, int, int,
                            const int *, int);

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
    size_t n_all = 0;                  // B*C*H*W the plane buffers hold
    size_t spart_n = 0;                // doubles in spart
    size_t rpart_n = 0;                // doubles in rpart
    size_t nimg = 0;                   // images the per-image buffers hold
    size_t rows_n = 0;                 // ints in band_rows
    void *pa[2] = {nullptr, nullptr};  // dual field buffer A: px, py (type S)
    void *pb[2] = {nullptr, nullptr};  // dual field buffer B: px, py (type S)
    void *g[2] = {nullptr, nullptr};   // G = grad(g)/dt: x and y planes (type M)
    double *u[2] = {nullptr, nullptr}; // flow state, double-buffered per step
    double *dprev = nullptr;
    double *spart = nullptr;
    double *rpart = nullptr;
    ImageDesc *desc = nullptr;         // per image
    int *band_rows = nullptr;          // band index of every sample, per image
    int *active = nullptr;             // per image: flow not yet complete
    unsigned int *nonfinite = nullptr; // per image
};

// Pinned host staging of the descriptor table, and an event marking the
// upload that last read it (the next call waits for it before rewriting).
struct DescStage {
    size_t bytes = 0;
    char *host = nullptr;
    hipEvent_t uploaded = nullptr;
    bool pending = false;
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
DescStage g_desc_stage[kMaxDevices];
HostStage g_stage[kMaxDevices];

// Benchmark timing of the Chambolle kernel: one event pair per ROF solve.
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

// Event pair for the next solve (created on demand, recycled after a drain).
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
    free_typed(s.desc);
    free_typed(s.band_rows);
    free_typed(s.active);
    free_typed(s.nonfinite);
    s.n_all = s.spart_n = s.rpart_n = s.nimg = s.rows_n = 0;
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

void free_desc_stage(DescStage &d)
{
    if (d.pending && d.uploaded)
        (void)hipEventSynchronize(d.uploaded);
    if (d.host)
        (void)hipHostFree(d.host);
    if (d.uploaded)
        (void)hipEventDestroy(d.uploaded);
    d = DescStage();
}

int ensure_scratch(Scratch &s, size_t elem_s, size_t elem_m, size_t n_all, size_t spart_n, size_t rpart_n,
                   size_t nimg, size_t rows_n)
{
    if (s.n_all >= n_all && s.spart_n >= spart_n && s.rpart_n >= rpart_n && s.nimg >= nimg && s.rows_n >= rows_n &&
        s.u[0])
        return TVSPEC_OK;
    // buffers may still be in use by earlier enqueued work
    HIP_TRY(hipDeviceSynchronize());
    n_all = n_all > s.n_all ? n_all : s.n_all;
    spart_n = spart_n > s.spart_n ? spart_n : s.spart_n;
    rpart_n = rpart_n > s.rpart_n ? rpart_n : s.rpart_n;
    nimg = nimg > s.nimg ? nimg : s.nimg;
    rows_n = rows_n > s.rows_n ? rows_n : s.rows_n;
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
    HIP_TRY(hipMalloc((void **)&s.desc, nimg * sizeof(ImageDesc)));
    HIP_TRY(hipMalloc((void **)&s.band_rows, rows_n * sizeof(int)));
    HIP_TRY(hipMalloc((void **)&s.active, nimg * sizeof(int)));
    HIP_TRY(hipMalloc((void **)&s.nonfinite, nimg * sizeof(unsigned int)));
    HIP_TRY(hipMemset(s.nonfinite, 0, nimg * sizeof(unsigned int)));
    HIP_TRY(hipDeviceSynchronize());
    s.n_all = n_all;
    s.spart_n = spart_n;
    s.rpart_n = rpart_n;
    s.nimg = nimg;
    s.rows_n = rows_n;
    return TVSPEC_OK;
}

// Copy the descriptor table and band rows to the device through the pinned
// staging buffer, ordered on stream st.
int upload_desc(int dev, const std::vector<ImageDesc> &desc, const std::vector<int> &rows, Scratch &sc,
                hipStream_t st)
{
    DescStage &d = g_desc_stage[dev];
    const size_t nd = desc.size() * sizeof(ImageDesc);
    const size_t nr = rows.size() * sizeof(int);
    if (d.pending) {
        HIP_TRY(hipEventSynchronize(d.uploaded));
        d.pending = false;
    }
    if (d.bytes < nd + nr) {
        if (d.host)
            HIP_TRY(hipHostFree(d.host));
        d.host = nullptr;
        d.bytes = 0;
        HIP_TRY(hipHostMalloc((void **)&d.host, nd + nr, hipHostMallocDefault));
        d.bytes = nd + nr;
    }
    if (!d.uploaded)
        HIP_TRY(hipEventCreateWithFlags(&d.uploaded, hipEventDisableTiming));
    std::memcpy(d.host, desc.data(), nd);
    std::memcpy(d.host + nd, rows.data(), nr);
    HIP_TRY(hipMemcpyAsync(sc.desc, d.host, nd, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sc.band_rows, d.host + nd, nr, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(d.uploaded, st));
    d.pending = true;
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// argument validation (host only, before any device call)

int validate_edges(const int *edges, int nb, int K)
{
    if (nb < 1 || nb > K)
        return fail(TVSPEC_EINVAL, "n_bands must be in [1, K]");
    if (edges[0] != 0 || edges[nb] != K)
        return fail(TVSPEC_EINVAL, "band edges must start at 0 and end at K");
    for (int j = 1; j <= nb; ++j)
        if (edges[j] <= edges[j - 1])
            return fail(TVSPEC_EINVAL, "band edges must be strictly increasing");
    return TVSPEC_OK;
}

int validate_shape(int B, int H, int W, int C, int iters)
{
    if (B < 1)
        return fail(TVSPEC_EINVAL, "B must be >= 1");
    if (H < 2 || W < 2)
        return fail(TVSPEC_EINVAL, "H and W must be >= 2");
    if (C < 1)
        return fail(TVSPEC_EINVAL, "C must be >= 1");
    if ((long long)B * C > 65535)
        return fail(TVSPEC_EINVAL, "B*C must be <= 65535");
    if ((long long)H * (long long)W > (1LL << 30))
        return fail(TVSPEC_EINVAL, "H*W must be <= 2^30");
    if ((long long)H * W * C * B > (1LL << 40))
        return fail(TVSPEC_EINVAL, "B*C*H*W too large");
    if (iters < 1)
        return fail(TVSPEC_EINVAL, "inner_iters must be >= 1");
    return TVSPEC_OK;
}

int validate_image(double dt, int K, const int *edges, int nb)
{
    if (!std::isfinite(dt) || !(dt > 0.0))
        return fail(TVSPEC_EINVAL, "dt must be finite and > 0");
    if (K < 1)
        return fail(TVSPEC_EINVAL, "K must be >= 1");
    return validate_edges(edges, nb, K);
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
// the decomposition of a batch of equal-size images, enqueued on a stream

struct Batch {
    const float *f;
    int B, H, W, C, iters;
    const double *dt;   // host [B]
    const int *K;       // host [B]
    const int *edges;   // host, concatenated n_bands[b]+1 entries per image
    const int *nb;      // host [B]
    double *bands, *S, *res, *stats;
    double tau;
    int warm, ipl;
    hipStream_t st;
};

template <typename S, typename M> int enqueue(int dev, const Batch &a, Scratch &sc)
{
    const int plane = a.H * a.W;
    const int BC = a.B * a.C;
    const size_t n_all = (size_t)plane * (size_t)BC;
    const int nblk = plane_blocks(plane);

    // descriptor table, band index rows, output offsets
    std::vector<ImageDesc> desc(a.B);
    std::vector<int> rows;
    int Kmax = 0;
    long long band_off = 0, s_off = 0;
    for (int b = 0, e0 = 0; b < a.B; ++b) {
        const int K = a.K[b], nb = a.nb[b];
        desc[b].dt = a.dt[b];
        desc[b].K = K;
        desc[b].nbands = nb;
        desc[b].band_off = band_off;
        desc[b].s_off = s_off;
        desc[b].row_off = (long long)rows.size();
        const int *e = a.edges + e0;
        rows.push_back(0); // sample 0 carries no phi
        for (int j = 0; j < nb; ++j)
            for (int k = e[j] + 1; k <= e[j + 1]; ++k)
                rows.push_back(j);
        band_off += (long long)nb * a.C * plane;
        s_off += (long long)a.C * K;
        e0 += nb + 1;
        Kmax = K > Kmax ? K : Kmax;
    }
    const size_t spart_n = (size_t)Kmax * BC * nblk;
    const size_t rpart_n = (size_t)BC * nblk * 3;
    int rc = ensure_scratch(sc, sizeof(S), sizeof(M), n_all, spart_n, rpart_n, (size_t)a.B, rows.size());
    if (rc != TVSPEC_OK)
        return rc;
    if ((rc = upload_desc(dev, desc, rows, sc, a.st)) != TVSPEC_OK)
        return rc;

    S *pbuf[2][2] = {{(S *)sc.pa[0], (S *)sc.pa[1]}, {(S *)sc.pb[0], (S *)sc.pb[1]}};
    M *gx = (M *)sc.g[0];
    M *gy = (M *)sc.g[1];

    int tb = 0;
    const int want = a.ipl > 0 ? a.ipl : 8;
    TileKernel<S, M> kt = tile_kernel<S, M>(want, &tb);
    const int ntx = (a.W + kTileX - 1) / kTileX;
    const int nty = (a.H + kTileY - 1) / kTileY;
    const int ntiles = ntx * nty;
    const int per_launch = a.ipl > 0 ? a.ipl : tb;

    hipLaunchKernelGGL(k_fill0, dim3(blocks_for((size_t)band_off, 4096)), dim3(kThreads), 0, a.st, a.bands,
                       (size_t)band_off);
    hipLaunchKernelGGL((k_init<S, M>), dim3(blocks_for(n_all, 4096)), dim3(kThreads), 0, a.st, a.f, sc.u[0], gx, gy,
                       pbuf[0][0], pbuf[0][1], a.H, a.W, a.C, n_all, sc.desc, sc.nonfinite, sc.active);
    HIP_TRY(hipGetLastError());

    int cur = 0;  // dual field buffer holding the current iterate
    int ucur = 0; // u buffer holding u_s (= s mod 2)
    for (int s = 0; s <= Kmax; ++s) {
        // timing: one event pair around the back-to-back Chambolle launches
        // of this solve (events between launches would perturb them)
        hipEvent_t e0 = nullptr, e1 = nullptr;
        long long live_planes = 0;
        if (g_timing.on) {
            for (int b = 0; b < a.B; ++b)
                live_planes += (s <= a.K[b]) ? a.C : 0;
            if ((rc = timing_pair(&e0, &e1)) != TVSPEC_OK)
                return rc;
            HIP_TRY(hipEventRecord(e0, a.st));
        }
        for (int done = 0; done < a.iters;) {
            // cold start: the first launch of a solve starts from p = 0
            const int zero_in = (!a.warm && done == 0) ? 1 : 0;
            const int it = (a.iters - done) < per_launch ? (a.iters - done) : per_launch;
            hipLaunchKernelGGL(kt, dim3(ntiles, BC), dim3(kTileThreads), 0, a.st, pbuf[cur][0], pbuf[cur][1], gx, gy,
                               pbuf[1 - cur][0], pbuf[1 - cur][1], a.H, a.W, ntx, ntiles, (S)a.tau, it, zero_in,
                               sc.active, a.C);
            if (g_timing.on) {
                ++g_timing.launches;
                g_timing.pixel_iters += live_planes * plane * it;
            }
            cur = 1 - cur;
            done += it;
        }
        if (g_timing.on)
            HIP_TRY(hipEventRecord(e1, a.st));
        hipLaunchKernelGGL((k_flow_step<S, M>), dim3(nblk, BC), dim3(kThreads), 0, a.st, pbuf[cur][0], pbuf[cur][1],
                           sc.u[ucur], sc.u[1 - ucur], sc.dprev, gx, gy, a.bands, a.res, sc.spart, sc.desc,
                           sc.band_rows, sc.active, a.H, a.W, a.C, BC, s);
        ucur = 1 - ucur;
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_check, dim3(nblk, BC), dim3(kThreads), 0, a.st, a.f, a.bands, a.res, sc.u[0], sc.u[1],
                       sc.desc, plane, a.C, sc.rpart);
    hipLaunchKernelGGL(k_reduce_s, dim3(Kmax, BC), dim3(kThreads), 0, a.st, sc.spart, sc.desc, a.C, BC, nblk, a.S);
    hipLaunchKernelGGL(k_report, dim3(a.B), dim3(kThreads), 0, a.st, sc.rpart, a.C, nblk, plane, a.stats,
                       sc.nonfinite);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int decompose_on_device(const Batch &a, int precision)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TVSPEC_EDEVICE, "device index out of range");
    Scratch &sc = g_scratch[dev][precision];
    switch (precision) {
    case TVSPEC_PRECISION_F32:
        return enqueue<float, float>(dev, a, sc);
    case TVSPEC_PRECISION_F64:
        return enqueue<double, double>(dev, a, sc);
    default:
        return enqueue<double, float>(dev, a, sc);
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

extern "C" int tvspec_decompose_batch_dev(const float *f, int B, int H, int W, int C, int inner_iters,
                                          const double *dt, const int *K, const int *band_edges, const int *n_bands,
                                          double *bands, double *S, double *residual, double *stats, double tau,
                                          int warm_start, int precision, int iters_per_launch, void *stream)
{
    g_last_error.clear();
    if (!f || !dt || !K || !band_edges || !n_bands || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    int rc = validate_shape(B, H, W, C, inner_iters);
    if (rc != TVSPEC_OK)
        return rc;
    for (int b = 0, e0 = 0; b < B; ++b) {
        if (n_bands[b] < 1 || n_bands[b] > K[b] || K[b] < 1)
            return fail(TVSPEC_EINVAL, "image " + std::to_string(b) + ": need K >= 1 and 1 <= n_bands <= K");
        if ((rc = validate_image(dt[b], K[b], band_edges + e0, n_bands[b])) != TVSPEC_OK)
            return fail(rc, "image " + std::to_string(b) + ": " + g_last_error);
        e0 += n_bands[b] + 1;
    }
    rc = validate_opts(tau, warm_start, precision, iters_per_launch);
    if (rc != TVSPEC_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Batch a{f, B, H, W, C, inner_iters, dt, K, band_edges, n_bands, bands, S, residual, stats, tau, warm_start,
            iters_per_launch, (hipStream_t)stream};
    return decompose_on_device(a, precision);
}

extern "C" int tvspec_decompose_dev(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                    const int *band_edges, int n_bands, double *bands, double *S, double *residual,
                                    double *stats, double tau, int warm_start, int precision, int iters_per_launch,
                                    void *stream)
{
    g_last_error.clear();
    if (!f || !band_edges || !bands || !S || !residual || !stats)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    int rc = validate_shape(1, H, W, C, inner_iters);
    if (rc != TVSPEC_OK)
        return rc;
    if ((rc = validate_image(dt, K, band_edges, n_bands)) != TVSPEC_OK)
        return rc;
    rc = validate_opts(tau, warm_start, precision, iters_per_launch);
    if (rc != TVSPEC_OK)
        return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Batch a{f, 1, H, W, C, inner_iters, &dt, &K, band_edges, &n_bands, bands, S, residual, stats, tau, warm_start,
            iters_per_launch, (hipStream_t)stream};
    return decompose_on_device(a, precision);
}

extern "C" int tvspec_decompose(const float *f, int H, int W, int C, double dt, int K, int inner_iters,
                                const int *band_edges, int n_bands, double *bands, double *S, double *residual)
{
    g_last_error.clear();
    if (!f || !band_edges || !bands || !S || !residual)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    int rc = validate_shape(1, H, W, C, inner_iters);
    if (rc != TVSPEC_OK)
        return rc;
    if ((rc = validate_image(dt, K, band_edges, n_bands)) != TVSPEC_OK)
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
    Batch a{h.f, 1, H, W, C, inner_iters, &dt, &K, band_edges, &n_bands, h.bands, h.S, h.res, h.stats,
            TVSPEC_DEFAULT_TAU, 0, 0, h.stream};
    rc = decompose_on_device(a, TVSPEC_DEFAULT_PRECISION);
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
        bool any = g_stage[d].stream || g_stage[d].f || g_desc_stage[d].host;
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
        free_desc_stage(g_desc_stage[d]);
        if (g_stage[d].stream) {
            (void)hipStreamDestroy(g_stage[d].stream);
            g_stage[d].stream = nullptr;
        }
    }
    (void)hipSetDevice(cur);
}
