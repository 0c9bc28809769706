// Tile kernels of the inner ROF solvers and the per-pixel arithmetic they
// share: Chambolle's dual fixed point (k_chambolle_tile) and the
// Chambolle-Pock primal-dual iteration (k_pdhg_tile), temporally blocked on
// LDS-staged 32 x 32 tiles.  Included by engine.hip inside
// namespace tvspec { namespace { ... } } (kept in a file of their own: the
// HBM counter records of the benchmark are tied to this file's text).
#ifndef TVSPEC_TILE_KERNELS_H
#define TVSPEC_TILE_KERNELS_H

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
        // float64 update with |a| and the reciprocal from the float32
        // hardware estimates (v_rsq_f32, v_rcp_f32), each refined by one
        // float64 Newton step (relative error ~1e-14; the float64 square
        // root and division sequences cost several times more):
        //     y ~ 1/sqrt(x),  s = x y,  |a| = s + s (1 - s y) / 2
        //     r ~ 1/den,      r' = r + r (1 - den r)
        // The estimate's argument is clamped to 1e-30 so that it stays a
        // normal float32; below that |a| comes out as ~1.5e15 x <= 1.5e-15
        // instead of sqrt(x) <= 1e-15, which moves 1 + tau |a| by less
        // than its rounding.
        const S x = ax * ax + ay * ay;
        const S y = (S)__builtin_amdgcn_rsqf(fmaxf((float)x, 1e-30f));
        const S sx = x * y;
        const S nrm = __builtin_fma(sx, __builtin_fma(-sx, S(0.5) * y, S(0.5)), sx);
        const S den = __builtin_fma(tau, nrm, S(1));
        const S r0 = (S)__builtin_amdgcn_rcpf((float)den);
        const S r = __builtin_fma(r0, __builtin_fma(-den, r0, S(1)), r0);
        px = __builtin_fma(tau, ax, px) * r;
        py = __builtin_fma(tau, ay, py) * r;
    }
}

// Temporally blocked Chambolle iterations.
//
// Chambolle's step needs a = grad w with w = div p - g/dt, g = u_k the data
// of the slot's current solve.  The float64 modes (S = double) form exactly
// that: w = div p - u_k/dt per pixel (u_k read once per launch from the
// float64 flow state; MIXED multiplies by the rounded 1/dt, F64 divides),
// then a = (w_right - w, w_down - w).  w is ~u/dt (up to ~1e3), and its
// float64 rounding (~1e-13) is far below what the bands see.  In float32
// (S = float) that rounding would bury the small gradients of flat regions,
// so F32 keeps the gradient form a = grad(div p) - G with G = grad(g)/dt
// formed in float64 once per solve and stored as float32: the same
// quantity, carrying only G's relative rounding.
//
// Grid: (number of BX x BY output tiles, slots * C); NT threads (1024 by
// default, so that every SIMD of the CU has four waves to interleave: the
// per-pixel chain of LDS reads, square root and reciprocal is long and a tile
// holds few pixels).  The workgroup stages the (BX+2TB) x (BY+2TB) region
// around its tile: the dual field and the data term of every region pixel
// live in registers of the thread that owns the pixel for all `iters`
// iterations; LDS only carries the values a neighbour needs.  The LDS planes
// carry a one-pixel ring that is never written, so neighbour reads need no
// tests.  One iteration on every region pixel, two barriers:
//     d   = (px - px_left) + (py - py_up)                      (div p)
//     w   = d - u_k/dt                                         (float64 modes)
//     a   = (w_right - w, w_down - w)  or  ((d_right - d) - Gx, (d_down - d) - Gy),
//           zero on the last column / row and outside the image
//     p  <- (p + tau a) / (1 + tau |a|)
// w (or d) goes through LDS between the two halves: px of the left pixel
// and py of the upper one for d, then w of the right and lower pixels for a.
// Pixels outside the image start with p = 0 and a = 0, so they keep p = 0;
// that realises the Neumann divergence (p_x = 0 on the last column and
// p_y = 0 on the last row is preserved by the update because a_x, a_y vanish
// there).  With zero_in set (first launch of a cold-started solve) the
// incoming dual field is taken as zero instead of being read.  The dual field
// is read from buffer `cur` of the slot and written to buffer 1 - cur.
// Channel planes of slots whose flow is complete (inactive) are skipped.
// The new dual vector of a pixel depends on the previous iterate within one
// pixel, so a region pixel at distance e from the region edge is exact while
// the iteration count is <= e: after iters <= TB iterations the BX x BY
// centre is exact and is written.
//
// The same cone says which rows are still needed: the update of iteration it
// (0-based) reaches the centre only from rows lo .. RY - 1 - lo, with lo =
// TB - iters + it + 1, and d only from rows lo .. RY - lo.  Where the region
// takes two passes of the workgroup (TB <= 5 at 32 x 32 tiles and 1024
// threads), every pass tests its rows and skips the others (their LDS values
// go stale, and nothing needed reads them); a wave whose pixels all lie
// outside issues nothing, which saves ~3.5% where two workgroups share a CU.
// With three or more passes the test is left out: it splits the
// straight-line passes the compiler interleaves, and with one workgroup per
// CU that interleaving hides more latency than the skipped rows save
// (measured at TB = 8 with several pixel-to-thread assignments).
template <typename S, typename M, int BX, int BY, int TB, int NT>
__global__ __launch_bounds__(NT) void k_chambolle_tile(const SlotDesc *__restrict__ slots, int cur, int H, int W,
                                                      int C, int ntx, int ntiles, S tau, int iters, int zero_in)
{
    const int slot = blockIdx.y / C;
    const int chan = blockIdx.y - slot * C;
    // Every descriptor field the launch uses is read before the activity
    // test, so the loads go out together and the workgroup waits for one
    // scalar-memory round trip instead of one per dependent use.
    const SlotDesc &sd = slots[slot];
    const int active = sd.active;
    const int kc = sd.k_cur;
    const void *v_pxi = sd.px[cur], *v_pyi = sd.py[cur];
    void *v_pxo = sd.px[1 - cur], *v_pyo = sd.py[1 - cur];
    const double *v_u0 = sd.u[0], *v_u1 = sd.u[1];
    const void *v_gx = sd.gx, *v_gy = sd.gy;
    const double dt = sd.dt;
    asm volatile("" ::"s"(active), "s"(kc), "s"(v_pxi), "s"(v_pyi), "s"(v_pxo), "s"(v_pyo), "s"(v_u0), "s"(v_u1),
                 "s"(v_gx), "s"(v_gy), "s"(dt));
    if (!active)
        return;
    constexpr bool kW = std::is_same<S, double>::value; // w-form data term
    constexpr int RX = BX + 2 * TB;
    constexpr int RY = BY + 2 * TB;
    constexpr int RN = RX * RY;
    constexpr int LX = RX + 2;            // LDS row pitch: region + zero ring
    constexpr int LN = LX * (RY + 2);
    constexpr int PPT = (RN + NT - 1) / NT;
    constexpr bool kSkip = PPT == 2;      // rows outside the cone are skipped
    __shared__ S s_px[LN];
    __shared__ S s_py[LN];
    __shared__ S s_d[LN];

    const size_t plane = (size_t)H * (size_t)W;
    const size_t coff = (size_t)chan * plane;
    const S *__restrict__ pxi = (const S *)v_pxi + coff;
    const S *__restrict__ pyi = (const S *)v_pyi + coff;
    const double *__restrict__ ui = ((kc & 1) ? v_u1 : v_u0) + coff;
    const M *__restrict__ gxi = (const M *)v_gx + coff;
    const M *__restrict__ gyi = (const M *)v_gy + coff;
    S *__restrict__ pxo = (S *)v_pxo + coff;
    S *__restrict__ pyo = (S *)v_pyo + coff;
    const double idt = 1.0 / dt;

    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs,
    // so give XCD x the x-th contiguous run of row-major tiles.
    const int b = blockIdx.x;
    const int L = ((ntiles & 7) == 0) ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
    const int ty = L / ntx;
    const int tx = L - ty * ntx;
    const int oy = ty * BY - TB;
    const int ox = tx * BX - TB;

    // zero ring (read by the outermost region pixels only)
    for (int e = threadIdx.x; e < 2 * LX + 2 * RY; e += NT) {
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

    // gq: u_k/dt (w-form) or Gx (gradient form); gy: Gy (gradient form only)
    S px[PPT], py[PPT], d[PPT], gq[PPT], gy[PPT];
    int li[PPT];     // LDS index of the pixel
    int rr[PPT];     // region row of the pixel (RY + 1 for the idle lanes of the last pass)
    S mx[PPT];       // 1 where a_x is live (inside the image, not its last column), else 0
    S my[PPT];       // 1 where a_y is live (inside the image, not its last row), else 0
    // Region load.  Every pixel's loads are issued before any loaded value
    // is used (the scaling and the LDS stores come in a second pass), so the
    // workgroup waits for one memory round trip rather than one per pixel.
    double uq[PPT];  // u_k (w-form) of the pixel, raw
    M g1[PPT], g2[PPT]; // Gx, Gy (gradient form), raw
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * NT;
        S vx = S(0), vy = S(0);
        double vu = 0.0;
        M vg1 = M(0), vg2 = M(0);
        bool ax_live = false, ay_live = false;
        int l = 0;
        rr[m] = RY + 1;
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            l = (ri + 1) * LX + (rj + 1);
            rr[m] = ri;
            if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                if (!zero_in) {
                    vx = pxi[q];
                    vy = pyi[q];
                }
                if constexpr (kW) {
                    vu = ui[q];
                } else {
                    vg1 = gxi[q];
                    vg2 = gyi[q];
                }
                ax_live = gj < W - 1;
                ay_live = gi < H - 1;
            }
        }
        li[m] = l;
        px[m] = vx;
        py[m] = vy;
        uq[m] = vu;
        g1[m] = vg1;
        g2[m] = vg2;
        d[m] = S(0);
        mx[m] = ax_live ? S(1) : S(0);
        my[m] = ay_live ? S(1) : S(0);
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        if constexpr (kW) {
            if constexpr (std::is_same<M, double>::value)
                gq[m] = uq[m] / dt;
            else
                gq[m] = uq[m] * idt;
            gy[m] = S(0);
        } else {
            gq[m] = (S)g1[m];
            gy[m] = (S)g2[m];
        }
        if (m < PPT - 1 || threadIdx.x + m * NT < RN) {
            s_px[li[m]] = px[m];
            s_py[li[m]] = py[m];
        }
    }
    __syncthreads();

    for (int it = 0; it < iters; ++it) {
        const int lo = TB - iters + it + 1;
        const unsigned span = (unsigned)(RY - 1 - 2 * lo);
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (kSkip ? (unsigned)(rr[m] - lo) <= span + 1u : (m < PPT - 1 || threadIdx.x + m * NT < RN)) {
                const int l = li[m];
                S dv = (px[m] - s_px[l - 1]) + (py[m] - s_py[l - LX]);
                if constexpr (kW)
                    dv = dv - gq[m];
                d[m] = dv;
                s_d[l] = dv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (kSkip ? (unsigned)(rr[m] - lo) <= span : (m < PPT - 1 || threadIdx.x + m * NT < RN)) {
                const int l = li[m];
                // unconditional LDS reads; the boundary masks multiply (a
                // select around the reads compiles to branches that expose
                // the LDS latency of every pixel)
                const S dr = s_d[l + 1];
                const S dd = s_d[l + LX];
                S ax, ay;
                if constexpr (kW) {
                    ax = (dr - d[m]) * mx[m];
                    ay = (dd - d[m]) * my[m];
                } else {
                    ax = ((dr - d[m]) - gq[m]) * mx[m];
                    ay = ((dd - d[m]) - gy[m]) * my[m];
                }
                chambolle_update<S, M>(px[m], py[m], ax, ay, tau);
                s_px[l] = px[m];
                s_py[l] = py[m];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * NT;
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

// Projection factor of the PDHG dual step: min(1, lam / |z|) for |z|^2 = x,
// so that z * factor is the projection of z onto the disc of radius lam
// (factor 1 for z = 0).
template <typename S, typename M> __device__ __forceinline__ S proj_factor(S x, S lam)
{
    if constexpr (std::is_same<S, M>::value) {
        using A = Arith<S>;
        const S f = lam * A::inv_(A::sqrt_(x)); // x = 0: lam * inf = inf
        return f < S(1) ? f : S(1);
    } else {
        // float32 reciprocal square root estimate refined by one float64
        // Newton step, as in the Chambolle update of this mode
        S y = (S)__builtin_amdgcn_rsqf((float)x);
        y = __builtin_fma(S(0.5) * y, __builtin_fma(-(x * y), y, S(1)), y);
        const S f = lam * y;
        return (x > S(1e-30) && f < S(1)) ? f : S(1);
    }
}

// Temporally blocked Chambolle-Pock primal-dual iterations for the ROF
// problem of the slot's current step (data g = u_k, weight lam = dt):
//     y    <- proj_{|y| <= lam}(y + sigma grad xbar)
//     x'   <- (x + tau div y + tau g) / (1 + tau)
//     xbar <- 2 x' - x,   x <- x'
// Same tiling, LDS ring, XCD-aware order, halo argument and row skipping as
// k_chambolle_tile (the new (x, xbar, y) of a pixel depends on the previous
// iterate within one pixel; iteration it needs y on rows lo - 1 .. RY - 1 -
// lo and x, xbar on rows lo .. RY - 1 - lo).  LDS carries xbar for the gradient (right and
// lower neighbours) and y for the divergence (left and upper neighbours).
// With solve_start set (first launch of a solve) x and xbar start at g and
// the dual field at zero (zero_y, cold start) or at the stored field (warm
// start); otherwise all three are read from buffer `cur`.  Pixels outside
// the image keep x = xbar = y = 0; grad xbar is masked to zero on the last
// column / row, which keeps y_x = 0 there (y_y on the last row) and gives
// the Neumann divergence.
template <typename S, typename M, int BX, int BY, int TB, int NT>
__global__ __launch_bounds__(NT) void k_pdhg_tile(const SlotDesc *__restrict__ slots, int cur, int H, int W, int C,
                                                 int ntx, int ntiles, S tau, S sigma, S inv1pt, int iters,
                                                 int solve_start, int zero_y)
{
    const int slot = blockIdx.y / C;
    const int chan = blockIdx.y - slot * C;
    // descriptor fields read together before the activity test, as in
    // k_chambolle_tile
    const SlotDesc &sd = slots[slot];
    const int active = sd.active;
    const int kc = sd.k_cur;
    const void *v_xi = sd.x[cur], *v_xbi = sd.xb[cur], *v_yxi = sd.px[cur], *v_yyi = sd.py[cur];
    void *v_xo = sd.x[1 - cur], *v_xbo = sd.xb[1 - cur], *v_yxo = sd.px[1 - cur], *v_yyo = sd.py[1 - cur];
    const double *v_u0 = sd.u[0], *v_u1 = sd.u[1];
    const double dt = sd.dt;
    asm volatile("" ::"s"(active), "s"(kc), "s"(v_xi), "s"(v_xbi), "s"(v_yxi), "s"(v_yyi), "s"(v_xo), "s"(v_xbo),
                 "s"(v_yxo), "s"(v_yyo), "s"(v_u0), "s"(v_u1), "s"(dt));
    if (!active)
        return;
    constexpr int RX = BX + 2 * TB;
    constexpr int RY = BY + 2 * TB;
    constexpr int RN = RX * RY;
    constexpr int LX = RX + 2;
    constexpr int LN = LX * (RY + 2);
    constexpr int PPT = (RN + NT - 1) / NT;
    constexpr bool kSkip = PPT == 2;      // rows outside the cone are skipped
    __shared__ S s_xb[LN];
    __shared__ S s_yx[LN];
    __shared__ S s_yy[LN];

    const size_t plane = (size_t)H * (size_t)W;
    const size_t coff = (size_t)chan * plane;
    const S lam = (S)dt;
    const double *__restrict__ g = ((kc & 1) ? v_u1 : v_u0) + coff;
    const S *__restrict__ xi = (const S *)v_xi + coff;
    const S *__restrict__ xbi = (const S *)v_xbi + coff;
    const S *__restrict__ yxi = (const S *)v_yxi + coff;
    const S *__restrict__ yyi = (const S *)v_yyi + coff;
    S *__restrict__ xo = (S *)v_xo + coff;
    S *__restrict__ xbo = (S *)v_xbo + coff;
    S *__restrict__ yxo = (S *)v_yxo + coff;
    S *__restrict__ yyo = (S *)v_yyo + coff;

    const int b = blockIdx.x;
    const int L = ((ntiles & 7) == 0) ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
    const int ty = L / ntx;
    const int tx = L - ty * ntx;
    const int oy = ty * BY - TB;
    const int ox = tx * BX - TB;

    for (int e = threadIdx.x; e < 2 * LX + 2 * RY; e += NT) {
        int li;
        if (e < LX)
            li = e;
        else if (e < 2 * LX)
            li = (RY + 1) * LX + (e - LX);
        else if (e < 2 * LX + RY)
            li = (e - 2 * LX + 1) * LX;
        else
            li = (e - 2 * LX - RY + 1) * LX + LX - 1;
        s_xb[li] = S(0);
        s_yx[li] = S(0);
        s_yy[li] = S(0);
    }

    S x[PPT], xb[PPT], yx[PPT], yy[PPT], gg[PPT], mx[PPT], my[PPT];
    double graw[PPT];
    int li[PPT];
    int rr[PPT];     // region row of the pixel (RY + 1 for the idle lanes of the last pass)
    // region load: all loads first, their uses in a second pass
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * NT;
        S vx = S(0), vxb = S(0), vyx = S(0), vyy = S(0);
        double vg = 0.0;
        bool ax_live = false, ay_live = false;
        int l = 0;
        rr[m] = RY + 1;
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            l = (ri + 1) * LX + (rj + 1);
            rr[m] = ri;
            if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                vg = g[q];
                if (!solve_start) {
                    vx = xi[q];
                    vxb = xbi[q];
                }
                if (!zero_y) {
                    vyx = yxi[q];
                    vyy = yyi[q];
                }
                ax_live = gj < W - 1;
                ay_live = gi < H - 1;
            }
        }
        li[m] = l;
        x[m] = vx;
        xb[m] = vxb;
        yx[m] = vyx;
        yy[m] = vyy;
        graw[m] = vg;
        mx[m] = ax_live ? S(1) : S(0);
        my[m] = ay_live ? S(1) : S(0);
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        gg[m] = (S)graw[m];
        if (solve_start) {
            x[m] = gg[m];
            xb[m] = gg[m];
        }
        if (m < PPT - 1 || threadIdx.x + m * NT < RN)
            s_xb[li[m]] = xb[m];
    }
    __syncthreads();

    for (int it = 0; it < iters; ++it) {
        const int lo = TB - iters + it + 1;
        const unsigned span = (unsigned)(RY - 1 - 2 * lo);
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (kSkip ? (unsigned)(rr[m] - lo + 1) <= span + 1u : (m < PPT - 1 || threadIdx.x + m * NT < RN)) {
                const int l = li[m];
                const S ax = (s_xb[l + 1] - xb[m]) * mx[m];
                const S ay = (s_xb[l + LX] - xb[m]) * my[m];
                const S zx = Arith<S>::fma_(sigma, ax, yx[m]);
                const S zy = Arith<S>::fma_(sigma, ay, yy[m]);
                const S f = proj_factor<S, M>(zx * zx + zy * zy, lam);
                yx[m] = zx * f;
                yy[m] = zy * f;
                s_yx[l] = yx[m];
                s_yy[l] = yy[m];
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (kSkip ? (unsigned)(rr[m] - lo) <= span : (m < PPT - 1 || threadIdx.x + m * NT < RN)) {
                const int l = li[m];
                const S d = (yx[m] - s_yx[l - 1]) + (yy[m] - s_yy[l - LX]);
                const S t = Arith<S>::fma_(tau, gg[m], Arith<S>::fma_(tau, d, x[m]));
                const S xn = t * inv1pt;
                const S xbn = xn + (xn - x[m]);
                x[m] = xn;
                xb[m] = xbn;
                s_xb[l] = xbn;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int idx = threadIdx.x + m * NT;
        if (idx < RN) {
            const int ri = idx / RX;
            const int rj = idx - ri * RX;
            const int gi = oy + ri;
            const int gj = ox + rj;
            if (ri >= TB && ri < TB + BY && rj >= TB && rj < TB + BX && gi < H && gj < W) {
                const size_t q = (size_t)gi * W + gj;
                xo[q] = x[m];
                xbo[q] = xb[m];
                yxo[q] = yx[m];
                yyo[q] = yy[m];
            }
        }
    }
}

#endif // TVSPEC_TILE_KERNELS_H
