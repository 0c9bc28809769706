/*
 * FP64 CPU oracle for the spectral total-variation decomposition of
 * Grossmann, Korolev, Gilboa, Schoenlieb, "Deeply Learned Spectral Total
 * Variation Decomposition" (arXiv 2006.10004).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Everything is double precision, scalar loops, no fused multiply-add
 * (build with -ffp-contract=off), true division and sqrt.  OpenMP, when
 * enabled, only splits independent per-pixel loops over rows; every
 * reduction runs serially in row-major order, so threaded and single-thread
 * results are bit-identical.
 *
 * What is computed, and where the paper defines it:
 *   - discrete isotropic TV in dual form, Sec. 2.1 Eq. (2): forward-difference
 *     gradient with Neumann boundary and the divergence that is its negative
 *     adjoint (the discretisation of Chambolle 2004, which the paper names as
 *     its CPU solver in Sec. 4.3);
 *   - one implicit Euler step of the TV flow Eq. (1), which is the ROF problem
 *     Eq. (8) with weight dt, solved by Chambolle's semi-implicit dual fixed
 *     point with step tau;
 *   - TV transform phi(t) = t u_tt(t), Eq. (3), by the central second
 *     difference on the time grid t_k = k dt;
 *   - spectrum S(t) = ||phi(t)||_L1, the unnumbered display after Eq. (3);
 *   - band integrals of phi, Eq. (7), right-endpoint rule on each [t_{k-1},t_k];
 *   - residual f_r(T) = u(T) - T u_t(T), Eq. (5), with a forward difference
 *     for u_t.
 *
 * Conventions (pixel (i,j): i = row 0..H-1, j = column 0..W-1, row-major,
 * column fastest; each channel of an image is processed independently):
 *   K  = number of spectral samples phi_1..phi_K; it needs u_0..u_{K+1},
 *        i.e. K+1 ROF solves.
 *   edges e_0 = 0 < e_1 < ... < e_B = K: band j (1-based) collects the
 *        samples k with e_{j-1} < k <= e_j.  The residual is returned on its
 *        own (the paper adds it to the last band; f = sum of bands + residual).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j) ((size_t)(i) * (size_t)W + (size_t)(j))

/* Number of threads the per-pixel loops use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward-difference gradient with Neumann boundary:
 *   gx(i,j) = u(i,j+1) - u(i,j) for j < W-1, and 0 on the last column;
 *   gy(i,j) = u(i+1,j) - u(i,j) for i < H-1, and 0 on the last row. */
void orc_grad(const double *u, int H, int W, double *gx, double *gy)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            gx[IDX(i, j)] = (j < W - 1) ? u[IDX(i, j + 1)] - u[IDX(i, j)] : 0.0;
            gy[IDX(i, j)] = (i < H - 1) ? u[IDX(i + 1, j)] - u[IDX(i, j)] : 0.0;
        }
    }
}

/* Discrete divergence, defined so that <grad u, p> = -<u, div p>:
 *   x part: px(i,0) on the first column, px(i,j) - px(i,j-1) inside,
 *           -px(i,W-2) on the last column; the y part likewise along rows.
 *   d = (x part) + (y part). */
void orc_div(const double *px, const double *py, int H, int W, double *d)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            double dx, dy;
            if (j == 0)
                dx = px[IDX(i, j)];
            else if (j == W - 1)
                dx = -px[IDX(i, j - 1)];
            else
                dx = px[IDX(i, j)] - px[IDX(i, j - 1)];
            if (i == 0)
                dy = py[IDX(i, j)];
            else if (i == H - 1)
                dy = -py[IDX(i - 1, j)];
            else
                dy = py[IDX(i, j)] - py[IDX(i - 1, j)];
            d[IDX(i, j)] = dx + dy;
        }
    }
}

/* Discrete isotropic total variation: sum over pixels of |grad u|. */
double orc_tv(const double *u, int H, int W)
{
    size_t n = (size_t)H * (size_t)W;
    double *gx = (double *)malloc(n * sizeof(double));
    double *gy = (double *)malloc(n * sizeof(double));
    double s = 0.0;
    orc_grad(u, H, W, gx, gy);
    for (size_t q = 0; q < n; ++q)
        s += sqrt(gx[q] * gx[q] + gy[q] * gy[q]);
    free(gx);
    free(gy);
    return s;
}

/* One ROF problem  min_v 0.5 ||g - v||^2 + lambda TV(v)  (Eq. (8) with
 * lambda = dt), by Chambolle's dual fixed point.  Every iteration updates all
 * pixels from the previous iterate:
 *     w  = div p - g / lambda
 *     a  = grad w
 *     p <- (p + tau a) / (1 + tau |a|)
 * and the primal solution is  v = g - lambda div p.
 * (px, py) hold the starting dual field on entry and the final one on exit;
 * v receives the primal solution. */
void orc_rof(const double *g, int H, int W, double lambda, double tau, int iters,
             double *px, double *py, double *v)
{
    size_t n = (size_t)H * (size_t)W;
    double *d = (double *)malloc(n * sizeof(double));
    double *w = (double *)malloc(n * sizeof(double));
    double *ax = (double *)malloc(n * sizeof(double));
    double *ay = (double *)malloc(n * sizeof(double));
    for (int it = 0; it < iters; ++it) {
        orc_div(px, py, H, W, d);
        int i;
#pragma omp parallel for schedule(static)
        for (i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                w[IDX(i, j)] = d[IDX(i, j)] - g[IDX(i, j)] / lambda;
        orc_grad(w, H, W, ax, ay);
#pragma omp parallel for schedule(static)
        for (i = 0; i < H; ++i) {
            for (int j = 0; j < W; ++j) {
                size_t q = IDX(i, j);
                double norm = sqrt(ax[q] * ax[q] + ay[q] * ay[q]);
                double den = 1.0 + tau * norm;
                px[q] = (px[q] + tau * ax[q]) / den;
                py[q] = (py[q] + tau * ay[q]) / den;
            }
        }
    }
    orc_div(px, py, H, W, d);
    for (size_t q = 0; q < n; ++q)
        v[q] = g[q] - lambda * d[q];
    free(d);
    free(w);
    free(ax);
    free(ay);
}

/* The same ROF problem by the first-order primal-dual algorithm of
 * Chambolle and Pock (2011, Algorithm 1; the paper's GPU baseline is a
 * primal-dual solver, Sec. 4.3), with operator grad, F = lambda ||.||_{2,1}
 * on the gradient field and G(v) = 0.5 ||v - g||^2:
 *     y    <- proj(y + sigma grad xbar),  proj(y) = y / max(1, |y| / lambda)
 *     x'   <- (x + tau div y + tau g) / (1 + tau)
 *     xbar <- x' + theta (x' - x),  theta = 1;   x <- x'
 * starting from x = xbar = g and the given y; v receives x after `iters`
 * iterations.  Convergence needs tau sigma ||grad||^2 <= 1 (||grad||^2 <=
 * 8).  (yx, yy) hold the starting dual field on entry and the final one on
 * exit. */
void orc_rof_pdhg(const double *g, int H, int W, double lambda, double tau, double sigma,
                  int iters, double *yx, double *yy, double *v)
{
    size_t n = (size_t)H * (size_t)W;
    double *x = (double *)malloc(n * sizeof(double));
    double *xb = (double *)malloc(n * sizeof(double));
    double *ax = (double *)malloc(n * sizeof(double));
    double *ay = (double *)malloc(n * sizeof(double));
    double *d = (double *)malloc(n * sizeof(double));
    memcpy(x, g, n * sizeof(double));
    memcpy(xb, g, n * sizeof(double));
    for (int it = 0; it < iters; ++it) {
        orc_grad(xb, H, W, ax, ay);
        int i;
#pragma omp parallel for schedule(static)
        for (i = 0; i < H; ++i) {
            for (int j = 0; j < W; ++j) {
                size_t q = IDX(i, j);
                double zx = yx[q] + sigma * ax[q];
                double zy = yy[q] + sigma * ay[q];
                double m = sqrt(zx * zx + zy * zy) / lambda;
                double s = m > 1.0 ? m : 1.0;
                yx[q] = zx / s;
                yy[q] = zy / s;
            }
        }
        orc_div(yx, yy, H, W, d);
#pragma omp parallel for schedule(static)
        for (i = 0; i < H; ++i) {
            for (int j = 0; j < W; ++j) {
                size_t q = IDX(i, j);
                double xn = (x[q] + tau * d[q] + tau * g[q]) / (1.0 + tau);
                xb[q] = xn + 1.0 * (xn - x[q]);
                x[q] = xn;
            }
        }
    }
    memcpy(v, x, n * sizeof(double));
    free(x);
    free(xb);
    free(ax);
    free(ay);
    free(d);
}

/* TV flow Eq. (1) by implicit Euler: u_0 = f, u_{s+1} = ROF(u_s, dt) for
 * s = 0..nsteps-1.  states receives u_0..u_nsteps, (nsteps+1) planes of H*W.
 * warm == 0: every solve starts its dual field from zero; warm != 0: the
 * dual field of solve s starts from the final one of solve s-1 (zero for
 * s = 0).  The paper does not say which; both are offered. */
void orc_tv_flow(const double *f, int H, int W, double dt, int nsteps, int iters,
                 double tau, int warm, double *states)
{
    size_t n = (size_t)H * (size_t)W;
    double *px = (double *)calloc(n, sizeof(double));
    double *py = (double *)calloc(n, sizeof(double));
    memcpy(states, f, n * sizeof(double));
    for (int s = 0; s < nsteps; ++s) {
        if (!warm) {
            memset(px, 0, n * sizeof(double));
            memset(py, 0, n * sizeof(double));
        }
        orc_rof(states + (size_t)s * n, H, W, dt, tau, iters, px, py,
                states + (size_t)(s + 1) * n);
    }
    free(px);
    free(py);
}

/* Spectral transform of a stored flow u_0..u_{K+1} (Eq. (3), the spectrum,
 * Eq. (5) and Eq. (7)):
 *   phi_k = t_k (u_{k-1} - 2 u_k + u_{k+1}) / dt^2,   t_k = k dt, k = 1..K
 *   S[k-1] = sum over pixels of |phi_k|
 *   band j = sum over e_{j-1} < k <= e_j of phi_k dt
 *   residual = u_K - T (u_{K+1} - u_K) / dt,          T = K dt
 * phi (optional, may be NULL) receives K planes. */
void orc_spectral(const double *states, int H, int W, double dt, int K,
                  const int *edges, int nbands, double *S, double *bands,
                  double *residual, double *phi)
{
    size_t n = (size_t)H * (size_t)W;
    double *ph = (double *)malloc(n * sizeof(double));
    memset(bands, 0, (size_t)nbands * n * sizeof(double));
    int band = 0;
    for (int k = 1; k <= K; ++k) {
        const double *um = states + (size_t)(k - 1) * n;
        const double *u0 = states + (size_t)k * n;
        const double *up = states + (size_t)(k + 1) * n;
        double tk = (double)k * dt;
        while (k > edges[band + 1])
            ++band;
        double s = 0.0;
        for (size_t q = 0; q < n; ++q) {
            ph[q] = tk * (um[q] - 2.0 * u0[q] + up[q]) / (dt * dt);
            s += fabs(ph[q]);
            bands[(size_t)band * n + q] += ph[q] * dt;
        }
        S[k - 1] = s;
        if (phi)
            memcpy(phi + (size_t)(k - 1) * n, ph, n * sizeof(double));
    }
    {
        const double *uK = states + (size_t)K * n;
        const double *uK1 = states + (size_t)(K + 1) * n;
        double T = (double)K * dt;
        for (size_t q = 0; q < n; ++q)
            residual[q] = uK[q] - T * (uK1[q] - uK[q]) / dt;
    }
    free(ph);
}

/* Band edges valid for K samples: e_0 = 0, strictly increasing, e_B = K. */
int orc_edges_valid(int K, const int *edges, int nbands)
{
    if (nbands < 1 || edges[0] != 0 || edges[nbands] != K)
        return 0;
    for (int j = 1; j <= nbands; ++j)
        if (edges[j] <= edges[j - 1])
            return 0;
    return 1;
}

/* One ROF solve of the flow by the selected solver: 0 = Chambolle's dual
 * fixed point (step tau), 1 = Chambolle-Pock primal-dual (steps tau, sigma);
 * (px, py) is the dual field carried between solves. */
static void rof_solve(int solver, const double *g, int H, int W, double lambda, double tau,
                      double sigma, int iters, double *px, double *py, double *v)
{
    if (solver == 1)
        orc_rof_pdhg(g, H, W, lambda, tau, sigma, iters, px, py, v);
    else
        orc_rof(g, H, W, lambda, tau, iters, px, py, v);
}

/* Full decomposition of a C x H x W float image (channels independent).
 * Same quantities as orc_tv_flow followed by orc_spectral (the ROF solves by
 * `solver`, as rof_solve), but the flow is
 * walked one step at a time with only u_{k-1}, u_k, u_{k+1} kept, so large
 * images do not need all K+2 states in memory.
 *   bands    [nbands][C][H][W]
 *   S        [C][K]            S[c][k-1] = S_c(t_k)
 *   residual [C][H][W]
 *   report   [2]: max |f - sum bands - residual|, and
 *                 max over c of |mean(u_{K+1}) - mean(f_c)|.
 * Returns 0, or -1 on invalid arguments. */
int orc_decompose_solver(const float *f, int H, int W, int C, double dt, int K, int iters,
                         int solver, double tau, double sigma, int warm, const int *edges,
                         int nbands, double *bands, double *S, double *residual, double *report)
{
    if (H < 2 || W < 2 || C < 1 || K < 1 || iters < 1 || !(dt > 0.0) || !(tau > 0.0) ||
        (solver != 0 && solver != 1) || (solver == 1 && !(sigma > 0.0)) ||
        !orc_edges_valid(K, edges, nbands))
        return -1;
    size_t n = (size_t)H * (size_t)W;
    double *um = (double *)malloc(n * sizeof(double));
    double *u0 = (double *)malloc(n * sizeof(double));
    double *up = (double *)malloc(n * sizeof(double));
    double *px = (double *)malloc(n * sizeof(double));
    double *py = (double *)malloc(n * sizeof(double));
    double recon = 0.0, drift = 0.0;
    for (int c = 0; c < C; ++c) {
        const float *fc = f + (size_t)c * n;
        double *rc = residual + (size_t)c * n;
        for (int j = 0; j < nbands; ++j)
            memset(bands + ((size_t)j * C + c) * n, 0, n * sizeof(double));
        memset(px, 0, n * sizeof(double));
        memset(py, 0, n * sizeof(double));
        for (size_t q = 0; q < n; ++q)
            u0[q] = (double)fc[q];
        /* u_0 -> u_1 */
        rof_solve(solver, u0, H, W, dt, tau, sigma, iters, px, py, up);
        int band = 0;
        for (int k = 1; k <= K; ++k) {
            /* shift the window: (u_{k-1}, u_k) <- (u_{k-1}, u_k) of this k */
            double *t = um;
            um = u0;
            u0 = up;
            up = t;
            if (!warm) {
                memset(px, 0, n * sizeof(double));
                memset(py, 0, n * sizeof(double));
            }
            rof_solve(solver, u0, H, W, dt, tau, sigma, iters, px, py, up); /* u_{k+1} */
            double tk = (double)k * dt;
            while (k > edges[band + 1])
                ++band;
            double *bj = bands + ((size_t)band * C + c) * n;
            double s = 0.0;
            for (size_t q = 0; q < n; ++q) {
                double phi = tk * (um[q] - 2.0 * u0[q] + up[q]) / (dt * dt);
                s += fabs(phi);
                bj[q] += phi * dt;
            }
            S[(size_t)c * K + (k - 1)] = s;
        }
        /* u0 = u_K, up = u_{K+1} */
        double T = (double)K * dt;
        for (size_t q = 0; q < n; ++q)
            rc[q] = u0[q] - T * (up[q] - u0[q]) / dt;
        double sf = 0.0, su = 0.0;
        for (size_t q = 0; q < n; ++q) {
            double acc = 0.0;
            for (int j = 0; j < nbands; ++j)
                acc += bands[((size_t)j * C + c) * n + q];
            double e = fabs((double)fc[q] - acc - rc[q]);
            if (e > recon)
                recon = e;
            sf += (double)fc[q];
            su += up[q];
        }
        double dm = fabs(su / (double)n - sf / (double)n);
        if (dm > drift)
            drift = dm;
    }
    report[0] = recon;
    report[1] = drift;
    free(um);
    free(u0);
    free(up);
    free(px);
    free(py);
    return 0;
}

/* orc_decompose_solver with Chambolle's dual fixed point. */
int orc_decompose(const float *f, int H, int W, int C, double dt, int K, int iters,
                  double tau, int warm, const int *edges, int nbands,
                  double *bands, double *S, double *residual, double *report)
{
    return orc_decompose_solver(f, H, W, C, dt, K, iters, 0, tau, 0.0, warm, edges, nbands, bands, S,
                                residual, report);
}
