// The decomposition engine: a table of image slots stepped through the flow.
//
// Every image being decomposed occupies a slot.  A slot's descriptor (kept
// in device memory, read by the kernels) holds pointers to the image's state
// and outputs and its position in the flow.  All slots of a table share the
// image size (H, W, C) and the number of Chambolle iterations per solve;
// each has its own dt, K, band edges and step counter.  One engine_step runs
// one ROF solve plus the fused outer update for every active slot of the
// table, so a slot can enter the table at any step boundary (continuous
// batching) and leaves it when its flow is complete.
#ifndef TVSPEC_ENGINE_H
#define TVSPEC_ENGINE_H

#include <hip/hip_runtime.h>

#include <cstddef>

#include "common.h"

namespace tvspec {

// Inner ROF solvers.
constexpr int kSolverChambolle = 0; // Chambolle's dual fixed point
constexpr int kSolverPDHG = 1;      // Chambolle-Pock primal-dual

struct SlotDesc {
    void *px[2], *py[2];  // dual field, ping-pong (state type of the mode)
    void *gx, *gy;        // F32 Chambolle: G = grad(g)/dt (float32); else unused
    void *x[2], *xb[2];   // PDHG: primal iterate and its extrapolation, ping-pong
    double *u[2];         // flow state; u_s lives in u[s % 2]
    double *dprev;        // D_{s-1}
    const float *f;       // [C][H][W]
    double *bands;        // [nbands][C][H][W]
    double *S;            // [C][K]
    double *res;          // [C][H][W]
    double *stats;        // [TVSPEC_NSTATS]
    double *spart;        // [K][C][nblk] step partials of S
    double *rpart;        // [C][nblk][3] check partials
    int *band_rows;       // [K + 1] band of every sample (entry 0 unused)
    unsigned int *nonfinite;
    double dt;
    int K;
    int nbands;
    int k_cur;            // next flow step (0 .. K); K + 1 once complete
    int active;           // 1 while k_cur <= K
};

// Inner-iteration precision modes (TVSPEC_PRECISION_*): bytes per element of
// the dual field (state) and of the stored data-term gradient G (F32 only; the
// float64 modes read the data term from the flow state, 0 bytes).
size_t state_elem(int precision);
size_t g_elem(int precision);

// Workgroups per channel plane of the per-pixel kernels (fixed per plane
// size, so partial sums are reproducible).
int plane_blocks(int plane);

// Device bytes of one slot's per-pixel engine buffers (dual field, G or the
// primal iterates, u, D, S and check partials), 256-byte aligned pieces.
size_t slot_scratch_bytes(int precision, int solver, int H, int W, int C, int K);

// Lay out those buffers in [base, base + slot_scratch_bytes) and fill the
// slot's pointers to them and its K; f, the outputs, band_rows, nonfinite,
// dt and nbands are set by the caller.
void slot_carve(SlotDesc &d, char *base, int precision, int solver, int H, int W, int C, int K);

// Tile shapes of the Chambolle tile kernel (results do not depend on the
// shape): 32 x 32 output pixels on 1024 threads, or 32 x 16 on 512 threads
// (twice the workgroups for small launches; TB 4, 5 or 8).
constexpr int kTileShapeSquare = 0;
constexpr int kTileShapeNarrow = 1;

struct StepConfig {
    int H, W, C;
    int iters;            // Chambolle iterations per ROF solve
    double tau;
    int warm;             // 0: every solve starts from p = 0
    int iters_per_launch; // 0: automatic
    int precision;
    int timed = 1;        // 0: never record benchmark timing (graph capture)
    int solver = kSolverChambolle;
    double sigma = 0.0;   // PDHG dual step (tau is its primal step)
    int tile = kTileShapeSquare; // Chambolle tile shape (the primal-dual solver uses the square one)
};

// Tile-kernel launches per engine_step over a table of nslots slots (the
// dual-field parity flips after a step when this is odd).
int tile_launches_per_step(const StepConfig &cfg, int nslots);

// u_0 = f, p = 0, bands = 0 (F32: G = grad(f)/dt), k_cur = 0, active = 1, for
// slots [first, first + count) of the table.
int engine_init(const StepConfig &cfg, SlotDesc *d_slots, int first, int count, hipStream_t st);

// One ROF solve and outer step for every active slot of a table of nslots
// (inactive slots cost an early exit).  *parity is the dual-field buffer
// holding the current iterate; it is updated.  live_planes counts the
// active slots' planes for the timing record.
int engine_step(const StepConfig &cfg, SlotDesc *d_slots, int nslots, int *parity, hipStream_t st,
                long long live_planes);

// S, stats and the reconstruction check of the completed slots [first,
// first + count); Kmax is the largest K among them.
int engine_finalize(const StepConfig &cfg, SlotDesc *d_slots, int first, int count, int Kmax, hipStream_t st);

// Benchmark timing (one event pair per engine_step around its tile launches).
int timing_enable(int on);
int timing_read(double *kernel_ms, long long *launches, long long *pixel_iters);

} // namespace tvspec

#endif // TVSPEC_ENGINE_H
