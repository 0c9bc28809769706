// tvspec_nn: the learned surrogate (include/tvspec_nn.h) on gfx950.
//
// Convolutions are implicit GEMMs on the matrix cores.  With pixels p and
// the reduction index k = tap * Cin + c (tap = 3 dy + dx), a 3x3 "same"
// convolution is Y[p][o] = sum_k A[p][k] Wt[o][k] with A[p][k] = X[p +
// (dy-1, dx-1)][c] (zero outside the image).  Channels-last storage makes
// the 8 consecutive k of one MFMA operand lane 8 consecutive channels of
// one pixel at one tap, i.e. one 16-byte load, as long as Cin is a multiple
// of 8.  v_mfma_f32_16x16x32_bf16 (gfx950) lane layout: A row l % 16 with k
// 8(l / 16) .. +7, B column l % 16 with the same k, result column l % 16,
// rows 4(l / 16) .. +3.
//
//   k_conv3x3      forward (and the input gradient, on flipped, transposed
//                  weights): a workgroup of 4 waves covers an 8 x 32 pixel
//                  tile x 16 NF output channels; each chunk of input
//                  channels is staged in LDS with its halo once and read by
//                  all 9 taps; the weight tiles go straight from global
//                  memory to LDS two k steps ahead; the decoder's
//                  concatenations can be read in place; bias, ReLU, a ReLU
//                  mask, an output scale and the encoder's 2 x 2 max pooling
//                  fused in the epilogue, which leaves through an LDS tile in
//                  16-byte pieces.
//   k_wgrad        weight gradient, reduction over pixels: a workgroup takes
//                  16 OW output x 16 WC input channels x all 9 taps over a
//                  range of 4 x 32 pixel tiles; each tile's dY and X (with
//                  its halo) are staged in LDS once, channels-last, and every
//                  tap's operand is the X tile read at a shift through the
//                  transposing LDS read (ds_read_b64_tr_b16); per-range
//                  partial sums are added in a fixed order by k_reduce_rows
//                  (deterministic).
//   the rest       packing, 2x2 max-pooling and its gradient, the gradient
//                  of the decoder's concatenations (which the convolutions and
//                  weight gradients read in place; ReLU masks fused), the
//                  normalised MSE loss and its gradient, Adam.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "tvspec_nn.h"

namespace tvspec {
namespace nn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kT = 256;

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        z[j] = (__bf16)0.0f;
    return z;
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const bf16x8 global_bf16x8;

// Sixteen zero bytes in global memory (never written): the source of the
// input loads of halo slots outside the image, so that every wave issues a
// fixed number of loads.  Kept in the global address space (not constant),
// so that those loads stay global_load rather than flat loads, which would
// also count against the LDS wait counter.
__device__ uint4 kZero16[1] = {{0u, 0u, 0u, 0u}};

// s_waitcnt vmcnt(N) lgkmcnt(0): at most N vector memory operations of this
// wave outstanding (they complete in issue order) and no LDS operation.
template <int N> __device__ __forceinline__ void wait_vm_lds()
{
    static_assert(N >= 0 && N < 64, "vmcnt is six bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}
// s_waitcnt lgkmcnt(0) alone.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }
// Keeps the compiler from moving memory operations across this point (it
// emits no instruction): the wait counts below rely on the issue order.
__device__ __forceinline__ void order_fence() { asm volatile("" ::: "memory"); }

// ---------------------------------------------------------------------------
// convolution (forward and input gradient)

// Y[p][o] = epilogue(sum_{tap, c} X[p + tap offset][c] Wt[o][tap][c]),
// Wt [Cout][9][Cin].  Epilogue: + bias[o] (bias != nullptr), max(., 0)
// (relu), zero where mask[p][o] <= 0 (mask != nullptr), times oscale[o]
// (oscale != nullptr); stored as bf16 or f32.
//
// Implicit GEMM over output pixels x output channels x (9 taps x Cin).  A
// workgroup of WAVES waves owns a (2 WAVES) x 32 tile of output pixels of
// one image and 16 NF output channels.  The input channels are taken in
// chunks of CC: the chunk's (2 WAVES + 2) x (32 + 2) input pixels are
// staged in LDS once, and all 9 taps read their operands from there (each
// input value leaves HBM/L2 1.2 to 1.3 times instead of 9).  A chunk's
// 9 CC values of k, tap-major (k = tap CC + c), make ceil(9 CC / 32) steps
// of 32 (zero-padded); the weight tile of a step (16 NF channels x 32 k) goes
// straight from global memory to LDS (global_load_lds_dwordx4, no registers
// in flight), kConvPrefetch steps ahead into kConvPrefetch + 1 rotating
// buffers.  Wave w computes output rows RPW w .. RPW w + RPW - 1 (2 RPW
// 16-pixel row fragments; RPW = 2) x NF column fragments of
// v_mfma_f32_16x16x32_bf16.  Measured
// variants that hold more in registers (8-wave workgroups, 64-wide k
// stages, weights two steps ahead in registers, 48-channel chunks) were all
// slower: each costs occupancy, and the lost workgroups per CU outweigh the
// latency they hide.  The next step's A fragments are read a step ahead only
// where the 16 registers cost no occupancy (kPrefA).
//
// LDS pixel pitch: CC bf16 padded to an odd multiple of 16 bytes, so the
// 16-byte operand reads of 8 (or 16) consecutive lanes, at consecutive
// pixels, fall in distinct banks.
constexpr int kTileX = 32;
constexpr int kHaloX = kTileX + 2;
constexpr int kConvPrefetch = 2;  // steps between issuing a weight tile and using it (3 measured 1.5% slower)
constexpr int kBPitch = 40;  // LDS row pitch of the weight tile (32 k + 8; 20 dwords: 4 x odd)

template <int CC, int WAVES, int RPW>
struct ConvShape {
    static_assert(CC % 8 == 0 && CC <= 64, "chunk of 8..64 channels");
    static constexpr int kThreads = 64 * WAVES;
    static constexpr int kTileY = RPW * WAVES;    // RPW output rows per wave
    static constexpr int kHaloPix = (kTileY + 2) * kHaloX;
    static constexpr int kPitch = ((CC / 8) % 2 == 1) ? CC : CC + 8;  // bf16 per pixel in LDS
    static constexpr int kSteps = (9 * CC + 31) / 32;
    static constexpr int kGroups = CC / 8;                              // 16-byte groups per pixel
    static constexpr int kItems = kHaloPix * kGroups;                   // 16-byte loads per chunk
    static constexpr int kItemsPerThread = (kItems + kThreads - 1) / kThreads;
};

// Optional output form of the network's last layer:
//   planar  the last layer (float32 output, one block of 16 channels)
//           writes the planar output [B][15][H][W] directly: bands as
//           computed, the residual channels 12..14 plus fout (f), and with
//           ipart the partial sums over each 8 x 32 tile, ipart[b][tile], of
//           |f - sum_j band_j - residual| over the 3 channels, taken on the
//           stored outputs (the reconstruction identity, Eq. (7)).
struct ConvIO {
    float *planar = nullptr;
    const float *fout = nullptr;
    double *ipart = nullptr;
};

// Waves per SIMD the last layer's shape keeps with its planar epilogue
// (which would otherwise cost it one: 5 -> 4).
template <bool F32OUT, int NF, int CC> constexpr int conv_min_waves()
{
    return (F32OUT && NF == 1 && CC == 16) ? 5 : 1;
}

template <bool F32OUT, int NF, int CC, int WAVES, int RPW>
__global__ __launch_bounds__(64 * WAVES, (conv_min_waves<F32OUT, NF, CC>())) void k_conv3x3(const __bf16 *__restrict__ X, const __bf16 *__restrict__ Wt,
                                                        const float *__restrict__ bias,
                                                        const __bf16 *__restrict__ mask,
                                                        const float *__restrict__ oscale, void *__restrict__ Y, int B,
                                                        int H, int W, int Cin, int Cout, int relu, int tiles_x,
                                                        int tiles_y, const __bf16 *__restrict__ Xlow, int Clow,
                                                        __bf16 *__restrict__ Ypool, ConvIO io)
{
    using CS = ConvShape<CC, WAVES, RPW>;
    constexpr int kRF = 2 * RPW;  // 16-pixel row fragments per wave
    using OutT = typename std::conditional<F32OUT, float, __bf16>::type;
    constexpr int kPitch = CS::kPitch;
    constexpr int kSteps = CS::kSteps;
    constexpr int kNT = CS::kThreads;
    constexpr int kTilePix = CS::kTileY * kTileX;
    constexpr int kOC = NF * 16;                                   // output channels of the tile
    constexpr int kOPitch = (((kOC * (int)sizeof(OutT) + 15) / 16) | 1) * 16;  // epilogue bytes per pixel
    constexpr int kXBytes = CS::kHaloPix * kPitch * 2;
    // a weight row (one output channel, 32 k) is five 16-byte slots, four of
    // data and one of padding; a buffer holds whole waves of slots
    static_assert(kBPitch == 40, "five 16-byte slots per weight row");
    constexpr int kWSlots = ((NF * 16 * 5 + kNT - 1) / kNT) * kNT;
    constexpr int kD = kWSlots / kNT;              // direct loads per wave per step
    constexpr int kXL = CS::kItemsPerThread;       // input loads per thread per chunk
    constexpr int kBBytes = kWSlots * 16;
    constexpr int kPD = kConvPrefetch;             // weights issued kPD steps ahead
    constexpr int kNB = kPD + 1;                   // rotating weight buffers
    static_assert(kPD == 2 || kPD == 3, "prefetch distance 2 or 3");
    static_assert(CS::kSteps >= kPD, "the prologue's steps lie in the first chunk");
    constexpr int kPlanarPitch = 80;               // planar epilogue: 16 floats + 16 bytes per pixel
    constexpr int kTileBytes = F32OUT ? (NF == 1 ? kTilePix * kPlanarPitch : 0) : kTilePix * kOPitch;
    constexpr int kSmem = (kXBytes + kNB * kBBytes > kTileBytes) ? kXBytes + kNB * kBBytes : kTileBytes;
    // input chunk and the weight buffers; after the last step, the
    // epilogue's output tile (bf16 outputs) in the same memory
    __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
    __bf16 *const sX = (__bf16 *)smem;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x;
    const int ty = (tile / tiles_x) % tiles_y;
    const int b = tile / (tiles_x * tiles_y);
    const int y0 = ty * CS::kTileY;
    const int x0 = tx * kTileX;
    const int co0 = blockIdx.y * (NF * 16);
    const int K = 9 * Cin;
    const int nchunks = Cin / CC;

    // input staging: item i = (halo pixel i / kGroups, 16-byte group i % kGroups)
    // (every thread issues kXL loads; slots outside the image or past the
    // chunk read kZero16)
    auto load_x = [&](int q, bf16x8 *v) {
#pragma unroll
        for (int j = 0; j < kXL; ++j) {
            const int i = threadIdx.x + j * kNT;
            const __bf16 *src = (const __bf16 *)kZero16;
            if (i < CS::kItems) {
                const int hp = i / CS::kGroups;
                const int cg = i - hp * CS::kGroups;
                const int hy = hp / kHaloX;
                const int hx = hp - hy * kHaloX;
                const int yy = y0 + hy - 1;
                const int xx = x0 + hx - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
                    const int c0 = q * CC + 8 * cg;
                    if (c0 < Clow)  // the upsampled half of a concatenated input
                        src = Xlow + ((size_t)((size_t)b * (H / 2) + yy / 2) * (W / 2) + xx / 2) * Clow + c0;
                    else
                        src = X + ((size_t)((size_t)b * H + yy) * W + xx) * (Cin - Clow) + (c0 - Clow);
                }
            }
            v[j] = *(const global_bf16x8 *)src;
        }
    };
    auto store_x = [&](const bf16x8 *v) {
#pragma unroll
        for (int j = 0; j < CS::kItemsPerThread; ++j) {
            const int i = threadIdx.x + j * kNT;
            if (i < CS::kItems) {
                const int hp = i / CS::kGroups;
                const int cg = i - hp * CS::kGroups;
                *(bf16x8 *)(&sX[hp * kPitch + 8 * cg]) = v[j];
            }
        }
    };
    // weight tile of step s of chunk q into buffer bb by direct loads: wave
    // w fills slots [64 (w kD + j), +64), j < kD; slot u is row u / 5 (output
    // channel co0 + u / 5), k group u % 5 (8 values of k at 8 (u % 5) of the
    // step).  Slots no MFMA reads (group 4, rows past 16 NF), rows of
    // channels >= Cout (they only feed outputs that are not stored) and k
    // past the chunk (their A operand is zero, and finite weights times zero
    // add exactly 0) read the first weights instead, so every source is Wt
    // plus a 32-bit offset.
    auto dma_w = [&](int q, int s, int bb) {
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            const int u = (wave * kD + j) * 64 + lane;
            const int row = u / 5;
            const int grp = u - row * 5;
            const int co = co0 + row;
            const int kc = s * 32 + grp * 8;  // k within the chunk
            int off = 0;
            if (grp < 4 && row < NF * 16 && co < Cout && kc < 9 * CC) {
                const int tap = kc / CC;
                off = co * K + tap * Cin + q * CC + (kc - tap * CC);
            }
            __builtin_amdgcn_global_load_lds(Wt + off,
                                             (lds_void *)(smem + kXBytes + bb * kBBytes + (wave * kD + j) * 1024), 16,
                                             0, 0);
        }
    };

    // this lane's row fragments: output row lr = 2 wave + (r >> 1), columns
    // 16 (r & 1) + r16; halo pixel of tap (0, 0)
    int hbase[kRF];
#pragma unroll
    for (int r = 0; r < kRF; ++r)
        hbase[r] = (RPW * wave + (r >> 1)) * kHaloX + 16 * (r & 1) + r16;

    floatx4 acc[kRF][NF];
#pragma unroll
    for (int r = 0; r < kRF; ++r)
#pragma unroll
        for (int c = 0; c < NF; ++c)
            acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    // Pipeline over the steps t = q kSteps + s (T in all): at the start of
    // step t the next chunk's input goes to registers (s = 0 only), then the
    // weights of step t + kPD (buffer (t + kPD) % kNB, last read in step t - 1,
    // whose closing barrier every wave has passed).  At the end of step t each
    // wave waits until the weights of step t + 1 have landed: loads complete in
    // issue order, so it waits until no more are outstanding than it issued
    // after them (the weights of steps t + 2 .. t + kPD, and the input loads
    // issued at the start of this chunk if that was after them, i.e. when s <
    // kPD - 1), then passes the barrier that makes every wave's slots visible.
    // A fragments (input tile) of step s of the current chunk: k = 32 s + 8 g
    // within the chunk.  The shapes whose occupancy allows the 16 registers
    // read them one step ahead.
    constexpr bool kPrefA = NF == 6 || (NF == 3 && CC == 16);
    auto load_a = [&](int s, bf16x8 *a) {
        const int kc = s * 32 + 8 * g;
        const bool kv = kc < 9 * CC;
        const int tap = kv ? kc / CC : 0;
        const int ch = kc - tap * CC;
        const int off = ((tap / 3) * kHaloX + (tap - (tap / 3) * 3)) * kPitch + ch;
#pragma unroll
        for (int r = 0; r < kRF; ++r)
            a[r] = kv ? *(const bf16x8 *)(&sX[hbase[r] * kPitch + off]) : zero8();
    };
    bf16x8 an[kRF];
    bf16x8 vx[kXL];
    const int T = nchunks * kSteps;
#pragma unroll
    for (int i = 0; i < kPD; ++i)
        dma_w(0, i, i);
    order_fence();
    load_x(0, vx);
    store_x(vx);
    wait_vm_lds<0>();
    __builtin_amdgcn_s_barrier();
    int bcur = 0;
    for (int q = 0; q < nchunks; ++q) {
        const bool next_chunk = q + 1 < nchunks;
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const int t = q * kSteps + s;
            const int bnext = bcur == 0 ? kNB - 1 : bcur - 1;  // (t + kPD) % kNB
            order_fence();
            if (s == 0 && next_chunk)
                load_x(q + 1, vx);
            order_fence();
            if (t + kPD < T) {
                if (s + kPD < kSteps)
                    dma_w(q, s + kPD, bnext);
                else
                    dma_w(q + 1, s + kPD - kSteps, bnext);
            }
            order_fence();
            // A fragments of step s; with kPrefA those of step s + 1 of the
            // same chunk are read now too, to land during this step's MFMAs
            bf16x8 a[kRF];
            if constexpr (kPrefA) {
                if (s == 0)
                    load_a(0, a);
                else {
#pragma unroll
                    for (int r = 0; r < kRF; ++r)
                        a[r] = an[r];
                }
                if (s + 1 < kSteps)
                    load_a(s + 1, an);
            } else {
                load_a(s, a);
            }
            const unsigned char *sBc = smem + kXBytes + bcur * kBBytes;
#pragma unroll
            for (int c = 0; c < NF; ++c) {
                const bf16x8 bfr = *(const bf16x8 *)(sBc + ((c * 16 + r16) * 5 + g) * 16);
#pragma unroll
                for (int r = 0; r < kRF; ++r)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bfr, acc[r][c], 0, 0, 0);
            }
            order_fence();
            // weights issued after those of step t + 1 (steps t + 2 .. t + kPD)
            const int nw = (t + 2 < T ? 1 : 0) + (kPD == 3 && t + 3 < T ? 1 : 0);
            if (next_chunk && s < kPD - 1) {
                if (nw == 2)
                    wait_vm_lds<2 * kD + kXL>();
                else if (nw == 1)
                    wait_vm_lds<kD + kXL>();
                else
                    wait_vm_lds<kXL>();
            } else {
                if (nw == 2)
                    wait_vm_lds<2 * kD>();
                else if (nw == 1)
                    wait_vm_lds<kD>();
                else
                    wait_vm_lds<0>();
            }
            __builtin_amdgcn_s_barrier();
            bcur = bcur == kNB - 1 ? 0 : bcur + 1;
        }
        if (next_chunk) {
            // every wave has read this chunk's tile (barrier above)
            store_x(vx);
            wait_lds();
            __builtin_amdgcn_s_barrier();
        }
    }

    // float32 outputs (the network's last layer: 15 channels, 60-byte pixels)
    // are stored directly, element by element: staging them costs that
    // kernel an occupancy step and saves nothing measurable.
    if constexpr (F32OUT && NF == 1) {
        if (io.planar) {
            // stage the tile [pixel][16 channels] (the last step's barrier
            // ended every read of the staging buffers), then one thread per
            // pixel: planar stores, residual = channel + f, identity term
#pragma unroll
            for (int r = 0; r < kRF; ++r) {
                const int ly = RPW * wave + (r >> 1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int lx = 16 * (r & 1) + 4 * g + i;
                    float v = acc[r][0][i] + (bias && r16 < Cout ? bias[r16] : 0.f);
                    if (relu)
                        v = v > 0.f ? v : 0.f;
                    if (oscale && r16 < Cout)
                        v *= oscale[r16];
                    *(float *)(smem + (ly * kTileX + lx) * kPlanarPitch + 4 * r16) = v;
                }
            }
            __syncthreads();
            __shared__ double s_red[WAVES];
            double sum = 0.0;
            const size_t HWs = (size_t)H * W;
            for (int pix = threadIdx.x; pix < kTilePix; pix += kNT) {
                const int ly = pix / kTileX;
                const int yy = y0 + ly;
                const int xx = x0 + pix - ly * kTileX;
                if (yy >= H || xx >= W)
                    continue;
                const size_t q = (size_t)yy * W + xx;
                const float *t = (const float *)(smem + pix * kPlanarPitch);
                float v[16];
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    v[k] = t[k];
                float *ob = io.planar + (size_t)b * 15 * HWs + q;
#pragma unroll
                for (int c = 0; c < 12; ++c)
                    ob[(size_t)c * HWs] = v[c];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float fc = io.fout[((size_t)b * 3 + c) * HWs + q];
                    const float rc = v[12 + c] + fc;
                    ob[(size_t)(12 + c) * HWs] = rc;
                    float d = fc;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        d -= v[3 * j + c];
                    d -= rc;
                    sum += fabsf(d);
                }
            }
            if (io.ipart) {
                for (int off = 32; off > 0; off >>= 1)
                    sum += __shfl_xor(sum, off, 64);
                if (lane == 0)
                    s_red[wave] = sum;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double tot = s_red[0];
                    for (int w = 1; w < WAVES; ++w)
                        tot += s_red[w];
                    io.ipart[tile] = tot;
                }
            }
            return;
        }
    }
    if constexpr (F32OUT) {
#pragma unroll
        for (int c = 0; c < NF; ++c) {
            const int co = co0 + c * 16 + r16;
            if (co >= Cout)
                continue;
            const float bv = bias ? bias[co] : 0.f;
            const float sv = oscale ? oscale[co] : 1.f;
#pragma unroll
            for (int r = 0; r < kRF; ++r) {
                const int yy = y0 + RPW * wave + (r >> 1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xx = x0 + 16 * (r & 1) + 4 * g + i;
                    if (yy >= H || xx >= W)
                        continue;
                    const size_t p = ((size_t)b * H + yy) * W + xx;
                    float v = acc[r][c][i] + bv;
                    if (relu)
                        v = v > 0.f ? v : 0.f;
                    if (mask && !((float)mask[p * Cout + co] > 0.f))
                        v = 0.f;
                    if (oscale)
                        v *= sv;
                    ((float *)Y)[p * Cout + co] = v;
                }
            }
        }
        return;
    }
    // bf16 outputs: epilogue in two phases.  (1) Every lane finishes its fragment values
    // (bias, ReLU, mask, scale) and writes them to an LDS tile [pixel][channel]
    // whose pixel pitch is an odd number of 16-byte units, so the four pixels
    // one write instruction covers fall in distinct banks.  (2) The tile
    // leaves in 16-byte pieces of consecutive channels of a pixel (whole rows
    // of consecutive memory when the workgroup holds every channel), or
    // element by element when the channel counts do not allow 16-byte pieces.
    // The last step's barrier ended every read of the staging buffers.  Without
    // an output scale, a ReLU mask is applied in (2) to whole 16-byte pieces,
    // read beside the output (same layout), instead of element by element in
    // (1): the masked elements become +0 either way.
    const int nch = Cout - co0 < kOC ? Cout - co0 : kOC;
    const bool wide = nch == kOC && (Cout * (int)sizeof(OutT)) % 16 == 0 && ((uintptr_t)Y & 15) == 0;
    const bool late_mask = mask && !oscale && wide && ((uintptr_t)mask & 15) == 0;
#pragma unroll
    for (int c = 0; c < NF; ++c) {
        const int ch = c * 16 + r16;
        const int co = co0 + ch;
        if (co >= Cout)
            continue;
        const float bv = bias ? bias[co] : 0.f;
        const float sv = oscale ? oscale[co] : 1.f;
#pragma unroll
        for (int r = 0; r < kRF; ++r) {
            const int ly = RPW * wave + (r >> 1);
            const int yy = y0 + ly;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int lx = 16 * (r & 1) + 4 * g + i;
                const int xx = x0 + lx;
                if (yy >= H || xx >= W)
                    continue;
                float v = acc[r][c][i] + bv;
                if (relu)
                    v = v > 0.f ? v : 0.f;
                if (mask && !late_mask && !((float)mask[(((size_t)b * H + yy) * W + xx) * Cout + co] > 0.f))
                    v = 0.f;
                if (oscale)
                    v *= sv;
                *(OutT *)(smem + (ly * kTileX + lx) * kOPitch + ch * (int)sizeof(OutT)) = (OutT)v;
            }
        }
    }
    __syncthreads();
    OutT *const Yt = (OutT *)Y;
    if (wide) {
        constexpr int kG = kOC * (int)sizeof(OutT) / 16;  // 16-byte pieces per pixel (co0 keeps them aligned)
        for (int e = threadIdx.x; e < kTilePix * kG; e += kNT) {
            const int pix = e / kG;
            const int j = e - pix * kG;
            const int ly = pix / kTileX;
            const int lx = pix - ly * kTileX;
            const int yy = y0 + ly;
            const int xx = x0 + lx;
            if (yy < H && xx < W) {
                const size_t o = (((size_t)b * H + yy) * W + xx) * Cout + co0;  // element offset of the pixel's block
                bf16x8 v = *(const bf16x8 *)(smem + pix * kOPitch + 16 * j);
                if (late_mask) {
                    const bf16x8 mv = *(const bf16x8 *)((const unsigned char *)(mask + o) + 16 * j);
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (!((float)mv[k] > 0.f))
                            v[k] = (__bf16)0.0f;
                }
                *(bf16x8 *)((unsigned char *)(Yt + o) + 16 * j) = v;
            }
        }
        if (Ypool) {
            // 2 x 2 max pooling of the staged tile (8 x 32 -> 4 x 16 pixels), as
            // k_maxpool takes it: the window's four values in row-major order,
            // compared in float (host: H, W even, no mask, every channel block full)
            constexpr int kPX = kTileX / 2;
            constexpr int kPY = CS::kTileY / 2;
            const int H2 = H / 2, W2 = W / 2;
            for (int e = threadIdx.x; e < kPY * kPX * kG; e += kNT) {
                const int pp = e / kG;
                const int j = e - pp * kG;
                const int py = pp / kPX;
                const int px = pp - py * kPX;
                const int yy = y0 / 2 + py;
                const int xx = x0 / 2 + px;
                if (yy < H2 && xx < W2) {
                    const unsigned char *t = smem + (2 * py * kTileX + 2 * px) * kOPitch + 16 * j;
                    bf16x8 m = *(const bf16x8 *)t;
                    const bf16x8 v1 = *(const bf16x8 *)(t + kOPitch);
                    const bf16x8 v2 = *(const bf16x8 *)(t + kTileX * kOPitch);
                    const bf16x8 v3 = *(const bf16x8 *)(t + (kTileX + 1) * kOPitch);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        float a = (float)m[k];
                        a = (float)v1[k] > a ? (float)v1[k] : a;
                        a = (float)v2[k] > a ? (float)v2[k] : a;
                        a = (float)v3[k] > a ? (float)v3[k] : a;
                        m[k] = (__bf16)a;
                    }
                    *(bf16x8 *)(Ypool + (((size_t)b * H2 + yy) * W2 + xx) * Cout + co0 + 8 * j) = m;
                }
            }
        }
    } else {
        for (int e = threadIdx.x; e < kTilePix * nch; e += kNT) {
            const int pix = e / nch;
            const int ch = e - pix * nch;
            const int ly = pix / kTileX;
            const int lx = pix - ly * kTileX;
            const int yy = y0 + ly;
            const int xx = x0 + lx;
            if (yy < H && xx < W)
                Yt[(((size_t)b * H + yy) * W + xx) * Cout + co0 + ch] =
                    *(const OutT *)(smem + pix * kOPitch + ch * (int)sizeof(OutT));
        }
    }
}

// Weights for the input gradient: Wd[c][tap][o] = W[o][8 - tap][c].
__global__ __launch_bounds__(kT) void k_flip_transpose(const __bf16 *__restrict__ W, __bf16 *__restrict__ Wd,
                                                       int Cout, int Cin)
{
    const size_t n = (size_t)Cout * 9 * Cin;
    for (size_t q = (size_t)blockIdx.x * kT + threadIdx.x; q < n; q += (size_t)gridDim.x * kT) {
        const int c = (int)(q % Cin);
        const int tap = (int)((q / Cin) % 9);
        const int o = (int)(q / ((size_t)9 * Cin));
        Wd[((size_t)c * 9 + (8 - tap)) * Cout + o] = W[q];
    }
}

// ---------------------------------------------------------------------------
// weight gradient
//
// dW[o][tap][c] = sum over pixels p of dY[p][o] X[p + offset(tap)][c]: a
// GEMM whose reduction index is the pixel.  A workgroup of WC waves owns
// 16 OW output channels x 16 WC input channels x all 9 taps and walks a
// range of pixel tiles (kGR rows x kGC columns of one image).  Per tile,
// the dY tile and the X tile with its one-pixel halo are staged in LDS once,
// channels-last as they are stored (16-byte pieces, from registers loaded
// one tile ahead), and every tap's operand is the X tile read at that tap's
// shift: each X value leaves L2 about 1.6 times per tile instead of 9.
//
// The MFMA operands need 8 consecutive pixels of one channel per lane, the
// transpose of that layout; ds_read_b64_tr_b16 (gfx950) delivers it.  In
// each group of 16 lanes it gives lane 4a + e, in slot j, element e of the 8
// bytes addressed by lane a + 4j.  So lane s of group g addresses pixel
// 8g + (s >> 2) (+ 4 for the operand's upper half) at the 4-channel piece
// s & 3 of a 16-channel fragment, and receives fragment row s at pixels
// 8g .. 8g + 3 (+ 4): exactly the operand layout of
// v_mfma_f32_16x16x32_bf16.  The 4 pixels of one group sit at a pitch that
// is an odd multiple of 32 bytes, so their 32-byte pieces fall in distinct
// banks.
//
// Wave w owns input channels 16 w .. 16 w + 15 of the tile: per pixel row
// it reads OW dY fragments and 9 shifted X fragments for 9 OW MFMAs.  The
// workgroups of the first channel tile also form the bias gradient (the sum
// of dY over the pixels) on wave 0, as products with a fragment of ones.
// Per-range partial sums are added in a fixed order by k_reduce_rows
// (deterministic).
constexpr int kGR = 4;          // pixel rows per tile
constexpr int kGC = 32;         // pixel columns per tile: one 32-wide MFMA k step per row
constexpr int kGHX = kGC + 2;   // X tile columns with the halo

typedef short short4v __attribute__((ext_vector_type(4)));
typedef short short8v __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) short4v lds_short4;

// One MFMA operand from two transposed reads, 4 pixel rows apart.
__device__ __forceinline__ bf16x8 tr_operand(const lds_u8 *p, int half)
{
    const short4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_short4 *)p);
    const short4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_short4 *)(p + half));
    const short8v v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, v);
}

// CAT: X is the concatenation [upsampled Xlow, X] of a decoder level, read in
// place (a separate instantiation, so the other layers keep the registers
// its addressing costs).
template <int OW, int WC, bool CAT>
__global__ __launch_bounds__(64 * WC, 2) void k_wgrad(const __bf16 *__restrict__ X, const __bf16 *__restrict__ dY,
                                                   float *__restrict__ part, size_t rs, int with_bias, int H, int W,
                                                   int Cin, int Cout, int n_ct, int tiles_x, int tiles_y, int tiles,
                                                   int tpr, const __bf16 *__restrict__ Xlow, int Clow)
{
    constexpr int kNT = 64 * WC;
    constexpr int kOT = 16 * OW;               // output channels of the workgroup
    constexpr int kCT = 16 * WC;               // input channels of the workgroup
    constexpr int kYP = 32 * (OW | 1);         // LDS bytes per pixel, dY tile
    constexpr int kXP = 32 * (WC | 1);         // LDS bytes per pixel, X tile
    constexpr int kYG = kOT / 8;               // 16-byte pieces per pixel
    constexpr int kXG = kCT / 8;
    constexpr int kYPix = kGR * kGC;
    constexpr int kXPix = (kGR + 2) * kGHX;
    constexpr int kYItems = kYPix * kYG;
    constexpr int kXItems = kXPix * kXG;
    constexpr int kYPer = (kYItems + kNT - 1) / kNT;
    constexpr int kXPer = (kXItems + kNT - 1) / kNT;
    constexpr int kYBytes = kYPix * kYP;
    __shared__ __attribute__((aligned(16))) unsigned char smem[kYBytes + kXPix * kXP];
    const lds_u8 *const sY = (const lds_u8 *)smem;
    const lds_u8 *const sX = sY + kYBytes;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r16 = lane & 15;
    const int g = lane >> 4;
    const int ct = blockIdx.x % n_ct;
    const int c0 = ct * kCT;
    const int o0 = (blockIdx.x / n_ct) * kOT;
    const int s = blockIdx.y;
    const int t0 = s * tpr;
    const int t1 = min(tiles, t0 + tpr);
    const int K = 9 * Cin;
    const bool do_bias = with_bias && ct == 0 && wave == 0;

    floatx4 acc[OW][9];
    floatx4 bacc[OW];
#pragma unroll
    for (int f = 0; f < OW; ++f) {
        bacc[f] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
            acc[f][tap] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    bf16x8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        ones[j] = (__bf16)1.0f;

    // tile t: image t / (tiles_y tiles_x), rows kGR ty .., columns kGC tx ..;
    // pieces outside the image or past the channel counts are zero
    bf16x8 vy[kYPer], vx[kXPer];
    auto load = [&](int t) {
        const int tx = t % tiles_x;
        const int ty = (t / tiles_x) % tiles_y;
        const int b = t / (tiles_x * tiles_y);
        const int y0 = ty * kGR;
        const int x0 = tx * kGC;
#pragma unroll
        for (int j = 0; j < kYPer; ++j) {
            const int i = threadIdx.x + j * kNT;
            const __bf16 *src = (const __bf16 *)kZero16;
            if (i < kYItems) {
                const int pix = i / kYG;
                const int grp = i - pix * kYG;
                const int r = pix / kGC;
                const int yy = y0 + r;
                const int xx = x0 + pix - r * kGC;
                const int o = o0 + 8 * grp;
                if (yy < H && xx < W && o < Cout)
                    src = dY + ((size_t)((size_t)b * H + yy) * W + xx) * Cout + o;
            }
            vy[j] = *(const global_bf16x8 *)src;
        }
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int i = threadIdx.x + j * kNT;
            const __bf16 *src = (const __bf16 *)kZero16;
            if (i < kXItems) {
                const int pix = i / kXG;
                const int grp = i - pix * kXG;
                const int hr = pix / kGHX;
                const int yy = y0 + hr - 1;
                const int xx = x0 + pix - hr * kGHX - 1;
                const int c = c0 + 8 * grp;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W && c < Cin) {
                    if constexpr (CAT) {
                        if (c < Clow)  // the upsampled half of the concatenation
                            src = Xlow + ((size_t)((size_t)b * (H / 2) + yy / 2) * (W / 2) + xx / 2) * Clow + c;
                        else
                            src = X + ((size_t)((size_t)b * H + yy) * W + xx) * (Cin - Clow) + (c - Clow);
                    } else {
                        src = X + ((size_t)((size_t)b * H + yy) * W + xx) * Cin + c;
                    }
                }
            }
            vx[j] = *(const global_bf16x8 *)src;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < kYPer; ++j) {
            const int i = threadIdx.x + j * kNT;
            if (i < kYItems) {
                const int pix = i / kYG;
                *(bf16x8 *)(smem + pix * kYP + 16 * (i - pix * kYG)) = vy[j];
            }
        }
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int i = threadIdx.x + j * kNT;
            if (i < kXItems) {
                const int pix = i / kXG;
                *(bf16x8 *)(smem + kYBytes + pix * kXP + 16 * (i - pix * kXG)) = vx[j];
            }
        }
    };

    // this lane's transposed-read addresses: pixel 8 g + (r16 >> 2) of a row
    // step, 4-channel piece r16 & 3 of a fragment
    const int kp = 8 * g + (r16 >> 2);
    const int cq = 8 * (r16 & 3);
    const lds_u8 *const pY = sY + kp * kYP + cq;
    const lds_u8 *const pX = sX + kp * kXP + 32 * wave + cq;

    if (t0 < t1)
        load(t0);
    for (int t = t0; t < t1; ++t) {
        store();
        __syncthreads();
        if (t + 1 < t1)
            load(t + 1);
#pragma unroll 1
        for (int r = 0; r < kGR; ++r) {
            bf16x8 a[OW];
#pragma unroll
            for (int f = 0; f < OW; ++f)
                a[f] = tr_operand(pY + r * kGC * kYP + 32 * f, 4 * kYP);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3;
                const int dx = tap - 3 * dy;
                const bf16x8 bx = tr_operand(pX + ((r + dy) * kGHX + dx) * kXP, 4 * kXP);
#pragma unroll
                for (int f = 0; f < OW; ++f)
                    acc[f][tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], bx, acc[f][tap], 0, 0, 0);
            }
            if (do_bias) {
#pragma unroll
                for (int f = 0; f < OW; ++f)
                    bacc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], ones, bacc[f], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // result lane layout: column r16 (input channel), rows 4 g .. 4 g + 3
    // (output channels) of each fragment
    // range s's row of the partial sums: the weight gradient [o][tap][c],
    // then (with_bias) the bias gradient [o]
    float *const out = part + (size_t)s * rs;
    const int c = c0 + 16 * wave + r16;
    if (c < Cin) {
#pragma unroll
        for (int f = 0; f < OW; ++f)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = o0 + 16 * f + 4 * g + i;
                if (o < Cout) {
#pragma unroll
                    for (int tap = 0; tap < 9; ++tap)
                        out[(size_t)o * K + tap * Cin + c] = acc[f][tap][i];
                }
            }
    }
    if (do_bias && r16 == 0) {
#pragma unroll
        for (int f = 0; f < OW; ++f)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = o0 + 16 * f + 4 * g + i;
                if (o < Cout)
                    out[(size_t)Cout * K + o] = bacc[f][i];
            }
    }
}

// Fixed-order sum of the rows of part [ns][n] (n a multiple of 4, part
// 16-byte aligned), in two stages so that narrow, tall partial arrays still
// fill the device:
//   stage 1 (k_reduce_groups): row g kRowGroup of part <- the sum of rows
//   g kRowGroup .. g kRowGroup + kRowGroup - 1 in order (in place; blockIdx.y
//   is the group g; each thread owns 4 consecutive columns);
//   stage 2 (k_reduce_rows): out[q] = sum over groups g in order of row
//   g kRowGroup (with one group, stage 1 is skipped and this is the plain
//   sum over rows).
constexpr int kRowGroup = 16;

__global__ __launch_bounds__(kT) void k_reduce_groups(float *__restrict__ part, int ns, size_t n)
{
    const int g = blockIdx.y;
    const int s0 = g * kRowGroup;
    const int s1 = min(ns, s0 + kRowGroup);
    const size_t n4 = n / 4;
    for (size_t q = (size_t)blockIdx.x * kT + threadIdx.x; q < n4; q += (size_t)gridDim.x * kT) {
        float4 a = ((const float4 *)(part + (size_t)s0 * n))[q];
        for (int s = s0 + 1; s < s1; ++s) {
            const float4 v = ((const float4 *)(part + (size_t)s * n))[q];
            a.x += v.x;
            a.y += v.y;
            a.z += v.z;
            a.w += v.w;
        }
        ((float4 *)(part + (size_t)s0 * n))[q] = a;
    }
}

// Where stage 2 puts column q of a weight-gradient row ([cout][9][cin], then
// the bias [cout]): into dw / db as they are, or into a layer's slice of the
// flat parameter gradient (weights [cout_r][9][cin_r] then bias [cout_r],
// the padding channels dropped).
struct RowOut {
    float *dw = nullptr, *db = nullptr, *flat = nullptr;
    size_t nw = 0;  // weight columns (cout 9 cin)
    int cin = 0, cin_r = 0, cout_r = 0;
};

__device__ __forceinline__ void put_col(const RowOut &w, size_t q, float v)
{
    if (!w.flat) {
        if (q < w.nw)
            w.dw[q] = v;
        else
            w.db[q - w.nw] = v;
        return;
    }
    if (q < w.nw) {
        const int c = (int)(q % w.cin);
        const int tap = (int)((q / w.cin) % 9);
        const int o = (int)(q / ((size_t)9 * w.cin));
        if (o < w.cout_r && c < w.cin_r)
            w.flat[((size_t)o * 9 + tap) * w.cin_r + c] = v;
    } else {
        const int o = (int)(q - w.nw);
        if (o < w.cout_r)
            w.flat[(size_t)w.cout_r * 9 * w.cin_r + o] = v;
    }
}

__global__ __launch_bounds__(kT) void k_reduce_rows(const float *__restrict__ part, int ns, int stride, size_t n,
                                                    RowOut out)
{
    const size_t n4 = n / 4;
    for (size_t q = (size_t)blockIdx.x * kT + threadIdx.x; q < n4; q += (size_t)gridDim.x * kT) {
        float4 a = ((const float4 *)part)[q];
        for (int s = stride; s < ns; s += stride) {
            const float4 v = ((const float4 *)(part + (size_t)s * n))[q];
            a.x += v.x;
            a.y += v.y;
            a.z += v.z;
            a.w += v.w;
        }
        put_col(out, 4 * q, a.x);
        put_col(out, 4 * q + 1, a.y);
        put_col(out, 4 * q + 2, a.z);
        put_col(out, 4 * q + 3, a.w);
    }
}

// ---------------------------------------------------------------------------
// layout, pooling, upsampling

// f [B][3][H][W] float -> x [B][H][W][8] bf16 holding 2 f - 1 (the input
// centred on zero, f in [0, 1] -> [-1, 1]), channels 3..7 zero.
__global__ __launch_bounds__(kT) void k_pack_input(const float *__restrict__ f, __bf16 *__restrict__ x, int B,
                                                   int H, int W)
{
    const long long HW = (long long)H * W;
    const long long P = B * HW;
    for (long long p = (long long)blockIdx.x * kT + threadIdx.x; p < P; p += (long long)gridDim.x * kT) {
        const long long b = p / HW;
        const long long q = p - b * HW;
        bf16x8 v = zero8();
#pragma unroll
        for (int c = 0; c < 3; ++c)
            v[c] = (__bf16)(2.f * f[(b * 3 + c) * HW + q] - 1.f);
        *(bf16x8 *)(x + (size_t)p * 8) = v;
    }
}

// 2x2 max pooling of [B][H][W][C] (C % 8 == 0).
__global__ __launch_bounds__(kT) void k_maxpool(const __bf16 *__restrict__ x, __bf16 *__restrict__ y, int B, int H,
                                                int W, int C)
{
    const int h = H / 2, w = W / 2, cg = C / 8;
    const long long n = (long long)B * h * w * cg;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < n; q += (long long)gridDim.x * kT) {
        const int c8 = (int)(q % cg);
        const long long o = q / cg;
        const int j = (int)(o % w);
        const int i = (int)((o / w) % h);
        const long long b = o / ((long long)w * h);
        const __bf16 *base = x + ((size_t)(b * H + 2 * i) * W + 2 * j) * C + c8 * 8;
        bf16x8 m = *(const bf16x8 *)base;
        const bf16x8 v1 = *(const bf16x8 *)(base + C);
        const bf16x8 v2 = *(const bf16x8 *)(base + (size_t)W * C);
        const bf16x8 v3 = *(const bf16x8 *)(base + (size_t)W * C + C);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            float a = (float)m[t];
            a = (float)v1[t] > a ? (float)v1[t] : a;
            a = (float)v2[t] > a ? (float)v2[t] : a;
            a = (float)v3[t] > a ? (float)v3[t] : a;
            m[t] = (__bf16)a;
        }
        *(bf16x8 *)(y + (size_t)o * C + c8 * 8) = m;
    }
}

// dx += dy routed to each window's first maximum (row-major window order),
// then dx *= (x > 0) over the window (the ReLU of the layer producing x).
__global__ __launch_bounds__(kT) void k_maxpool_bwd(const __bf16 *__restrict__ x, const __bf16 *__restrict__ dy,
                                                    __bf16 *__restrict__ dx, int B, int H, int W, int C)
{
    const int h = H / 2, w = W / 2;
    const long long n = (long long)B * h * w * C;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < n; q += (long long)gridDim.x * kT) {
        const int c = (int)(q % C);
        const long long o = q / C;
        const int j = (int)(o % w);
        const int i = (int)((o / w) % h);
        const long long b = o / ((long long)w * h);
        size_t idx[4];
        idx[0] = ((size_t)(b * H + 2 * i) * W + 2 * j) * C + c;
        idx[1] = idx[0] + C;
        idx[2] = idx[0] + (size_t)W * C;
        idx[3] = idx[2] + C;
        int am = 0;
        float mv = (float)x[idx[0]];
#pragma unroll
        for (int t = 1; t < 4; ++t) {
            const float v = (float)x[idx[t]];
            if (v > mv) {
                mv = v;
                am = t;
            }
        }
        const float g = (float)dy[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float v = (float)dx[idx[t]] + (t == am ? g : 0.f);
            if (!((float)x[idx[t]] > 0.f))
                v = 0.f;
            dx[idx[t]] = (__bf16)v;
        }
    }
}

// Gradient of the concatenation [nearest-upsampled low, skip] in its two
// sources: dlow = (sum of the 4 children's first C1 channels) * (low > 0),
// dskip = (last C2 channels) * (skip > 0).
__global__ __launch_bounds__(kT) void k_up_concat_bwd(const __bf16 *__restrict__ dcat, const __bf16 *__restrict__ low,
                                                      const __bf16 *__restrict__ skip, __bf16 *__restrict__ dlow,
                                                      __bf16 *__restrict__ dskip, int B, int H, int W, int C1, int C2)
{
    const int C = C1 + C2;
    const int h = H / 2, w = W / 2;
    const long long nl = (long long)B * h * w * C1;
    const long long ns = (long long)B * H * W * C2;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < nl + ns; q += (long long)gridDim.x * kT) {
        if (q < nl) {
            const int c = (int)(q % C1);
            const long long o = q / C1;
            const int j = (int)(o % w);
            const int i = (int)((o / w) % h);
            const long long b = o / ((long long)w * h);
            const size_t base = ((size_t)(b * H + 2 * i) * W + 2 * j) * C + c;
            float a = (float)dcat[base] + (float)dcat[base + C];
            a += (float)dcat[base + (size_t)W * C] + (float)dcat[base + (size_t)W * C + C];
            dlow[q] = (__bf16)((float)low[q] > 0.f ? a : 0.f);
        } else {
            const long long r = q - nl;
            const int c = (int)(r % C2);
            const long long p = r / C2;
            const float v = (float)dcat[(size_t)p * C + C1 + c];
            dskip[r] = (__bf16)((float)skip[r] > 0.f ? v : 0.f);
        }
    }
}

// ---------------------------------------------------------------------------
// loss

constexpr int kOutC = TVSPEC_NET_OUT_CHANNELS;  // 15
constexpr int kOutPad = 16;                       // channels of the last layer's output
constexpr int kGroups = TVSPEC_NET_BANDS + 1;     // 4 bands + residual, 3 channels each

// t [P][16] float from bands [B][4][3][H][W] and residual [B][3][H][W]
// (float64).  The residual output is f plus the last layer's channels 12..14,
// so those channels are trained towards r - f (the sign-flipped sum of the
// bands), computed here in float64 before the rounding.
__global__ __launch_bounds__(kT) void k_pack_target(const double *__restrict__ bands, const double *__restrict__ res,
                                                    const float *__restrict__ f, float *__restrict__ t, int B,
                                                    long long HW)
{
    const long long P = B * HW;
    for (long long p = (long long)blockIdx.x * kT + threadIdx.x; p < P; p += (long long)gridDim.x * kT) {
        const long long b = p / HW;
        const long long q = p - b * HW;
        float *tp = t + (size_t)p * kOutPad;
        for (int j = 0; j < TVSPEC_NET_BANDS; ++j)
            for (int c = 0; c < 3; ++c)
                tp[3 * j + c] = (float)bands[((b * TVSPEC_NET_BANDS + j) * 3 + c) * HW + q];
        for (int c = 0; c < 3; ++c)
            tp[12 + c] = (float)(res[(b * 3 + c) * HW + q] - (double)f[(b * 3 + c) * HW + q]);
        tp[15] = 0.f;
    }
}

__device__ __forceinline__ double block_sum_d(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// err[b] = (sum of part[b][0..nblk)) / (3 HW), one block per image: thread
// t adds entries t, t + 256, ... in order, then the block's fixed-order
// tree (so the value is deterministic; a megapixel image has 16384 tile
// partials, which one thread alone adds too slowly).  Grid (B).
__global__ __launch_bounds__(kT) void k_identity_total(const double *__restrict__ part, int nblk, long long HW,
                                                       float *__restrict__ err)
{
    __shared__ double sh[kT / 64];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kT)
        s += part[(size_t)b * nblk + k];
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0)
        err[b] = (float)(s / (3.0 * (double)HW));
}

__device__ __forceinline__ float block_sum(float v, float *sh)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// part[b][j][blk][2] = block sums of (o - t)^2 and t^2 over band j of image b.
__global__ __launch_bounds__(kT) void k_loss_partial(const float *__restrict__ o, const float *__restrict__ t,
                                                     long long HW, float *__restrict__ part)
{
    __shared__ float sh[4];
    const int b = blockIdx.y;
    const int nblk = gridDim.x;
    float num[kGroups], den[kGroups];
#pragma unroll
    for (int j = 0; j < kGroups; ++j)
        num[j] = den[j] = 0.f;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < HW; q += (long long)nblk * kT) {
        const float *op = o + (size_t)(b * HW + q) * kOutPad;
        const float *tp = t + (size_t)(b * HW + q) * kOutPad;
#pragma unroll
        for (int j = 0; j < kGroups; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float e = op[3 * j + c] - tp[3 * j + c];
                num[j] += e * e;
                den[j] += tp[3 * j + c] * tp[3 * j + c];
            }
    }
#pragma unroll
    for (int j = 0; j < kGroups; ++j) {
        const float a = block_sum(num[j], sh);
        const float d = block_sum(den[j], sh);
        if (threadIdx.x == 0) {
            part[((size_t)(b * kGroups + j) * nblk + blockIdx.x) * 2] = a;
            part[((size_t)(b * kGroups + j) * nblk + blockIdx.x) * 2 + 1] = d;
        }
    }
}

// nd[b][j][2] = totals (fixed order), the denominator raised by the floor
// kappa 3 HW scale_j^2 (the energy of a group whose RMS is its output
// scale); loss[0] = (1/(5B)) sum num/den.  One block: thread t totals the
// pairs t, t + 256, ...; the loss terms are then added in a fixed order.
__global__ __launch_bounds__(kT) void k_loss_total(const float *__restrict__ part, int B, int nblk,
                                                   const float *__restrict__ oscale, float kappa, long long HW,
                                                   float *__restrict__ nd, float *__restrict__ loss)
{
    __shared__ double sl[kT];
    double l = 0.0;
    for (int bj = threadIdx.x; bj < B * kGroups; bj += kT) {
        const double sj = oscale[3 * (bj % kGroups)];
        double a = 0.0, d = (double)kappa * 3.0 * (double)HW * sj * sj;
        for (int k = 0; k < nblk; ++k) {
            a += part[((size_t)bj * nblk + k) * 2];
            d += part[((size_t)bj * nblk + k) * 2 + 1];
        }
        nd[2 * bj] = (float)a;
        nd[2 * bj + 1] = (float)d;
        l += d > 0.0 ? a / d : 0.0;
    }
    sl[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kT; ++i)
            t += sl[i];
        loss[0] = (float)(t / (double)(B * kGroups));
    }
}

// do = 2 (o - t) / (den_bj 5 B) times the output scale of the channel (the
// gradient before the scale), as bf16 [P][16] (channel 15 zero).
__global__ __launch_bounds__(kT) void k_loss_grad(const float *__restrict__ o, const float *__restrict__ t,
                                                  const float *__restrict__ nd, const float *__restrict__ oscale,
                                                  int B, long long HW, __bf16 *__restrict__ dO)
{
    const long long n = B * HW * kOutPad;
    const float scale = 2.f / (float)(B * kGroups);
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < n; q += (long long)gridDim.x * kT) {
        const int c = (int)(q % kOutPad);
        const long long b = q / (HW * kOutPad);
        float v = 0.f;
        if (c < kOutC) {
            const float den = nd[2 * (b * kGroups + c / 3) + 1];
            v = den > 0.f ? scale * (o[q] - t[q]) / den * oscale[c] : 0.f;
        }
        dO[q] = (__bf16)v;
    }
}

// err[b] = mean over channels c and pixels of |f - sum_j band_j - residual|
// for out [B][15][H][W] (channel 3j + c band j, 12 + c residual) and f
// [B][3][H][W]: the reconstruction identity of the decomposition, Eq. (7),
// as the network's output satisfies it.  One block per image.
__global__ __launch_bounds__(kT) void k_identity_error(const float *__restrict__ f, const float *__restrict__ out,
                                                       long long HW, float *__restrict__ err)
{
    __shared__ float sh[4];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (long long q = threadIdx.x; q < 3 * HW; q += kT) {
        const int c = (int)(q / HW);
        const long long pix = q - c * HW;
        const float *ob = out + (size_t)b * kOutC * HW;
        float r = f[((size_t)b * 3 + c) * HW + pix];
        for (int j = 0; j < TVSPEC_NET_BANDS; ++j)
            r -= ob[(size_t)(3 * j + c) * HW + pix];
        r -= ob[(size_t)(12 + c) * HW + pix];
        acc += fabsf(r);
    }
    const float t = block_sum((float)acc, sh);
    if (threadIdx.x == 0)
        err[b] = t / (float)(3 * HW);
}

// ---------------------------------------------------------------------------
// parameters

// Adam on flat float32 arrays (Kingma and Ba, with bias correction).
// The gradient is multiplied by *gscale (the clipping factor, 1 without
// clipping) as it is read.
__global__ __launch_bounds__(kT) void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                             float *__restrict__ v, long long n, float lr, float b1, float b2,
                                             float eps, float c1, float c2, const float *__restrict__ gscale)
{
    const float gs = *gscale;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < n; q += (long long)gridDim.x * kT) {
        const float gq = g[q] * gs;
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
    }
}

// Gradient-norm clipping, deterministic: part[blk] = sum of g^2 over the
// block's grid-stride share (double), then one block totals the partials in
// order and sets
//   norm = sqrt(total);  avg <- norm on the first step;
//   scale = (clip > 0 and norm > clip avg) ? clip avg / norm : 1;
//   avg <- 0.99 avg + 0.01 min(norm, clip avg)  (clip > 0)
// state = {norm, avg, scale, steps} (float, float, float, float count).
constexpr int kNormBlocks = 512;

__global__ __launch_bounds__(kT) void k_sumsq(const float *__restrict__ g, long long n, double *__restrict__ part)
{
    __shared__ double sh[kT / 64];
    double a = 0.0;
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < n; q += (long long)gridDim.x * kT) {
        const double x = g[q];
        a += x * x;
    }
    const double t = block_sum_d(a, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = t;
}

__global__ __launch_bounds__(64) void k_clip_scale(const double *__restrict__ part, int nblk, float clip,
                                                   float *__restrict__ state)
{
    if (threadIdx.x != 0)
        return;
    double t = 0.0;
    for (int k = 0; k < nblk; ++k)
        t += part[k];
    const float norm = (float)sqrt(t);
    const bool first = state[3] == 0.f;
    float avg = first ? norm : state[1];
    float scale = 1.f;
    if (clip > 0.f) {
        const float lim = clip * avg;
        if (norm > lim && norm > 0.f)
            scale = lim / norm;
        avg = 0.99f * avg + 0.01f * fminf(norm, lim);
    }
    state[0] = norm;
    state[1] = avg;
    state[2] = scale;
    state[3] += 1.f;
}

// One layer's parameter shapes for k_requant_all.
struct LayerDev {
    long long off;   // its slice of the flat parameters: weights [cout_r][9][cin_r], then bias [cout_r]
    long long start; // its first element in the launch's index space (cout 9 cin + cout elements each)
    __bf16 *wq;      // [cout][9][cin] (padding channels zero)
    __bf16 *wd;      // [cin][9][cout], taps reversed: the input gradient's weights
    float *bias;     // [cout]
    int cout, cin, cout_r, cin_r;
};
constexpr int kMaxLayers = 16;

// From the float32 master parameters, for every layer at once: the bf16
// weights of the forward convolution, the same weights flipped and
// transposed for the input gradient (Wd[c][8 - tap][o] = W[o][tap][c]) and
// the float32 bias, each padded with zeros to the stored channel counts.
__global__ __launch_bounds__(kT) void k_requant_all(const float *__restrict__ master,
                                                    const LayerDev *__restrict__ tab, int nl, long long total)
{
    __shared__ LayerDev t[kMaxLayers];
    for (int i = threadIdx.x; i < nl; i += kT)
        t[i] = tab[i];
    __syncthreads();
    for (long long q = (long long)blockIdx.x * kT + threadIdx.x; q < total; q += (long long)gridDim.x * kT) {
        int li = 0;
        while (li + 1 < nl && t[li + 1].start <= q)
            ++li;
        const LayerDev &l = t[li];
        const long long e = q - l.start;
        const long long n = (long long)l.cout * 9 * l.cin;
        const float *wm = master + l.off;
        if (e < n) {
            const int c = (int)(e % l.cin);
            const int tap = (int)((e / l.cin) % 9);
            const int o = (int)(e / (9LL * l.cin));
            const __bf16 v = (__bf16)((o < l.cout_r && c < l.cin_r) ? wm[((size_t)o * 9 + tap) * l.cin_r + c] : 0.f);
            l.wq[e] = v;
            l.wd[((size_t)c * 9 + (8 - tap)) * l.cout + o] = v;
        } else {
            const int o = (int)(e - n);
            l.bias[o] = o < l.cout_r ? wm[(size_t)l.cout_r * 9 * l.cin_r + o] : 0.f;
        }
    }
}

int grid_for(long long n)
{
    long long b = (n + kT - 1) / kT;
    if (b < 1)
        b = 1;
    if (b > 65536)
        b = 65536;
    return (int)b;
}

// ---------------------------------------------------------------------------
// workspace shared by the raw convolution entry points and the network

struct Work {
    size_t part_bytes = 0;
    float *part = nullptr;
    size_t wd_bytes = 0;
    __bf16 *wd = nullptr;
};

int ensure(void **p, size_t *have, size_t bytes)
{
    if (*p && *have >= bytes)
        return TVSPEC_OK;
    if (*p)
        HIP_TRY(hipDeviceSynchronize());
    if (*p)
        (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    HIP_TRY(hipMalloc(p, bytes));
    *have = bytes;
    return TVSPEC_OK;
}

template <int NF, int CC, int WAVES, int RPW>
void conv_launch_w(const __bf16 *x, int B, int H, int W, int Cin, const __bf16 *w, const float *bias, int Cout,
                   int relu, const __bf16 *mask, void *y, bool f32, hipStream_t st, const float *oscale,
                   const __bf16 *xlow, int clow, __bf16 *ypool, const ConvIO &io)
{
    const int tiles_x = (W + kTileX - 1) / kTileX;
    constexpr int kTileY = RPW * WAVES;
    const int tiles_y = (H + kTileY - 1) / kTileY;
    const dim3 grid((unsigned)((long long)tiles_x * tiles_y * B), (unsigned)((Cout + NF * 16 - 1) / (NF * 16)));
    if (f32)
        hipLaunchKernelGGL((k_conv3x3<true, NF, CC, WAVES, RPW>), grid, dim3(64 * WAVES), 0, st, x, w, bias, mask, oscale,
                           y, B, H, W, Cin, Cout, relu, tiles_x, tiles_y, xlow, clow, nullptr, io);
    else
        hipLaunchKernelGGL((k_conv3x3<false, NF, CC, WAVES, RPW>), grid, dim3(64 * WAVES), 0, st, x, w, bias, mask,
                           oscale, y, B, H, W, Cin, Cout, relu, tiles_x, tiles_y, xlow, clow, ypool, io);
}

// Four waves per workgroup, two output rows per wave (8 x 32 pixel tiles):
// 8-wave workgroups (16 x 32) were measured slower on every layer of the
// network (half the workgroups per CU, barriers over twice the waves), and so
// were four rows per wave at NF 3 (fewer operand reads per MFMA, but 2
// instead of 3 waves per SIMD: forward pass 1.21 against 1.16 ms).
template <int NF, int CC>
void conv_launch(const __bf16 *x, int B, int H, int W, int Cin, const __bf16 *w, const float *bias, int Cout,
                 int relu, const __bf16 *mask, void *y, bool f32, hipStream_t st, const float *oscale,
                 const __bf16 *xlow, int clow, __bf16 *ypool, const ConvIO &io)
{
    conv_launch_w<NF, CC, 4, 2>(x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, ypool,
                                io);
}

// Column fragments per wave (NF) and input channels per LDS chunk (CC),
// chosen from measurements of every (NF, CC) on the network's layers: the
// widest chunk Cin allows (32, else 16, else 8) is fastest at every NF.  A
// wide layer (NF 6 or 4, 96 or 64 output channels per workgroup) whose Cin
// is not a multiple of 32 is narrowed to NF <= 3 (wide columns with narrow
// chunks were no faster and hold more registers), as is one whose image
// gives fewer than 512 workgroups.  NF divides Cout / 16 where it can.
void conv_shape(int B, int H, int W, int Cin, int Cout, int *nf, int *cc)
{
    const int n = (Cout + 15) / 16;
    int f = 1;
    for (int c : {6, 4, 3, 2})
        if (n % c == 0) {
            f = c;
            break;
        }
    if (n > 1 && f == 1)
        f = 6;  // partly empty last column block
    // a small image gives few pixel tiles: narrower column blocks double the
    // workgroups where wide ones would leave CUs idle
    const long long tiles = (long long)B * ((H + 7) / 8) * ((W + kTileX - 1) / kTileX);
    if (f >= 4 && tiles * ((n + f - 1) / f) < 512)
        f = n % 3 == 0 ? 3 : (n % 2 == 0 ? 2 : f);
    // wide column blocks need 32-channel chunks; the widest chunk the input
    // allows is the fastest at every width (measured per layer: NF 3 with
    // 32-channel chunks 10-18% faster than with 16)
    if (f >= 4 && Cin % 32 != 0)
        f = n % 3 == 0 ? 3 : (n % 2 == 0 ? 2 : 3);
    *nf = f;
    *cc = Cin % 32 == 0 ? 32 : (Cin % 16 == 0 ? 16 : 8);
}

template <int NF>
void conv_launch_cc(int cc, const __bf16 *x, int B, int H, int W, int Cin, const __bf16 *w, const float *bias,
                    int Cout, int relu, const __bf16 *mask, void *y, bool f32, hipStream_t st, const float *oscale,
                    const __bf16 *xlow, int clow, __bf16 *ypool, const ConvIO &io)
{
    switch (cc) {
    case 32: conv_launch<NF, 32>(x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, ypool, io); break;
    case 16: conv_launch<NF, 16>(x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, ypool, io); break;
    default: conv_launch<NF, 8>(x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, ypool, io); break;
    }
}

// With xlow != nullptr the input is the concatenation [nearest 2x upsampling
// of xlow ([B][H/2][W/2][clow]), x ([B][H][W][Cin - clow])] along channels,
// read in place (H, W even; clow a multiple of the chunk width, checked).
// With ypool != nullptr the 2 x 2 max pooling of y ([B][H/2][W/2][Cout],
// H and W even) is written too: by the convolution's epilogue where its
// tile allows (bf16, no mask, every channel block full, 16-byte aligned),
// else by k_maxpool afterwards; the values are the same either way.
int conv_fwd(const __bf16 *x, int B, int H, int W, int Cin, const __bf16 *w, const float *bias, int Cout, int relu,
             const __bf16 *mask, void *y, bool f32, hipStream_t st, const float *oscale = nullptr,
             const __bf16 *xlow = nullptr, int clow = 0, __bf16 *ypool = nullptr, const ConvIO &io = ConvIO())
{
    int nf = 1, cc = 8;
    conv_shape(B, H, W, Cin, Cout, &nf, &cc);
    if (io.planar && (!f32 || Cout != 16 || nf != 1 || !io.fout))
        return fail(TVSPEC_EINVAL, "planar network output: the last layer's shape only");
    if (xlow && (clow <= 0 || clow >= Cin || clow % cc != 0 || (Cin - clow) % 8 != 0 || H % 2 || W % 2))
        return fail(TVSPEC_EINVAL, "fused concatenation: chunk width must divide the low-resolution channels");
    if (ypool && (H % 2 || W % 2 || f32 || Cout % 8))
        return fail(TVSPEC_EINVAL, "pooled output: needs even H, W and bf16 output with Cout a multiple of 8");
    const bool fuse_pool = ypool && !mask && Cout % (nf * 16) == 0 && ((uintptr_t)y & 15) == 0 &&
                           ((uintptr_t)ypool & 15) == 0;
    __bf16 *yp = fuse_pool ? ypool : nullptr;
    switch (nf) {
    case 1: conv_launch_cc<1>(cc, x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, yp, io); break;
    case 2: conv_launch_cc<2>(cc, x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, yp, io); break;
    case 3: conv_launch_cc<3>(cc, x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, yp, io); break;
    case 4: conv_launch_cc<4>(cc, x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, yp, io); break;
    default: conv_launch_cc<6>(cc, x, B, H, W, Cin, w, bias, Cout, relu, mask, y, f32, st, oscale, xlow, clow, yp, io); break;
    }
    if (ypool && !fuse_pool) {
        const long long cnt = (long long)B * (H / 2) * (W / 2) * (Cout / 8);
        hipLaunchKernelGGL(k_maxpool, dim3(grid_for(cnt)), dim3(kT), 0, st, (const __bf16 *)y, ypool, B, H, W, Cout);
    }
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int conv_dgrad(Work &wk, const __bf16 *dy, int B, int H, int W, int Cout, const __bf16 *w, int Cin,
               const __bf16 *mask, __bf16 *dx, hipStream_t st)
{
    const size_t nw = (size_t)Cout * 9 * Cin;
    TVSPEC_TRY(ensure((void **)&wk.wd, &wk.wd_bytes, nw * sizeof(__bf16)));
    hipLaunchKernelGGL(k_flip_transpose, dim3(grid_for((long long)nw)), dim3(kT), 0, st, w, wk.wd, Cout, Cin);
    return conv_fwd(dy, B, H, W, Cout, wk.wd, nullptr, Cin, 0, mask, dx, false, st);
}

// Column q of the fixed-order sum of the ns rows of part [ns][n] goes where
// `out` says (overwrites part).
void reduce_rows(float *part, int ns, size_t n, const RowOut &out, hipStream_t st)
{
    const long long n4 = (long long)(n / 4);
    int stride = 1;
    if (ns > kRowGroup) {
        const int groups = (ns + kRowGroup - 1) / kRowGroup;
        hipLaunchKernelGGL(k_reduce_groups, dim3(grid_for(n4), groups), dim3(kT), 0, st, part, ns, n);
        stride = kRowGroup;
    }
    hipLaunchKernelGGL(k_reduce_rows, dim3(grid_for(n4)), dim3(kT), 0, st, part, ns, stride, n, out);
}

// Output and input channels per workgroup of the weight gradient: 16 OW and
// 16 WC with OW, WC in {1, 3, 4}, each the one that pads the channel count
// least (the larger on a tie); OW is then capped at WC, since the wider
// output tiles need the registers that fewer threads per workgroup spend on
// the next tile's loads.
int wgrad_width(int C)
{
    int best = 4, best_pad = 1 << 30;
    for (int m : {4, 3, 1}) {
        const int pad = (C + 16 * m - 1) / (16 * m) * 16 * m;
        if (pad < best_pad) {
            best = m;
            best_pad = pad;
        }
    }
    return best;
}

template <int OW, int WC>
void wgrad_launch(dim3 grid, const __bf16 *x, const __bf16 *dy, float *part, size_t rs, int with_bias, int H, int W,
                  int Cin, int Cout, int n_ct, int tiles_x, int tiles_y, int tiles, int tpr, const __bf16 *xlow,
                  int clow, hipStream_t st)
{
    if (xlow)
        hipLaunchKernelGGL((k_wgrad<OW, WC, true>), grid, dim3(64 * WC), 0, st, x, dy, part, rs, with_bias, H, W,
                           Cin, Cout, n_ct, tiles_x, tiles_y, tiles, tpr, xlow, clow);
    else
        hipLaunchKernelGGL((k_wgrad<OW, WC, false>), grid, dim3(64 * WC), 0, st, x, dy, part, rs, with_bias, H, W,
                           Cin, Cout, n_ct, tiles_x, tiles_y, tiles, tpr, xlow, clow);
}

// Weight gradient [Cout][9][Cin] and, with out.db or out.flat, the bias
// gradient, summed over the pixel ranges in one fixed-order reduction and
// written where `out` says (out.nw and out.cin are filled in here).  With
// xlow the input is the concatenation [nearest 2x upsampling of xlow
// ([B][H/2][W/2][clow]), x ([B][H][W][Cin - clow])], read in place (H, W
// even, clow a multiple of 8).
int conv_wgrad(Work &wk, const __bf16 *x, const __bf16 *dy, int B, int H, int W, int Cin, int Cout, RowOut out,
               hipStream_t st, const __bf16 *xlow = nullptr, int clow = 0)
{
    if (xlow && (clow <= 0 || clow >= Cin || clow % 8 || H % 2 || W % 2))
        return fail(TVSPEC_EINVAL, "weight gradient of a concatenated input: bad shapes");
    if (!xlow)
        clow = 0;
    const int WC = wgrad_width(Cin);
    const int OW = wgrad_width(Cout) > WC ? (WC == 1 ? 1 : 3) : wgrad_width(Cout);
    const int n_ot = (Cout + 16 * OW - 1) / (16 * OW);
    const int n_ct = (Cin + 16 * WC - 1) / (16 * WC);
    const int tiles_x = (W + kGC - 1) / kGC, tiles_y = (H + kGR - 1) / kGR;
    const long long tiles = (long long)B * tiles_x * tiles_y;
    const int K = 9 * Cin;
    const size_t n = (size_t)Cout * K;
    const int with_bias = (out.db || out.flat) ? 1 : 0;
    const size_t rs = n + (with_bias ? (size_t)Cout : 0);  // a multiple of 4 (Cin, Cout multiples of 8)
    out.nw = n;
    out.cin = Cin;
    const long long per_range = (long long)n_ot * n_ct;
    // pixel ranges: ~1024 workgroups in all, as long as the partial sums stay
    // within 64 MB, but at least enough to give every CU one workgroup
    long long ns = 1024 / per_range;
    const long long cap = (64LL << 20) / (long long)(rs * sizeof(float));
    ns = ns > cap ? cap : ns;
    const long long floor_ns = (256 + per_range - 1) / per_range;
    ns = ns < floor_ns ? floor_ns : ns;
    ns = ns > tiles ? tiles : ns;
    ns = ns < 1 ? 1 : ns;
    const long long tpr = (tiles + ns - 1) / ns;
    ns = (tiles + tpr - 1) / tpr;
    const size_t need = (size_t)ns * rs * sizeof(float);
    TVSPEC_TRY(ensure((void **)&wk.part, &wk.part_bytes, need));
    const dim3 grid((unsigned)per_range, (unsigned)ns);
    const int ti = (int)tiles, tp = (int)tpr;
#define TVSPEC_WG(ow, wc)                                                                                       \
    if (OW == ow && WC == wc)                                                                                   \
        wgrad_launch<ow, wc>(grid, x, dy, wk.part, rs, with_bias, H, W, Cin, Cout, n_ct, tiles_x, tiles_y, ti, tp, \
                             xlow, clow, st);
    TVSPEC_WG(1, 1) TVSPEC_WG(1, 3) TVSPEC_WG(1, 4) TVSPEC_WG(3, 3) TVSPEC_WG(3, 4) TVSPEC_WG(4, 4)
#undef TVSPEC_WG
    reduce_rows(wk.part, (int)ns, rs, out, st);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

std::mutex g_raw_mu;
std::map<int, Work> g_raw_work;  // per device

int raw_work(Work **wk)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    *wk = &g_raw_work[dev];
    return TVSPEC_OK;
}

// ---------------------------------------------------------------------------
// the network

struct Layer {
    const char *name;
    int cin_r, cout_r;   // real channel counts (parameter shapes)
    int cin, cout;       // as stored (input padded to 8, output to 16)
    long long off;       // offset of the weights in the flat parameter vector
    __bf16 *wq = nullptr;
    __bf16 *wd = nullptr;  // flipped, transposed copy for the input gradient
    float *bias = nullptr;
};

struct Act {
    __bf16 *a = nullptr;  // activation
    __bf16 *g = nullptr;  // its gradient
    int H = 0, W = 0, C = 0;
};

} // namespace
} // namespace nn
} // namespace tvspec

struct tvspec_net {
    int dev = 0;
    int H = 0, W = 0, maxB = 0;
    std::vector<tvspec::nn::Layer> L;
    long long nparams = 0;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    long long step = 0;
    float kappa = 0.f;        // loss denominator floor (0: the paper's loss)
    float gclip = 0.f;        // gradient-norm clip factor (0: off)
    double *gpart = nullptr;  // [kNormBlocks] sum-of-squares partials
    float *gstate = nullptr;  // {norm, running average, scale, steps}
    // activations: x0, e1a, e1b, p1, e2a, e2b, p2, e3a, e3b, p3, e4a, e4b, c3, d3a, d3b, c2, d2a, d2b, c1, d1a, d1b
    tvspec::nn::Act A[21];
    float *out = nullptr;     // [P][16]
    float *tgt = nullptr;     // [P][16]
    __bf16 *dout = nullptr;   // [P][16]
    float *lpart = nullptr, *nd = nullptr, *loss = nullptr;
    double *ipart = nullptr;  // [max_batch][otiles] identity-error partials
    float *oscale = nullptr;  // [16] output channel scales (1 by default)
    int lblk = 0;
    int otiles = 0;           // 8 x 32 output tiles per image (identity partials of the forward pass)
    tvspec::nn::LayerDev *ltab = nullptr;  // the layers' shapes for k_requant_all
    long long lcount = 0;                  // elements k_requant_all covers
    tvspec::nn::Work wk;
    std::vector<void *> allocs;
    std::mutex mu;
};

namespace tvspec {
namespace nn {
namespace {

enum { X0, E1A, E1B, P1, E2A, E2B, P2, E3A, E3B, P3, E4A, E4B, C3, D3A, D3B, C2, D2A, D2B, C1, D1A, D1B };

constexpr int kW0 = 48, kW1 = 96, kW2 = 192, kW3 = 384;

int net_alloc(tvspec_net *n, void **p, size_t bytes)
{
    HIP_TRY(hipMalloc(p, bytes));
    n->allocs.push_back(*p);
    return TVSPEC_OK;
}

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double normal(uint64_t &s)
{
    // Box-Muller on two uniforms in (0, 1]
    const double u1 = ((splitmix(s) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix(s) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

int requant_all(tvspec_net *n, hipStream_t st)
{
    hipLaunchKernelGGL(k_requant_all, dim3(grid_for(n->lcount)), dim3(kT), 0, st, n->master, n->ltab,
                       (int)n->L.size(), n->lcount);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

// The first decoder convolution of each level reads the upsampled lower
// level and the skip tensor in place (so does its weight gradient: no
// concatenated tensor is ever written).  training: leave the output in
// n->out ([P][16]); otherwise the last layer writes the planar output
// `planar` (with the identity partials into ipart[b][tile] unless ipart is
// null).
int forward(tvspec_net *n, const float *f, int B, hipStream_t st, bool training, float *planar = nullptr,
            double *ipart = nullptr)
{
    Act *A = n->A;
    const int H = n->H, W = n->W;
    hipLaunchKernelGGL(k_pack_input, dim3(grid_for((long long)B * H * W)), dim3(kT), 0, st, f, A[X0].a, B, H, W);
    auto conv = [&](int li, int in, int out) {
        const Layer &l = n->L[li];
        return conv_fwd(A[in].a, B, A[in].H, A[in].W, l.cin, l.wq, l.bias, l.cout, 1, nullptr, A[out].a, false, st);
    };
    // convolution li followed by 2 x 2 max pooling into `pooled`
    auto conv_pool = [&](int li, int in, int out, int pooled) {
        const Layer &l = n->L[li];
        return conv_fwd(A[in].a, B, A[in].H, A[in].W, l.cin, l.wq, l.bias, l.cout, 1, nullptr, A[out].a, false, st,
                        nullptr, nullptr, 0, A[pooled].a);
    };
    TVSPEC_TRY(conv(0, X0, E1A));
    TVSPEC_TRY(conv_pool(1, E1A, E1B, P1));
    TVSPEC_TRY(conv(2, P1, E2A));
    TVSPEC_TRY(conv_pool(3, E2A, E2B, P2));
    TVSPEC_TRY(conv(4, P2, E3A));
    TVSPEC_TRY(conv_pool(5, E3A, E3B, P3));
    TVSPEC_TRY(conv(6, P3, E4A));
    TVSPEC_TRY(conv(7, E4A, E4B));
    // decoder level: concatenation [upsampled low, skip] -> conv li -> out
    auto up_conv = [&](int low, int skip, int /*cat*/, int li, int out) -> int {
        const Layer &l = n->L[li];
        return conv_fwd(A[skip].a, B, A[skip].H, A[skip].W, l.cin, l.wq, l.bias, l.cout, 1, nullptr, A[out].a, false,
                        st, nullptr, A[low].a, A[low].C);
    };
    TVSPEC_TRY(up_conv(E4B, E3B, C3, 8, D3A));
    TVSPEC_TRY(conv(9, D3A, D3B));
    TVSPEC_TRY(up_conv(D3B, E2B, C2, 10, D2A));
    TVSPEC_TRY(conv(11, D2A, D2B));
    TVSPEC_TRY(up_conv(D2B, E1B, C1, 12, D1A));
    TVSPEC_TRY(conv(13, D1A, D1B));
    const Layer &lo = n->L[14];
    ConvIO io;
    if (!training && planar) {
        io.planar = planar;
        io.fout = f;
        io.ipart = ipart;
    }
    TVSPEC_TRY(conv_fwd(A[D1B].a, B, H, W, lo.cin, lo.wq, lo.bias, lo.cout, 0, nullptr, n->out, true, st,
                        n->oscale, nullptr, 0, nullptr, io));
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

// Loss of the last forward pass against bands/residual; leaves dL/dout in n->dout.
int loss_and_grad(tvspec_net *n, const float *f, const double *bands, const double *res, int B, hipStream_t st)
{
    const long long HW = (long long)n->H * n->W;
    hipLaunchKernelGGL(k_pack_target, dim3(grid_for(B * HW)), dim3(kT), 0, st, bands, res, f, n->tgt, B, HW);
    hipLaunchKernelGGL(k_loss_partial, dim3(n->lblk, B), dim3(kT), 0, st, n->out, n->tgt, HW, n->lpart);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(kT), 0, st, n->lpart, B, n->lblk, n->oscale, n->kappa, HW, n->nd,
                       n->loss);
    hipLaunchKernelGGL(k_loss_grad, dim3(grid_for(B * HW * kOutPad)), dim3(kT), 0, st, n->out, n->tgt, n->nd,
                       n->oscale, B, HW, n->dout);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int backward(tvspec_net *n, int B, hipStream_t st)
{
    Act *A = n->A;
    Work &wk = n->wk;
    // layer li: input activation `in`, gradient of its (masked) output dz;
    // writes the layer's parameter gradients and, if din >= 0, the gradient
    // of its input masked by mask_in (the input's own ReLU) or unmasked
    // (a decoder level's first layer: `in` is the concatenation, whose
    // weight gradient reads the lower level `low` and the skip tensor `skip`
    // in place, and whose input gradient goes to the two sources: the skip
    // channels straight into the skip tensor's gradient with its ReLU mask,
    // the upsampled channels into the concatenation's gradient buffer, from
    // which k_up_concat_bwd sums each 2 x 2 block into the lower level's)
    auto layer = [&](int li, int in, const __bf16 *dz, int din, bool mask_in, int low = -1, int skip = -1) -> int {
        const Layer &l = n->L[li];
        RowOut go;  // straight into the layer's slice of the flat gradient
        go.flat = n->grad + l.off;
        go.cout_r = l.cout_r;
        go.cin_r = l.cin_r;
        if (low >= 0) {
            const int cl = A[low].C, cs = A[skip].C;
            TVSPEC_TRY(conv_wgrad(wk, A[skip].a, dz, B, A[in].H, A[in].W, l.cin, l.cout, go, st, A[low].a, cl));
            TVSPEC_TRY(conv_fwd(dz, B, A[in].H, A[in].W, l.cout, l.wd + (size_t)cl * 9 * l.cout, nullptr, cs, 0,
                                A[skip].a, A[skip].g, false, st));
            TVSPEC_TRY(conv_fwd(dz, B, A[in].H, A[in].W, l.cout, l.wd, nullptr, cl, 0, nullptr, A[in].g, false, st));
            const long long cnt = (long long)B * A[low].H * A[low].W * cl;
            hipLaunchKernelGGL(k_up_concat_bwd, dim3(grid_for(cnt)), dim3(kT), 0, st, A[in].g, A[low].a, A[skip].a,
                               A[low].g, A[skip].g, B, A[in].H, A[in].W, cl, 0);
            return TVSPEC_OK;
        }
        TVSPEC_TRY(conv_wgrad(wk, A[in].a, dz, B, A[in].H, A[in].W, l.cin, l.cout, go, st));
        // input gradient: the forward kernel on the layer's flipped weights
        if (din >= 0)
            TVSPEC_TRY(conv_fwd(dz, B, A[in].H, A[in].W, l.cout, l.wd, nullptr, l.cin, 0,
                                mask_in ? A[in].a : nullptr, A[din].g, false, st));
        return TVSPEC_OK;
    };
    auto pool_bwd = [&](int x, int p) {
        const long long cnt = (long long)B * A[p].H * A[p].W * A[p].C;
        hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid_for(cnt)), dim3(kT), 0, st, A[x].a, A[p].g, A[x].g, B, A[x].H,
                           A[x].W, A[x].C);
    };
    TVSPEC_TRY(layer(14, D1B, n->dout, D1B, true));
    TVSPEC_TRY(layer(13, D1A, A[D1B].g, D1A, true));
    TVSPEC_TRY(layer(12, C1, A[D1A].g, C1, false, D2B, E1B));
    TVSPEC_TRY(layer(11, D2A, A[D2B].g, D2A, true));
    TVSPEC_TRY(layer(10, C2, A[D2A].g, C2, false, D3B, E2B));
    TVSPEC_TRY(layer(9, D3A, A[D3B].g, D3A, true));
    TVSPEC_TRY(layer(8, C3, A[D3A].g, C3, false, E4B, E3B));
    TVSPEC_TRY(layer(7, E4A, A[E4B].g, E4A, true));
    TVSPEC_TRY(layer(6, P3, A[E4A].g, P3, false));
    pool_bwd(E3B, P3);
    TVSPEC_TRY(layer(5, E3A, A[E3B].g, E3A, true));
    TVSPEC_TRY(layer(4, P2, A[E3A].g, P2, false));
    pool_bwd(E2B, P2);
    TVSPEC_TRY(layer(3, E2A, A[E2B].g, E2A, true));
    TVSPEC_TRY(layer(2, P1, A[E2A].g, P1, false));
    pool_bwd(E1B, P1);
    TVSPEC_TRY(layer(1, E1A, A[E1B].g, E1A, true));
    TVSPEC_TRY(layer(0, X0, A[E1A].g, -1, false));
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

int check_batch(tvspec_net *n, int B)
{
    if (B < 1 || B > n->maxB)
        return fail(TVSPEC_EINVAL, "B must be in [1, max_batch]");
    return TVSPEC_OK;
}

} // namespace
} // namespace nn
} // namespace tvspec

using namespace tvspec;
using namespace tvspec::nn;

// ---------------------------------------------------------------------------
// C ABI

extern "C" int tvspec_nn_conv3x3(const void *x, int B, int H, int W, int Cin, const void *w, const float *bias,
                                 int Cout, int relu, void *y, int y_f32, void *stream)
{
    g_last_error.clear();
    if (!x || !w || !y)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (B < 1 || H < 1 || W < 1 || Cin < 8 || Cin % 8 || Cout < 16 || Cout % 16 || (relu != 0 && relu != 1) ||
        (y_f32 != 0 && y_f32 != 1) || (long long)B * H * W > (1LL << 31))
        return fail(TVSPEC_EINVAL, "need B, H, W >= 1, Cin a multiple of 8, Cout a multiple of 16");
    return conv_fwd((const __bf16 *)x, B, H, W, Cin, (const __bf16 *)w, bias, Cout, relu, nullptr, y, y_f32 == 1,
                    (hipStream_t)stream);
}

extern "C" int tvspec_nn_conv3x3_dgrad(const void *dy, int B, int H, int W, int Cout, const void *w, int Cin,
                                       const void *mask, void *dx, void *stream)
{
    g_last_error.clear();
    if (!dy || !w || !dx)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (B < 1 || H < 1 || W < 1 || Cout < 8 || Cout % 8 || Cin < 16 || Cin % 16 ||
        (long long)B * H * W > (1LL << 31))
        return fail(TVSPEC_EINVAL, "need B, H, W >= 1, Cout a multiple of 8, Cin a multiple of 16");
    std::lock_guard<std::mutex> lock(g_raw_mu);
    Work *wk = nullptr;
    TVSPEC_TRY(raw_work(&wk));
    return conv_dgrad(*wk, (const __bf16 *)dy, B, H, W, Cout, (const __bf16 *)w, Cin, (const __bf16 *)mask,
                      (__bf16 *)dx, (hipStream_t)stream);
}

extern "C" int tvspec_nn_conv3x3_wgrad(const void *x, const void *dy, int B, int H, int W, int Cin, int Cout,
                                       float *dw, float *db, void *stream)
{
    g_last_error.clear();
    if (!x || !dy || !dw)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (B < 1 || H < 1 || W < 1 || Cin < 8 || Cin % 8 || Cout < 8 || Cout % 8 || (long long)B * H * W > (1LL << 31))
        return fail(TVSPEC_EINVAL, "need B, H, W >= 1, Cin and Cout multiples of 8");
    std::lock_guard<std::mutex> lock(g_raw_mu);
    Work *wk = nullptr;
    TVSPEC_TRY(raw_work(&wk));
    RowOut out;
    out.dw = dw;
    out.db = db;
    return conv_wgrad(*wk, (const __bf16 *)x, (const __bf16 *)dy, B, H, W, Cin, Cout, out, (hipStream_t)stream);
}

extern "C" int tvspec_net_create(int H, int W, int max_batch, unsigned long long seed, tvspec_net **out)
{
    g_last_error.clear();
    if (!out)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    *out = nullptr;
    if (H < 8 || W < 8 || H % 8 || W % 8 || max_batch < 1 || (long long)max_batch * H * W > (1LL << 31))
        return fail(TVSPEC_EINVAL, "need H, W multiples of 8 (>= 8) and max_batch >= 1");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto n = new tvspec_net();
    n->dev = dev;
    n->H = H;
    n->W = W;
    n->maxB = max_batch;
    struct Spec {
        const char *name;
        int cin, cout;
    } spec[15] = {{"e1a", 3, kW0},         {"e1b", kW0, kW0},       {"e2a", kW0, kW1},       {"e2b", kW1, kW1},
                  {"e3a", kW1, kW2},       {"e3b", kW2, kW2},       {"e4a", kW2, kW3},       {"e4b", kW3, kW3},
                  {"d3a", kW3 + kW2, kW2}, {"d3b", kW2, kW2},       {"d2a", kW2 + kW1, kW1}, {"d2b", kW1, kW1},
                  {"d1a", kW1 + kW0, kW0}, {"d1b", kW0, kW0},       {"out", kW0, kOutC}};
    long long off = 0;
    auto cleanup = [&](int rc) {
        for (void *p : n->allocs)
            (void)hipFree(p);
        delete n;
        return rc;
    };
    for (int i = 0; i < 15; ++i) {
        Layer l;
        l.name = spec[i].name;
        l.cin_r = spec[i].cin;
        l.cout_r = spec[i].cout;
        l.cin = (spec[i].cin + 7) / 8 * 8;
        l.cout = (spec[i].cout + 15) / 16 * 16;
        l.off = off;
        off += (long long)l.cout_r * 9 * l.cin_r + l.cout_r;
        int rc = net_alloc(n, (void **)&l.wq, (size_t)l.cout * 9 * l.cin * sizeof(__bf16));
        if (rc == TVSPEC_OK)
            rc = net_alloc(n, (void **)&l.bias, (size_t)l.cout * sizeof(float));
        if (rc == TVSPEC_OK)
            rc = net_alloc(n, (void **)&l.wd, (size_t)l.cout * 9 * l.cin * sizeof(__bf16));
        if (rc != TVSPEC_OK)
            return cleanup(rc);
        n->L.push_back(l);
    }
    n->nparams = off;
    {
        LayerDev tab[kMaxLayers];
        long long start = 0;
        for (size_t i = 0; i < n->L.size(); ++i) {
            const Layer &l = n->L[i];
            tab[i] = LayerDev{l.off, start, l.wq, l.wd, l.bias, l.cout, l.cin, l.cout_r, l.cin_r};
            start += (long long)l.cout * 9 * l.cin + l.cout;
        }
        n->lcount = start;
        int rc = net_alloc(n, (void **)&n->ltab, n->L.size() * sizeof(LayerDev));
        if (rc == TVSPEC_OK && hipMemcpy(n->ltab, tab, n->L.size() * sizeof(LayerDev), hipMemcpyHostToDevice) !=
                                   hipSuccess)
            rc = fail(TVSPEC_EDEVICE, "hipMemcpy failed");
        if (rc != TVSPEC_OK)
            return cleanup(rc);
    }
    const size_t pb = (size_t)off * sizeof(float);
    for (float **p : {&n->master, &n->grad, &n->m, &n->v}) {
        const int rc = net_alloc(n, (void **)p, pb);
        if (rc != TVSPEC_OK)
            return cleanup(rc);
    }
    struct ASpec {
        int lvl, C;
    } as[21] = {{0, 8},         {0, kW0}, {0, kW0}, {1, kW0},       {1, kW1}, {1, kW1}, {2, kW1},
                {2, kW2},       {2, kW2}, {3, kW2}, {3, kW3},       {3, kW3}, {2, kW3 + kW2}, {2, kW2},
                {2, kW2},       {1, kW2 + kW1}, {1, kW1}, {1, kW1}, {0, kW1 + kW0}, {0, kW0}, {0, kW0}};
    for (int i = 0; i < 21; ++i) {
        Act &a = n->A[i];
        a.H = H >> as[i].lvl;
        a.W = W >> as[i].lvl;
        a.C = as[i].C;
        const size_t bytes = (size_t)max_batch * a.H * a.W * a.C * sizeof(__bf16);
        // a concatenation is only ever read in place: it has a gradient but
        // no stored activation
        const bool cat = i == C3 || i == C2 || i == C1;
        int rc = cat ? TVSPEC_OK : net_alloc(n, (void **)&a.a, bytes);
        if (rc == TVSPEC_OK)
            rc = net_alloc(n, (void **)&a.g, bytes);
        if (rc != TVSPEC_OK)
            return cleanup(rc);
    }
    const size_t P = (size_t)max_batch * H * W;
    n->lblk = (int)std::min<long long>(1024, ((long long)H * W + kT - 1) / kT);
    n->otiles = ((H + 7) / 8) * ((W + kTileX - 1) / kTileX);
    int rc = net_alloc(n, (void **)&n->out, P * kOutPad * sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->tgt, P * kOutPad * sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->dout, P * kOutPad * sizeof(__bf16));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->lpart, (size_t)max_batch * kGroups * n->lblk * 2 * sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->nd, (size_t)max_batch * kGroups * 2 * sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->ipart, (size_t)max_batch * n->otiles * sizeof(double));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->gpart, kNormBlocks * sizeof(double));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->gstate, 4 * sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->loss, sizeof(float));
    if (rc == TVSPEC_OK)
        rc = net_alloc(n, (void **)&n->oscale, kOutPad * sizeof(float));
    if (rc != TVSPEC_OK)
        return cleanup(rc);
    {
        const float ones[kOutPad] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 0.f};
        if (hipMemcpy(n->oscale, ones, sizeof(ones), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(TVSPEC_EDEVICE, "output scale upload failed"));
        if (hipMemset(n->gstate, 0, 4 * sizeof(float)) != hipSuccess)
            return cleanup(fail(TVSPEC_EDEVICE, "clip state reset failed"));
    }
    // He-normal weights, zero biases; the output layer starts at zero, so the
    // first outputs are 0 and every band's loss term starts at 1
    std::vector<float> h((size_t)off, 0.f);
    uint64_t s = seed;
    for (const Layer &l : n->L) {
        if (&l == &n->L.back())
            continue;
        const double sd = std::sqrt(2.0 / (9.0 * l.cin_r));
        for (long long q = 0; q < (long long)l.cout_r * 9 * l.cin_r; ++q)
            h[(size_t)(l.off + q)] = (float)(sd * normal(s));
    }
    if (hipMemcpy(n->master, h.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, pb) != hipSuccess || hipMemset(n->v, 0, pb) != hipSuccess)
        return cleanup(fail(TVSPEC_EDEVICE, "parameter upload failed"));
    if ((rc = requant_all(n, nullptr)) != TVSPEC_OK)
        return cleanup(rc);
    if (hipDeviceSynchronize() != hipSuccess)
        return cleanup(fail(TVSPEC_EDEVICE, "device synchronisation failed"));
    *out = n;
    return TVSPEC_OK;
}

extern "C" int tvspec_net_num_params(tvspec_net *net, long long *n)
{
    g_last_error.clear();
    if (!net || !n)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    *n = net->nparams;
    return TVSPEC_OK;
}

extern "C" int tvspec_net_get_params(tvspec_net *net, float *host, long long n)
{
    g_last_error.clear();
    if (!net || !host)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (n != net->nparams)
        return fail(TVSPEC_EINVAL, "n must equal tvspec_net_num_params");
    std::lock_guard<std::mutex> lock(net->mu);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(host, net->master, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
    return TVSPEC_OK;
}

extern "C" int tvspec_net_set_params(tvspec_net *net, const float *host, long long n)
{
    g_last_error.clear();
    if (!net || !host)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (n != net->nparams)
        return fail(TVSPEC_EINVAL, "n must equal tvspec_net_num_params");
    std::lock_guard<std::mutex> lock(net->mu);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(net->master, host, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(net->m, 0, (size_t)n * sizeof(float)));
    HIP_TRY(hipMemset(net->v, 0, (size_t)n * sizeof(float)));
    HIP_TRY(hipMemset(net->gstate, 0, 4 * sizeof(float)));
    net->step = 0;
    TVSPEC_TRY(requant_all(net, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return TVSPEC_OK;
}

extern "C" int tvspec_net_set_output_scale(tvspec_net *net, const float *scale)
{
    g_last_error.clear();
    if (!net || !scale)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    float h[kOutPad];
    for (int c = 0; c < kOutC; ++c) {
        if (!(scale[c] > 0.f) || !std::isfinite(scale[c]))
            return fail(TVSPEC_EINVAL, "output scales must be finite and > 0");
        h[c] = scale[c];
    }
    h[kOutC] = 0.f;
    std::lock_guard<std::mutex> lock(net->mu);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(net->oscale, h, sizeof(h), hipMemcpyHostToDevice));
    return TVSPEC_OK;
}

extern "C" int tvspec_net_set_loss_floor(tvspec_net *net, float kappa)
{
    g_last_error.clear();
    if (!net)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (!(kappa >= 0.f) || !std::isfinite(kappa))
        return fail(TVSPEC_EINVAL, "kappa must be finite and >= 0");
    std::lock_guard<std::mutex> lock(net->mu);
    net->kappa = kappa;
    return TVSPEC_OK;
}

extern "C" int tvspec_net_set_grad_clip(tvspec_net *net, float clip)
{
    g_last_error.clear();
    if (!net)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (!(clip == 0.f || clip >= 1.f) || !std::isfinite(clip))
        return fail(TVSPEC_EINVAL, "clip must be 0 (off) or finite and >= 1");
    std::lock_guard<std::mutex> lock(net->mu);
    net->gclip = clip;
    return TVSPEC_OK;
}

extern "C" int tvspec_net_grad_stats(tvspec_net *net, float *norm, float *avg, float *scale)
{
    g_last_error.clear();
    if (!net || !norm || !avg || !scale)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lock(net->mu);
    float h[4];
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(h, net->gstate, sizeof(h), hipMemcpyDeviceToHost));
    *norm = h[0];
    *avg = h[1];
    *scale = h[2];
    return TVSPEC_OK;
}

extern "C" int tvspec_net_forward_checked(tvspec_net *net, const float *f, int B, float *out, float *err,
                                         void *stream)
{
    g_last_error.clear();
    if (!net || !f || !out)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(check_batch(net, B));
    std::lock_guard<std::mutex> lock(net->mu);
    hipStream_t st = (hipStream_t)stream;
    TVSPEC_TRY(forward(net, f, B, st, false, out, err ? net->ipart : nullptr));
    const long long HW = (long long)net->H * net->W;
    if (err)
        hipLaunchKernelGGL(k_identity_total, dim3(B), dim3(kT), 0, st, net->ipart, net->otiles, HW, err);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

extern "C" int tvspec_net_forward(tvspec_net *net, const float *f, int B, float *out, void *stream)
{
    return tvspec_net_forward_checked(net, f, B, out, nullptr, stream);
}

extern "C" int tvspec_net_loss_grad(tvspec_net *net, const float *f, const double *bands, const double *residual,
                                    int B, float *loss, float *grads, void *stream)
{
    g_last_error.clear();
    if (!net || !f || !bands || !residual || !loss)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    TVSPEC_TRY(check_batch(net, B));
    std::lock_guard<std::mutex> lock(net->mu);
    hipStream_t st = (hipStream_t)stream;
    TVSPEC_TRY(forward(net, f, B, st, true));
    TVSPEC_TRY(loss_and_grad(net, f, bands, residual, B, st));
    TVSPEC_TRY(backward(net, B, st));
    HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    if (grads)
        HIP_TRY(hipMemcpyAsync(grads, net->grad, (size_t)net->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return TVSPEC_OK;
}

extern "C" int tvspec_net_train_step(tvspec_net *net, const float *f, const double *bands, const double *residual,
                                     int B, float lr, float *loss, void *stream)
{
    g_last_error.clear();
    if (!net || !f || !bands || !residual)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (!(lr > 0.f) || !std::isfinite(lr))
        return fail(TVSPEC_EINVAL, "lr must be finite and > 0");
    TVSPEC_TRY(check_batch(net, B));
    std::lock_guard<std::mutex> lock(net->mu);
    hipStream_t st = (hipStream_t)stream;
    TVSPEC_TRY(forward(net, f, B, st, true));
    TVSPEC_TRY(loss_and_grad(net, f, bands, residual, B, st));
    TVSPEC_TRY(backward(net, B, st));
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)net->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)net->step));
    hipLaunchKernelGGL(k_sumsq, dim3(kNormBlocks), dim3(kT), 0, st, net->grad, net->nparams, net->gpart);
    hipLaunchKernelGGL(k_clip_scale, dim3(1), dim3(64), 0, st, net->gpart, kNormBlocks, net->gclip, net->gstate);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(net->nparams)), dim3(kT), 0, st, net->master, net->grad, net->m, net->v,
                       net->nparams, lr, b1, b2, 1e-8f, c1, c2, net->gstate + 2);
    TVSPEC_TRY(requant_all(net, st));
    if (!loss)
        return TVSPEC_OK;
    HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return TVSPEC_OK;
}

extern "C" int tvspec_net_last_loss(tvspec_net *net, float *loss, void *stream)
{
    g_last_error.clear();
    if (!net || !loss)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lock(net->mu);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return TVSPEC_OK;
}

extern "C" int tvspec_net_identity_error(const float *f, const float *out, int B, int H, int W, float *err,
                                         void *stream)
{
    g_last_error.clear();
    if (!f || !out || !err)
        return fail(TVSPEC_EINVAL, "null pointer argument");
    if (B < 1 || B > 65535 || H < 1 || W < 1)
        return fail(TVSPEC_EINVAL, "need 1 <= B <= 65535 and H, W >= 1");
    hipLaunchKernelGGL(k_identity_error, dim3(B), dim3(kT), 0, (hipStream_t)stream, f, out, (long long)H * W, err);
    HIP_TRY(hipGetLastError());
    return TVSPEC_OK;
}

extern "C" int tvspec_net_destroy(tvspec_net *net)
{
    g_last_error.clear();
    if (!net)
        return TVSPEC_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(net->dev);
    (void)hipDeviceSynchronize();
    for (void *p : net->allocs)
        (void)hipFree(p);
    if (net->wk.part)
        (void)hipFree(net->wk.part);
    if (net->wk.wd)
        (void)hipFree(net->wk.wd);
    (void)hipSetDevice(cur);
    delete net;
    return TVSPEC_OK;
}
