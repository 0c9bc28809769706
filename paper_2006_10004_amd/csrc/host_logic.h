// Host-side logic of the tvspec library that needs no GPU runtime: error
// text, argument validation of the C ABI, the band of every spectral sample
// and the server's pool allocator.  Kept free of HIP headers so that it can
// also be built and checked on its own with the host sanitizers.
#ifndef TVSPEC_HOST_LOGIC_H
#define TVSPEC_HOST_LOGIC_H

#include <algorithm>
#include <cstddef>
#include <map>
#include <string>

#include "tvspec.h"

namespace tvspec {

// Text of the last error on the calling thread.
extern thread_local std::string g_last_error;

inline int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// Argument validation of the C ABI (host only, before any device work); each
// returns TVSPEC_OK or TVSPEC_EINVAL with the reason in g_last_error.
//   validate_shape  B images of C x H x W, inner_iters: B, C >= 1, H, W >= 2,
//                   B*C <= 65535 (grid rows), H*W <= 2^30, B*C*H*W <= 2^40,
//                   iters >= 1
//   validate_image  dt finite and > 0, K >= 1, band edges (nb + 1 ints,
//                   host): 1 <= nb <= K, 0 = e_0 < e_1 < ... < e_nb = K
//   validate_opts   0 < tau <= 0.25, warm in {0, 1}, a precision mode,
//                   0 <= iters_per_launch <= 16 (F32) or 8
//   validate_tile_shape  TVSPEC_TILE_SQUARE or _NARROW; the narrow shape
//                   only with the Chambolle solver and iters_per_launch <= 8
int validate_shape(int B, int H, int W, int C, int iters);
int validate_image(double dt, int K, const int *edges, int nb);
int validate_opts(double tau, int warm, int precision, int ipl);
int validate_tile_shape(int tile_shape, int solver, int ipl);

// Round up to a multiple of 256 bytes.
inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// The band of every spectral sample k = 0..K for validated edges (the
// paper's Eq. (7): sample k belongs to band j when e_j < k <= e_{j+1});
// rows has K + 1 entries, entry 0 (no phi at t_0) is 0.
void band_rows_of(const int *edges, int nbands, int *rows);

// First-fit allocator of 256-byte-aligned ranges of the pool.
//   reset(cap)        one free range [0, cap)
//   alloc(n, &off)    the lowest-offset free range of at least align256(n)
//                     bytes; false if none
//   release(off, n)   returns a range alloc gave out (same n), merging it
//                     with free neighbours
class RangeAlloc {
  public:
    void reset(size_t cap)
    {
        free_.clear();
        free_[0] = cap;
        used_ = peak_ = 0;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            const size_t o = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest)
                free_[o + n] = rest;
            *off = o;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align256(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
        used_ -= n;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_; // offset -> length
    size_t used_ = 0, peak_ = 0;
};

} // namespace tvspec

#endif // TVSPEC_HOST_LOGIC_H
