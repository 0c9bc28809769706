// Shared host-side helpers of the tvspec library: error text and HIP checks.
#ifndef TVSPEC_COMMON_H
#define TVSPEC_COMMON_H

#include <hip/hip_runtime.h>

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
int validate_shape(int B, int H, int W, int C, int iters);
int validate_image(double dt, int K, const int *edges, int nb);
int validate_opts(double tau, int warm, int precision, int ipl);

} // namespace tvspec

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::tvspec::fail(e_ == hipErrorOutOfMemory ? TVSPEC_ENOMEM : TVSPEC_EDEVICE, \
                                  std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

#define TVSPEC_TRY(expr)                                                                      \
    do {                                                                                      \
        int rc_ = (expr);                                                                     \
        if (rc_ != TVSPEC_OK)                                                                 \
            return rc_;                                                                       \
    } while (0)

#endif // TVSPEC_COMMON_H
