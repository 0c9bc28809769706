// Shared host-side helpers of the tvspec library: HIP error checks (the rest
// of the host logic is in host_logic.h).
#ifndef TVSPEC_COMMON_H
#define TVSPEC_COMMON_H

#include <hip/hip_runtime.h>

#include <string>

#include "host_logic.h"
#include "tvspec.h"


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
