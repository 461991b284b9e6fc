// host.hpp -- host-side helpers of libmsst: error reporting, device queries,
// launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "msst.h"

namespace msst {

ms_status set_error(ms_status code, const char* fmt, ...);
void clear_error();

// Validates that the current device is a gfx950 and returns its compute
// unit count (cached per device).  MS_ERR_UNSUPPORTED / MS_ERR_DEVICE on
// failure.
ms_status device_cu_count(int* cus);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace msst

#define MS_REQUIRE(cond, ...)                                                  \
    do {                                                                       \
        if (!(cond)) return msst::set_error(MS_ERR_INVALID_ARGUMENT, __VA_ARGS__); \
    } while (0)

#define MS_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return msst::set_error(MS_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define MS_LAUNCHED()                                                                  \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return msst::set_error(MS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)
