// common.hip -- library-wide entry points: version, errors, device checks and
// the Philox fill used to check the generator block for block.
#include <mutex>
#include <string.h>

#include "device.hpp"
#include "host.hpp"

namespace msst {

static thread_local char g_error[512] = "";

ms_status set_error(ms_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_error[0] = 0; }

ms_status device_cu_count(int* cus) {
    static std::mutex mu;
    static int cached[64];
    static int checked[64];
    int dev = 0;
    MS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(MS_ERR_UNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!checked[dev]) {
        hipDeviceProp_t prop;
        MS_HIP(hipGetDeviceProperties(&prop, dev));
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return set_error(MS_ERR_UNSUPPORTED, "device %d is %s; libmsst is built for gfx950", dev,
                             prop.gcnArchName);
        cached[dev] = prop.multiProcessorCount;
        checked[dev] = 1;
    }
    *cus = cached[dev];
    return MS_OK;
}

__global__ void philox_fill_kernel(uint64_t seed, uint32_t tag, uint64_t id0, int64_t n_ids,
                                   uint32_t c0, int32_t n_draws, uint32_t* out) {
    const int64_t total = n_ids * (int64_t)n_draws;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n_draws;
        const uint32_t j = (uint32_t)(t - i * n_draws);
        const Rng r = make_rng(seed, tag, id0 + (uint64_t)i);
        const uint4 w = r.block(c0 + j);
        uint4* o = reinterpret_cast<uint4*>(out) + t;
        *o = w;
    }
}

}  // namespace msst

extern "C" {

int32_t ms_abi_version(void) { return MS_ABI_VERSION; }

const char* ms_last_error(void) { return msst::g_error; }

ms_status ms_philox_fill(uint64_t seed, uint32_t tag, uint64_t id0, int64_t n_ids, uint32_t c0,
                         int32_t n_draws, uint32_t* out_dev, void* stream) {
    MS_REQUIRE(out_dev != nullptr, "ms_philox_fill: out_dev is NULL");
    MS_REQUIRE(n_ids > 0 && n_draws > 0, "ms_philox_fill: n_ids and n_draws must be positive");
    MS_REQUIRE(n_ids * (int64_t)n_draws < ((int64_t)1 << 31), "ms_philox_fill: too many blocks");
    MS_REQUIRE(((uintptr_t)out_dev & 15u) == 0, "ms_philox_fill: out_dev must be 16-byte aligned");
    int cus = 0;
    ms_status st = msst::device_cu_count(&cus);
    if (st != MS_OK) return st;
    const int64_t total = n_ids * (int64_t)n_draws;
    int64_t blocks = (total + 255) / 256;
    if (blocks > (int64_t)cus * 16) blocks = (int64_t)cus * 16;
    hipLaunchKernelGGL(msst::philox_fill_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, seed, tag, id0, n_ids, c0, n_draws, out_dev);
    MS_LAUNCHED();
    msst::clear_error();
    return MS_OK;
}

}  // extern "C"
