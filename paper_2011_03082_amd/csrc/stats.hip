// stats.hip -- deterministic FP64 image statistics (mean, RMSE against a
// reference, per-sample variance) for the matched-error comparison of the
// plain and sphere-traced estimators.
#include "device.hpp"
#include "host.hpp"

namespace msst {

constexpr int kStatBlocks = 512;

__global__ void image_stats_partial(const float* sum, const float* comp, const float* sumsq, const float* ref,
                                    int64_t n, double inv_spp, double* partial) {
    __shared__ double red[256][4];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const double s = (double)sum[p] + (comp ? (double)comp[p] : 0.0);
        const double m = s * inv_spp;
        a0 += m;
        if (ref) {
            const double e = m - (double)ref[p];
            a1 += e * e;
            a3 += (double)ref[p];
        }
        if (sumsq) a2 += (double)sumsq[p] * inv_spp - m * m;
    }
    red[threadIdx.x][0] = a0;
    red[threadIdx.x][1] = a1;
    red[threadIdx.x][2] = a2;
    red[threadIdx.x][3] = a3;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 4; ++k) red[threadIdx.x][k] += red[threadIdx.x + off][k];
        __syncthreads();
    }
    if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void image_stats_final(const double* partial, int nb, int64_t n, double* out) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b * 4 + k];
    s /= (double)n;
    out[k] = k == 1 ? sqrt(s) : s;
}

}  // namespace msst

extern "C" {

ms_status ms_image_stats_workspace_size(int64_t n_pixels, size_t* bytes) {
    MS_REQUIRE(bytes != nullptr, "ms_image_stats_workspace_size: bytes is NULL");
    *bytes = (size_t)msst::kStatBlocks * 4 * sizeof(double);
    return MS_OK;
}

ms_status ms_image_stats(const float* sum_dev, const float* comp_dev, const float* sumsq_dev, const float* ref_dev,
                         int64_t n_pixels, int32_t spp, double* out_dev, void* workspace_dev, size_t workspace_bytes,
                         void* stream) {
    using namespace msst;
    MS_REQUIRE(sum_dev && out_dev, "ms_image_stats: NULL array");
    MS_REQUIRE(n_pixels > 0 && spp > 0, "ms_image_stats: n_pixels and spp must be positive");
    MS_REQUIRE(workspace_dev != nullptr, "ms_image_stats: workspace is NULL");
    if (workspace_bytes < (size_t)kStatBlocks * 4 * sizeof(double))
        return set_error(MS_ERR_WORKSPACE_TOO_SMALL, "ms_image_stats: workspace too small");
    int cus;
    ms_status st = device_cu_count(&cus);
    if (st != MS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double* partial = reinterpret_cast<double*>(workspace_dev);
    hipLaunchKernelGGL(image_stats_partial, dim3(kStatBlocks), dim3(256), 0, s, sum_dev, comp_dev, sumsq_dev, ref_dev,
                       n_pixels, 1.0 / (double)spp, partial);
    hipLaunchKernelGGL(image_stats_final, dim3(1), dim3(64), 0, s, partial, kStatBlocks, n_pixels, out_dev);
    MS_LAUNCHED();
    clear_error();
    return MS_OK;
}

}  // extern "C"
