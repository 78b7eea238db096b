// Raw Philox4x32-10 blocks and Gaussian slot draws, exposed so that the
// variation streams of the reconstruction can be checked bit for bit.
#include "hf_device.hpp"
#include "hf_internal.hpp"

namespace hf {
namespace {

__global__ void k_philox(const uint32_t *__restrict__ ctr, uint64_t seed, uint32_t *__restrict__ out, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const U4 c{ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3]};
    const U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * k] = r.x;
    out[4 * k + 1] = r.y;
    out[4 * k + 2] = r.z;
    out[4 * k + 3] = r.w;
}

template <typename T>
__global__ void k_gauss(uint64_t seed, const int64_t *__restrict__ g, const int32_t *__restrict__ v,
                        const int32_t *__restrict__ slot, int64_t n, double *__restrict__ z) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    z[k] = (double)gauss_slot<T>(seed, (uint64_t)g[k], (uint32_t)v[k], (uint32_t)slot[k]);
}

}  // namespace

hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctr, seed, out, n);
    return hipGetLastError();
}

hipError_t launch_gauss(uint64_t seed, const int64_t *g, const int32_t *v, const int32_t *slot, int64_t n,
                        int precision, double *z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (precision == HF_PREC_MIXED)
        hipLaunchKernelGGL(k_gauss<float>, grid, dim3(256), 0, s, seed, g, v, slot, n, z);
    else
        hipLaunchKernelGGL(k_gauss<double>, grid, dim3(256), 0, s, seed, g, v, slot, n, z);
    return hipGetLastError();
}

}  // namespace hf
