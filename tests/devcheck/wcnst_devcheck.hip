// GPU check of the device arithmetic's ranged reciprocal and square root:
// each argument through recip_ranged / sqrt_ranged and through the IEEE
// division and root, on the device, for a test to compare bit for bit.
#include <hip/hip_runtime.h>

#include "wcnst_device.hpp"

namespace {

__global__ void ranged_math(const double* __restrict__ x, double* __restrict__ out, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    out[i] = wcnst::recip_ranged(v);
    out[(size_t)n + i] = 1.0 / v;
    out[(size_t)2 * n + i] = wcnst::sqrt_ranged(v);
    out[(size_t)3 * n + i] = sqrt(v);
}

}  // namespace

extern "C" {

// x: n host doubles.  out: 4 n host doubles (recip_ranged, 1/x, sqrt_ranged,
// sqrt).  Returns 0, or the HIP error code of the first failing call.
int dc_ranged_math(const double* x, int n, double* out)
{
    if (n <= 0) return 0;
    double *dx = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dx, (size_t)n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dout, (size_t)4 * n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(dx, x, (size_t)n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        ranged_math<<<(n + 255) / 256, 256>>>(dx, dout, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)4 * n * sizeof(double), hipMemcpyDeviceToHost);
    hipFree(dx);
    hipFree(dout);
    return (int)e;
}

}  // extern "C"
