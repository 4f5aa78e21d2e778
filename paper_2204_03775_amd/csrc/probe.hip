// Streaming bandwidth probes (declared in include/wave_probe.h).  Each
// thread moves float4s in a grid-stride loop; launches fill every CU
// several times over.
#include <hip/hip_runtime.h>

#include "wave_probe.h"

namespace {

struct alignas(16) f4 {
    float v[4];
};

__global__ __launch_bounds__(256) void copy_k(const f4 *__restrict__ s, f4 *__restrict__ d,
                                              long long n4)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (long long)gridDim.x * blockDim.x)
        d[i] = s[i];
}

__global__ __launch_bounds__(256) void r3w1_k(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                              const f4 *__restrict__ c, f4 *__restrict__ d,
                                              long long n4)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (long long)gridDim.x * blockDim.x) {
        const f4 x = a[i], y = b[i], z = c[i];
        f4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            o.v[e] = x.v[e] + y.v[e] + z.v[e];
        d[i] = o;
    }
}

bool bad(const void *p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15u); }

int grid_for(long long n4)
{
    long long g = (n4 + 255) / 256;
    return int(g < 256 * 64 ? g : 256 * 64);  // up to 64 blocks per CU
}

}  // namespace

extern "C" int probe_copy(const float *src, float *dst, int64_t n, void *stream)
{
    if (bad(src) || bad(dst) || n <= 0 || (n & 3))
        return -1;
    const long long n4 = n / 4;
    hipLaunchKernelGGL(copy_k, dim3(grid_for(n4)), dim3(256), 0, (hipStream_t)stream,
                       (const f4 *)src, (f4 *)dst, n4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_read3_write1(const float *a, const float *b, const float *c, float *d,
                                  int64_t n, void *stream)
{
    if (bad(a) || bad(b) || bad(c) || bad(d) || n <= 0 || (n & 3))
        return -1;
    const long long n4 = n / 4;
    hipLaunchKernelGGL(r3w1_k, dim3(grid_for(n4)), dim3(256), 0, (hipStream_t)stream,
                       (const f4 *)a, (const f4 *)b, (const f4 *)c, (f4 *)d, n4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}
