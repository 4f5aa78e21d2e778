// Streaming bandwidth probes (declared in include/wave_probe.h).  Each
// thread moves float4s in a grid-stride loop; launches fill every CU
// several times over.
#include <hip/hip_runtime.h>

#include "wave_probe.h"

namespace {

struct alignas(16) f4 {
    float v[4];
};

// Each thread moves U float4s per iteration (independent loads in flight),
// streamed non-temporally like the propagator's once-read data.
constexpr int U = 4;

__device__ __forceinline__ f4 ldnt(const f4 *p)
{
    f4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        o.v[e] = __builtin_nontemporal_load(&p->v[e]);
    return o;
}

__device__ __forceinline__ void stnt(f4 *p, const f4 &v)
{
#pragma unroll
    for (int e = 0; e < 4; ++e)
        __builtin_nontemporal_store(v.v[e], &p->v[e]);
}

__global__ __launch_bounds__(256) void copy_k(const f4 *__restrict__ s, f4 *__restrict__ d,
                                              long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x * U;
    for (long long base = (long long)blockIdx.x * blockDim.x * U + threadIdx.x; base < n4;
         base += stride) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * blockDim.x;
            if (i < n4)
                v[u] = ldnt(s + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * blockDim.x;
            if (i < n4)
                stnt(d + i, v[u]);
        }
    }
}

__global__ __launch_bounds__(256) void r3w1_k(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                              const f4 *__restrict__ c, f4 *__restrict__ d,
                                              long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x * U;
    for (long long base = (long long)blockIdx.x * blockDim.x * U + threadIdx.x; base < n4;
         base += stride) {
        f4 x[U], y[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * blockDim.x;
            if (i < n4) {
                x[u] = ldnt(a + i);
                y[u] = ldnt(b + i);
                z[u] = ldnt(c + i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * blockDim.x;
            if (i < n4) {
                f4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    o.v[e] = x[u].v[e] + y[u].v[e] + z[u].v[e];
                stnt(d + i, o);
            }
        }
    }
}

bool bad(const void *p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15u); }

int grid_for(long long n4)
{
    long long g = (n4 + 256 * U - 1) / (256 * U);
    return int(g < 256 * 16 ? g : 256 * 16);  // up to 16 blocks per CU
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
