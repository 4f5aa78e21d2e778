// Streaming bandwidth probes (declared in include/wave_probe.h).  Each
// thread moves float4s in a grid-stride loop.
#include <hip/hip_runtime.h>

#include "wave_probe.h"

namespace {

struct alignas(16) f4 {
    float v[4];
};

// Each thread keeps U float4 loads in flight, U grid strides apart, and
// the grid holds 2 work-groups of 256 threads per CU: the fastest of the
// launch shapes tried on MI355X (1..16 loads per thread, 256..1024 threads,
// 1..8 work-groups per CU).  Accesses are non-temporal, like the
// propagator's once-read data.
constexpr int U = 2;
constexpr int kThreads = 256;
constexpr int kBlocksPerCu = 2;

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

__global__ __launch_bounds__(kThreads) void copy_k(const f4 *__restrict__ s, f4 *__restrict__ d,
                                                   long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride * U) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4)
                v[u] = ldnt(s + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4)
                stnt(d + i + u * stride, v[u]);
    }
}

__global__ __launch_bounds__(kThreads) void r3w1_k(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                   const f4 *__restrict__ c, f4 *__restrict__ d,
                                                   long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride * U) {
        f4 x[U], y[U], z[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4) {
                x[u] = ldnt(a + i + u * stride);
                y[u] = ldnt(b + i + u * stride);
                z[u] = ldnt(c + i + u * stride);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4) {
                f4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    o.v[e] = x[u].v[e] + y[u].v[e] + z[u].v[e];
                stnt(d + i + u * stride, o);
            }
    }
}

struct alignas(16) d2 {
    double v[2];
};

// o = a + b + c + d, g += o (FP64): four FP32 reads, an FP64 read and write
// and an FP32 write per element, 36 bytes: the access mix of the fused
// adjoint step (phi^{m+1}, phi^{m+2}, k and the forward level in; phi^m and
// the FP64 gradient accumulator out).
__global__ __launch_bounds__(kThreads) void adjmix_k(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                     const f4 *__restrict__ c, const f4 *__restrict__ d,
                                                     d2 *__restrict__ g, f4 *__restrict__ o, long long n4)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride * U) {
        f4 x[U];
        d2 g0[U], g1[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4) {
                const long long j = i + u * stride;
                const f4 p = ldnt(a + j), q = ldnt(b + j), r = ldnt(c + j), t = ldnt(d + j);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    x[u].v[e] = p.v[e] + q.v[e] + r.v[e] + t.v[e];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    g0[u].v[e] = __builtin_nontemporal_load(&g[2 * j].v[e]);
                    g1[u].v[e] = __builtin_nontemporal_load(&g[2 * j + 1].v[e]);
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * stride < n4) {
                const long long j = i + u * stride;
                stnt(o + j, x[u]);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    __builtin_nontemporal_store(g0[u].v[e] + (double)x[u].v[e], &g[2 * j].v[e]);
                    __builtin_nontemporal_store(g1[u].v[e] + (double)x[u].v[2 + e], &g[2 * j + 1].v[e]);
                }
            }
    }
}

// Synchronisation between work-groups of one cooperative launch, as the
// library's single-launch batch does it between steps: nsteps barriers
// across the whole grid (ring = 0), or waits for the two ring neighbours'
// step counters (ring = 1), each work-group arriving with an agent-scope
// release and leaving after an agent-scope acquire.  words: [0] arrivals,
// [1] barriers opened, [2] abort, [3] spare, [4 + b] steps done by
// work-group b; all zero at launch.  Every wait gives up once the wall
// clock passes the deadline and raises words[2].
__global__ __launch_bounds__(256) void sync_k(int *words, int nsteps, int ring, unsigned long long timeout)
{
    __shared__ int stop;
    const unsigned long long deadline = wall_clock64() + timeout;
    unsigned *count = reinterpret_cast<unsigned *>(words);
    unsigned *gen = reinterpret_cast<unsigned *>(words + 1);
    int *abort = words + 2;
    int *done = words + 4;
    const int nb = gridDim.x, b = blockIdx.x;
    const int l = (b + nb - 1) % nb, r = (b + 1) % nb;
    auto give_up = [&]() {
        return wall_clock64() > deadline || __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    unsigned g = 0;
    for (int j = 0; j < nsteps; ++j) {
        __syncthreads();
        if (threadIdx.x == 0) {
            stop = 0;
            if (ring) {
                __hip_atomic_store(done + b, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                while (__hip_atomic_load(done + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= j ||
                       __hip_atomic_load(done + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= j) {
                    if (give_up()) {
                        stop = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            } else {
                const unsigned a = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (a + 1 == (unsigned)nb) {
                    __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                        if (give_up()) {
                            stop = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                ++g;
            }
            if (stop)
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (stop)
            return;
    }
}

__global__ void empty_k() {}

// The step's plane march without its arithmetic.  A work-group owns a tile
// of 256 cells x 8 rows of a padded field (4 ghost planes and rows on each
// side, rows `pitch4` float4 apart, interior x from float4 `x04`) and a
// chunk of zc planes.  For every plane z of the chunk, in march order, it
// reads a at the plane four ahead of the march (as the step's register queue
// does), b and k at plane z, and writes b = a + b + k over b at plane z (the
// step overwrites u^{n-1} in place): 16 bytes per cell.  The next plane's
// values are loaded before the current plane is stored.  Cache policies are
// the step's: a (u^n, which neighbouring tiles read again) with the default
// policy, b and k read and b written non-temporally.  Work-groups are
// mapped to tiles as the step kernels map them (contiguous runs per XCD).
// down: every chunk is marched from its top plane.
__global__ __launch_bounds__(512) void step_stream_k(const f4 *__restrict__ a, f4 *__restrict__ b,
                                                     const f4 *__restrict__ k, int nx4, int ny, int nz,
                                                     long long pitch4, long long plane4, int x04, int zc,
                                                     int ntx, int nty, int nwg, int down)
{
    const int per = gridDim.x >> 3;
    const int lid = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (lid >= nwg)
        return;
    const int tx = lid % ntx, rest = lid / ntx, ty = rest % nty, ch = rest / nty;
    const int z0 = ch * zc, z1 = min(z0 + zc, nz), len = z1 - z0;
    const int col = tx * 64 + (int)(threadIdx.x % 64), row = ty * 8 + (int)(threadIdx.x / 64);
    if (col >= nx4 || row >= ny)
        return;
    const long long off = (long long)(row + 4) * pitch4 + x04 + col;
    const int dz = down ? -1 : 1;
    const int zs = down ? z1 - 1 : z0;
    auto at = [&](int z) { return (long long)(z + 4) * plane4 + off; };
    f4 an = a[at(zs + 4 * dz)], bn = ldnt(b + at(zs)), kn = ldnt(k + at(zs));
    for (int l = 0; l < len; ++l) {
        const int z = zs + l * dz;
        const f4 x = an, y = bn, w = kn;
        if (l + 1 < len) {
            an = a[at(z + 5 * dz)];
            bn = ldnt(b + at(z + dz));
            kn = ldnt(k + at(z + dz));
        }
        f4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            o.v[e] = x.v[e] + y.v[e] + w.v[e];
        stnt(b + at(z), o);
    }
}

// The same for the 16-bit storage forms (2-byte cells; a padded field has
// nz + 8 planes of ny + 8 rows of `pitch` cells, interior x from cell x0).
// Tiles of 32 x TY threads, each thread 4 consecutive cells (8 bytes) in RY
// rows, and z-chunks of zc planes, as the 16-bit step kernels tile a grid.
// Two levels (UV false): read u four planes ahead of the march (default
// policy) and p, k at the plane (non-temporal), write p = u ^ p ^ k in place
// (non-temporal): 8 bytes per cell.  u and step change (UV true): read u
// ahead and d (default policy, as the step reads its change) and k at the
// plane, write o = u ^ k into the other level buffer and d = d ^ u in place:
// 10 bytes per cell.  Bitwise XOR keeps the check
// exact for any bit pattern.  Out-of-range cells get an offset past the
// plane's buffer resource, so they read zero and store nothing.
typedef unsigned u2raw __attribute__((vector_size(8)));
constexpr int kRawWord3 = 0x00020000;  // raw (stride 0) 32-bit buffer access
constexpr int kPolKeep = 0, kPolStream = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane16(const void *f, long long plane_bytes, int z)
{
    const char *p = reinterpret_cast<const char *>(f) + (long long)(z + 4) * plane_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, (int)plane_bytes, kRawWord3);
}

template <int TY, int RY, bool UV>
__global__ __launch_bounds__(32 * TY) void step_stream16_k(const void *u, void *p, void *o, const void *k,
                                                           int nxq, int ny, int nz, long long pitch,
                                                           long long plane_bytes, int x0, int zc, int ntx,
                                                           int nty, int nwg, int down)
{
    const int per = gridDim.x >> 3;
    const int lid = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (lid >= nwg)
        return;
    const int tx = lid % ntx, rest = lid / ntx, ty = rest % nty, ch = rest / nty;
    const int z0 = ch * zc, z1 = min(z0 + zc, nz), len = z1 - z0;
    const int q = tx * 32 + (int)(threadIdx.x % 32);
    const int r0 = (ty * TY + (int)(threadIdx.x / 32)) * RY;
    unsigned off[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r)
        off[r] = (q < nxq && r0 + r < ny) ? 2u * unsigned((r0 + r + 4) * pitch + x0 + 4 * q) : 0xffffffffu;
    const int dz = down ? -1 : 1;
    const int zs = down ? z1 - 1 : z0;
    u2raw un[RY], pn[RY], kn[RY];
    auto load = [&](int z) {
        const __amdgpu_buffer_rsrc_t ru = plane16(u, plane_bytes, z + 4 * dz);
        const __amdgpu_buffer_rsrc_t rp = plane16(p, plane_bytes, z);
        const __amdgpu_buffer_rsrc_t rk = plane16(k, plane_bytes, z);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            un[r] = __builtin_amdgcn_raw_buffer_load_b64(ru, off[r], 0, kPolKeep);
            pn[r] = __builtin_amdgcn_raw_buffer_load_b64(rp, off[r], 0, UV ? kPolKeep : kPolStream);
            kn[r] = __builtin_amdgcn_raw_buffer_load_b64(rk, off[r], 0, kPolStream);
        }
    };
    load(zs);
    for (int l = 0; l < len; ++l) {
        const int z = zs + l * dz;
        u2raw a[RY], b[RY], c[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            a[r] = un[r];
            b[r] = pn[r];
            c[r] = kn[r];
        }
        if (l + 1 < len)
            load(z + dz);
        const __amdgpu_buffer_rsrc_t rp = plane16(p, plane_bytes, z);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if constexpr (UV) {
                __builtin_amdgcn_raw_buffer_store_b64(a[r] ^ c[r], plane16(o, plane_bytes, z), off[r], 0,
                                                      kPolStream);
                __builtin_amdgcn_raw_buffer_store_b64(b[r] ^ a[r], rp, off[r], 0, kPolStream);
            } else {
                __builtin_amdgcn_raw_buffer_store_b64(a[r] ^ b[r] ^ c[r], rp, off[r], 0, kPolStream);
            }
        }
    }
}

// The fused adjoint step's access pattern without its arithmetic: FP32
// fields c (phi^{m+1}) and a (the forward level) read four planes ahead of
// the march with the default policy, p (phi^{m+2}) and k at the plane
// non-temporally, the FP64 accumulator g (8-byte cells, same layout) read
// and written at the plane with the default policy, and p overwritten in
// place non-temporally: 36 bytes per cell.  Tiles of 32 x TY threads, each
// thread 4 cells of one row (128 cells x TY rows), z-chunks of zc planes,
// as the adjoint kernel tiles a grid.  p = c ^ a ^ p ^ k and the two
// 16-byte halves of a thread's accumulator cells XORed with c and a.
typedef unsigned u4raw __attribute__((vector_size(16)));

template <int TY>
__global__ __launch_bounds__(32 * TY) void adjoint_stream_k(const float *c, const float *a, float *p,
                                                            const float *k, double *g, int nxq, int ny, int nz,
                                                            long long pitch, long long plane_bytes, int x0, int zc,
                                                            int ntx, int nty, int nwg, int down)
{
    const int per = gridDim.x >> 3;
    const int lid = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (lid >= nwg)
        return;
    const int tx = lid % ntx, rest = lid / ntx, ty = rest % nty, ch = rest / nty;
    const int z0 = ch * zc, z1 = min(z0 + zc, nz), len = z1 - z0;
    const int q = tx * 32 + (int)(threadIdx.x % 32);
    const int row = ty * TY + (int)(threadIdx.x / 32);
    const bool in = q < nxq && row < ny;
    const long long cell = (long long)(row + 4) * pitch + x0 + 4 * q;
    const unsigned off = in ? 4u * unsigned(cell) : 0xffffffffu;    // FP32 fields
    const unsigned goff = in ? 8u * unsigned(cell) : 0xffffffffu;   // accumulator
    const long long gplane = 2 * plane_bytes;
    const int dz = down ? -1 : 1;
    const int zs = down ? z1 - 1 : z0;
    auto grs = [&](int z) {
        const char *b = reinterpret_cast<const char *>(g) + (long long)(z + 4) * gplane;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(b), (short)0, (int)gplane, kRawWord3);
    };
    u4raw cn, an, pn, kn, g0, g1;
    auto load = [&](int z) {
        cn = __builtin_amdgcn_raw_buffer_load_b128(plane16(c, plane_bytes, z + 4 * dz), off, 0, kPolKeep);
        an = __builtin_amdgcn_raw_buffer_load_b128(plane16(a, plane_bytes, z + 4 * dz), off, 0, kPolKeep);
        pn = __builtin_amdgcn_raw_buffer_load_b128(plane16(p, plane_bytes, z), off, 0, kPolStream);
        kn = __builtin_amdgcn_raw_buffer_load_b128(plane16(k, plane_bytes, z), off, 0, kPolStream);
        g0 = __builtin_amdgcn_raw_buffer_load_b128(grs(z), goff, 0, kPolKeep);
        g1 = __builtin_amdgcn_raw_buffer_load_b128(grs(z), goff + 16u, 0, kPolKeep);
    };
    load(zs);
    for (int l = 0; l < len; ++l) {
        const int z = zs + l * dz;
        const u4raw vc = cn, va = an, vp = pn, vk = kn, w0 = g0, w1 = g1;
        if (l + 1 < len)
            load(z + dz);
        __builtin_amdgcn_raw_buffer_store_b128(vc ^ va ^ vp ^ vk, plane16(p, plane_bytes, z), off, 0, kPolStream);
        __builtin_amdgcn_raw_buffer_store_b128(w0 ^ vc, grs(z), goff, 0, kPolKeep);
        __builtin_amdgcn_raw_buffer_store_b128(w1 ^ va, grs(z), goff + 16u, 0, kPolKeep);
    }
}

bool bad(const void *p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15u); }

int grid_for(long long n4)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const long long g = (n4 + kThreads - 1) / kThreads;
    return int(g < (long long)kBlocksPerCu * cus ? g : (long long)kBlocksPerCu * cus);
}

}  // namespace

extern "C" int probe_copy(const float *src, float *dst, int64_t n, void *stream)
{
    if (bad(src) || bad(dst) || n <= 0 || (n & 3))
        return -1;
    const long long n4 = n / 4;
    hipLaunchKernelGGL(copy_k, dim3(grid_for(n4)), dim3(kThreads), 0, (hipStream_t)stream,
                       (const f4 *)src, (f4 *)dst, n4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_read3_write1(const float *a, const float *b, const float *c, float *d,
                                  int64_t n, void *stream)
{
    if (bad(a) || bad(b) || bad(c) || bad(d) || n <= 0 || (n & 3))
        return -1;
    const long long n4 = n / 4;
    hipLaunchKernelGGL(r3w1_k, dim3(grid_for(n4)), dim3(kThreads), 0, (hipStream_t)stream,
                       (const f4 *)a, (const f4 *)b, (const f4 *)c, (f4 *)d, n4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_adjoint_mix(const float *a, const float *b, const float *c, const float *d, double *g,
                                 float *o, int64_t n, void *stream)
{
    if (bad(a) || bad(b) || bad(c) || bad(d) || bad(g) || bad(o) || n <= 0 || (n & 3))
        return -1;
    const long long n4 = n / 4;
    hipLaunchKernelGGL(adjmix_k, dim3(grid_for(n4)), dim3(kThreads), 0, (hipStream_t)stream,
                       (const f4 *)a, (const f4 *)b, (const f4 *)c, (const f4 *)d, (d2 *)g, (f4 *)o, n4);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_sync(int *words, int blocks, int nsteps, int ring, double timeout_s, void *stream)
{
    int dev = 0, khz = 0, coop = 0;
    if (!words || blocks < 2 || nsteps < 0 || !(timeout_s >= 0.0) ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop || khz < 1)
        return -1;
    unsigned long long timeout = (unsigned long long)(timeout_s * khz * 1000.0);
    void *args[] = {&words, &nsteps, &ring, &timeout};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(sync_k), dim3(blocks), dim3(256), args, 0,
                                   (hipStream_t)stream) != hipSuccess)
        return -5;
    return 0;
}

extern "C" int probe_empty(int blocks, void *stream)
{
    if (blocks < 1)
        return -1;
    hipLaunchKernelGGL(empty_k, dim3(blocks), dim3(256), 0, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_step_stream(const float *a, float *b, const float *k, int nx, int ny, int nz, int64_t pitch,
                                 int64_t x0, int zc, int down, void *stream)
{
    if (bad(a) || bad(b) || bad(k) || nx < 4 || (nx & 3) || ny < 1 || nz < 1 || zc < 1 || (pitch & 3) ||
        (x0 & 3) || x0 < 4 || pitch < x0 + nx + 4)
        return -1;
    const int nx4 = nx / 4;
    const int ntx = (nx4 + 63) / 64, nty = (ny + 7) / 8, nch = (nz + zc - 1) / zc;
    const long long nwg = (long long)ntx * nty * nch;
    if (nwg > (1ll << 30))
        return -1;
    const long long pitch4 = pitch / 4, plane4 = pitch4 * (ny + 8);
    const int grid = int((nwg + 7) / 8 * 8);
    hipLaunchKernelGGL(step_stream_k, dim3(grid), dim3(512), 0, (hipStream_t)stream, (const f4 *)a, (f4 *)b,
                       (const f4 *)k, nx4, ny, nz, pitch4, plane4, int(x0 / 4), zc, ntx, nty, int(nwg), down ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int probe_step_stream16(const void *u, void *p, void *o, const void *k, int nx, int ny, int nz,
                                   int64_t pitch, int64_t x0, int zc, int ty, int ry, int down, void *stream)
{
    auto bad8 = [](const void *q) { return !q || (reinterpret_cast<uintptr_t>(q) & 7u); };
    if (bad8(u) || bad8(p) || bad8(k) || (o && bad8(o)) || nx < 4 || (nx & 3) || ny < 1 || nz < 1 || zc < 1 ||
        (pitch & 3) || (x0 & 3) || x0 < 4 || pitch < x0 + nx + 4)
        return -1;
    const long long plane_bytes = (long long)pitch * (ny + 8) * 2;
    if (plane_bytes >= (1ll << 31))
        return -1;
    const int nxq = nx / 4;
    const int ntx = (nxq + 31) / 32, nty = (ny + ty * ry - 1) / (ty * ry), nch = (nz + zc - 1) / zc;
    const long long nwg = (long long)ntx * nty * nch;
    if (nwg > (1ll << 30))
        return -1;
    const int grid = int((nwg + 7) / 8 * 8);
#define STREAM16(TY, RY)                                                                                     \
    if (ty == TY && ry == RY) {                                                                              \
        if (o)                                                                                               \
            hipLaunchKernelGGL((step_stream16_k<TY, RY, true>), dim3(grid), dim3(32 * TY), 0,                \
                               (hipStream_t)stream, u, p, o, k, nxq, ny, nz, (long long)pitch, plane_bytes,  \
                               int(x0), zc, ntx, nty, int(nwg), down ? 1 : 0);                               \
        else                                                                                                 \
            hipLaunchKernelGGL((step_stream16_k<TY, RY, false>), dim3(grid), dim3(32 * TY), 0,               \
                               (hipStream_t)stream, u, p, o, k, nxq, ny, nz, (long long)pitch, plane_bytes,  \
                               int(x0), zc, ntx, nty, int(nwg), down ? 1 : 0);                               \
        return hipGetLastError() == hipSuccess ? 0 : -5;                                                     \
    }
    STREAM16(8, 1)
    STREAM16(8, 2)
    STREAM16(16, 1)
    STREAM16(16, 2)
    STREAM16(32, 1)
#undef STREAM16
    return -1;
}

extern "C" int probe_adjoint_stream(const float *c, const float *a, float *p, const float *k, double *g, int nx,
                                    int ny, int nz, int64_t pitch, int64_t x0, int zc, int ty, int down,
                                    void *stream)
{
    if (bad(c) || bad(a) || bad(p) || bad(k) || bad(g) || nx < 4 || (nx & 3) || ny < 1 || nz < 1 || zc < 1 ||
        (pitch & 3) || (x0 & 3) || x0 < 4 || pitch < x0 + nx + 4 || (ty != 8 && ty != 16))
        return -1;
    const long long plane_bytes = (long long)pitch * (ny + 8) * 4;
    if (2 * plane_bytes >= (1ll << 31))
        return -1;
    const int nxq = nx / 4;
    const int ntx = (nxq + 31) / 32, nty = (ny + ty - 1) / ty, nch = (nz + zc - 1) / zc;
    const long long nwg = (long long)ntx * nty * nch;
    if (nwg > (1ll << 30))
        return -1;
    const int grid = int((nwg + 7) / 8 * 8);
    if (ty == 8)
        hipLaunchKernelGGL(adjoint_stream_k<8>, dim3(grid), dim3(256), 0, (hipStream_t)stream, c, a, p, k, g, nxq,
                           ny, nz, (long long)pitch, plane_bytes, int(x0), zc, ntx, nty, int(nwg), down ? 1 : 0);
    else
        hipLaunchKernelGGL(adjoint_stream_k<16>, dim3(grid), dim3(512), 0, (hipStream_t)stream, c, a, p, k, g,
                           nxq, ny, nz, (long long)pitch, plane_bytes, int(x0), zc, ntx, nty, int(nwg),
                           down ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}
