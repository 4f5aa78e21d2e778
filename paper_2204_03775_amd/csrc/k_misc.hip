// Kernels outside the time step: the k range check at set-up, batch
// counter clearing, and the adjoint run's receiver injection, misfit
// reduction and gradient output.

#include "wave_dev.h"

namespace wavek {

// Adds k * trace_grad[row][r] at the receiver cells: one thread per distinct
// cell, summing its receivers in a fixed order (deterministic, no atomics).
// With s_val set, the source value of the forward step that made this level
// is k at the source cell times a fixed wavelet value, so its derivative
// with respect to that k adds lambda s / k = phi s / k^2 there (lambda =
// phi / k): thread src_thread takes it -- the thread of the receiver cell
// that is also the source cell (after its own add), or thread ncells.
__global__ void inject_receivers(float *phi, const float *__restrict__ k, const long long *__restrict__ cell_off,
                                 const int *__restrict__ cell_start, const int *__restrict__ cell_rec,
                                 int ncells, const float *__restrict__ tg_row, const float *__restrict__ s_val,
                                 long long src_off, int src_thread, double *acc)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    float v = 0.f;
    if (c < ncells) {
        float s = 0.f;
        for (int i = cell_start[c]; i < cell_start[c + 1]; ++i)
            s += tg_row[cell_rec[i]];
        const long long o = cell_off[c];
        v = fmaf(k[o], s, phi[o]);
        phi[o] = v;
    } else if (c == ncells && s_val) {
        v = phi[src_off];
    }
    if (s_val && c == src_thread) {
        const double kk = k[src_off];
        acc[src_off] += (double)v * (double)*s_val / (kk * kk);
    }
}

// k = (v dt)^2 per cell, formed in FP64 and rounded once to FP32 (dense
// [n] arrays).
__global__ __launch_bounds__(256) void velocity_to_k(const float *__restrict__ v, long long n, double dt,
                                                    float *k)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double vd = (double)v[i] * dt;
        k[i] = (float)(vd * vd);
    }
}

// misfit = 0.5 sum (traces - d_obs)^2 in FP64 (one work-group, fixed
// summation order, differences taken exactly); residual = traces - d_obs
// rounded to FP32 when requested.
__global__ __launch_bounds__(1024) void misfit_kernel(const float *__restrict__ tr,
                                                      const float *__restrict__ obs, long long n,
                                                      float *residual, double *out)
{
    __shared__ double part[1024];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const double r = (double)tr[i] - (double)obs[i];  // exact
        if (residual)
            residual[i] = (float)r;  // == the FP32 difference
        acc += r * r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = 0.5 * part[0];
}

// dense[z][y][x] (+)= acc at the interior cells of the field layout; with
// v set, the chain rule to velocity: dJ/dv = dJ/dk * 2 dt^2 v (k = (v dt)^2).
__global__ __launch_bounds__(256) void grad_to_dense(const double *__restrict__ acc, double *dense, int nx,
                                                    int ny, int nz, int px, int x0, long long plane,
                                                    int accumulate, const float *__restrict__ v,
                                                    double two_dt2)
{
    const long long n = (long long)nx * ny * nz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / ((long long)nx * ny));
        double g = acc[(long long)(z + kGhost) * plane + (long long)(y + kGhost) * px + x0 + x];
        if (v)
            g *= two_dt2 * (double)v[i];
        dense[i] = accumulate ? dense[i] + g : g;
    }
}

// Clears both ticket sets at the start of a batched run (a kernel rather
// than a memset, so that it can sit in a captured graph).
__global__ void clear_counters(int *c)
{
    if (threadIdx.x < 16)
        c[threadIdx.x] = 0;
}

// Zero n ints (a kernel, not a memset, so that it can sit in a captured graph).
__global__ __launch_bounds__(256) void zero_ints(int *p, long long n)
{
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        p[i] = 0;
}

// Max, min and a non-finite flag of an FP32 k over the interior, as float
// bit patterns (valid for non-negative values; negatives raise the flag).
__global__ __launch_bounds__(256) void k_range(const float *__restrict__ k, int nx, int ny, int nz,
                                               int px, int x0, long long plane, unsigned *out)
{
    __shared__ unsigned smax[256], smin[256], sbad[256];
    unsigned mx = 0u, mn = 0x7f800000u, bad = 0u;
    const long long n = (long long)nx * ny * nz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / ((long long)nx * ny));
        const float v = k[(long long)(z + kGhost) * plane + (long long)(y + kGhost) * px + x0 + x];
        if (!(v >= 0.f) || !(v < INFINITY)) {
            bad = 1u;
        } else {
            const unsigned b = __float_as_uint(v);
            mx = max(mx, b);
            mn = min(mn, b);
        }
    }
    const int t = threadIdx.x;
    smax[t] = mx;
    smin[t] = mn;
    sbad[t] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            smax[t] = max(smax[t], smax[t + s]);
            smin[t] = min(smin[t], smin[t + s]);
            sbad[t] |= sbad[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        atomicMax(&out[0], smax[0]);
        atomicMin(&out[1], smin[0]);
        atomicOr(&out[2], sbad[0]);
    }
}

// Counts non-finite values: the interior of a field (FP32 or 16-bit bits,
// by storage type) into out[0], n trace values into out[1].
__global__ __launch_bounds__(256) void count_nonfinite(const void *__restrict__ field, int kind, int nx,
                                                      int ny, int nz, int px, int x0, long long plane,
                                                      const float *__restrict__ traces, long long n,
                                                      int *out)
{
    const long long cells = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    int bad_f = 0, bad_t = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / ((long long)nx * ny));
        const long long p = (long long)(z + kGhost) * plane + (long long)(y + kGhost) * px + x0 + x;
        if (kind == WAVE_F32) {
            bad_f += !isfinite(static_cast<const float *>(field)[p]);
        } else {
            const unsigned b = static_cast<const unsigned short *>(field)[p];
            const unsigned e = (kind == WAVE_F16 || kind == WAVE_F16_UV) ? 0x7c00u : 0x7f80u;
            bad_f += (b & e) == e;  // all-ones exponent: infinity or NaN
        }
    }
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad_t += !isfinite(traces[i]);
    if (bad_f)
        atomicAdd(&out[0], bad_f);
    if (bad_t)
        atomicAdd(&out[1], bad_t);
}

}  // namespace wavek
