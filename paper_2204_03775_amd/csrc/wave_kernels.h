// Kernel declarations for the host code of libwave.so (wave.hip); the
// kernels are defined in wave_step.h (instantiated by the k_*.hip units)
// and k_misc.hip.
#pragma once

#include "wave_dev.h"

namespace wavek {

// kernels (defined in the k_*.hip translation units)
template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_tiled(StepArgs a);
template <int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_tiled_cached(StepArgs a);
template <int MODE, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void adjoint_tiled(StepArgs a);
template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_batch(const ShotDesc *__restrict__ shots, BatchItems it,
                                                       int j);
template <int KIND, int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_batch_run(const ShotDesc *__restrict__ shots, BatchItems it,
                                                           RunSync rs);
template <int TXV, int TY, int RY>
__global__ __launch_bounds__(TXV *TY) void step_flow(const ShotDesc *__restrict__ shots, FlowPlan p);
template <int KIND>
__global__ __launch_bounds__(256) void step_naive(StepArgs a);
template <int KIND>
__global__ void sample_naive(const void *__restrict__ f, const long long *__restrict__ off, int nrec,
                             float *row, const int *exps, int slot);
template <int SRC, int DST>
__global__ __launch_bounds__(256) void convert_interior(const void *__restrict__ src, void *dst, int nx,
                                                        int ny, int nz, int spx, int sx0, long long sp,
                                                        int dpx, int dx0, long long dp, float scale,
                                                        const int *exps, int slot);
__global__ void clear_counters(int *c);
__global__ __launch_bounds__(256) void zero_ints(int *p, long long n);
__global__ __launch_bounds__(256) void k_range(const float *__restrict__ k, int nx, int ny, int nz,
                                               int px, int x0, long long plane, unsigned *out);
__global__ void inject_receivers(float *phi, const float *__restrict__ k,
                                 const long long *__restrict__ cell_off,
                                 const int *__restrict__ cell_start, const int *__restrict__ cell_rec,
                                 int ncells, const float *__restrict__ tg_row, const float *__restrict__ s_val,
                                 long long src_off, int src_thread, double *acc);
__global__ __launch_bounds__(256) void velocity_to_k(const float *__restrict__ v, long long n, double dt,
                                                    float *k);
__global__ __launch_bounds__(1024) void misfit_kernel(const float *__restrict__ tr,
                                                      const float *__restrict__ obs, long long n,
                                                      float *residual, double *out);
__global__ __launch_bounds__(256) void count_nonfinite(const void *__restrict__ field, int kind, int nx,
                                                      int ny, int nz, int px, int x0, long long plane,
                                                      const float *__restrict__ traces, long long n,
                                                      int *out);
__global__ __launch_bounds__(256) void grad_to_dense(const double *__restrict__ acc, double *dense, int nx,
                                                    int ny, int nz, int px, int x0, long long plane,
                                                    int accumulate, const float *__restrict__ v,
                                                    double two_dt2);

}  // namespace wavek
