// F32-storage step kernels: the tiled kernel for every tile shape (streaming
// and cache-resident load policies), the naive kernel and its receiver
// sampler.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY)                                                  \
    template __global__ void step_tiled<WAVE_F32, TXV, TY, RY>(StepArgs); \
    template __global__ void step_tiled_cached<TXV, TY, RY>(StepArgs);
WAVE_TILE_SHAPES(INST)
#undef INST
template __global__ void step_naive<WAVE_F32>(StepArgs);
template __global__ void sample_naive<WAVE_F32>(const void *__restrict__, const long long *__restrict__, int,
                                                float *, const int *, int);

}  // namespace wavek
