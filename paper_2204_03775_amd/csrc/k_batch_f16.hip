// F16-storage batched (persistent, many shots per launch) step kernels, one
// per tile shape.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY) \
    template __global__ void step_batch<WAVE_F16, TXV, TY, RY>(const ShotDesc *__restrict__, BatchItems, int); \
    template __global__ void step_batch_run<WAVE_F16, TXV, TY, RY>(const ShotDesc *__restrict__, BatchItems, RunSync);
WAVE_TILE_SHAPES(INST)
#undef INST

}  // namespace wavek
