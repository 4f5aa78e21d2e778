// Data-flow batched step kernels (FP32, every step of a group of shots in
// one launch), one per tile shape.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY) \
    template __global__ void step_flow<TXV, TY, RY>(const ShotDesc *__restrict__, FlowPlan);
WAVE_TILE_SHAPES(INST)
#undef INST

}  // namespace wavek
