// Adjoint and imaging steps of the gradient run as separate passes (FP32),
// one per tile shape.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY)                                              \
    template __global__ void adjoint_tiled<kAdj, TXV, TY, RY>(StepArgs); \
    template __global__ void adjoint_tiled<kImg, TXV, TY, RY>(StepArgs);
WAVE_TILE_SHAPES(INST)
#undef INST

}  // namespace wavek
