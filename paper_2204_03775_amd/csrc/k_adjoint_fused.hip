// Fused adjoint step + imaging term of the gradient run (FP32), one per tile
// shape.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY) template __global__ void adjoint_tiled<kFus, TXV, TY, RY>(StepArgs);
WAVE_TILE_SHAPES(INST)
#undef INST

}  // namespace wavek
