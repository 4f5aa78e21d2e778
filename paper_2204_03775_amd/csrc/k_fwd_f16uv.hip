// F16_UV step kernels (16-bit u^n and step change d^n): the tiled kernel for
// every tile shape and the naive kernel.
#include "wave_step.h"

namespace wavek {

#define INST(TXV, TY, RY) template __global__ void step_tiled<WAVE_F16_UV, TXV, TY, RY>(StepArgs);
WAVE_TILE_SHAPES(INST)
#undef INST
template __global__ void step_naive<WAVE_F16_UV>(StepArgs);

}  // namespace wavek
