// Storage conversions of the interior (16-bit encode / decode, FP32 copy).
#include "wave_step.h"

namespace wavek {

#define INST(S, D)                                                                                   \
    template __global__ void convert_interior<S, D>(const void *__restrict__, void *, int, int, int, int, \
                                                    int, long long, int, int, long long, float,         \
                                                    const int *, int);
INST(WAVE_F32, WAVE_F16)
INST(WAVE_F32, WAVE_BF16)
INST(WAVE_F16, WAVE_F32)
INST(WAVE_BF16, WAVE_F32)
INST(WAVE_F32, WAVE_F32)
#undef INST

}  // namespace wavek
