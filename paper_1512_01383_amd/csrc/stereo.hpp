// stereo.hpp -- launcher of the stereo matching-cost kernel (stereo.hip).
#pragma once
#include <hip/hip_runtime.h>

// costs [D][H][W] of the pair left / right ([H][W]); see sl_stereo_costs
hipError_t launch_stereo_costs(const float *left, const float *right, int H, int W, int D,
                               float trunc, float *out, hipStream_t st);
