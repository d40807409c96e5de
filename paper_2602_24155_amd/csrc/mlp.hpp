// Host interface of the learned policy's network (kernels in mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/crfrob.h"

namespace crf {
// Scores of `rows` host input rows (CR_MLP_INPUTS floats each) into host y, on the GPU.
bool mlp_score(cr_mlp *m, const float *x, int rows, float *y, hipStream_t stream, std::string &err);
}  // namespace crf
