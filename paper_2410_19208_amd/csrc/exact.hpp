// The exact projection X_+ = U max(D, 0) U^T of Thm 1, computed on the GPU (exact.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "psdproj.h"

namespace psd {

size_t exact_workspace_bytes(int n, int precision);
psdproj_status exact_projection(int n, int precision, const void* X, int64_t ldx, void* P, int64_t ldp,
                                void* workspace, size_t workspace_bytes, psdproj_result* result_dev, hipStream_t s);

}  // namespace psd
