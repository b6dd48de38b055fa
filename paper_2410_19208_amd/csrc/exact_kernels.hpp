// Launchers of the exact-projection kernels (k_exact.hip), used by exact.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "psdproj.h"

namespace psd {

int exact_sumsq_blocks(int n, int* rows);
void launch_gemm64(int n, const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                   double alpha, const double* D, int64_t ldd, double beta, hipStream_t s);
void launch_ex_norm(int n, bool fp64, const void* X, int64_t ldx, double* part, double* out, psdproj_result* res,
                    hipStream_t s);
void launch_ex_scale(int n, bool fp64, const void* X, int64_t ldx, const double* out, double* X64, double* S,
                     hipStream_t s);
void launch_ex_poly(int n, double* W, double a2, hipStream_t s);
void launch_ex_final(int n, bool fp64, const double* Q, void* P, int64_t ldp, hipStream_t s);
void launch_ex_trace(int n, const double* S, psdproj_result* res, hipStream_t s);

}  // namespace psd
