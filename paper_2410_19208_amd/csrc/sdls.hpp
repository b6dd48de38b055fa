// Launchers of the SDLS dual-gradient kernels (k_sdls.hip), used by the solver in sdls.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace psd {

// number of trace partial blocks for order n (and the rows each covers)
int sdls_trace_blocks(int n, int* rows_per_block);
void launch_sdls_form(bool fp64, const void* C, int64_t ldc, const void* A, int64_t lda, int64_t astride, int m,
                      const double* y, double inv_rho, void* X, int64_t ldx, int n, hipStream_t s);
void launch_sdls_trace(bool fp64, const void* A, int64_t lda, int64_t astride, int m, const void* P, int64_t ldp,
                       int n, double* part, hipStream_t s);
void launch_sdls_update(const double* part, int nblk, int m, const double* b, double beta, double* y, double* g,
                        double* out, hipStream_t s);

}  // namespace psd
