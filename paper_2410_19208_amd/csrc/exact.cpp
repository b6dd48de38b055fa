// The exact projection X_+ = U max(D, 0) U^T of Thm 1 on the GPU, without an eigendecomposition:
// X_+ = (X + |X|) / 2 with |X| = X sign(X), and sign(X) by the scaled Newton-Schulz iteration
// (Chen & Chow, "A stable scaling of Newton-Schulz for improving the sign function computation of
// a Hermitian matrix", 2014):  S_0 = X / ||X||_F (every |eigenvalue| in (0, 1]), and
//   S_{k+1} = (a_k / 2) S_k (3 I - a_k^2 S_k^2),  a_k = sqrt(3 / (1 + l_k + l_k^2)),
//   l_{k+1} = (a_k l_k / 2) (3 - a_k^2 l_k^2),
// which maps the spectrum of |S_k| in [l_k, 1] into [l_{k+1}, 1] and converges quadratically once
// l_k is near 1.  Eigenvalues with |lambda| >= l_0 ||X||_F are converged when l_k reaches 1 to
// round-off; one below it contributes at most |lambda| / 2 <= l_0 ||X||_F / 2 to the error of
// X_+.  l_0 is 1e-13 for FP64 storage and 1e-9 otherwise; the iteration count follows from l_0
// alone, so the host schedules it without reading anything back.  Every product is an n x n FP64
// GEMM on the matrix cores (k_gemm64): 2 per iteration and one for X S, O(n^3) in all -- the
// cost the randomized projections avoid.
#include <hip/hip_runtime.h>

#include <cmath>

#include "exact.hpp"
#include "exact_kernels.hpp"
#include "runtime.hpp"

namespace psd {

namespace {
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int iteration_count(double l0) {
  double l = l0;
  int k = 0;
  while (1.0 - l > 1e-15 && k < 200) {
    const double a = std::sqrt(3.0 / (1.0 + l + l * l));
    l = 0.5 * a * l * (3.0 - a * a * l * l);
    ++k;
  }
  return k + 1;   // one more at the fixed point absorbs the round-off of the last steps
}
}  // namespace

size_t exact_workspace_bytes(int n, int precision) {
  (void)precision;
  const size_t M = al256((size_t)n * n * 8);
  int R = 1;
  const int nb = exact_sumsq_blocks(n, &R);
  return 4 * M + al256((size_t)nb * 8) + 256;
}

psdproj_status exact_projection(int n, int precision, const void* X, int64_t ldx, void* P, int64_t ldp,
                                void* workspace, size_t workspace_bytes, psdproj_result* res, hipStream_t s) {
  if (n < 1 || !X || !P || !workspace || !res || ldx < n || ldp < n) return PSDPROJ_E_INVALID;
  if (workspace_bytes < exact_workspace_bytes(n, precision)) return PSDPROJ_E_NOMEM;
  const bool fp64 = precision == PSDPROJ_FP64;
  const size_t M = al256((size_t)n * n * 8);
  unsigned char* w = (unsigned char*)workspace;
  double* X64 = (double*)w;
  double* S = (double*)(w + M);
  double* T1 = (double*)(w + 2 * M);
  double* T2 = (double*)(w + 3 * M);
  int R = 1;
  const int nb = exact_sumsq_blocks(n, &R);
  double* part = (double*)(w + 4 * M);
  double* out = (double*)(w + 4 * M + al256((size_t)nb * 8));
  {
    ProfScope t(K_EXACT_MISC, s);
    launch_ex_norm(n, fp64, X, ldx, part, out, res, s);
    launch_ex_scale(n, fp64, X, ldx, out, X64, S, s);
  }
  double l = fp64 ? 1e-13 : 1e-9;
  const int K = iteration_count(l);
  for (int k = 0; k < K; ++k) {
    const double a = std::sqrt(3.0 / (1.0 + l + l * l));
    {
      ProfScope t(K_GEMM64, s);
      launch_gemm64(n, S, n, S, n, T1, n, 1.0, nullptr, n, 0.0, s);          // T1 = S^2
    }
    {
      ProfScope t(K_EXACT_MISC, s);
      launch_ex_poly(n, T1, a * a, s);                                         // T1 = 3I - a^2 S^2
    }
    {
      ProfScope t(K_GEMM64, s);
      launch_gemm64(n, S, n, T1, n, T2, n, 0.5 * a, nullptr, n, 0.0, s);     // T2 = (a/2) S T1
    }
    double* t = S; S = T2; T2 = t;
    l = std::fmin(1.0, 0.5 * a * l * (3.0 - a * a * l * l));
  }
  {
    ProfScope t(K_EXACT_MISC, s);
    launch_ex_trace(n, S, res, s);
  }
  {
    ProfScope t(K_GEMM64, s);
    launch_gemm64(n, X64, n, S, n, T1, n, 0.5, X64, n, 0.5, s);             // Q = (X + X S) / 2
  }
  {
    ProfScope t(K_EXACT_MISC, s);
    launch_ex_final(n, fp64, T1, P, ldp, s);                                 // P = (Q + Q^T) / 2
  }
  return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_E_DEVICE;
}

}  // namespace psd

extern "C" {

psdproj_status psdproj_exact_workspace(int64_t n, int32_t precision, size_t* bytes) {
  if (n < 1 || n > 65535 || !bytes || precision < PSDPROJ_FP64 || precision > PSDPROJ_BF16X3) return PSDPROJ_E_INVALID;
  *bytes = psd::exact_workspace_bytes((int)n, precision);
  return PSDPROJ_OK;
}

psdproj_status psdproj_exact(int64_t n, int32_t precision, const void* A, int64_t lda, void* P, int64_t ldp,
                             void* workspace, size_t workspace_bytes, psdproj_result* result_dev,
                             psdproj_stream_t stream) {
  if (n < 1 || n > 65535 || precision < PSDPROJ_FP64 || precision > PSDPROJ_BF16X3) return PSDPROJ_E_INVALID;
  if (((uintptr_t)workspace & 255) || ((uintptr_t)A & 15) || ((uintptr_t)P & 15)) return PSDPROJ_E_INVALID;
  return psd::exact_projection((int)n, precision, A, lda, P, ldp, workspace, workspace_bytes, result_dev,
                               (hipStream_t)stream);
}

}  // extern "C"
