// Kernels of the dual gradient descent for the SDLS problem (Alg. 6, supplementary SDP section):
//   k_sdls_form:   X = C/rho + sum_i y_i A_i (line 5), FP64 per element, stored in T;
//   k_sdls_trace:  per-block partial sums of Tr(A_i^T P) = sum_jk A_i[j][k] P[j][k] (line 14; A_i
//                  symmetric), FP64;
//   k_sdls_update: g_i = (sum of the partials in block order) - b_i, y_i -= beta g_i (line 15),
//                  ||g||_2; one workgroup, fixed order, so the iterates do not depend on scheduling.
// The projection between form and trace is the library's own (Alg. 2 / Alg. 3 run in place on X).
// All three are streaming kernels bound by HBM: form reads m + 1 matrices and writes one, trace
// reads m + 1.
#include "common.hpp"
#include "sdls.hpp"

namespace psd {

constexpr int SD_THREADS = 256;
constexpr int SD_CHUNK = 8;   // constraints accumulated per sweep of the trace kernel

// Block (x, y) covers columns 256 x .. 256 x + 255 of row y.
template <typename T>
__global__ __launch_bounds__(SD_THREADS) void k_sdls_form(const T* __restrict__ C, int64_t ldc,
                                                          const T* __restrict__ A, int64_t lda, int64_t astride,
                                                          int m, const double* __restrict__ y, double inv_rho,
                                                          T* __restrict__ X, int64_t ldx, int n) {
  const int64_t i = blockIdx.y;
  const int j = blockIdx.x * SD_THREADS + threadIdx.x;
  if (j >= n) return;
  const gmem<const T>* Ag = gp(A) + i * lda + j;
  double acc = (double)gp(C)[i * ldc + j] * inv_rho;
  for (int t = 0; t < m; ++t) acc = fma(y[t], (double)Ag[(int64_t)t * astride], acc);
  gp(X)[i * ldx + j] = (T)acc;
}

// Block b covers rows [b R, (b+1) R); part[t * nblk + b] = its share of Tr(A_t P).
template <typename T>
__global__ __launch_bounds__(SD_THREADS) void k_sdls_trace(const T* __restrict__ A, int64_t lda, int64_t astride,
                                                           int m, const T* __restrict__ P, int64_t ldp, int n,
                                                           int rows_per_block, double* __restrict__ part) {
  __shared__ double red[SD_CHUNK][SD_THREADS / WAVE];
  const int nblk = gridDim.x, b = blockIdx.x;
  const int r0 = b * rows_per_block, r1 = min(n, r0 + rows_per_block);
  const gmem<const T>* Ag = gp(A);
  const gmem<const T>* Pg = gp(P);
  const int wave = wave_id(), lane = threadIdx.x & 63;
  for (int t0 = 0; t0 < m; t0 += SD_CHUNK) {
    double acc[SD_CHUNK];
#pragma unroll
    for (int u = 0; u < SD_CHUNK; ++u) acc[u] = 0.0;
    for (int64_t i = r0; i < r1; ++i)
      for (int j = threadIdx.x; j < n; j += SD_THREADS) {
        const double pv = (double)Pg[i * ldp + j];
#pragma unroll
        for (int u = 0; u < SD_CHUNK; ++u)
          if (t0 + u < m) acc[u] = fma((double)Ag[(int64_t)(t0 + u) * astride + i * lda + j], pv, acc[u]);
      }
#pragma unroll
    for (int u = 0; u < SD_CHUNK; ++u) {
      const double w = wave_allsum(acc[u]);
      if (lane == 0) red[u][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x < SD_CHUNK && t0 + (int)threadIdx.x < m) {
      double s = 0.0;
      for (int w = 0; w < SD_THREADS / WAVE; ++w) s += red[threadIdx.x][w];
      part[(int64_t)(t0 + threadIdx.x) * nblk + b] = s;
    }
    __syncthreads();
  }
}

// One workgroup.  out[0] = ||g||_2; g and y updated in place.
__global__ __launch_bounds__(SD_THREADS) void k_sdls_update(const double* __restrict__ part, int nblk, int m,
                                                            const double* __restrict__ bvec, double beta,
                                                            double* __restrict__ y, double* __restrict__ g,
                                                            double* __restrict__ out) {
  __shared__ double red[SD_THREADS / WAVE];
  double sq = 0.0;
  for (int t = threadIdx.x; t < m; t += SD_THREADS) {
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += part[(int64_t)t * nblk + k];
    const double gt = s - bvec[t];
    g[t] = gt;
    y[t] -= beta * gt;
    sq = fma(gt, gt, sq);
  }
  const double w = wave_allsum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < SD_THREADS / WAVE; ++k) s += red[k];
    out[0] = sqrt(s);
  }
}

int sdls_trace_blocks(int n, int* rows_per_block) {
  const int R = max(1, (n + 1023) / 1024);
  *rows_per_block = R;
  return (n + R - 1) / R;
}

void launch_sdls_form(bool fp64, const void* C, int64_t ldc, const void* A, int64_t lda, int64_t astride, int m,
                      const double* y, double inv_rho, void* X, int64_t ldx, int n, hipStream_t s) {
  const dim3 grid((n + SD_THREADS - 1) / SD_THREADS, n);
  if (fp64)
    hipLaunchKernelGGL(k_sdls_form<double>, grid, dim3(SD_THREADS), 0, s, (const double*)C, ldc,
                       (const double*)A, lda, astride, m, y, inv_rho, (double*)X, ldx, n);
  else
    hipLaunchKernelGGL(k_sdls_form<float>, grid, dim3(SD_THREADS), 0, s, (const float*)C, ldc,
                       (const float*)A, lda, astride, m, y, inv_rho, (float*)X, ldx, n);
}

void launch_sdls_trace(bool fp64, const void* A, int64_t lda, int64_t astride, int m, const void* P, int64_t ldp,
                       int n, double* part, hipStream_t s) {
  int R = 1;
  const int nblk = sdls_trace_blocks(n, &R);
  if (fp64)
    hipLaunchKernelGGL(k_sdls_trace<double>, dim3(nblk), dim3(SD_THREADS), 0, s, (const double*)A, lda, astride, m,
                       (const double*)P, ldp, n, R, part);
  else
    hipLaunchKernelGGL(k_sdls_trace<float>, dim3(nblk), dim3(SD_THREADS), 0, s, (const float*)A, lda, astride, m,
                       (const float*)P, ldp, n, R, part);
}

void launch_sdls_update(const double* part, int nblk, int m, const double* b, double beta, double* y, double* g,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sdls_update, dim3(1), dim3(SD_THREADS), 0, s, part, nblk, m, b, beta, y, g, out);
}

}  // namespace psd
