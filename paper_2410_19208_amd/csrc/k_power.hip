// Alg. 4 (power iteration for sigma_1) and Alg. 5 (alpha = |sigma_1(X) - sigma_1(X - sigma_1 I)|).
//
// One launch of k_gemv computes y = X v - shift v with v = y_prev * inv_prev (the previous
// product scaled to unit norm; the first product uses the raw Gaussian start vector) and the
// norm ||y||.  The shift of Alg. 5 line 2 is applied to the vector, so X - sigma_1 I is never
// formed.  Vectors and accumulation are FP64 for every storage precision of A.
// The norm is reduced deterministically: each block writes its partial sum of squares, and
// the last block to finish (integer ticket counter) adds the partials in block order.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int GEMV_THREADS = 256;
constexpr int ROWS_PER_WAVE = GEMV_ROWS / 4;   // 8

template <typename T>
__device__ void gemv_block(const Prob& p, int t, int last) {
  const int n = p.n, ld = p.ld;
  const int pp = p.iscal[I_PP] & 1;                 // ping-pong: read vec[pp], write vec[1-pp]
  const double* __restrict__ vin = p.vec + (int64_t)pp * ld;
  double* __restrict__ vout = p.vec + (int64_t)(1 - pp) * ld;
  const double inv = p.scal[S_INV];
  const double shift = p.scal[S_SHIFT];
  const T* __restrict__ A = (const T*)p.A;
  const int64_t lda = p.lda;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int row0 = t * GEMV_ROWS + wave * ROWS_PER_WAVE;
  __shared__ double red[4];

  double acc[ROWS_PER_WAVE];
#pragma unroll
  for (int q = 0; q < ROWS_PER_WAVE; ++q) acc[q] = 0.0;
  int rows[ROWS_PER_WAVE];
#pragma unroll
  for (int q = 0; q < ROWS_PER_WAVE; ++q) rows[q] = min(row0 + q, n - 1);   // clamp; masked below
  // Rows that do not start 16-byte aligned are read with scalar loads (n4 = 0); otherwise
  // 4-wide vector loads cover [0, n4) and scalar loads the tail [n4, n).
  const int n4 = p.avec ? (n & ~3) : 0;
  for (int j = lane * 4; j < n4; j += WAVE * 4) {
    const double v0 = vin[j] * inv, v1 = vin[j + 1] * inv, v2 = vin[j + 2] * inv, v3 = vin[j + 3] * inv;
#pragma unroll
    for (int q = 0; q < ROWS_PER_WAVE; ++q) {
      const T* src = A + (int64_t)rows[q] * lda + j;
      if constexpr (sizeof(T) == 4) {
        const f32x4 a = __builtin_nontemporal_load((const f32x4*)src);
        acc[q] += (double)a[0] * v0 + (double)a[1] * v1 + (double)a[2] * v2 + (double)a[3] * v3;
      } else {
        const f64x2 a = __builtin_nontemporal_load((const f64x2*)src);
        const f64x2 b = __builtin_nontemporal_load((const f64x2*)(src + 2));
        acc[q] += a[0] * v0 + a[1] * v1 + b[0] * v2 + b[1] * v3;
      }
    }
  }
  for (int j = n4 + lane; j < n; j += WAVE) {
    const double vj = vin[j] * inv;
#pragma unroll
    for (int q = 0; q < ROWS_PER_WAVE; ++q) acc[q] += (double)A[(int64_t)rows[q] * lda + j] * vj;
  }
  double ss = 0.0;
#pragma unroll
  for (int q = 0; q < ROWS_PER_WAVE; ++q) {
    const double s = wave_sum(acc[q]);
    const int row = row0 + q;
    if (row < n) {
      const double y = s - shift * (vin[row] * inv);
      if (lane == 0) vout[row] = y;
      ss += y * y;
    }
  }
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nblk = (n + GEMV_ROWS - 1) / GEMV_ROWS;
    p.vpart[t] = red[0] + red[1] + red[2] + red[3];
    __threadfence();
    const int ticket = atomicAdd(&p.iscal[I_COUNTER], 1);
    if (ticket == nblk - 1) {
      __threadfence();
      const volatile double* vp = p.vpart;
      double tot = 0.0;
      for (int b = 0; b < nblk; ++b) tot += vp[b];
      const double nrm = sqrt(tot);
      p.scal[S_NRM] = nrm;
      p.scal[S_INV] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
      if (last == 1) p.scal[S_SIGMA1] = nrm;
      if (last == 2) p.scal[S_SIGMA2] = nrm;
      p.iscal[I_COUNTER] = 0;
      p.iscal[I_PP] = p.iscal[I_PP] + 1;
    }
  }
}

__global__ __launch_bounds__(GEMV_THREADS) void k_gemv(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                       int nprob, int last) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (p.prec == F64) gemv_block<double>(p, t, last);
  else gemv_block<float>(p, t, last);
}

// alpha = |sigma1 - sigma2| (Alg. 5 line 4); E_ALPHA unless positive and finite.
__global__ void k_alpha(const Prob* __restrict__ probs, const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  if (threadIdx.x != 0) return;
  const double a = fabs(p.scal[S_SIGMA1] - p.scal[S_SIGMA2]);
  p.scal[S_ALPHA] = a;
  if (!(a > 0.0) || !isfinite(a)) set_status(p, PSDPROJ_E_ALPHA);
}

// Per-run initialisation of the device scalars (no memset nodes: a kernel clears them).
__global__ void k_setup(const Prob* __restrict__ probs, const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  for (int i = threadIdx.x; i < NISCAL; i += blockDim.x) p.iscal[i] = 0;
  for (int i = threadIdx.x; i < NSCAL; i += blockDim.x) p.scal[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0 && p.variant == PSDPROJ_SCALED && p.alpha_mode == 0) p.scal[S_ALPHA] = p.alpha_in;
}

__global__ void k_finalize(const Prob* __restrict__ probs, const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  if (threadIdx.x != 0) return;
  psdproj_result out;
  out.status = p.iscal[I_STATUS];
  out.r_plus = p.iscal[I_RPLUS];
  out.alpha_used = (p.variant == PSDPROJ_SCALED) ? p.scal[S_ALPHA] : 0.0;
  out.sigma1 = p.scal[S_SIGMA1];
  out.sigma2 = p.scal[S_SIGMA2];
  *p.res = out;
}

int tiles_gemv(const Prob& p) { return (p.n + GEMV_ROWS - 1) / GEMV_ROWS; }
int tiles_vec(const Prob& p) { return (p.ld + 1023) / 1024; }
int tiles_omega(const Prob& p) { return (int)(((int64_t)p.rpad * p.ld + 1023) / 1024); }

void launch_gemv(const Launch& L, int last) {
  hipLaunchKernelGGL(k_gemv, dim3(L.grid), dim3(GEMV_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, last);
}
void launch_alpha(const Launch& L) {
  hipLaunchKernelGGL(k_alpha, dim3(L.grid), dim3(64), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_setup(const Launch& L) {
  hipLaunchKernelGGL(k_setup, dim3(L.grid), dim3(64), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_finalize(const Launch& L) {
  hipLaunchKernelGGL(k_finalize, dim3(L.grid), dim3(64), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
