// CholeskyQR2 orthonormalisation of the sketch (the economy-QR "orth" step of Alg. 1):
//   G = Y^T Y, G = R^T R, Q1 = Y R^-1; then once more on Q1.
// The range of Q equals the range of Y for any invertible R, which is all the method uses.
//
// k_chol: one workgroup per problem factors G (FP64, upper triangle) and inverts R.
// A column whose Schur pivot is below tol * (its Gram diagonal) lies in the span of the
// previous columns to working precision; it is dropped (its row and column of R^-1 are zero),
// which leaves the range unchanged.
// k_apply: out = in * F for an n x r_pad panel and an r_pad x r_pad FP64 matrix F.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int CHOL_THREADS = 256;

__global__ __launch_bounds__(CHOL_THREADS) void k_chol(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                       int nprob, int round) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int r = p.r, rp = p.rpad;
  double* __restrict__ G = p.G;      // input Gram (column-major, ld rp)
  double* __restrict__ H = p.H;      // working copy -> R in its upper triangle
  double* __restrict__ F = p.F;      // R^-1
  int* __restrict__ drop = p.drop;
  __shared__ double rowj[PSDPROJ_MAX_RANK];
  __shared__ double s_piv;
  __shared__ int s_drop, s_ndrop;
  const double tol = (p.prec == F64) ? 1e-26 : 1e-13;

  for (int64_t e = threadIdx.x; e < (int64_t)rp * rp; e += CHOL_THREADS) H[e] = G[e];
  if (threadIdx.x == 0) s_ndrop = 0;
  __syncthreads();

  for (int j = 0; j < r; ++j) {
    if (threadIdx.x == 0) {
      const double d = H[(int64_t)j * rp + j];
      const double g0 = G[(int64_t)j * rp + j];
      const int dr = !(g0 > 0.0) || !(d > tol * g0) || !isfinite(d);
      s_drop = dr;
      s_piv = dr ? 0.0 : sqrt(d);
      drop[j] = dr;
      s_ndrop += dr;
    }
    __syncthreads();
    const int dr = s_drop;
    const double piv = s_piv;
    for (int k = j + 1 + threadIdx.x; k < r; k += CHOL_THREADS) {
      const double v = dr ? 0.0 : H[(int64_t)k * rp + j] / piv;
      H[(int64_t)k * rp + j] = v;
      rowj[k] = v;
    }
    if (threadIdx.x == 0) H[(int64_t)j * rp + j] = dr ? 1.0 : piv;
    __syncthreads();
    if (!dr) {
      // trailing update of the upper triangle: H[a][b] -= R[j][a] R[j][b], j < a <= b < r
      for (int b = j + 1 + threadIdx.x; b < r; b += CHOL_THREADS) {
        const double rb = rowj[b];
        double* colb = H + (int64_t)b * rp;
        for (int a = j + 1; a <= b; ++a) colb[a] -= rowj[a] * rb;
      }
    }
    __syncthreads();
  }

  // Triangular inverse, bottom-up by rows: F[i][j] = -(sum_{k=i+1..j} R[i][k] F[k][j]) / R[i][i].
  for (int64_t e = threadIdx.x; e < (int64_t)rp * rp; e += CHOL_THREADS) F[e] = 0.0;
  __syncthreads();
  for (int i = r - 1; i >= 0; --i) {
    const int di = drop[i];
    const double inv = di ? 0.0 : 1.0 / H[(int64_t)i * rp + i];
    for (int k = i + 1 + threadIdx.x; k < r; k += CHOL_THREADS) rowj[k] = H[(int64_t)k * rp + i];
    __syncthreads();
    if (!di) {
      for (int j = i + threadIdx.x; j < r; j += CHOL_THREADS) {
        if (j == i) { F[(int64_t)i * rp + i] = inv; continue; }
        const double* colj = F + (int64_t)j * rp;
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += rowj[k] * colj[k];
        F[(int64_t)j * rp + i] = -s * inv;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    p.iscal[I_NDROP] = s_ndrop;
    if (s_ndrop >= r && round == 0 && p.variant == PSDPROJ_SCALED) set_status(p, PSDPROJ_E_BREAKDOWN);
  }
}

// out[row][c] = sum_k in[row][k] F[k][c] for one tile of APPLY_ROWS rows.
// round 0: in = pass output Y, out = Q1.  round 1: in = Q1, out = Q (pass operand, with
// the BF16 split for BF16X3).  round 2: in = Q, F = V_keep diag(sqrt w), out = the
// row-major rebuild factor (columns >= r_plus are zero).
template <typename T>
__device__ void apply_tile(const Prob& p, int round, int tile) {
  constexpr int KT = 32;                         // F rows staged per LDS pass
  constexpr int CPT = PSDPROJ_MAX_RANK / 4;      // max columns per thread
  __shared__ double Fs[KT][PSDPROJ_MAX_RANK + 1];
  const int rp = p.rpad, ld = p.ld;
  const T* in = (const T*)((round == 0) ? p.y : (round == 1) ? p.q1 : p.zm);
  const int ncols = (round == 2) ? p.rwpad : rp;
  const int rplus = (round == 2) ? p.iscal[I_RPLUS] : rp;
  const int row_l = threadIdx.x & (APPLY_ROWS - 1);
  const int cgrp = threadIdx.x / APPLY_ROWS;     // 4 column groups, strided
  const int row = tile * APPLY_ROWS + row_l;
  double acc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) acc[c] = 0.0;
  const int kmax = (round == 2) ? p.r : p.r;
  for (int k0 = 0; k0 < kmax; k0 += KT) {
    __syncthreads();
    for (int e = threadIdx.x; e < KT * ncols; e += 256) {
      const int kk = e / ncols, c = e - kk * ncols;
      const int k = k0 + kk;
      double f = 0.0;
      if (k < p.r && c < rp) f = (round == 2 && c >= rplus) ? 0.0 : p.F[(int64_t)c * rp + k];
      Fs[kk][c] = f;
    }
    __syncthreads();
    const int kn = min(KT, kmax - k0);
    for (int kk = 0; kk < kn; ++kk) {
      const double x = (double)in[(int64_t)(k0 + kk) * ld + row];
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = c * 4 + cgrp;
        if (col < ncols) acc[c] += x * Fs[kk][col];
      }
    }
  }
  // store
  if (round == 2) {
    const int64_t o = (int64_t)row * p.rwpad;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = c * 4 + cgrp;
      if (col >= ncols) continue;
      if (p.prec == F64) {
        ((double*)p.wf)[o + col] = acc[c];
      } else {
        const float f = (float)acc[c];
        ((float*)p.wf)[o + col] = f;
        if (p.prec == B3) {
          const bf16 h = (bf16)f;
          p.whi[o + col] = h;
          p.wlo[o + col] = (bf16)(f - (float)h);
        }
      }
    }
  } else {
    T* out = (T*)((round == 0) ? p.q1 : p.zm);
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = c * 4 + cgrp;
      if (col >= rp) continue;
      const int64_t o = (int64_t)col * ld + row;
      const T v = (T)acc[c];
      out[o] = v;
      if (round == 1 && p.prec == B3) {
        const bf16 h = (bf16)(float)v;
        p.zhi[o] = h;
        p.zlo[o] = (bf16)((float)v - (float)h);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_apply(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                               int nprob, int round) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (t * APPLY_ROWS >= p.ld) return;
  if (p.prec == F64) apply_tile<double>(p, round, t);
  else apply_tile<float>(p, round, t);
}

int tiles_small(const Prob&) { return 1; }
int tiles_apply(const Prob& p) { return p.ld / APPLY_ROWS; }

void launch_chol(const Launch& L, int round) {
  hipLaunchKernelGGL(k_chol, dim3(L.grid), dim3(CHOL_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
}
void launch_apply(const Launch& L, int round) {
  hipLaunchKernelGGL(k_apply, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob, round);
}

}  // namespace psd
