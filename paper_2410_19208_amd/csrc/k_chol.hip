// CholeskyQR2 orthonormalisation of the sketch (the economy-QR "orth" step of Alg. 1):
//   G = Y^T Y, G = R^T R, Q1 = Y R^-1; then once more on Q1.
// The range of Q equals the range of Y for any invertible R, which is all the method uses.
//
// k_chol (one workgroup of 16 waves per problem): right-looking Cholesky with the upper
// triangle of G held in registers as 16x16 FP64 tiles (tile t of the upper triangle lives in
// wave t mod 16; lane l holds row l%16, columns 4*(l/16)..+3 of it).  Step j broadcasts the
// pivot row through LDS (double-buffered, one barrier per step) and every lane applies the
// rank-1 update to its own elements.  A column whose Schur pivot is below tol * (its Gram
// diagonal) lies in the span of the previous columns to working precision; it is dropped
// (zero row of R, zero column of Q), which leaves the range unchanged.  R goes to H, and the
// inverses of R's 16x16 diagonal blocks to the diagonal blocks of F.
//
// k_apply, rounds 0/1: Q = Y R^-1 by blocked forward substitution on v_mfma_f64_16x16x4f64,
//   Q_J = (Y_J - sum_{I<J} Q_I R_IJ) R_JJ^-1   (16-column blocks; each wave owns 16 rows).
// k_apply, round 2: the rebuild factor W = Q F with F = V_keep diag(sqrt(w)) (row-major out).
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int CH_WAVES = SYM_WAVES;
constexpr int CH_THREADS = SYM_THREADS;
constexpr int CH_SLOTS = SYM_SLOTS;

__global__ __launch_bounds__(CH_THREADS) void k_chol(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob, int round) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int r = p.r, rp = p.rpad, nb = rp / 16, nt = nb * (nb + 1) / 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, kg = lane >> 4;
  const double* __restrict__ G = p.G;
  double* __restrict__ H = p.H;
  double* __restrict__ F = p.F;
  __shared__ double rowbuf[2][PSDPROJ_MAX_RANK];
  __shared__ double g0[PSDPROJ_MAX_RANK];
  __shared__ int dflag[PSDPROJ_MAX_RANK];
  const double tol = (p.prec == F64) ? 1e-26 : 1e-13;

  for (int j = tid; j < rp; j += CH_THREADS) g0[j] = (j < r) ? G[(int64_t)j * rp + j] : 0.0;

  double reg[CH_SLOTS][4];
  int tI[CH_SLOTS], tJ[CH_SLOTS];
#pragma unroll
  for (int s = 0; s < CH_SLOTS; ++s) {
    const int t = wave + s * CH_WAVES;
    int I = nb, J = nb;  // inactive slot: beyond every index
    if (t < nt) upper_tile(t, nb, I, J);
    tI[s] = I;
    tJ[s] = J;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 16 * I + li, b = 16 * J + 4 * kg + q;
      reg[s][q] = (t < nt) ? G[(int64_t)b * rp + a] : 0.0;
    }
  }
  __syncthreads();

  int ndrop = 0;
  for (int j = 0; j < r; ++j) {
    double* buf = rowbuf[j & 1];
    const int jb = j >> 4, ji = j & 15;
    // owners publish row j (columns b >= j) of the current Schur complement
#pragma unroll
    for (int s = 0; s < CH_SLOTS; ++s) {
      if (tI[s] == jb && li == ji) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int b = 16 * tJ[s] + 4 * kg + q;
          if (b >= j) buf[b] = reg[s][q];
        }
      }
    }
    __syncthreads();
    const double d = buf[j], gj = g0[j];
    const bool dr = !(gj > 0.0) || !(d > tol * gj) || !isfinite(d);
    const double piv = dr ? 0.0 : sqrt(d);
    const double ip = dr ? 0.0 : 1.0 / piv;
    ndrop += dr;
    if (tid == 0) dflag[j] = dr;
#pragma unroll
    for (int s = 0; s < CH_SLOTS; ++s) {
      if (tJ[s] >= nb || tJ[s] < jb) continue;       // inactive, or entirely left of column j
      const int a = 16 * tI[s] + li;
      if (a < j) continue;                            // rows of R already final
      const double ua = buf[a] * ip;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 16 * tJ[s] + 4 * kg + q;
        if (a == j) {
          if (b > j) reg[s][q] = buf[b] * ip;
          else if (b == j) reg[s][q] = dr ? 1.0 : piv;
        } else if (b > j) {
          reg[s][q] -= ua * (buf[b] * ip);
        }
      }
    }
  }
  for (int j = r + tid; j < rp; j += CH_THREADS) dflag[j] = 1;
  // R (upper triangle, zero-padded) to H
#pragma unroll
  for (int s = 0; s < CH_SLOTS; ++s) {
    if (tJ[s] >= nb) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 16 * tI[s] + li, b = 16 * tJ[s] + 4 * kg + q;
      if (a <= b) H[(int64_t)b * rp + a] = (a < r && b < r) ? reg[s][q] : ((a == b) ? 1.0 : 0.0);
      else H[(int64_t)b * rp + a] = 0.0;
    }
  }
  __syncthreads();
  // inverses of the 16x16 diagonal blocks of R: wave I, lane c < 16 solves R_II x = e_c
  if (wave < nb && lane < 16) {
    const int I = wave, c = lane, base = 16 * I;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = 0.0;
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      if (i > c) continue;
      const int gi = base + i;
      double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = i + 1; k < 16; ++k)
        if (k <= c) s -= H[(int64_t)(base + k) * rp + gi] * x[k];
      x[i] = dflag[gi] ? 0.0 : s / H[(int64_t)gi * rp + gi];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) F[(int64_t)(base + c) * rp + base + i] = x[i];
  }
  if (tid == 0) p.iscal[I_NDROP] = ndrop;
  (void)round;
}

// ------------------------------------------------------------------ apply
constexpr int AP_WAVES = 4;
constexpr int AP_THREADS = AP_WAVES * WAVE;

template <typename T>
__device__ void apply_tri(const Prob& p, int round, int tile, double* Qs) {
  const int rp = p.rpad, nb = rp / 16, ld = p.ld, qld = rp + 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, kg = lane >> 4;
  const int rowbase = tile * APPLY_ROWS + wave * 16;
  const T* __restrict__ in = (const T*)((round == 0) ? p.y : p.q1);
  T* __restrict__ out = (T*)((round == 0) ? p.q1 : p.zm);
  const double* __restrict__ R = p.H;
  const double* __restrict__ Dinv = p.F;
  double* Qw = Qs + (size_t)wave * 16 * qld;   // this wave's 16 rows, row-major
  for (int J = 0; J < nb; ++J) {
    f64x4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = (double)in[(int64_t)(16 * J + li) * ld + rowbase + 4 * v + kg];
    for (int I = 0; I < J; ++I) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 16 * I + 4 * kk + kg;
        const double a = Qw[li * qld + k];
        const double b = R[(int64_t)(16 * J + li) * rp + k];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Qw[(4 * v + kg) * qld + 16 * J + li] = acc[v];
    __syncthreads();
    f64x4 q = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + kg;
      const double a = Qw[li * qld + 16 * J + k];
      const double b = Dinv[(int64_t)(16 * J + li) * rp + 16 * J + k];
      q = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, q, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rowbase + 4 * v + kg;
      const int64_t o = (int64_t)(16 * J + li) * ld + row;
      Qw[(4 * v + kg) * qld + 16 * J + li] = q[v];
      const T val = (T)q[v];
      out[o] = val;
      if (round == 1 && p.prec == B3) {
        const bf16 h = (bf16)(float)val;
        p.zhi[o] = h;
        p.zlo[o] = (bf16)((float)val - (float)h);
      }
    }
    __syncthreads();
  }
}

// W = Q F, F = V_keep diag(sqrt(w)) (columns >= r_plus are zero); row-major output.
template <typename T>
__device__ void apply_factor(const Prob& p, int tile) {
  const int rp = p.rpad, nb = rp / 16, ld = p.ld, kw = p.rwpad;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, kg = lane >> 4;
  const int rowbase = tile * APPLY_ROWS + wave * 16;
  const int rplus = min(max(p.iscal[I_RPLUS], 0), rp);
  const T* __restrict__ Q = (const T*)p.zm;
  const double* __restrict__ F = p.F;
  for (int J = 0; J < kw / 16; ++J) {
    f64x4 acc = {0, 0, 0, 0};
    if (16 * J < rplus) {
      const bool colok = (16 * J + li) < rplus;
      for (int I = 0; I < nb; ++I) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 16 * I + 4 * kk + kg;
          const double a = (double)Q[(int64_t)k * ld + rowbase + li];
          const double b = colok ? F[(int64_t)(16 * J + li) * rp + k] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t o = (int64_t)(rowbase + 4 * v + kg) * kw + 16 * J + li;
      if (p.prec == F64) {
        ((double*)p.wf)[o] = acc[v];
      } else {
        const float f = (float)acc[v];
        ((float*)p.wf)[o] = f;
        if (p.prec == B3) {
          const bf16 h = (bf16)f;
          p.whi[o] = h;
          p.wlo[o] = (bf16)(f - (float)h);
        }
      }
    }
  }
}

__global__ __launch_bounds__(AP_THREADS) void k_apply(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                      int nprob, int round) {
  extern __shared__ double qs_smem[];
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (t * APPLY_ROWS >= p.ld) return;
  if (round == 2) {
    if (p.prec == F64) apply_factor<double>(p, t);
    else apply_factor<float>(p, t);
  } else {
    if (p.prec == F64) apply_tri<double>(p, round, t, qs_smem);
    else apply_tri<float>(p, round, t, qs_smem);
  }
}

int tiles_small(const Prob&) { return 1; }
int tiles_apply(const Prob& p) { return p.ld / APPLY_ROWS; }

static size_t apply_smem() { return (size_t)AP_WAVES * 16 * (PSDPROJ_MAX_RANK + 2) * sizeof(double); }

void apply_init() {
  hipFuncSetAttribute((const void*)k_apply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)apply_smem());
}

void launch_chol(const Launch& L, int round) {
  hipLaunchKernelGGL(k_chol, dim3(L.grid), dim3(CH_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
}
void launch_apply(const Launch& L, int round) {
  hipLaunchKernelGGL(k_apply, dim3(L.grid), dim3(AP_THREADS), apply_smem(), L.stream, L.probs, L.tstart, L.nprob,
                     round);
}

}  // namespace psd
