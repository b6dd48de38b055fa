// Householder tridiagonalisation C = Q_H T Q_H^T of the compressed matrix (first half of the
// symmetric eigensolve of Alg. 2 line 2 / Alg. 3 line 3), FP64, one workgroup per problem.
//
// The symmetric matrix lives in registers as upper-triangle 16x16 tiles (see SYM_* in
// common.hpp).  Step j (j = 0 .. r-3):
//   1. the owners of row j publish it through LDS (double-buffered);
//   2. every wave forms the reflector H_j = I - tau v v^T that maps C[j+1:, j] to beta e_1
//      (redundantly, identical arithmetic in every wave, so no extra barrier);
//   3. p = tau C2 v (C2 = trailing block) as per-tile partial row and column sums written to
//      LDS and summed in a fixed order, K = tau/2 p^T v, w = p - K v;
//   4. C2 -= v w^T + w v^T on the registers.
// Outputs: diagonal d and off-diagonal e of T, tau_j, the reflector vectors v (entries j+2..r-1)
// in column j of H, the Gershgorin interval, and the Sturm count nu of eigenvalues below the
// clamp threshold (0 for Alg. 2, 1 for Alg. 3): only the r - nu eigenpairs above it are kept.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

template <int NS>   // register slots per wave (14: r_pad <= 224, 17: r_pad = 256)
__global__ __launch_bounds__(SYM_THREADS) void k_tridiag(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                         int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int r = p.r, rp = p.rpad, nb = rp / 16, nt = nb * (nb + 1) / 2;
  const int tid = threadIdx.x, wave = wave_id(), lane = tid & 63, li = lane & 15, kg = lane >> 4;
  __shared__ double rowbuf[2][PSDPROJ_MAX_RANK];
  __shared__ double rpart[(PSDPROJ_MAX_RANK / 16) * (PSDPROJ_MAX_RANK / 16 + 1) / 2][16];
  __shared__ double cpart[(PSDPROJ_MAX_RANK / 16) * (PSDPROJ_MAX_RANK / 16 + 1) / 2][16];
  __shared__ double pvec[PSDPROJ_MAX_RANK];

  double reg[NS][4];
  int tI[NS], tJ[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int t = wave + s * SYM_WAVES;
    int I = nb, J = nb;
    if (t < nt) upper_tile(t, nb, I, J);
    tI[s] = I;
    tJ[s] = J;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 16 * I + li, b = 16 * J + 4 * kg + q;
      reg[s][q] = (t < nt) ? p.C[(int64_t)b * rp + a] : 0.0;
    }
  }

  for (int j = 0; j + 2 < r; ++j) {
    double* buf = rowbuf[j & 1];
    const int jb = j >> 4, ji = j & 15;
    // 1. publish row j (the 16-column strips of row block jb; entries left of j are not read)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (tI[s] == jb && tJ[s] < nb && li == ji) {
        double* dst = buf + 16 * tJ[s] + 4 * kg;
        *(double2*)dst = double2{reg[s][0], reg[s][1]};
        *(double2*)(dst + 2) = double2{reg[s][2], reg[s][3]};
      }
    }
    __syncthreads();
    // 2. reflector: x = buf[j+1 ..], sigma = ||x[1:]||^2 (wave reduction, same in every wave)
    double part = 0.0;
    for (int i = j + 2 + lane; i < r; i += WAVE) part += buf[i] * buf[i];
    const double sigma = wave_sum(part);
    const double alpha = buf[j + 1];
    double tau = 0.0, beta = alpha, sc = 0.0;
    if (sigma > 0.0) {
      const double mu = sqrt(alpha * alpha + sigma);
      beta = (alpha <= 0.0) ? mu : -mu;
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      p.td[j] = buf[j];
      p.te[j] = beta;
      p.tau[j] = tau;
    }
    for (int i = j + 2 + tid; i < r; i += SYM_THREADS) p.H[(int64_t)j * rp + i] = buf[i] * sc;
    if (tau != 0.0) {
      // v_i: 0 (i <= j), 1 (i = j+1), buf[i] * sc (i >= j+2)
      // 3a. per-tile partial sums of C2 v (rows) and of C2^T v over the tile's rows (columns)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (tJ[s] >= nb || 16 * tJ[s] + 15 <= j) continue;   // (uniform) no trailing columns here
        const int t = wave + s * SYM_WAVES;
        const int a = 16 * tI[s] + li;
        const int b0 = 16 * tJ[s] + 4 * kg;
        const double2 x01 = *(const double2*)(buf + b0);
        const double2 x23 = *(const double2*)(buf + b0 + 2);
        const double xb[4] = {x01.x, x01.y, x23.x, x23.y};
        // v restricted to the trailing block; padding (>= r) is zero in buf and in the registers
        const double va = (a > j + 1) ? buf[a] * sc : (a == j + 1 ? 1.0 : 0.0);
        const double ma = (a > j) ? 1.0 : 0.0;
        double rs = 0.0, cs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int b = b0 + q;
          const double vb = (b > j + 1) ? xb[q] * sc : (b == j + 1 ? 1.0 : 0.0);
          const double x = (b > j) ? reg[s][q] * ma : 0.0;
          rs += x * vb;
          cs[q] = x * va;
        }
        // row sums: add over the 4 lane groups holding the same row
        rs += __shfl_xor(rs, 16, 64);
        rs += __shfl_xor(rs, 32, 64);
        if (kg == 0) rpart[t][li] = rs;
        if (tI[s] != tJ[s]) {
          // column sums: add over the 16 rows of the tile
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double c = cs[q];
            c += __shfl_xor(c, 1, 64);
            c += __shfl_xor(c, 2, 64);
            c += __shfl_xor(c, 4, 64);
            c += __shfl_xor(c, 8, 64);
            if (li == 0) cpart[t][4 * kg + q] = c;
          }
        }
      }
      __syncthreads();
      // 3b. p_i = tau * (sum over tiles of row block i/16 + transposed tiles of column block i/16)
      for (int i = r + tid; i < rp; i += SYM_THREADS) pvec[i] = 0.0;   // padding stays zero
      for (int i = j + 1 + tid; i < r; i += SYM_THREADS) {
        const int ib = i >> 4, ii = i & 15;
        double s = 0.0;
        // tiles (ib, J) for J >= ib: tile index of (ib, J)
        const int trow = ib * nb - ib * (ib - 1) / 2;   // index of (ib, ib)
        for (int J = ib; J < nb; ++J) {
          if (16 * J + 15 <= j) continue;
          s += rpart[trow + (J - ib)][ii];
        }
        for (int I = 0; I < ib; ++I) {
          if (16 * ib + 15 <= j) continue;
          const int tix = I * nb - I * (I - 1) / 2 + (ib - I);
          s += cpart[tix][ii];
        }
        pvec[i] = tau * s;
      }
      __syncthreads();
      // K = tau/2 p^T v (wave reduction, same in every wave)
      double dp = 0.0;
      for (int i = j + 1 + lane; i < r; i += WAVE) {
        const double vi = (i > j + 1) ? buf[i] * sc : 1.0;
        dp += pvec[i] * vi;
      }
      const double K = 0.5 * tau * wave_sum(dp);
      // 4. C2 -= v w^T + w v^T, w = p - K v
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (tJ[s] >= nb || 16 * tJ[s] + 15 <= j) continue;
        const int a = 16 * tI[s] + li;
        const int b0 = 16 * tJ[s] + 4 * kg;
        const double2 x01 = *(const double2*)(buf + b0);
        const double2 x23 = *(const double2*)(buf + b0 + 2);
        const double xb[4] = {x01.x, x01.y, x23.x, x23.y};
        const double2 p01 = *(const double2*)(pvec + b0);
        const double2 p23 = *(const double2*)(pvec + b0 + 2);
        const double pb[4] = {p01.x, p01.y, p23.x, p23.y};
        // rows/columns outside the trailing block get zero v and w (no update there)
        const double va = (a > j + 1) ? buf[a] * sc : (a == j + 1 ? 1.0 : 0.0);
        const double wa = (a > j) ? pvec[a] - K * va : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int b = b0 + q;
          const double vb = (b > j + 1) ? xb[q] * sc : (b == j + 1 ? 1.0 : 0.0);
          const double wb = (b > j) ? pb[q] - K * vb : 0.0;
          reg[s][q] -= va * wb + wa * vb;
        }
      }
    }
    // rows >= j+1 of the registers are consistent for the next step; the rpart/cpart/pvec
    // buffers are rewritten only after the next step's first barrier.
  }
  // last 2x2 (or 1x1) block
  if (r >= 2) {
    const int j = r - 2;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (tI[s] >= nb) continue;
      const int a = 16 * tI[s] + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 16 * tJ[s] + 4 * kg + q;
        if (a == j && b == j) p.td[j] = reg[s][q];
        if (a == j && b == j + 1) p.te[j] = reg[s][q];
        if (a == j + 1 && b == j + 1) p.td[j + 1] = reg[s][q];
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (tI[s] == 0 && tJ[s] == 0 && li == 0 && kg == 0) p.td[0] = reg[s][0];
  }
  if (tid == 0) {
    if (r >= 2) p.tau[r - 2] = 0.0;
    p.tau[r - 1] = 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    // Gershgorin interval, norm, pivmin, squared off-diagonals, Sturm count at the threshold
    double gl = 1e308, gu = -1e308, emax2 = 0.0;
    for (int i = 0; i < r; ++i) {
      const double el = (i > 0) ? fabs(p.te[i - 1]) : 0.0;
      const double er = (i + 1 < r) ? fabs(p.te[i]) : 0.0;
      gl = fmin(gl, p.td[i] - el - er);
      gu = fmax(gu, p.td[i] + el + er);
      if (i + 1 < r) emax2 = fmax(emax2, p.te[i] * p.te[i]);
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    const double slack = 2.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
    gl -= slack + 1e-300;
    gu += slack + 1e-300;
    for (int i = 0; i + 1 < r; ++i) p.evals[PSDPROJ_MAX_RANK + i] = p.te[i] * p.te[i];  // e^2 scratch
    p.scal[S_TNORM] = tnorm;
    p.scal[8] = gl;
    p.scal[9] = gu;
    p.scal[10] = pivmin;
    const double thr = (p.variant == PSDPROJ_SCALED) ? 1.0 : 0.0;
    p.scal[S_THRESH] = thr;
    int nu = isfinite(tnorm) ? sturm_count(p.td, p.evals + PSDPROJ_MAX_RANK, r, thr, pivmin) : r;
    if (nu < 0) nu = 0;
    if (nu > r) nu = r;
    p.iscal[I_NU] = nu;
  }
}

void launch_tridiag(const Launch& L) {
  if (L.maxnb <= 14)
    hipLaunchKernelGGL(k_tridiag<14>, dim3(L.grid), dim3(SYM_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
  else
    hipLaunchKernelGGL(k_tridiag<17>, dim3(L.grid), dim3(SYM_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
