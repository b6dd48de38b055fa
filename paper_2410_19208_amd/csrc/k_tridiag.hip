// Householder tridiagonalisation C = Q_H T Q_H^T of the compressed matrix (first half of the
// symmetric eigensolve of Alg. 2 line 2 / Alg. 3 line 3), FP64, one workgroup per problem.
//
// The upper-triangle 16x16 tiles of the symmetric r_pad x r_pad matrix live in registers.  A
// wave owns whole column blocks, paired as J and nb-1-J so every wave holds nb+1 tiles; lane l
// of a tile holds row l/4, columns 4*(l%4) .. +3.  Step j (j = 0 .. r-3):
//   1. the owners of row j publish it through LDS (double-buffered);
//   2. every wave forms the reflector H_j = I - tau v v^T that maps C[j+1:, j] to beta e_1
//      (redundantly, identical arithmetic in every wave, so no extra barrier);
//   3. p = tau C2 v (C2 = trailing block): per tile, the row sums C_IJ v_J (a quad reduction
//      with DPP moves) go to LDS; the column sums C_IJ^T v_I accumulate in registers over a
//      column block and are reduced once per block (16-lane reduce-scatter); p_i adds the nb
//      row-block terms and the column-block term in a fixed order; K = tau/2 p^T v,
//      w = p - K v;
//   4. C2 -= v w^T + w v^T on the registers.
// Tiles left of or above the trailing block are skipped (wave-uniform tests).
// Outputs: diagonal d and off-diagonal e of T, tau_j, the reflector vectors v (entries j+2..r-1)
// in column j of H, the Gershgorin interval, and the Sturm count nu of eigenvalues below the
// clamp threshold (0 for Alg. 2, 1 for Alg. 3): only the r - nu eigenpairs above it are kept.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int TD_WAVES = 8;
constexpr int TD_THREADS = TD_WAVES * WAVE;
constexpr int TD_NB = PSDPROJ_MAX_RANK / 16;   // 16 column blocks at most

// Column sums of a tile block: c[q] of lane l is a partial sum for column 4*(l%4) + q over the
// rows held by lane l; the 16 lanes sharing l%4 are added.  Halving over lane bits 5 and 4,
// then rotations by 4 and 8 within each 16-lane row (bits 3 and 2); afterwards the lanes with
// bits 2 and 3 clear hold the sum for column 4*(l%4) + ((l >> 4) & 3) in c[0].  Fixed order.
__device__ __forceinline__ void colsum16(double (&c)[4], int lane) {
  {
    const bool up = (lane & 32) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double lo = c[k], hi = c[k + 2];
      const double keep = up ? hi : lo, send = up ? lo : hi;
      c[k] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool up = (lane & 16) != 0;
    const double keep = up ? c[1] : c[0], send = up ? c[0] : c[1];
    c[0] = keep + __shfl_xor(send, 16, 64);
  }
  c[0] += dpp_f64<DPP_ROR4>(c[0]);
  c[0] += dpp_f64<DPP_ROR8>(c[0]);
}

template <int NS>   // register slots per wave: nb + 1 (15: r_pad <= 224, 17: r_pad = 256)
__global__ __launch_bounds__(TD_THREADS) void k_tridiag(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                        int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int r = p.r, rp = p.rpad, nb = rp / 16;
  const gmem<const double>* __restrict__ Cm = gp((const double*)p.C);
  gmem<double>* __restrict__ Hm = gp(p.H);
  gmem<double>* __restrict__ tdm = gp(p.td);
  gmem<double>* __restrict__ tem = gp(p.te);
  gmem<double>* __restrict__ taum = gp(p.tau);
  const int tid = threadIdx.x, wave = wave_id(), lane = tid & 63, lr = lane >> 2, lc = lane & 3;
  __shared__ double rowbuf[2][PSDPROJ_MAX_RANK];
  __shared__ double rpart[TD_NB][TD_NB][16];   // [I][J][row]: C_IJ v_J
  __shared__ double cpart[TD_NB][16];          // [J][col]: sum over I < J of C_IJ^T v_I
  __shared__ double pvec[PSDPROJ_MAX_RANK];

  // column blocks of this wave: bA = wave, bB = nb-1-wave (bB used only when bB > bA)
  const int bA = wave, bB = nb - 1 - wave;
  const bool hasA = bA <= bB;
  const bool hasB = bA < bB;
  // slot s: s <= bA -> tile (s, bA); else tile (s - bA - 1, bB)
  auto slot_ij = [&](int s, int& I, int& J) {
    if (s <= bA) { I = s; J = bA; }
    else { I = s - bA - 1; J = bB; }
  };
  auto slot_ok = [&](int s) { return s <= bA ? hasA : (hasB && s - bA - 1 <= bB); };

  double reg[NS][4];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    int I, J;
    slot_ij(s, I, J);
    const bool ok = slot_ok(s);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 16 * I + lr, b = 16 * J + 4 * lc + q;
      reg[s][q] = ok ? Cm[(int64_t)b * rp + a] : 0.0;
    }
  }

  for (int j = 0; j + 2 < r; ++j) {
    double* buf = rowbuf[j & 1];
    const int jb = j >> 4, ji = j & 15;
    // 1. publish row j: slot I = jb of every column block J >= jb (entries left of j unused)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      int I, J;
      slot_ij(s, I, J);
      if (slot_ok(s) && I == jb && lr == ji) {
        double* dst = buf + 16 * J + 4 * lc;
        *(double2*)dst = double2{reg[s][0], reg[s][1]};
        *(double2*)(dst + 2) = double2{reg[s][2], reg[s][3]};
      }
    }
    lds_barrier();
    // 2. reflector: x = buf[j+1 ..], sigma = ||x[1:]||^2 (wave reduction, same in every wave)
    double part = 0.0;
    for (int i = j + 2 + lane; i < r; i += WAVE) part += buf[i] * buf[i];
    const double sigma = wave_allsum(part);
    const double alpha = buf[j + 1];
    double tau = 0.0, beta = alpha, sc = 0.0;
    if (sigma > 0.0) {
      const double mu = sqrt(alpha * alpha + sigma);
      beta = (alpha <= 0.0) ? mu : -mu;
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      tdm[j] = buf[j];
      tem[j] = beta;
      taum[j] = tau;
    }
    for (int i = j + 2 + tid; i < r; i += TD_THREADS) Hm[(int64_t)j * rp + i] = buf[i] * sc;
    if (tau == 0.0) continue;   // uniform: every wave computed the same tau
    // v_i: 0 (i <= j), 1 (i = j+1), buf[i] * sc (i >= j+2); padding (>= r) is zero in buf
    auto vval = [&](int i, double x) { return (i > j + 1) ? x * sc : (i == j + 1 ? 1.0 : 0.0); };

    // 3a. row sums per tile -> rpart; column sums per column block -> cpart
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int J = blk ? bB : bA;
      const bool have = blk ? hasB : hasA;
      if (!have || 16 * J + 15 <= j) continue;   // uniform: no trailing columns in this block
      const int b0 = 16 * J + 4 * lc;
      const double2 x01 = *(const double2*)(buf + b0);
      const double2 x23 = *(const double2*)(buf + b0 + 2);
      const double vb[4] = {vval(b0, x01.x), vval(b0 + 1, x01.y), vval(b0 + 2, x23.x), vval(b0 + 3, x23.y)};
      double cs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        int I, JJ;
        slot_ij(s, I, JJ);
        if ((s <= bA) != (blk == 0) || !slot_ok(s)) continue;   // compile-time slot, uniform block
        if (16 * I + 15 <= j) continue;                          // uniform: rows all above the block
        const int a = 16 * I + lr;
        const double va = vval(a, buf[a]);
        const bool ra = a > j;
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double x = (ra && b0 + q > j) ? reg[s][q] : 0.0;
          rs += x * vb[q];
          if (I != J) cs[q] += x * va;
        }
        rs += dpp_f64<DPP_XOR1>(rs);
        rs += dpp_f64<DPP_XOR2>(rs);
        if (lc == 0) rpart[I][J][lr] = rs;
      }
      colsum16(cs, lane);
      if ((lane & 12) == 0) cpart[J][4 * lc + ((lane >> 4) & 3)] = cs[0];
    }
    lds_barrier();
    // 3b. p_i = tau * (sum_{J >= i/16} C_{i/16,J} v_J + sum_{I < i/16} C_{I,i/16}^T v_I)
    for (int i = tid; i < rp; i += TD_THREADS) {
      double s = 0.0;
      if (i > j && i < r) {
        const int ib = i >> 4, ii = i & 15;
#pragma unroll
        for (int J = 0; J < TD_NB; ++J) {
          const double t = rpart[ib][J][ii];   // in bounds for every J; stale entries are not added
          s += (J >= ib && J < nb) ? t : 0.0;
        }
        s += cpart[ib][ii];
        s *= tau;
      }
      pvec[i] = s;   // zero outside the trailing block and in the padding
    }
    lds_barrier();
    // K = tau/2 p^T v (wave reduction, same in every wave)
    double dp = 0.0;
    for (int i = j + 1 + lane; i < r; i += WAVE) dp += pvec[i] * vval(i, buf[i]);
    const double K = 0.5 * tau * wave_allsum(dp);
    // 4. C2 -= v w^T + w v^T, w = p - K v (zero outside the trailing block)
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int J = blk ? bB : bA;
      const bool have = blk ? hasB : hasA;
      if (!have || 16 * J + 15 <= j) continue;
      const int b0 = 16 * J + 4 * lc;
      const double2 x01 = *(const double2*)(buf + b0);
      const double2 x23 = *(const double2*)(buf + b0 + 2);
      const double2 p01 = *(const double2*)(pvec + b0);
      const double2 p23 = *(const double2*)(pvec + b0 + 2);
      const double xb[4] = {x01.x, x01.y, x23.x, x23.y};
      const double pb[4] = {p01.x, p01.y, p23.x, p23.y};
      double vb[4], wb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        vb[q] = vval(b0 + q, xb[q]);
        wb[q] = pb[q] - K * vb[q];   // pvec is zero for b <= j
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        int I, JJ;
        slot_ij(s, I, JJ);
        if ((s <= bA) != (blk == 0) || !slot_ok(s)) continue;
        if (16 * I + 15 <= j) continue;
        const int a = 16 * I + lr;
        const double va = vval(a, buf[a]);
        const double wa = pvec[a] - K * va;
#pragma unroll
        for (int q = 0; q < 4; ++q) reg[s][q] -= va * wb[q] + wa * vb[q];
      }
    }
    // rows >= j+1 of the registers are consistent for the next step; rpart/cpart/pvec are
    // rewritten only after the next step's first barrier.
  }
  // last 2x2 (or 1x1) block
  if (r >= 2) {
    const int j = r - 2;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!slot_ok(s)) continue;
      int I, J;
      slot_ij(s, I, J);
      const int a = 16 * I + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 16 * J + 4 * lc + q;
        if (a == j && b == j) p.td[j] = reg[s][q];
        if (a == j && b == j + 1) p.te[j] = reg[s][q];
        if (a == j + 1 && b == j + 1) p.td[j + 1] = reg[s][q];
      }
    }
  } else {
    if (wave == 0 && lane == 0) p.td[0] = reg[0][0];
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
    hipLaunchKernelGGL(k_tridiag<15>, dim3(L.grid), dim3(TD_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
  else
    hipLaunchKernelGGL(k_tridiag<17>, dim3(L.grid), dim3(TD_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
