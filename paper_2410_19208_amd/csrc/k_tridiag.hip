// Householder tridiagonalisation C = Q_H T Q_H^T of the compressed matrix (first half of the
// symmetric eigensolve of Alg. 2 line 2 / Alg. 3 line 3), FP64, one workgroup per problem.
//
// The upper-triangle 16x16 tiles of the symmetric r_pad x r_pad matrix live in registers.  A
// wave owns whole column blocks, paired as J and nb-1-J so every wave holds nb+1 tiles; lane l
// of a tile holds row l/4, columns 4*(l%4) .. +3.  Step j (j = 0 .. r-3), three barriers:
//   1. row j is in LDS (published by its owners at the end of the previous step, with the
//      per-wave sums of squares of its entries past the subdiagonal); every wave forms the
//      reflector H_j = I - tau v v^T mapping C[j+1:, j] to beta e_1 with identical arithmetic,
//      and a private LDS copy of v;
//   2. products with the trailing block C2: per tile the row sums C_IJ v_J (quad reduction)
//      go to LDS, the column sums C_IJ^T v_I accumulate over a column block and are reduced
//      once per block, and each wave adds its part of v^T C2 v;
//   3. one thread per row: p_i = tau (C2 v)_i from the row-block and column-block terms in a
//      fixed order, K = tau/2 p^T v = tau^2/2 v^T C2 v, w = p - K v, shared through LDS;
//   4. C2 -= v w^T + w v^T on the registers; the owners of row j+1 publish it.
// v and w vanish outside C2, so the products and the update need no masks; tiles left of or
// above C2 are skipped (wave-uniform tests).
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
  c[0] += dpp_perm_f64<DPP_ROR4>(c[0]);
  c[0] += dpp_perm_f64<DPP_ROR8>(c[0]);
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
  __shared__ double rowbuf[2][PSDPROJ_MAX_RANK];        // row j of the reduced matrix (double-buffered)
  __shared__ double sqp[2][TD_WAVES];                   // per-wave parts of ||row j, columns >= j+2||^2
  __shared__ double rpart[TD_NB][TD_NB / 2][16][2];     // [I][J/2][row][J%2]: C_IJ v_J (zero where J < I)
  __shared__ double cpart[TD_NB][16];                   // [J][col]: sum over I < J of C_IJ^T v_I
  __shared__ double kpart[TD_WAVES];                    // per-wave parts of v^T C2 v
  __shared__ double2 vw[PSDPROJ_MAX_RANK];              // (v_i, w_i)
  __shared__ double vpw[TD_WAVES][PSDPROJ_MAX_RANK];    // per-wave copy of v (no barrier needed)
  double* __restrict__ vp = vpw[wave];

  for (int e = tid; e < TD_NB * 16 * TD_NB; e += TD_THREADS) (&rpart[0][0][0][0])[e] = 0.0;

  // column blocks of this wave: bA = wave, bB = nb-1-wave (bB used only when bB > bA).  bA is
  // re-read through an empty asm at the start of each phase so that the per-slot conditions
  // derived from it are scalar compares made where they are used, not lane masks kept live
  // across the whole loop.
  int bA = wave;
  auto refresh = [&] { __asm__ volatile("" : "+s"(bA)); };
  auto blkJ = [&](int blk) { return blk ? nb - 1 - bA : bA; };
  auto blk_has = [&](int blk) { return blk ? bA < nb - 1 - bA : bA <= nb - 1 - bA; };
  // slot s: s <= bA -> tile (s, bA); else tile (s - bA - 1, bB)
  auto slot_ij = [&](int s, int& I, int& J) {
    if (s <= bA) { I = s; J = bA; }
    else { I = s - bA - 1; J = nb - 1 - bA; }
  };
  auto slot_ok = [&](int s) { return s <= bA ? blk_has(0) : (blk_has(1) && s - bA - 1 <= nb - 1 - bA); };
  constexpr int SA_END = NS < 8 ? NS : 8;   // bA <= (nb - 1) / 2 <= 7 whenever block A exists
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

  // Row jn of the registers -> rowbuf[jn & 1]; the squares of its entries in columns >= jn+2
  // summed per wave -> sqp[jn & 1][wave] (zero from waves holding none of the row).
  auto publish_part = [&](int s, int jn, double& sq) {
    int I, J;
    slot_ij(s, I, J);
    if (I == (jn >> 4) && lr == (jn & 15)) {   // scalar test first, then the lane test
      const int b0 = 16 * J + 4 * lc;
      double* dst = rowbuf[jn & 1] + b0;
      *(double2*)dst = double2{reg[s][0], reg[s][1]};
      *(double2*)(dst + 2) = double2{reg[s][2], reg[s][3]};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (b0 + q >= jn + 2) sq = fma(reg[s][q], reg[s][q], sq);
    }
  };
  auto publish_sq = [&](int jn, double sq) {
    sq += dpp_perm_f64<DPP_XOR1>(sq);
    sq += dpp_perm_f64<DPP_XOR2>(sq);
    if (lane == 4 * (jn & 15)) sqp[jn & 1][wave] = sq;
  };
  {
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (slot_ok(s)) publish_part(s, 0, sq);
    publish_sq(0, sq);
  }

  for (int j = 0; j + 2 < r; ++j) {
    lds_barrier();
    const double* __restrict__ buf = rowbuf[j & 1];
    // block index of column j in a scalar register, so that the per-slot tests below are
    // scalar compares and branches
    const int jb = __builtin_amdgcn_readfirstlane(j) >> 4;
    // 1. reflector H_j = I - tau v v^T mapping C[j+1:, j] to beta e_1 (same arithmetic in
    //    every wave): alpha = C[j+1][j], sigma = ||C[j+2:, j]||^2; tau = 0 when sigma = 0.
    //    sqrt and the two reciprocals are hardware estimates refined by Goldschmidt / Newton
    //    steps (no IEEE division on the chain).
    double sigma = 0.0;
#pragma unroll
    for (int w = 0; w < TD_WAVES; ++w) sigma += sqp[j & 1][w];
    const double alpha = buf[j + 1];
    const double x2 = fma(alpha, alpha, sigma);
    const double y0 = __builtin_amdgcn_rsq(x2);
    double g = x2 * y0, h = 0.5 * y0;
    const double e0 = fma(-h, g, 0.5);
    g = fma(g, e0, g);
    h = fma(h, e0, h);
    g = fma(fma(-g, g, x2), h, g);
    g = fma(fma(-g, g, x2), h, g);   // g = sqrt(alpha^2 + sigma)
    double bt = (alpha <= 0.0) ? g : -g;
    double rb = rcp_f64(bt), ra = rcp_f64(alpha - bt);
    if (!(x2 > 1e-280 && x2 < 1e280)) {   // far from 1: IEEE sqrt and division (same in all lanes)
      const double mu = sqrt(x2);
      bt = (alpha <= 0.0) ? mu : -mu;
      rb = 1.0 / bt;
      ra = 1.0 / (alpha - bt);
    }
    const bool refl = sigma > 0.0;
    const double beta = refl ? bt : alpha;
    const double tau = refl ? (bt - alpha) * rb : 0.0;
    const double sc = refl ? ra : 0.0;
    // v_i: 0 (i <= j), 1 (i = j+1), C[i][j] * sc (i >= j+2); zero in the padding (>= r).
    // With tau = 0 the step below leaves the registers unchanged (w = 0).
    auto vval = [&](int i, double x) { return (i > j + 1) ? x * sc : (i == j + 1 ? 1.0 : 0.0); };
    {
      const int i0 = 4 * lane;
      if (i0 < rp) {
        const double2 x01 = *(const double2*)(buf + i0);
        const double2 x23 = *(const double2*)(buf + i0 + 2);
        *(double2*)(vp + i0) = double2{vval(i0, x01.x), vval(i0 + 1, x01.y)};
        *(double2*)(vp + i0 + 2) = double2{vval(i0 + 2, x23.x), vval(i0 + 3, x23.y)};
      }
    }
    lds_wave_sync();

    // 2. products with the trailing block C2 (v vanishes outside it, so no masking): per tile
    //    the row sums C_IJ v_J (quad reduction) -> rpart; the column sums C_IJ^T v_I over a
    //    column block -> cpart; v^T C2 v from the lane partials -> kpart.
    double kv = 0.0;
    refresh();
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int J = blkJ(blk);
      const bool have = blk_has(blk);
      if (!have || J < jb) continue;   // uniform: no trailing columns in this block
      const int b0 = 16 * J + 4 * lc;
      const double2 v01 = *(const double2*)(vp + b0);
      const double2 v23 = *(const double2*)(vp + b0 + 2);
      const double vb[4] = {v01.x, v01.y, v23.x, v23.y};
      double cs[4] = {0.0, 0.0, 0.0, 0.0};
      // The block's slots hold row blocks 0 .. J in slot order; they are taken from I = J down
      // to I = jb, and v at the next slot's rows is loaded one slot ahead into the other of two
      // registers chosen by slot parity (both start with the first slot's value), so that no
      // copies are needed where the skipped slots above the block join the chain.
      const int slo = blk ? bA + 1 : 0, shi = slo + J;   // slots of this block
      double vx[2];
      vx[0] = vx[1] = vp[16 * J + lr];
#pragma unroll
      for (int s = (blk ? NS : SA_END) - 1; s >= blk; --s) {   // block A slots: s <= bA <= 7
        if (s > shi) continue;              // above the block (before the chain starts)
        const int I = s - slo;
        if (s < slo || I < jb) break;       // end of the block or of the trailing rows
        const double va = vx[s & 1];
        vx[(s + 1) & 1] = vp[16 * max(I - 1, 0) + lr];
        double rs = reg[s][0] * vb[0];
        rs = fma(reg[s][1], vb[1], rs);
        rs = fma(reg[s][2], vb[2], rs);
        rs = fma(reg[s][3], vb[3], rs);
        kv = fma(va, rs, kv);
        const double vc = (I != J) ? va : 0.0;   // the diagonal tile has no mirrored part
#pragma unroll
        for (int q = 0; q < 4; ++q) cs[q] = fma(reg[s][q], vc, cs[q]);
        rs += dpp_perm_f64<DPP_XOR1>(rs);
        rs += dpp_perm_f64<DPP_XOR2>(rs);
        rpart[I][J >> 1][lr][J & 1] = rs;   // the four lanes of the quad store the same sum
      }
      // the tiles above the diagonal count twice in v^T C2 v: once more through the column sums
#pragma unroll
      for (int q = 0; q < 4; ++q) kv = fma(cs[q], vb[q], kv);
      colsum16(cs, lane);
      if ((lane & 12) == 0) cpart[J][4 * lc + ((lane >> 4) & 3)] = cs[0];
    }
    kv = wave_allsum(kv);
    if (lane == 0) kpart[wave] = kv;
    lds_barrier();

    // 3. p = tau C2 v, K = tau/2 p^T v = tau^2/2 v^T C2 v, w = p - K v -> vv, wv (shared);
    //    v_j (entries j+2 ..) into column j of H, and d_j, e_j, tau_j.
    if (tid < rp) {
      const int i = tid, ib = i >> 4, ii = i & 15;
      double s = 0.0;
#pragma unroll
      for (int J = 0; J < TD_NB; J += 2) {
        const double2 t = *(const double2*)&rpart[ib][J >> 1][ii][0];   // consecutive rows: no bank conflicts
        s += t.x;
        s += t.y;
      }
      s += cpart[ib][ii];
      double vcv = 0.0;
#pragma unroll
      for (int w = 0; w < TD_WAVES; ++w) vcv += kpart[w];
      const double K = 0.5 * tau * tau * vcv;
      const double vi = vval(i, buf[i]);
      const double pi_ = (i > j && i < r) ? tau * s : 0.0;
      vw[i] = double2{vi, pi_ - K * vi};
      if (i >= j + 2 && i < r) Hm[(int64_t)j * rp + i] = vi;
      if (i == 0) {
        tdm[j] = buf[j];
        tem[j] = beta;
        taum[j] = tau;
      }
    }
    lds_barrier();

    // 4. C2 -= v w^T + w v^T on the registers (v, w vanish outside C2), and row j+1 published
    //    for the next step.
    double sq = 0.0;
    const int jn = __builtin_amdgcn_readfirstlane(j + 1);
    refresh();
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int J = blkJ(blk);
      const bool have = blk_has(blk);
      if (!have || J < jb) continue;
      const int b0 = 16 * J + 4 * lc;
      double vb[4], wb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 t = vw[b0 + q];
        vb[q] = t.x;
        wb[q] = t.y;
      }
      const int slo = blk ? bA + 1 : 0, shi = slo + J;   // slots of this block, as above
      double2 tx[2];
      tx[0] = tx[1] = vw[16 * J + lr];
#pragma unroll
      for (int s = (blk ? NS : SA_END) - 1; s >= blk; --s) {
        if (s > shi) continue;
        const int I = s - slo;
        if (s < slo || I < jb) break;
        const double2 t = tx[s & 1];
        tx[(s + 1) & 1] = vw[16 * max(I - 1, 0) + lr];
        const double va = t.x, wa = t.y;
#pragma unroll
        for (int q = 0; q < 4; ++q) reg[s][q] = fma(-va, wb[q], fma(-wa, vb[q], reg[s][q]));
      }
    }
    {
      // the tiles of row block jn/16: slot jn/16 of block A, slot bA+1+jn/16 of block B
      const int nbI = jn >> 4;
      const int sA = (blk_has(0) && nbI <= bA) ? nbI : -1;
      const int sB = (blk_has(1) && nbI <= nb - 1 - bA) ? bA + 1 + nbI : -1;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s != sA && s != sB) continue;
        const int J = (s == sA) ? bA : nb - 1 - bA;
        if (lr == (jn & 15)) {
          const int b0 = 16 * J + 4 * lc;
          double* dst = rowbuf[jn & 1] + b0;
          *(double2*)dst = double2{reg[s][0], reg[s][1]};
          *(double2*)(dst + 2) = double2{reg[s][2], reg[s][3]};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (b0 + q >= jn + 2) sq = fma(reg[s][q], reg[s][q], sq);
        }
      }
    }
    publish_sq(jn, sq);
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
    p.scal[S_GL] = gl;
    p.scal[S_GU] = gu;
    p.scal[S_PIVMIN] = pivmin;
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
