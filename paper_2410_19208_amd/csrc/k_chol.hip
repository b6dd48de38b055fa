// CholeskyQR2 orthonormalisation of the sketch (the economy-QR "orth" step of Alg. 1):
//   G = Y^T Y, G = R^T R, Q1 = Y R^-1; then once more on Q1.
// The range of Q equals the range of Y for any invertible R, which is all the method uses.
//
// k_chol (one workgroup of 8 waves per problem): blocked right-looking Cholesky on
// 16x16 FP64 tiles.  The upper-triangle tiles of G live in registers (tile t in wave t mod 8)
// in the result layout of v_mfma_f64_16x16x4f64 (lane l holds rows 4v + l/16,
// column l%16), which is also that instruction's B-operand layout.  For each block column J:
//   A. the owner of tile (J,J) factors it in registers by row operations on [W_JJ | I] (lane c
//      holds column c of W_JJ, lane 16 + c column c of I; pivots and multipliers broadcast
//      with readlane), which leaves R_JJ on the left and R_JJ^-T on the right;
//   B. the panel tiles become R_JK = R_JJ^-T W_JK (MFMA; B operand straight from registers);
//   C. the trailing tiles take W_KL -= R_JK^T R_JL (MFMA; operands from the panel in LDS).
// A column whose Schur pivot is below tol * (its Gram diagonal) lies in the span of the
// previous columns to working precision; it is dropped (zero row of R and zero column of
// R_JJ^-1, hence a zero column of Q), which leaves the range unchanged.  R goes to H, the
// inverses of the diagonal blocks to the diagonal blocks of F, both row-major (the apply
// kernels read 16 consecutive columns per row with 16 lanes).
//
// k_apply, rounds 0/1: Q = Y R^-1 by blocked forward substitution on v_mfma_f64_16x16x4f64,
//   Q_J = (Y_J - sum_{I<J} Q_I R_IJ) R_JJ^-1   (16-column blocks; each wave owns 16 rows, held
//   in registers).
// k_apply, round 2: the rebuild factor W = Q F with F = V_keep diag(sqrt(w)) (row-major out).
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int CH_WAVES = 8;
// Every Schur pivot at least CQ_WELL times its Gram diagonal: the column-scaled condition
// number of Y is then at most about sqrt(r / CQ_WELL), and Q = Y R^-1 is orthonormal to about
// r eps / CQ_WELL, so one CholeskyQR round suffices where only the range is needed.
constexpr double CQ_WELL = 1e-6;
constexpr int CH_THREADS = CH_WAVES * WAVE;
constexpr int NBMAX = PSDPROJ_MAX_RANK / 16;

// NS register slots per wave: 14 cover r_pad <= 224 (105 tiles), 17 cover r_pad = 256 (136).
template <int NS>
__global__ __launch_bounds__(CH_THREADS) void k_chol(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob, int arg) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int round = arg & ORTH_ROUND_MASK;
  if (round == 1 && orth_single(p, arg)) return;   // second CholeskyQR round not needed
  const int r = p.r, rp = p.rpad, nb = rp / 16, nt = nb * (nb + 1) / 2;
  const int tid = threadIdx.x, wave = wave_id(), lane = tid & 63, li = lane & 15, kg = lane >> 4;
  const gmem<const double>* __restrict__ G = gp((const double*)p.G);
  gmem<double>* __restrict__ H = gp(p.H);
  gmem<double>* __restrict__ F = gp(p.F);
  __shared__ double panel[NBMAX][16][17];   // R_JK of the current block row, row-major
  __shared__ double dsm[16][17];            // diagonal tile being factored
  __shared__ double dinv[16][17];           // R_JJ^-1
  __shared__ double g0[PSDPROJ_MAX_RANK];
  __shared__ int dflag[PSDPROJ_MAX_RANK];
  __shared__ int wflag[PSDPROJ_MAX_RANK];   // Schur pivot below CQ_WELL x Gram diagonal
  const double tol = (p.prec == F64) ? 1e-26 : 1e-13;

  for (int j = tid; j < rp; j += CH_THREADS) g0[j] = (j < r) ? G[(int64_t)j * rp + j] : 0.0;

  f64x4 reg[NS];
  int tI[NS], tJ[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int t = wave + s * CH_WAVES;
    int I = nb, J = nb;  // inactive slot
    if (t < nt) upper_tile(t, nb, I, J);
    tI[s] = I;
    tJ[s] = J;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * I + 4 * v + kg, b = 16 * J + li;
      reg[s][v] = (t < nt) ? G[(int64_t)b * rp + a] : 0.0;
    }
  }
  lds_barrier();

  for (int J = 0; J < nb; ++J) {
    // ---- A: factor the diagonal tile (owner wave), R_JJ and R_JJ^-1 into LDS
    const int tdiag = J * nb - J * (J - 1) / 2;
    if (wave == tdiag % CH_WAVES) {
      const int sd = tdiag / CH_WAVES;
      f64x4 dt = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == sd) dt = reg[s];
      // tile -> LDS (result layout), then lane c < 16 takes column c into registers
#pragma unroll
      for (int v = 0; v < 4; ++v) dsm[4 * v + kg][li] = dt[v];
      lds_wave_sync();
      // Right-looking Cholesky of the tile by row operations on [W | I]: lane c < 16 holds
      // column c of W, lane 16 + c column c of the identity (lanes >= 32 hold zeros).  Step jj
      // scales row jj by 1/sqrt(pivot) and subtracts R[jj][i] times it from every row i > jj;
      // the left half becomes R and the right half R^-T, so lane 16 + i ends with row i of
      // X = R_JJ^-1, and the inverse costs no broadcasts of its own.  The pivot and the
      // multipliers R[jj][i] (row jj of lane i) are broadcast with readlane.  A dropped row jj
      // (1/pivot taken as 0) gives a zero row of R with a unit diagonal and a zero column of X.
      double col[16];
#pragma unroll
      for (int a = 0; a < 16; ++a)
        col[a] = (lane < 16) ? dsm[a][li] : ((lane == 16 + a) ? 1.0 : 0.0);
      int drops = 0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const double d = bcast_f64(col[jj], jj);
        const double gj = g0[16 * J + jj];
        const bool dr = !(gj > 0.0) || !(d > tol * gj) || !isfinite(d);
        // sqrt(d) and 1/sqrt(d) from the hardware reciprocal-square-root estimate: one
        // Goldschmidt step, then a Newton correction of each (no IEEE sqrt or division)
        const double y0 = __builtin_amdgcn_rsq(d);
        double g = d * y0, h = 0.5 * y0;
        const double e0 = fma(-h, g, 0.5);
        g = fma(g, e0, g);
        h = fma(h, e0, h);
        g = fma(fma(-g, g, d), h, g);
        double ip = 2.0 * h;
        ip = fma(ip, fma(-g, ip, 1.0), ip);
        const double piv = dr ? 0.0 : g;
        ip = dr ? 0.0 : ip;
        const double nrm = col[jj] * ip;   // row jj scaled; R[jj][c] in lane c > jj
#pragma unroll
        for (int a = jj + 1; a < 16; ++a) col[a] -= bcast_f64(nrm, a) * nrm;
        col[jj] = (lane == jj) ? (dr ? 1.0 : piv) : nrm;
        drops |= (dr ? 1 : 0) << jj;
      }
      // R_JJ (upper, zero below; lane c holds column c) and its inverse (lane 16 + i holds row i)
      // to LDS; R_JJ back to the owner's registers
      lds_wave_sync();
      if (lane < 16) {
#pragma unroll
        for (int a = 0; a < 16; ++a) dsm[a][lane] = (a <= lane) ? col[a] : 0.0;
        dflag[16 * J + lane] = (drops >> lane) & 1;
        // the Schur pivot of column lane is R[lane][lane]^2 (read back from this lane's store)
        const double rjj = dsm[lane][lane];
        wflag[16 * J + lane] = (rjj * rjj >= CQ_WELL * g0[16 * J + lane]) ? 0 : 1;
      } else if (lane < 32) {
#pragma unroll
        for (int a = 0; a < 16; ++a) dinv[lane - 16][a] = col[a];
      }
      lds_wave_sync();
#pragma unroll
      for (int v = 0; v < 4; ++v) dt[v] = dsm[4 * v + kg][li];
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == sd) reg[s] = dt;
    }
    lds_barrier();
    if (wave == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = 4 * e + kg, c = li;
        F[(int64_t)(16 * J + a) * rp + 16 * J + c] = dinv[a][c];   // row-major
      }
    }
    // Per-lane LDS offset (row kg, column li of a 16x17 tile), re-materialised every block so
    // that per-slot addresses are not hoisted out of the loop (they would occupy registers).
    int lofs = kg * 17 + li;
    __asm__ volatile("" : "+v"(lofs));
    const double* pan = &panel[0][0][0];
    const double* dv = &dinv[0][0];
    // ---- B: panel tiles R_JK = R_JJ^-T W_JK for K > J
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (tI[s] != J || tJ[s] >= nb || tJ[s] == J) continue;
      f64x4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = dv[kk * 68 + lofs];   // (R_JJ^-T)[li][4kk+kg]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, reg[s][kk], acc, 0, 0, 0);
      }
      reg[s] = acc;
      const int K = tJ[s];
#pragma unroll
      for (int v = 0; v < 4; ++v) panel[K][4 * v + kg][li] = acc[v];
    }
    lds_barrier();
    // ---- C: trailing tiles W_KL -= R_JK^T R_JL, J < K <= L
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (tI[s] <= J || tJ[s] >= nb) continue;
      const int K = tI[s], L = tJ[s];
      f64x4 acc = reg[s];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = pan[K * 272 + kk * 68 + lofs];   // (R_JK^T)[li][4kk+kg]
        const double b = pan[L * 272 + kk * 68 + lofs];   // R_JL[4kk+kg][li]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, b, acc, 0, 0, 0);
      }
      reg[s] = acc;
    }
    // the next block's step A reads only its owner's registers; the panel is rewritten after
    // the next barrier
  }
  // R (upper-triangle tiles, now all final in registers) to H
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (tJ[s] >= nb) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * tI[s] + 4 * v + kg, b = 16 * tJ[s] + li;
      H[(int64_t)a * rp + b] = reg[s][v];   // row-major
    }
  }
  lds_barrier();
  if (tid == 0) {
    int ndrop = 0, nweak = 0;
    for (int j = 0; j < r; ++j) {
      ndrop += dflag[j];
      nweak += dflag[j] | wflag[j];
    }
    p.iscal[I_NDROP] = ndrop;
    if (round == 0) p.iscal[I_WELL] = (nweak == 0) ? 1 : 0;
  }
}

// ------------------------------------------------------------------ apply
constexpr int AP_WAVES = 4;
constexpr int AP_THREADS = AP_WAVES * WAVE;

// Both rounds keep a wave's 16 rows of Q in registers in the A-operand layout of
// v_mfma_f64_16x16x4f64: qa[I][kk] of lane (li, kg) is Q[row li][16I + 4kk + kg].  The loops
// over column blocks are unrolled to NB (the largest block count of the launch), so qa is
// indexed by constants; blocks past the problem's nb are skipped (J) or contribute exact
// zeros (I).  A 16x17 LDS scratch per wave turns result-layout blocks into operand layout.

// Result-layout block x (lane: rows 4v + kg, column li) -> operand layout (lane: row li,
// columns 4kk + kg), through the wave's scratch.
__device__ __forceinline__ f64x4 to_operand(f64x4 x, double* sc, int li, int kg) {
#pragma unroll
  for (int v = 0; v < 4; ++v) sc[(4 * v + kg) * 17 + li] = x[v];
  lds_wave_sync();
  f64x4 out;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) out[kk] = sc[li * 17 + 4 * kk + kg];
  lds_wave_sync();
  return out;
}

template <typename T, int NB>
__device__ __forceinline__ void apply_tri(const Prob& p, int round, bool single, int tile, double* scratch) {
  const int rp = p.rpad, nb = rp / 16, ld = p.ld;
  const int wave = wave_id(), lane = threadIdx.x & 63, li = lane & 15, kg = lane >> 4;
  const int rowbase = tile * APPLY_ROWS + wave * 16;
  // round 0 maps Y to Q1 (or, when the second round is skipped, straight to the pass operand);
  // round 1 maps Q1 to the pass operand
  const bool final_out = (round == 1) || single;
  const gmem<const T>* __restrict__ in = gp((const T*)((round == 0) ? p.y : p.q1));
  gmem<T>* __restrict__ out = gp((T*)(final_out ? p.zm : p.q1));
  const gmem<const double>* __restrict__ R = gp((const double*)p.H);
  const gmem<const double>* __restrict__ Dinv = gp((const double*)p.F);
  gmem<bf16>* __restrict__ zhi = gp(p.zhi);
  gmem<bf16>* __restrict__ zlo = gp(p.zlo);
  double* sc = scratch + wave * 16 * 17;
  double qa[NB][4];
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    if (J < nb) {   // uniform
      const gmem<const double>* col = R + (int64_t)kg * rp + 16 * J + li;   // R[kg + 4m][16J + li]
      f64x4 acc0, acc1 = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc0[v] = (double)in[(int64_t)(16 * J + li) * ld + rowbase + 4 * v + kg];
      double dj[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) dj[kk] = Dinv[(int64_t)(16 * J + 4 * kk + kg) * rp + 16 * J + li];
      // Y_J - sum_{I<J} Q_I R_IJ, as two chains (even and odd I) added at the end
#pragma unroll
      for (int I = 0; I < J; ++I) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double b = col[(int64_t)(16 * I + 4 * kk) * rp];
          if (I & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-qa[I][kk], b, acc1, 0, 0, 0);
          else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(-qa[I][kk], b, acc0, 0, 0, 0);
        }
        if (I & 1) __builtin_amdgcn_sched_barrier(0);   // loads run at most two row blocks ahead
      }
      const f64x4 w = to_operand(acc0 + acc1, sc, li, kg);
      f64x4 q = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) q = __builtin_amdgcn_mfma_f64_16x16x4f64(w[kk], dj[kk], q, 0, 0, 0);
      const f64x4 qo = to_operand(q, sc, li, kg);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) qa[J][kk] = qo[kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t o = (int64_t)(16 * J + li) * ld + rowbase + 4 * v + kg;
        const T val = (T)q[v];
        out[o] = val;
        if (final_out && p.prec == B3) {
          const bf16 h = (bf16)(float)val;
          const int64_t oz = zsplit_index(rowbase + 4 * v + kg, 16 * J + li, ld);
          zhi[oz] = h;
          zlo[oz] = (bf16)((float)val - (float)h);
        }
      }
    }
  }
}

// W = Q F, F = V_keep diag(sqrt(w)) (columns >= r_plus are zero); row-major output.
template <typename T, int NB>
__device__ __forceinline__ void apply_factor(const Prob& p, int tile) {
  const int rp = p.rpad, nb = rp / 16, ld = p.ld, kw = p.rwpad;
  const int wave = wave_id(), lane = threadIdx.x & 63, li = lane & 15, kg = lane >> 4;
  const int rowbase = tile * APPLY_ROWS + wave * 16;
  const int rplus = min(max(p.iscal[I_RPLUS], 0), rp);
  const gmem<const T>* __restrict__ Q = gp((const T*)p.zm);
  const gmem<const double>* __restrict__ Fm = gp((const double*)p.F);
  gmem<T>* __restrict__ wf = gp((T*)p.wf);
  gmem<bf16>* __restrict__ whi = gp(p.whi);
  gmem<bf16>* __restrict__ wlo = gp(p.wlo);
  double qa[NB][4];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    if (I < nb) {   // uniform
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) qa[I][kk] = (double)Q[(int64_t)(16 * I + 4 * kk + kg) * ld + rowbase + li];
    } else {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) qa[I][kk] = 0.0;
    }
  }
#pragma unroll 1
  for (int J = 0; J < kw / 16; ++J) {
    f64x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    if (16 * J < rplus) {
      const gmem<const double>* col = Fm + (int64_t)kg * rp + 16 * J + li;   // F[kg + 4m][16J + li]
      // opaque to loop-invariant code motion, which would otherwise precompute all 4*NB load
      // addresses outside the J loop (2*4*NB registers)
      __asm__ volatile("" : "+v"(col));
      auto load = [&](double (&b)[4], int I) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) b[kk] = col[(int64_t)(16 * I + 4 * kk) * rp];
      };
      auto mfma4 = [&](const double (&b)[4], int I) {   // one chain per parity of I
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (I & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[I][kk], b[kk], acc1, 0, 0, 0);
          else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[I][kk], b[kk], acc0, 0, 0, 0);
        }
      };
      if (nb == NB) {
        // loads run two row blocks ahead of the MFMAs (a ring of three register blocks); the
        // scheduling barrier keeps each prefetch ahead of the MFMAs that follow it
        double ring[3][4];
        load(ring[0], 0);
        load(ring[1], 1);
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          if (I + 2 < NB) load(ring[(I + 2) % 3], I + 2);
          __builtin_amdgcn_sched_barrier(0);
          mfma4(ring[I % 3], I);
        }
      } else {
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          if (I < nb) {   // uniform
            double b[4];
            load(b, I);
            mfma4(b, I);
          }
        }
      }
    }
    f64x4 a = acc0 + acc1;
    // W's columns >= r_plus must be zero (the rebuild reads whole 16/32-column groups); F holds
    // other data there, and output column li depends on column li of F only
    if (16 * J + li >= rplus) a = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t o = (int64_t)(rowbase + 4 * v + kg) * kw + 16 * J + li;
      const T val = (T)a[v];
      wf[o] = val;
      if (p.prec == B3) {
        const bf16 h = (bf16)(float)val;
        whi[o] = h;
        wlo[o] = (bf16)((float)val - (float)h);
      }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(AP_THREADS) void k_apply(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                      int nprob, int arg) {
  __shared__ double scratch[AP_WAVES * 16 * 17];
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int round = arg & ORTH_ROUND_MASK;
  const bool single = orth_single(p, arg);
  if (round == 1 && single) return;   // the first round already wrote the pass operand
  const int t = blockIdx.x - tstart[pi];
  if (t * APPLY_ROWS >= p.ld) return;
  if (p.prec == F64) apply_tri<double, NB>(p, round, single, t, scratch);
  else apply_tri<float, NB>(p, round, single, t, scratch);
}

template <int NB>
__global__ __launch_bounds__(AP_THREADS) void k_apply_factor(const Prob* __restrict__ probs,
                                                             const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (t * APPLY_ROWS >= p.ld) return;
  if (p.prec == F64) apply_factor<double, NB>(p, t);
  else apply_factor<float, NB>(p, t);
}

int tiles_small(const Prob&) { return 1; }
int tiles_apply(const Prob& p) { return p.ld / APPLY_ROWS; }

void apply_init() {}

void launch_chol(const Launch& L, int round) {
  if (L.maxnb <= 14)
    hipLaunchKernelGGL(k_chol<14>, dim3(L.grid), dim3(CH_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
  else
    hipLaunchKernelGGL(k_chol<17>, dim3(L.grid), dim3(CH_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
}
void launch_apply(const Launch& L, int round) {
  if (round == 2) {
    if (L.maxnb <= 14)
      hipLaunchKernelGGL(k_apply_factor<14>, dim3(L.grid), dim3(AP_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
    else
      hipLaunchKernelGGL(k_apply_factor<16>, dim3(L.grid), dim3(AP_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
  } else if (L.maxnb <= 14) {
    hipLaunchKernelGGL(k_apply<14>, dim3(L.grid), dim3(AP_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
  } else {
    hipLaunchKernelGGL(k_apply<16>, dim3(L.grid), dim3(AP_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, round);
  }
}

}  // namespace psd
