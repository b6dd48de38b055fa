// Alg. 4 (power iteration for sigma_1) and Alg. 5 (alpha = |sigma_1(X) - sigma_1(X - sigma_1 I)|).
//
// Two forms of Alg. 5.  Sequential (N > PAIRED_MAX): the first power iteration, then the
// second on X - sigma_1 I, 2 (N + 1) products.  Paired (N <= PAIRED_MAX): both runs over N + 1
// products with two vectors each, so A is read half as often: the first run as written, and
// beside it a Krylov basis of the second run's start vector under shifts mu_j that follow the
// first run's estimate of sigma_1, from which the second run's iterates are formed at the end
// (k_alpha2).
//
// One launch of k_gemv computes y = X v - shift v with v = y_prev * inv_prev (the previous
// product scaled to unit norm; the first product uses the raw Gaussian start vector) and the
// norm ||y||.  The shift of Alg. 5 is applied to the vector, so X - sigma_1 I is never formed.
// Vectors and accumulation are FP64 for every storage precision of A.
//
// X is symmetric, so only its upper triangle is read: k_gemv gives one workgroup per 256 x 256
// tile X_IJ (I <= J) and, from one read of it, forms both X_IJ v_J (row sums, contribution to
// block row I) and X_IJ^T v_I (column sums, contribution to block row J; skipped on the
// diagonal tile).  That halves the HBM bytes of a product.  Each block row gets exactly nb
// contributions, stored in a partial array; k_gemv_finish (one workgroup per block row) adds
// them in a fixed order, applies the shift and stores the row's sum of squares, and the last
// block row to finish (integer ticket) adds those in block order and forms the norm.  No
// result depends on scheduling.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int GEMV_THREADS = 256;   // 4 waves x 64 rows of a tile

// Tile t -> (I, J), I <= J: t enumerates the lower-triangle pairs (a, b), b <= a, row by row,
// and (I, J) = (b, a).
__device__ __forceinline__ void gemv_tile_ij(int t, int& I, int& J) {
  int a = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  J = a;
  I = t - a * (a + 1) / 2;
}

// One halving stage: lanes with bit D set keep the upper M/2 rows, the others the lower M/2,
// and each adds its partner's (lane ^ D) copy of the rows it keeps.
template <int M, int D, int RB>
__device__ __forceinline__ void halve(double (&x)[RB], int lane) {
  const bool up = (lane & D) != 0;
#pragma unroll
  for (int k = 0; k < M / 2; ++k) {
    const double lo = x[k], hi = x[k + M / 2];
    const double keep = up ? hi : lo;
    const double send = up ? lo : hi;
    x[k] = keep + __shfl_xor(send, D, 64);
  }
  if constexpr (M > 2) halve<M / 2, D / 2, RB>(x, lane);
}

// Sum of x over the 64 lanes of a wave for RB rows at once: after the call, x[0] of lane l
// holds the full sum of row l >> (6 - log2 RB).  Recursive halving over lane bits 5, 4, ...
// then a butterfly over the remaining low bits; the addition order is fixed.
template <int RB>
__device__ __forceinline__ void reduce_scatter(double (&x)[RB], int lane) {
  halve<RB, 32, RB>(x, lane);
#pragma unroll
  for (int d = 32 / RB; d > 0; d >>= 1) x[0] += __shfl_xor(x[0], d, 64);
}

// Fixed-order sum of the nb contributions of block row b, shift, store, sum of squares; the
// last block row also forms the norm.  The contributions are loaded FIN_CHUNK at a time (all
// issued before the first is added, from clamped addresses) and added in block order; the
// last block row's threads load the nb row sums of squares in parallel and thread 0 adds them
// in block order from LDS.
constexpr int FIN_CHUNK = 32;
__global__ __launch_bounds__(GEMV_THREADS) void k_gemv_finish(const Prob* __restrict__ probs,
                                                              const int* __restrict__ tstart, int nprob, int last) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int b = blockIdx.x - tstart[pi];
  __shared__ double red[GEMV_THREADS / WAVE];
  __shared__ double rows[GEMV_THREADS];
  __shared__ int is_last;
  const int n = p.n, ld = p.ld;
  const int nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  const int pp = p.iscal[I_PP] & 1;
  const gmem<const double>* __restrict__ vin = gp((const double*)p.vec) + (int64_t)pp * ld;
  gmem<double>* __restrict__ vout = gp(p.vec) + (int64_t)(1 - pp) * ld;
  const double inv = p.scal[S_INV];
  const double shift = p.scal[S_SHIFT];
  const int x = threadIdx.x;
  const int row = b * GEMV_TILE + x;
  const gmem<const double>* __restrict__ part = gp((const double*)p.gvp) + (int64_t)b * nb * GEMV_TILE;
  const int ncontrib = p.csr ? 1 : nb;   // a sparse product gives one contribution per row
  double y = 0.0;
  if (row < n) {
    double s = 0.0;
    for (int c0 = 0; c0 < ncontrib; c0 += FIN_CHUNK) {
      double t[FIN_CHUNK];
#pragma unroll
      for (int k = 0; k < FIN_CHUNK; ++k) t[k] = part[(int64_t)min(c0 + k, ncontrib - 1) * GEMV_TILE + x];
#pragma unroll
      for (int k = 0; k < FIN_CHUNK; ++k)
        if (c0 + k < ncontrib) s += t[k];
    }
    y = s - shift * (vin[row] * inv);
    vout[row] = y;
  }
  const double ss = wave_sum(y * y);
  if ((x & 63) == 0) red[x >> 6] = ss;
  __syncthreads();
  if (x == 0) {
    double tot = 0.0;
    for (int w = 0; w < GEMV_THREADS / WAVE; ++w) tot += red[w];
    p.vpart[b] = tot;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    is_last = (atomicAdd(&p.iscal[I_COUNTER], 1) == nb - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double t2 = 0.0;
  for (int r0 = 0; r0 < nb; r0 += GEMV_THREADS) {
    if (r0 + x < nb) rows[x] = p.vpart[r0 + x];
    __syncthreads();
    if (x == 0)
      for (int r = 0; r < GEMV_THREADS && r0 + r < nb; ++r) t2 += rows[r];
    __syncthreads();
  }
  if (x == 0) {
    const double nrm = sqrt(t2);
    p.scal[S_NRM] = nrm;
    p.scal[S_INV] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    if (last == 1) p.scal[S_SIGMA1] = nrm;
    if (last == 2) p.scal[S_SIGMA2] = nrm;
    p.iscal[I_COUNTER] = 0;
    p.iscal[I_PP] = p.iscal[I_PP] + 1;
  }
}

// Paired form of Alg. 5, after product j (block row b; one thread per row):
//   first run:  v_{j+1} = X v_j (v_j = vec[pp] / ||.||, as in k_gemv_finish without shift);
//   second run: b_{j+1} = X bhat_j - mu_j bhat_j, bhat_j = b_j / rho_j, stored as basis slot j+1.
// The last block row to finish adds both sums of squares in block order and sets
// nu_j = ||X v_j||, rho_{j+1} = ||b_{j+1}||, the inverse norms the next product scales by, and
// the next shift: mu_1 = mu_0 = tr(X)/n (v_0 is not normalised, so nu_0 is no estimate of
// sigma_1), mu_{j+1} = nu_j after that.  After product N, nu_N is sigma_1 of the first run.
// Both rows' partials are added in the same fixed order as k_gemv_finish's.
__global__ __launch_bounds__(GEMV_THREADS) void k_gemv2_finish(const Prob* __restrict__ probs,
                                                               const int* __restrict__ tstart, int nprob, int j) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int b = blockIdx.x - tstart[pi];
  __shared__ double red[2][GEMV_THREADS / WAVE];
  __shared__ double rows[2][GEMV_THREADS];
  __shared__ int is_last;
  const int n = p.n, ld = p.ld;
  const int nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  const int pp = p.iscal[I_PP] & 1;
  gmem<double>* __restrict__ vout = gp(p.vec) + (int64_t)(1 - pp) * ld;
  const gmem<const double>* __restrict__ bj = gp((const double*)p.bh) + (int64_t)j * ld;
  gmem<double>* __restrict__ bnext = gp(p.bh) + (int64_t)(j + 1) * ld;
  const double invb = p.scal[S_INVB];
  const double mu = p.scal[S_MU];
  const int x = threadIdx.x;
  const int row = b * GEMV_TILE + x;
  const int64_t vstride = (int64_t)nb * nb * GEMV_TILE;
  const int ncontrib = p.csr ? 1 : nb;
  double y[2] = {0.0, 0.0};
  if (row < n) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const gmem<const double>* __restrict__ part = gp((const double*)p.gvp) + w * vstride + (int64_t)b * nb * GEMV_TILE;
      double s = 0.0;
      for (int c0 = 0; c0 < ncontrib; c0 += FIN_CHUNK) {
        double t[FIN_CHUNK];
#pragma unroll
        for (int k = 0; k < FIN_CHUNK; ++k) t[k] = part[(int64_t)min(c0 + k, ncontrib - 1) * GEMV_TILE + x];
#pragma unroll
        for (int k = 0; k < FIN_CHUNK; ++k)
          if (c0 + k < ncontrib) s += t[k];
      }
      y[w] = s;
    }
    y[1] = y[1] - mu * (bj[row] * invb);
    vout[row] = y[0];
    bnext[row] = y[1];
  }
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const double ss = wave_sum(y[w] * y[w]);
    if ((x & 63) == 0) red[w][x >> 6] = ss;
  }
  __syncthreads();
  if (x == 0) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      double tot = 0.0;
      for (int q = 0; q < GEMV_THREADS / WAVE; ++q) tot += red[w][q];
      p.vpart[w * nb + b] = tot;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    is_last = (atomicAdd(&p.iscal[I_COUNTER], 1) == nb - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double t2[2] = {0.0, 0.0};
  for (int r0 = 0; r0 < nb; r0 += GEMV_THREADS) {
    if (r0 + x < nb) {
      rows[0][x] = p.vpart[r0 + x];
      rows[1][x] = p.vpart[nb + r0 + x];
    }
    __syncthreads();
    if (x == 0)
      for (int r = 0; r < GEMV_THREADS && r0 + r < nb; ++r) {
        t2[0] += rows[0][r];
        t2[1] += rows[1][r];
      }
    __syncthreads();
  }
  if (x == 0) {
    const double nu = sqrt(t2[0]), rho = sqrt(t2[1]);
    p.scal[S_NRM] = nu;
    p.scal[S_INV] = (nu > 0.0) ? 1.0 / nu : 0.0;
    p.scal[S_INVB] = (rho > 0.0) ? 1.0 / rho : 0.0;
    p.pw[j + 1] = rho;
    p.pw[PAIRED_MAX + 2 + j] = mu;
    p.scal[S_MU] = (j == 0) ? p.scal[S_MU0] : nu;
    if (j == p.alpha_iters) p.scal[S_SIGMA1] = nu;
    p.iscal[I_COUNTER] = 0;
    p.iscal[I_PP] = p.iscal[I_PP] + 1;
  }
}

// Paired form of Alg. 5, the end: the second run's iterates are (X - sigma_1 I)^m b_0 up to
// scale, and from X bhat_j = rho_{j+1} bhat_{j+1} + mu_j bhat_j the product with X - sigma_1 I
// maps coefficients c over the basis to c'_{j+1} += rho_{j+1} c_j, c'_j += (mu_j - sigma_1) c_j.
// Thread 0 of every block applies that map N times to e_0 (rescaling by the largest magnitude
// after each), giving z_N, and once more, giving z_{N+1}; the block's rows of both are formed
// from the basis and their sums of squares added in block order by the last block:
// sigma_2 = ||z_{N+1}|| / ||z_N|| (0 when z_N vanishes, as Alg. 4 stops at a zero product),
// alpha = |sigma_1 - sigma_2|.  With the shifts tracking sigma_1 the coefficients stay within
// a small factor of ||z||, so the result agrees with the two runs made one after the other to
// near FP64 rounding.
__global__ __launch_bounds__(256) void k_alpha2(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int blk = blockIdx.x - tstart[pi];
  const int G = tstart[pi + 1] - tstart[pi];
  const int N = p.alpha_iters;
  __shared__ double cz[2][PAIRED_MAX + 2];
  __shared__ double cw[2][PAIRED_MAX + 2];   // thread 0's coefficient vectors (no per-lane arrays)
  __shared__ double red[2][256 / WAVE];
  __shared__ double rows[2][256];
  __shared__ int is_last;
  const int x = threadIdx.x;
  const double s1 = p.scal[S_SIGMA1];
  if (x == 0) {
    const double* rho = p.pw;
    const double* mu = p.pw + PAIRED_MAX + 2;
    double* c = cw[0];
    double* d = cw[1];
    for (int i = 0; i < N + 2; ++i) c[i] = 0.0;
    c[0] = 1.0;
    auto apply = [&]() {
      for (int i = 0; i < N + 2; ++i) d[i] = 0.0;
      for (int i = 0; i <= N; ++i) {
        d[i + 1] += rho[i + 1] * c[i];
        d[i] += (mu[i] - s1) * c[i];
      }
    };
    for (int m = 0; m < N; ++m) {
      apply();
      double big = 0.0;
      for (int i = 0; i < N + 2; ++i) big = fmax(big, fabs(d[i]));
      const double sc = (big > 0.0) ? 1.0 / big : 0.0;
      for (int i = 0; i < N + 2; ++i) c[i] = d[i] * sc;
    }
    apply();
    // fold bhat_i = b_i / rho_i into the coefficients (rho_0 = 1: b_0 is used as drawn; a zero
    // rho_i means b_i and every later basis vector are zero)
    for (int i = 0; i < N + 2; ++i) {
      const double ir = (rho[i] > 0.0) ? 1.0 / rho[i] : 0.0;
      cz[0][i] = c[i] * ir;
      cz[1][i] = d[i] * ir;
    }
  }
  __syncthreads();
  double ss[2] = {0.0, 0.0};
  for (int e = x; e < 1024; e += 256) {
    const int i = blk * 1024 + e;
    if (i >= p.n) break;
    double z0 = 0.0, z1 = 0.0;
    for (int k = 0; k < N + 2; ++k) {
      const double bv = p.bh[(int64_t)k * p.ld + i];
      z0 = fma(cz[0][k], bv, z0);
      z1 = fma(cz[1][k], bv, z1);
    }
    ss[0] = fma(z0, z0, ss[0]);
    ss[1] = fma(z1, z1, ss[1]);
  }
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const double t = wave_sum(ss[w]);
    if ((x & 63) == 0) red[w][x >> 6] = t;
  }
  __syncthreads();
  if (x == 0) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      double tot = 0.0;
      for (int q = 0; q < 256 / WAVE; ++q) tot += red[w][q];
      p.vpart[w * G + blk] = tot;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    is_last = (atomicAdd(&p.iscal[I_COUNTER], 1) == G - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double t2[2] = {0.0, 0.0};
  for (int r0 = 0; r0 < G; r0 += 256) {
    if (r0 + x < G) {
      rows[0][x] = p.vpart[r0 + x];
      rows[1][x] = p.vpart[G + r0 + x];
    }
    __syncthreads();
    if (x == 0)
      for (int r = 0; r < 256 && r0 + r < G; ++r) {
        t2[0] += rows[0][r];
        t2[1] += rows[1][r];
      }
    __syncthreads();
  }
  if (x == 0) {
    const double s2 = (t2[0] > 0.0) ? sqrt(t2[1]) / sqrt(t2[0]) : 0.0;
    p.scal[S_SIGMA2] = s2;
    const double a = fabs(s1 - s2);
    p.scal[S_ALPHA] = a;
    if (!(a > 0.0) || !isfinite(a)) set_status(p, PSDPROJ_E_ALPHA);
    p.iscal[I_COUNTER] = 0;
  }
}

// Stream one wave's 64 rows of a tile in batches of RB rows, NBUF of them in flight in register
// buffers (the loop is fully unrolled, so the loads of batches bt+1 .. bt+NBUF-1 are in flight
// while batch bt is used and no copy between the buffers forces an early wait; the arithmetic
// and its order do not depend on NBUF), against NV vectors at once (one element
// of A read, NV row and NV column terms formed).  VEC: rows start and end 16-byte aligned,
// so a 16-byte chunk lies wholly inside or wholly past column n; chunks past n read the row's
// first chunk instead (their v_J entries are zero, and their column sums belong to columns
// past n, never read).  Otherwise element loads at clamped addresses with the values past
// column n zeroed.  Rows past n are loaded clamped to row n-1; their row sums land in partial
// slots that are never read and their column terms are multiplied by a zero v_I.
// The vector entries are waited for only once two batches of A are in flight, so the tile's
// stream starts without waiting for them.
template <typename T, int RB, bool VEC, int NV>
__device__ __forceinline__ void gemv_stream(const gmem<const T>* __restrict__ A, int64_t lda, int n, int rw, int c0,
                                            const gmem<const double>* const (&vin)[NV], const double (&inv)[NV],
                                            bool diag, double (&yc)[NV][4], gmem<double>* const (&rowout)[NV],
                                            int lane) {
  constexpr int NBT = 64 / RB;
  constexpr int LOGRB = (RB == 16) ? 4 : (RB == 8) ? 3 : 2;
  // batches in flight: three for two vectors (the products' 2 waves per SIMD have registers for
  // a third buffer), two for one vector (3 waves per SIMD)
  constexpr int NBUF = (NV == 2 && sizeof(T) == 4) ? 3 : 2;
  T a[NBUF][RB][4];
  auto load = [&](T (&dst)[RB][4], int r0) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = (int64_t)min(r0 + q, n - 1) * lda;
      if constexpr (VEC) {
        if constexpr (sizeof(T) == 4) {
          const f32x4 x = __builtin_nontemporal_load((const gmem<f32x4>*)(A + row + (c0 < n ? c0 : 0)));
#pragma unroll
          for (int e = 0; e < 4; ++e) dst[q][e] = x[e];
        } else {
          const f64x2 x0 = __builtin_nontemporal_load((const gmem<f64x2>*)(A + row + (c0 < n ? c0 : 0)));
          const f64x2 x1 = __builtin_nontemporal_load((const gmem<f64x2>*)(A + row + (c0 + 2 < n ? c0 + 2 : 0)));
          dst[q][0] = x0[0]; dst[q][1] = x0[1]; dst[q][2] = x1[0]; dst[q][3] = x1[1];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const T x = A[row + min(c0 + e, n - 1)];
          dst[q][e] = (c0 + e < n) ? x : (T)0;
        }
      }
    }
  };
  // raw vector entries (unconditional loads, no branch per load), used only once two batches
  // of A are in flight
  double vjr[NV][4], vrr[NV];
#pragma unroll
  for (int w = 0; w < NV; ++w) {
#pragma unroll
    for (int e = 0; e < 4; ++e) vjr[w][e] = vin[w][min(c0 + e, n - 1)];
    vrr[w] = vin[w][min(rw + lane, n - 1)];
  }
#pragma unroll
  for (int b = 0; b + 1 < NBUF; ++b) load(a[b], rw + b * RB);
  double vj[NV][4], vrow[NV];
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt) {
    // keep the scheduler from hoisting later batches' loads (they would need more buffers)
    __builtin_amdgcn_sched_barrier(0);
    if (bt + NBUF - 1 < NBT) load(a[(bt + NBUF - 1) % NBUF], rw + (bt + NBUF - 1) * RB);
    if (bt == 0) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int w = 0; w < NV; ++w) {
#pragma unroll
        for (int e = 0; e < 4; ++e) vj[w][e] = (c0 + e < n) ? vjr[w][e] * inv[w] : 0.0;
        // v_I of row rw + lane (zero past n and on the diagonal tile, whose transpose is itself)
        vrow[w] = (!diag && rw + lane < n) ? vrr[w] * inv[w] : 0.0;
      }
    }
    double rs[NV][RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      double x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = (double)a[bt % NBUF][q][e];
#pragma unroll
      for (int w = 0; w < NV; ++w) {
        rs[w][q] = x[0] * vj[w][0] + x[1] * vj[w][1] + x[2] * vj[w][2] + x[3] * vj[w][3];
        const double vi = bcast_f64(vrow[w], bt * RB + q);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          yc[w][e] += x[e] * vi;
          // pin the column update to its row: otherwise it is deferred past the row sums and
          // every converted row stays live
          __asm__ volatile("" : "+v"(yc[w][e]));
        }
      }
    }
#pragma unroll
    for (int w = 0; w < NV; ++w) {
      reduce_scatter<RB>(rs[w], lane);
      if ((lane & ((64 / RB) - 1)) == 0) rowout[w][bt * RB + (lane >> (6 - LOGRB))] = rs[w][0];
    }
  }
}

// RB rows per load batch: 8 for FP32 storage, 4 for FP64 (32 VGPRs of A per buffer, so the
// kernel keeps 3 waves per SIMD).  NV = 1: the product of Alg. 4 (vector vec[pp] / ||.||);
// NV = 2: that product and the one of basis vector j of the paired form of Alg. 5, whose
// partials follow the first vector's (nb x nb x GEMV_TILE further on).
template <typename T, int RB, int NV>
__device__ __forceinline__ void gemv_tile(const Prob& p, int t, int j) {
  const int n = p.n, ld = p.ld;
  const int nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  int I, J;
  gemv_tile_ij(t, I, J);
  const bool diag = (I == J);
  const int pp = p.iscal[I_PP] & 1;                 // ping-pong: read vec[pp], write vec[1-pp]
  const gmem<const double>* vin[NV];
  double inv[NV];
  vin[0] = gp((const double*)p.vec) + (int64_t)pp * ld;
  inv[0] = p.scal[S_INV];
  if constexpr (NV == 2) {
    vin[1] = gp((const double*)p.bh) + (int64_t)j * ld;
    inv[1] = p.scal[S_INVB];
  }
  const int wave = wave_id(), lane = threadIdx.x & 63;
  __shared__ double cred[NV][GEMV_THREADS / WAVE][GEMV_TILE];

  // lane owns columns c0 .. c0+3 of the tile, the wave rows rw .. rw+63
  const int c0 = J * GEMV_TILE + 4 * lane;
  const int rw = I * GEMV_TILE + wave * 64;
  double yc[NV][4];
#pragma unroll
  for (int w = 0; w < NV; ++w)
#pragma unroll
    for (int e = 0; e < 4; ++e) yc[w][e] = 0.0;
  const int64_t vstride = (int64_t)nb * nb * GEMV_TILE;
  gmem<double>* gvp[NV];
  gmem<double>* rowout[NV];
#pragma unroll
  for (int w = 0; w < NV; ++w) {
    gvp[w] = gp(p.gvp) + w * vstride;
    rowout[w] = gvp[w] + ((int64_t)I * nb + J) * GEMV_TILE + wave * 64;
  }
  if (rw < n) {
    const gmem<const T>* __restrict__ A = gp((const T*)p.A);
    if (p.avec)
      gemv_stream<T, RB, true, NV>(A, p.lda, n, rw, c0, vin, inv, diag, yc, rowout, lane);
    else
      gemv_stream<T, RB, false, NV>(A, p.lda, n, rw, c0, vin, inv, diag, yc, rowout, lane);
  }
  // column sums: this wave's rows -> LDS, then the 4 waves in order (an LDS-only barrier: the
  // row-sum stores need not land first)
#pragma unroll
  for (int w = 0; w < NV; ++w)
#pragma unroll
    for (int e = 0; e < 4; ++e) cred[w][wave][4 * lane + e] = yc[w][e];
  lds_barrier();
  if (!diag) {
    const int c = threadIdx.x;
#pragma unroll
    for (int w = 0; w < NV; ++w)
      gvp[w][((int64_t)J * nb + I) * GEMV_TILE + c] = cred[w][0][c] + cred[w][1][c] + cred[w][2][c] + cred[w][3][c];
  }
}

// Sparse A (CSR, both triangles): block row b, one row per thread, y_i = sum_k a_ik v_k in FP64 over
// the row's nonzeros in storage order; the row's one contribution goes to slot 0 of its partials
// (for NV = 2 also the basis vector's, in the second partial array).  Indices outside [0, n) or
// [0, nnz) are skipped and set E_INVALID (nnz travels in lda).
template <typename T, int NV>
__device__ __forceinline__ void spmv_rows(const Prob& p, int b, int j) {
  const int n = p.n, ld = p.ld, nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  const int pp = p.iscal[I_PP] & 1;
  const gmem<const double>* vin[NV];
  double inv[NV];
  vin[0] = gp((const double*)p.vec) + (int64_t)pp * ld;
  inv[0] = p.scal[S_INV];
  if constexpr (NV == 2) {
    vin[1] = gp((const double*)p.bh) + (int64_t)j * ld;
    inv[1] = p.scal[S_INVB];
  }
  const int i = b * GEMV_TILE + threadIdx.x;
  if (i >= n) return;
  const gmem<const int32_t>* rowptr = gp(p.rowptr);
  const gmem<const int32_t>* colidx = gp(p.colidx);
  const gmem<const T>* vals = gp((const T*)p.A);
  const int64_t k0 = max((int64_t)rowptr[i], (int64_t)0), k1 = min((int64_t)rowptr[i + 1], p.lda);
  double y[NV];
#pragma unroll
  for (int w = 0; w < NV; ++w) y[w] = 0.0;
  bool bad = false;
  for (int64_t k = k0; k < k1; ++k) {
    const int c = colidx[k];
    if ((unsigned)c >= (unsigned)n) { bad = true; continue; }
    const double a = (double)vals[k];
#pragma unroll
    for (int w = 0; w < NV; ++w) y[w] = fma(a, vin[w][c] * inv[w], y[w]);
  }
  if (bad) set_status(p, PSDPROJ_E_INVALID);
  const int64_t vstride = (int64_t)nb * nb * GEMV_TILE;
#pragma unroll
  for (int w = 0; w < NV; ++w) gp(p.gvp)[w * vstride + (int64_t)b * nb * GEMV_TILE + threadIdx.x] = y[w];
}

template <int NV>
__device__ __forceinline__ void gemv_block(const Prob* __restrict__ probs, const int* __restrict__ tstart, int nprob,
                                           int j) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (p.csr) {
    if (p.prec == F64) spmv_rows<double, NV>(p, t, j);
    else spmv_rows<float, NV>(p, t, j);
    return;
  }
  const int G = tstart[pi + 1] - tstart[pi];   // this problem's workgroups
  for (int u = t; u < p.gv_tiles; u += G) {
    if (p.prec == F64) gemv_tile<double, 4, NV>(p, u, j);
    else gemv_tile<float, 8, NV>(p, u, j);
    if (u + G < p.gv_tiles) lds_barrier();     // the next tile rewrites the column-sum stage
  }
}

__global__ __launch_bounds__(GEMV_THREADS) void k_gemv(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                       int nprob) {
  gemv_block<1>(probs, tstart, nprob, 0);
}

// Paired form of Alg. 5, product j: X v_j (first run) and X b_j (basis of the second run)
// from one read of A.
__global__ __launch_bounds__(GEMV_THREADS) void k_gemv2(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                        int nprob, int j) {
  gemv_block<2>(probs, tstart, nprob, j);
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

int gemv_tile_count(const Prob& p) {
  const int nb = (p.n + GEMV_TILE - 1) / GEMV_TILE;
  return p.csr ? nb : nb * (nb + 1) / 2;
}
int tiles_gemv(const Prob& p) {
  return p.csr ? gemv_tile_count(p) : (gemv_tile_count(p) + GV_PER_WG - 1) / GV_PER_WG;
}
int tiles_gemv_rows(const Prob& p) { return (p.n + GEMV_TILE - 1) / GEMV_TILE; }
int tiles_vec(const Prob& p) { return (p.ld + 1023) / 1024; }
int tiles_omega(const Prob& p) { return (int)(((int64_t)p.rpad * p.ld + 1023) / 1024); }

void launch_gemv(const Launch& L, int last) {
  (void)last;
  hipLaunchKernelGGL(k_gemv, dim3(L.grid), dim3(GEMV_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_gemv_finish(const Launch& L, int last) {
  hipLaunchKernelGGL(k_gemv_finish, dim3(L.grid), dim3(GEMV_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, last);
}
void launch_gemv2(const Launch& L, int j) {
  hipLaunchKernelGGL(k_gemv2, dim3(L.grid), dim3(GEMV_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, j);
}
void launch_gemv2_finish(const Launch& L, int j) {
  hipLaunchKernelGGL(k_gemv2_finish, dim3(L.grid), dim3(GEMV_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob, j);
}
void launch_alpha2(const Launch& L) {
  hipLaunchKernelGGL(k_alpha2, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
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
