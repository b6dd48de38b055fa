// Alg. 4 (power iteration for sigma_1) and Alg. 5 (alpha = |sigma_1(X) - sigma_1(X - sigma_1 I)|).
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

// Stream one wave's 64 rows of a tile in batches of RB rows, double-buffered in registers (the
// loop is fully unrolled, so the loads of batch bt+1 are in flight while batch bt is used and
// no copy between the buffers forces an early wait).  VEC: rows start and end 16-byte aligned,
// so a 16-byte chunk lies wholly inside or wholly past column n; chunks past n read the row's
// first chunk instead (their v_J entries are zero, and their column sums belong to columns
// past n, never read).  Otherwise element loads at clamped addresses with the values past
// column n zeroed.  Rows past n are loaded clamped to row n-1; their row sums land in partial
// slots that are never read and their column terms are multiplied by a zero v_I.
// The vector entries are waited for only once two batches of A are in flight, so the tile's
// stream starts without waiting for them.
template <typename T, int RB, bool VEC>
__device__ __forceinline__ void gemv_stream(const gmem<const T>* __restrict__ A, int64_t lda, int n, int rw, int c0,
                                            const gmem<const double>* __restrict__ vin, double inv, bool diag,
                                            double (&yc)[4], gmem<double>* __restrict__ rowout, int lane) {
  constexpr int NBT = 64 / RB;
  constexpr int LOGRB = (RB == 16) ? 4 : (RB == 8) ? 3 : 2;
  T a[2][RB][4];
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
  double vjr[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) vjr[e] = vin[min(c0 + e, n - 1)];
  const double vrr = vin[min(rw + lane, n - 1)];
  load(a[0], rw);
  double vj[4], vrow = 0.0;
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt) {
    // keep the scheduler from hoisting later batches' loads (they would need more buffers)
    __builtin_amdgcn_sched_barrier(0);
    if (bt + 1 < NBT) load(a[(bt + 1) & 1], rw + (bt + 1) * RB);
    if (bt == 0) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 4; ++e) vj[e] = (c0 + e < n) ? vjr[e] * inv : 0.0;
      // v_I of row rw + lane (zero past n and on the diagonal tile, whose transpose is itself)
      vrow = (!diag && rw + lane < n) ? vrr * inv : 0.0;
    }
    double rs[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      double x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = (double)a[bt & 1][q][e];
      rs[q] = x[0] * vj[0] + x[1] * vj[1] + x[2] * vj[2] + x[3] * vj[3];
      const double vi = bcast_f64(vrow, bt * RB + q);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        yc[e] += x[e] * vi;
        // pin the column update to its row: otherwise it is deferred past the row sums and
        // every converted row stays live
        __asm__ volatile("" : "+v"(yc[e]));
      }
    }
    reduce_scatter<RB>(rs, lane);
    if ((lane & ((64 / RB) - 1)) == 0) rowout[bt * RB + (lane >> (6 - LOGRB))] = rs[0];
  }
}

// RB rows per load batch: 8 for FP32 storage, 4 for FP64 (32 VGPRs of A per buffer, so the
// kernel keeps 3 waves per SIMD).
template <typename T, int RB>
__device__ __forceinline__ void gemv_tile(const Prob& p, int t) {
  const int n = p.n, ld = p.ld;
  const int nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  int I, J;
  gemv_tile_ij(t, I, J);
  const bool diag = (I == J);
  const int pp = p.iscal[I_PP] & 1;                 // ping-pong: read vec[pp], write vec[1-pp]
  const gmem<const double>* __restrict__ vin = gp((const double*)p.vec) + (int64_t)pp * ld;
  const double inv = p.scal[S_INV];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  __shared__ double cred[GEMV_THREADS / WAVE][GEMV_TILE];

  // lane owns columns c0 .. c0+3 of the tile, the wave rows rw .. rw+63
  const int c0 = J * GEMV_TILE + 4 * lane;
  const int rw = I * GEMV_TILE + wave * 64;
  double yc[4] = {0.0, 0.0, 0.0, 0.0};
  gmem<double>* __restrict__ gvp = gp(p.gvp);
  gmem<double>* __restrict__ rowout = gvp + ((int64_t)I * nb + J) * GEMV_TILE + wave * 64;
  if (rw < n) {
    const gmem<const T>* __restrict__ A = gp((const T*)p.A);
    if (p.avec)
      gemv_stream<T, RB, true>(A, p.lda, n, rw, c0, vin, inv, diag, yc, rowout, lane);
    else
      gemv_stream<T, RB, false>(A, p.lda, n, rw, c0, vin, inv, diag, yc, rowout, lane);
  }
  // column sums: this wave's rows -> LDS, then the 4 waves in order (an LDS-only barrier: the
  // row-sum stores need not land first)
#pragma unroll
  for (int e = 0; e < 4; ++e) cred[wave][4 * lane + e] = yc[e];
  lds_barrier();
  if (!diag) {
    const int c = threadIdx.x;
    gvp[((int64_t)J * nb + I) * GEMV_TILE + c] = cred[0][c] + cred[1][c] + cred[2][c] + cred[3][c];
  }
}

// Sparse A (CSR, both triangles): block row b, one row per thread, y_i = sum_k a_ik v_k in FP64 over
// the row's nonzeros in storage order; the row's one contribution goes to slot 0 of its partials.
// Indices outside [0, n) or [0, nnz) are skipped and set E_INVALID (nnz travels in lda).
template <typename T>
__device__ __forceinline__ void spmv_rows(const Prob& p, int b) {
  const int n = p.n, ld = p.ld, nb = (n + GEMV_TILE - 1) / GEMV_TILE;
  const int pp = p.iscal[I_PP] & 1;
  const gmem<const double>* __restrict__ vin = gp((const double*)p.vec) + (int64_t)pp * ld;
  const double inv = p.scal[S_INV];
  const int i = b * GEMV_TILE + threadIdx.x;
  if (i >= n) return;
  const gmem<const int32_t>* rowptr = gp(p.rowptr);
  const gmem<const int32_t>* colidx = gp(p.colidx);
  const gmem<const T>* vals = gp((const T*)p.A);
  const int64_t k0 = max((int64_t)rowptr[i], (int64_t)0), k1 = min((int64_t)rowptr[i + 1], p.lda);
  double y = 0.0;
  bool bad = false;
  for (int64_t k = k0; k < k1; ++k) {
    const int j = colidx[k];
    if ((unsigned)j >= (unsigned)n) { bad = true; continue; }
    y = fma((double)vals[k], vin[j] * inv, y);
  }
  if (bad) set_status(p, PSDPROJ_E_INVALID);
  gp(p.gvp)[(int64_t)b * nb * GEMV_TILE + threadIdx.x] = y;
}

__global__ __launch_bounds__(GEMV_THREADS) void k_gemv(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                       int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (p.csr) {
    if (p.prec == F64) spmv_rows<double>(p, t);
    else spmv_rows<float>(p, t);
    return;
  }
  const int G = tstart[pi + 1] - tstart[pi];   // this problem's workgroups
  for (int u = t; u < p.gv_tiles; u += G) {
    if (p.prec == F64) gemv_tile<double, 4>(p, u);
    else gemv_tile<float, 8>(p, u);
    if (u + G < p.gv_tiles) lds_barrier();     // the next tile rewrites the column-sum stage
  }
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
