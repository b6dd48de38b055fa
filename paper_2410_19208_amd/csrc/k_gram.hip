// Gram products of n x r panels in FP64: G = Y^T Y (CholeskyQR rounds) and the compressed
// matrix C = Q^T M(Q) (Alg. 2 line 2 / Alg. 3 line 3), on v_mfma_f64_16x16x4f64.
//
// A workgroup computes one 32x32 tile of the r_pad x r_pad result over one chunk of
// GRAM_CHUNK rows; the chunk partials are summed in a fixed order by k_gram_reduce, so the
// result is deterministic.  For the symmetric Grams only the upper tiles are computed.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

__device__ __forceinline__ void gram_operands(const Prob& p, int mode, const void*& X, const void*& Y) {
  if (mode == 0) { X = p.y; Y = p.y; }
  else if (mode == 1) { X = p.q1; Y = p.q1; }
  else { X = p.zm; Y = p.y; }
}

template <typename T>
__device__ __forceinline__ void load4(const T* src, double out[4]) {
  if constexpr (sizeof(T) == 4) {
    float4 v = *(const float4*)src;
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
  } else {
    double2 a = *(const double2*)src, b = *(const double2*)(src + 2);
    out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
  }
}

template <typename T>
__device__ void gram_tile(const Prob& p, int mode, int tile, int chunk) {
  const int nt = p.rpad / GRAM_TILE;
  int ti, tj;
  if (mode == 2) { ti = tile / nt; tj = tile % nt; }
  else {  // upper tiles ti <= tj, enumerated row by row
    ti = 0;
    int rem = tile;
    while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
    tj = ti + rem;
  }
  const void* Xv; const void* Yv;
  gram_operands(p, mode, Xv, Yv);
  const T* X = (const T*)Xv;
  const T* Y = (const T*)Yv;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int li = lane & 15, kg = lane >> 4;
  const int ci = ti * GRAM_TILE + (wave >> 1) * 16 + li;   // X column (row of the result)
  const int cj = tj * GRAM_TILE + (wave & 1) * 16 + li;    // Y column (column of the result)
  const int r0 = chunk * GRAM_CHUNK;
  const int r1 = min(p.ld, r0 + GRAM_CHUNK);
  const int64_t ld = p.ld;
  f64x4 acc = {0, 0, 0, 0};
#pragma unroll 4
  for (int k = r0; k < r1; k += 16) {
    double a[4], b[4];
    load4<T>(X + (int64_t)ci * ld + k + kg * 4, a);
    load4<T>(Y + (int64_t)cj * ld + k + kg * 4, b);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
  }
  // lane holds result rows acc_row(kg, v) of the wave's 16x16 block, column li
  double* out = p.gpart + (int64_t)chunk * p.rpad * p.rpad;
  const int row0 = ti * GRAM_TILE + (wave >> 1) * 16;
  const int col = tj * GRAM_TILE + (wave & 1) * 16 + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[(int64_t)col * p.rpad + row0 + acc_row<true>(kg, v)] = acc[v];
}

__global__ __launch_bounds__(256) void k_gram(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                              int nprob, int arg) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int mode = arg & ORTH_ROUND_MASK;
  if (mode == 1 && orth_single(p, arg)) return;   // second CholeskyQR round not needed
  const int t = blockIdx.x - tstart[pi];
  const int nt = p.rpad / GRAM_TILE;
  const int ntiles = (mode == 2) ? nt * nt : nt * (nt + 1) / 2;
  if (t >= ntiles * p.ngchunk) return;
  const int chunk = t / ntiles, tile = t - chunk * ntiles;
  if (p.prec == F64) gram_tile<double>(p, mode, tile, chunk);
  else gram_tile<float>(p, mode, tile, chunk);
}

// Sum the chunk partials (fixed order), complete the symmetric result, zero outside r x r.
// One entry per thread (the sums over the chunks are the long part; more workgroups spread
// them over more CUs).
// Mode 2 symmetrises: C <- (C + C^T)/2.  A non-finite entry sets E_NONFINITE.
constexpr int GRED_PER_BLOCK = 256;
__global__ __launch_bounds__(256) void k_gram_reduce(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob, int arg) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int mode = arg & ORTH_ROUND_MASK;
  if (mode == 1 && orth_single(p, arg)) return;
  const int rp = p.rpad;
  const int64_t RR = (int64_t)rp * rp;
  double* dst = (mode == 2) ? p.C : p.G;
  const int64_t base = (int64_t)(blockIdx.x - tstart[pi]) * GRED_PER_BLOCK;
  bool bad = false;
  for (int e = threadIdx.x; e < GRED_PER_BLOCK; e += 256) {
    const int64_t idx = base + e;
    if (idx >= RR) break;
    const int j = (int)(idx / rp), i = (int)(idx - (int64_t)j * rp);
    double v = 0.0;
    if (i < p.r && j < p.r) {
      if (mode == 2) {
        double sij = 0.0, sji = 0.0;
        for (int c = 0; c < p.ngchunk; ++c) {
          sij += p.gpart[c * RR + (int64_t)j * rp + i];
          sji += p.gpart[c * RR + (int64_t)i * rp + j];
        }
        v = 0.5 * (sij + sji);
      } else {
        int a = i, b = j;
        if (i / GRAM_TILE > j / GRAM_TILE) { a = j; b = i; }  // lower tile: mirror of the upper one
        for (int c = 0; c < p.ngchunk; ++c) v += p.gpart[c * RR + (int64_t)b * rp + a];
      }
      if (!isfinite(v)) bad = true;
    }
    dst[idx] = v;
  }
  if (bad) set_status(p, PSDPROJ_E_NONFINITE);
}

int tiles_gram(const Prob& p, bool full) {
  const int nt = p.rpad / GRAM_TILE;
  return (full ? nt * nt : nt * (nt + 1) / 2) * p.ngchunk;
}

void launch_gram(const Launch& L, int mode) {
  hipLaunchKernelGGL(k_gram, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob, mode);
}
void launch_gram_reduce(const Launch& L, int mode) {
  hipLaunchKernelGGL(k_gram_reduce, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob, mode);
}

}  // namespace psd
