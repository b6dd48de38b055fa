// Philox4x32-10 test matrices and start vectors (Alg. 1 line 1, Alg. 4 line 1).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key bumped by the Weyl constants between rounds.  Counter/key/element
// conventions are those documented in psdproj.h.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c.x;
    uint64_t p1 = (uint64_t)M1 * c.z;
    U4 o;
    o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    o.y = (uint32_t)p1;
    o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    o.w = (uint32_t)p0;
    c = o;
  }
  return c;
}

__device__ __forceinline__ U4 philox_at(uint64_t seed, uint32_t stream, uint64_t c) {
  U4 ctr{(uint32_t)c, (uint32_t)(c >> 32), stream, 0u};
  return philox10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)(v >> 11) * 0x1.0p-53 + 0x1.0p-54;
}

// Element g of a Gaussian stream: Box-Muller on the two uniforms of counter g/2.
__device__ __forceinline__ double gauss_at(uint64_t seed, uint32_t stream, uint64_t g) {
  U4 w = philox_at(seed, stream, g >> 1);
  double u1 = unit53(w.x, w.y);
  double u2 = unit53(w.z, w.w);
  double rad = sqrt(-2.0 * log(u1));
  double ang = 2.0 * M_PI * u2;
  return (g & 1) ? rad * sin(ang) : rad * cos(ang);
}

// Structured test matrix (the subsampled randomized Hadamard transform, the structured
// alternative of Sec. 3.1's footnote), entries +1 / -1:
//   Omega[i][j] = d_i (-1)^popcount(i & s_j),  d_i from the low bit of word x0 of counter i,
//   stream 3, and s_j = pi(j) for a permutation pi of [0, 2^m) (m = max(1, ceil(log2 n))): a
//   four-round Feistel network on w = m + (m mod 2) bits, round t adding F_t(R) = low w/2 bits of
//   word x0 of counter t 2^(w/2) + R (stream 4) into the left half, re-applied while the value is
//   at least 2^m (cycle walking keeps it a permutation).
__device__ __forceinline__ uint32_t feistel(uint64_t seed, uint32_t x, int m) {
  const int h = (m + (m & 1)) >> 1;
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = (x >> h) & mask, R = x & mask;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint32_t f = philox_at(seed, 4u, ((uint64_t)t << h) + R).x & mask;
    const uint32_t nl = R;
    R = L ^ f;
    L = nl;
  }
  return (L << h) | R;
}

__device__ __forceinline__ uint32_t srht_column(uint64_t seed, uint32_t j, int m) {
  uint32_t y = feistel(seed, j, m);
  while (y >= (1u << m)) y = feistel(seed, y, m);   // ends: the walk follows a cycle through j
  return y;
}

__device__ __forceinline__ double srht_at(uint64_t seed, int i, uint32_t s) {
  const double d = (philox_at(seed, 3u, (uint64_t)i).x & 1u) ? -1.0 : 1.0;
  return (__builtin_popcount((uint32_t)i & s) & 1) ? -d : d;
}

__device__ __forceinline__ void split_bf16(float x, bf16& hi, bf16& lo) {
  hi = (bf16)x;
  lo = (bf16)(x - (float)hi);
}

// Omega panel (column-major, ld), zero outside n x r.
__global__ __launch_bounds__(256) void k_omega(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                               int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int64_t total = (int64_t)p.rpad * p.ld;
  const int64_t base = (int64_t)(blockIdx.x - tstart[pi]) * 1024;
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int64_t idx = base + e;
    if (idx >= total) break;
    const int j = (int)(idx / p.ld), i = (int)(idx % p.ld);
    double v = 0.0;
    if (i < p.n && j < p.r)
      v = p.sketch ? srht_at(p.seed, i, srht_column(p.seed, (uint32_t)j, p.srht_m))
                   : gauss_at(p.seed, 0u, (uint64_t)j * (uint64_t)p.n + (uint64_t)i);
    if (p.prec == F64) {
      ((double*)p.zm)[idx] = v;
    } else {
      float f = (float)v;
      ((float*)p.zm)[idx] = f;
      if (p.prec == B3) {
        const int64_t oz = zsplit_index(i, j, p.ld);
        split_bf16(f, p.zhi[oz], p.zlo[oz]);
      }
    }
  }
}

// Start vector of a power iteration (stream 1 or 2) into vec[0..ld), and reset the
// per-iteration scalars: inverse norm 1 (the first product uses the raw Gaussian vector).
__global__ __launch_bounds__(256) void k_power_init(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                    int nprob, int which) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int base = (blockIdx.x - tstart[pi]) * 1024;
  double* v = p.vec + (int64_t)(p.iscal[I_PP] & 1) * p.ld;   // the vector the next product reads
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int i = base + e;
    if (i >= p.ld) break;
    v[i] = (i < p.n) ? gauss_at(p.seed, (uint32_t)(1 + which), (uint64_t)i) : 0.0;
  }
  if (blockIdx.x == tstart[pi] && threadIdx.x == 0) {
    p.scal[S_INV] = 1.0;
    p.scal[S_SHIFT] = (which == 0) ? 0.0 : p.scal[S_SIGMA1];
  }
}

// Diagonal entry X_ii (dense in the storage type; CSR: the stored entries of row i in column i,
// added in storage order, indices outside the arrays skipped).
__device__ __forceinline__ double diag_entry(const Prob& p, int i) {
  if (p.csr) {
    const int64_t k0 = max((int64_t)p.rowptr[i], (int64_t)0), k1 = min((int64_t)p.rowptr[i + 1], p.lda);
    double d = 0.0;
    for (int64_t k = k0; k < k1; ++k)
      if (p.colidx[k] == i) d += (p.prec == F64) ? ((const double*)p.A)[k] : (double)((const float*)p.A)[k];
    return d;
  }
  const int64_t o = (int64_t)i * p.lda + i;
  return (p.prec == F64) ? ((const double*)p.A)[o] : (double)((const float*)p.A)[o];
}

// Start of Alg. 5 in its paired form: the first run's start vector (stream 1) into the vector
// the next product reads, the second run's (stream 2) into basis slot 0, and the shift of the
// basis' first two products, mu_0 = tr(X)/n: each block adds its rows' diagonal entries in a
// fixed order and the last block to finish (integer ticket) adds the block sums in block order.
__global__ __launch_bounds__(256) void k_power_init2(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int blk = blockIdx.x - tstart[pi];
  const int G = tstart[pi + 1] - tstart[pi];
  const int base = blk * 1024;
  double* v = p.vec + (int64_t)(p.iscal[I_PP] & 1) * p.ld;
  __shared__ double red[256 / 64];
  __shared__ double rows[256];
  __shared__ int is_last;
  const int x = threadIdx.x;
  double ds = 0.0;
  for (int e = x; e < 1024; e += 256) {
    const int i = base + e;
    if (i >= p.ld) break;
    const bool in = i < p.n;
    v[i] = in ? gauss_at(p.seed, 1u, (uint64_t)i) : 0.0;
    p.bh[i] = in ? gauss_at(p.seed, 2u, (uint64_t)i) : 0.0;
    if (in) ds += diag_entry(p, i);
  }
  const double ws = wave_sum(ds);
  if ((x & 63) == 0) red[x >> 6] = ws;
  __syncthreads();
  if (x == 0) {
    double tot = 0.0;
    for (int w = 0; w < 256 / 64; ++w) tot += red[w];
    p.vpart[blk] = tot;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    is_last = (atomicAdd(&p.iscal[I_COUNTER], 1) == G - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double tr = 0.0;
  for (int r0 = 0; r0 < G; r0 += 256) {
    if (r0 + x < G) rows[x] = p.vpart[r0 + x];
    __syncthreads();
    if (x == 0)
      for (int r = 0; r < 256 && r0 + r < G; ++r) tr += rows[r];
    __syncthreads();
  }
  if (x == 0) {
    const double mu0 = tr / (double)p.n;
    p.scal[S_INV] = 1.0;
    p.scal[S_INVB] = 1.0;
    p.scal[S_MU0] = mu0;
    p.scal[S_MU] = mu0;
    p.pw[0] = 1.0;
    p.iscal[I_COUNTER] = 0;
  }
}

__global__ void k_words(uint64_t seed, uint32_t stream, uint64_t c0, int64_t count, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  U4 w = philox_at(seed, stream, c0 + (uint64_t)i);
  out[4 * i + 0] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

__global__ void k_gauss(uint64_t seed, uint32_t stream, uint64_t start, int64_t count, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[i] = gauss_at(seed, stream, start + (uint64_t)i);
}

// the n x r structured test matrix, column-major (entry (i, j) at out[j n + i])
__global__ void k_srht(uint64_t seed, int n, int r, int m, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * r) return;
  const int j = (int)(e / n), i = (int)(e - (int64_t)j * n);
  out[e] = srht_at(seed, i, srht_column(seed, (uint32_t)j, m));
}

// ---------------------------------------------------------------- launchers
void launch_omega(const Launch& L) {
  hipLaunchKernelGGL(k_omega, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_power_init(const Launch& L, int which) {
  hipLaunchKernelGGL(k_power_init, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob, which);
}
void launch_power_init2(const Launch& L) {
  hipLaunchKernelGGL(k_power_init2, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_words(uint64_t seed, uint32_t stream_id, uint64_t c0, int64_t count, uint32_t* out, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_words, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, seed, stream_id, c0, count, out);
}
void launch_gauss(uint64_t seed, uint32_t stream_id, uint64_t start, int64_t count, double* out, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_gauss, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, seed, stream_id, start, count, out);
}

void launch_srht(uint64_t seed, int n, int r, double* out, hipStream_t s) {
  int m = 1;
  while ((int64_t(1) << m) < n) ++m;
  const int64_t count = (int64_t)n * r;
  if (count <= 0) return;
  hipLaunchKernelGGL(k_srht, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, seed, n, r, m, out);
}

}  // namespace psd
