// Passes over A: Y = M(Z) with M(Z) = A Z (Alg. 2) or (A Z + alpha Z)/alpha (Alg. 3, the
// scaled matrix B = (A + alpha I)/alpha applied without forming it).  Used for the sketch
// (Z = Omega), the power iterations (Z = Q) and the compression pass (Z = Q).
//
// Design (gfx950): a workgroup of 4 waves owns BM rows of A and every column of the n x r
// panel.  A streams from HBM straight into registers in MFMA operand order (each lane reads
// KPL consecutive elements of one row); the BK x r slice of Z is staged through LDS and
// shared by the 4 waves.  K is split into `split` chunks; with split = 8 the chunk index
// equals the XCD of the workgroup (blocks are dealt round-robin to the 8 XCDs), so each
// XCD's L2 holds only its own 1/8 of Z.  Partials are summed in a fixed order by
// k_pass_reduce, so results do not depend on scheduling.
//
// Precisions: FP64 -> v_mfma_f64_16x16x4f64; FP32 -> v_mfma_f32_16x16x4f32; BF16X3 ->
// v_mfma_f32_16x16x32_bf16 on the splits x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
// accumulating hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term, ~2^-16 relative, is dropped).
#include "common.hpp"
#include "launch.hpp"

namespace psd {

template <int PREC> struct PassCfg;
template <> struct PassCfg<F64> {
  typedef double TA; typedef f64x4 Acc;
  static constexpr int RB = 1, BM = PASS_BM_D, BK = PASS_BK_D, ESZ = 8, NBUF = 1;
};
template <> struct PassCfg<F32> {
  typedef float TA; typedef f32x4 Acc;
  static constexpr int RB = 2, BM = PASS_BM_F, BK = PASS_BK_F, ESZ = 4, NBUF = 1;
};
template <> struct PassCfg<B3> {
  typedef float TA; typedef f32x4 Acc;
  static constexpr int RB = 2, BM = PASS_BM_F, BK = PASS_BK_F, ESZ = 2, NBUF = 2;
};

template <int PREC, int NCB>
__global__ __launch_bounds__(PASS_THREADS, 2) void k_pass(const Prob* __restrict__ probs,
                                                         const int* __restrict__ tstart, int nprob) {
  typedef PassCfg<PREC> C;
  typedef typename C::TA TA;
  typedef typename C::Acc Acc;
  constexpr int RB = C::RB, BM = C::BM, BK = C::BK, KPL = BK / 4, NC = NCB * 16;
  constexpr int CSTRIDE = BK * C::ESZ + 16;   // bytes per LDS column (padded against bank conflicts)
  constexpr int CH = BK * C::ESZ / 16;         // 16-byte chunks per column
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::NBUF * NC * CSTRIDE];

  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (t >= p.npass_tiles) return;
  const int s = t % p.split;
  const int m0 = (t / p.split) * BM;
  const int n = p.n, ld = p.ld;
  const int kbeg = s * p.kchunk;
  const int kend = min(n, kbeg + p.kchunk);
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int lrow = lane & 15, kg = lane >> 4;
  const TA* __restrict__ A = (const TA*)p.A;
  const int64_t lda = p.lda;

  Acc acc[RB][NCB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = Acc{0, 0, 0, 0};

  const bool rows_full = (m0 + BM <= n) && p.avec;
  int rowg[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) rowg[rb] = m0 + wave * 16 * RB + rb * 16 + lrow;

  for (int kk = kbeg; kk < kend; kk += BK) {
    // ---- A fragments: lane (row, kg) holds A[row][kk + kg*KPL .. + KPL)
    TA a[RB][KPL];
    const int c0 = kk + kg * KPL;
    if (rows_full && kk + BK <= n) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const TA* src = A + (int64_t)rowg[rb] * lda + c0;
        if constexpr (PREC == F64) {
#pragma unroll
          for (int v = 0; v < KPL; v += 2) {
            f64x2 x = __builtin_nontemporal_load((const f64x2*)(src + v));
            a[rb][v] = x[0]; a[rb][v + 1] = x[1];
          }
        } else {
#pragma unroll
          for (int v = 0; v < KPL; v += 4) {
            f32x4 x = __builtin_nontemporal_load((const f32x4*)(src + v));
            a[rb][v] = x[0]; a[rb][v + 1] = x[1]; a[rb][v + 2] = x[2]; a[rb][v + 3] = x[3];
          }
        }
      }
    } else {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < KPL; ++v) {
          const int col = c0 + v;
          a[rb][v] = (rowg[rb] < n && col < n) ? A[(int64_t)rowg[rb] * lda + col] : (TA)0;
        }
    }

    // ---- Z slice [kk, kk+BK) x [0, NC) into LDS (column-major, padded)
    for (int c = threadIdx.x; c < C::NBUF * NC * CH; c += PASS_THREADS) {
      const int buf = c / (NC * CH);
      const int rem = c - buf * NC * CH;
      const int col = rem / CH, ch = rem - col * CH;
      const unsigned char* src;
      if constexpr (PREC == B3) {
        const bf16* z = buf ? p.zlo : p.zhi;
        src = (const unsigned char*)(z + (int64_t)col * ld + kk) + ch * 16;
      } else {
        src = (const unsigned char*)((const TA*)p.zm + (int64_t)col * ld + kk) + ch * 16;
      }
      *(uint4*)(lds + (buf * NC + col) * CSTRIDE + ch * 16) = *(const uint4*)src;
    }
    __syncthreads();

    // ---- MFMA over the slice
    if constexpr (PREC == B3) {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
        bf16x8 ahi[RB], alo[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float x = a[rb][ks * 8 + e];
            const bf16 h = (bf16)x;
            ahi[rb][e] = h;
            alo[rb][e] = (bf16)(x - (float)h);
          }
        const int koff = (kg * KPL + ks * 8) * 2;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int col = cb * 16 + lrow;
          const bf16x8 bhi = *(const bf16x8*)(lds + col * CSTRIDE + koff);
          const bf16x8 blo = *(const bf16x8*)(lds + (NC + col) * CSTRIDE + koff);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], bhi, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], blo, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[rb], bhi, acc[rb][cb], 0, 0, 0);
          }
        }
      }
    } else if constexpr (PREC == F32) {
#pragma unroll
      for (int t4 = 0; t4 < KPL; t4 += 4) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int col = cb * 16 + lrow;
          const float4 b = *(const float4*)(lds + col * CSTRIDE + (kg * KPL + t4) * 4);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][t4 + 0], b.x, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][t4 + 1], b.y, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][t4 + 2], b.z, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][t4 + 3], b.w, acc[rb][cb], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int t2 = 0; t2 < KPL; t2 += 2) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int col = cb * 16 + lrow;
          const double2 b = *(const double2*)(lds + col * CSTRIDE + (kg * KPL + t2) * 8);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][t2 + 0], b.x, acc[rb][cb], 0, 0, 0);
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][t2 + 1], b.y, acc[rb][cb], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- partial tile: lane holds rows acc_row(kg, v) of its 16-row block, column cb*16 + lrow
  TA* __restrict__ out = (TA*)p.part + (int64_t)s * p.rpad * ld;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int rbase = m0 + wave * 16 * RB + rb * 16;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      TA* dst = out + (int64_t)(cb * 16 + lrow) * ld + rbase;
      if constexpr (PREC == F64) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[acc_row<true>(kg, v)] = acc[rb][cb][v];
      } else {
        *(float4*)(dst + 4 * kg) = float4{acc[rb][cb][0], acc[rb][cb][1], acc[rb][cb][2], acc[rb][cb][3]};
      }
    }
  }
}

// Y = sum_s part[s] in fixed order; scaled: Y = (Y + alpha Z) / alpha.  Zero outside n x r.
template <typename T>
__device__ __forceinline__ void reduce_body(const Prob& p, int64_t base) {
  const int64_t P = (int64_t)p.rpad * p.ld;
  const T* part = (const T*)p.part;
  const T* z = (const T*)p.zm;
  T* y = (T*)p.y;
  const bool scaled = (p.variant == PSDPROJ_SCALED);
  const T alpha = (T)p.scal[S_ALPHA];
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int64_t idx = base + e;
    if (idx >= P) break;
    const int col = (int)(idx / p.ld), row = (int)(idx - (int64_t)col * p.ld);
    T v = 0;
    if (col < p.r && row < p.n) {
      for (int s = 0; s < p.split; ++s) v += part[(int64_t)s * P + idx];
      if (scaled) v = (v + alpha * z[idx]) / alpha;
    }
    y[idx] = v;
  }
}

__global__ __launch_bounds__(256) void k_pass_reduce(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int64_t base = (int64_t)(blockIdx.x - tstart[pi]) * 1024;
  if (p.prec == F64) reduce_body<double>(p, base);
  else reduce_body<float>(p, base);
}

// ---------------------------------------------------------------- tile counts and launchers
int tiles_pass(const Prob& p) {
  const int bm = (p.prec == F64) ? PASS_BM_D : PASS_BM_F;
  return ((p.n + bm - 1) / bm) * p.split;
}
int tiles_reduce(const Prob& p) { return (int)(((int64_t)p.rpad * p.ld + 1023) / 1024); }

template <int PREC>
static void launch_pass_prec(const Launch& L, int ncb) {
  switch (ncb) {
#define PSD_CASE(N) case N: hipLaunchKernelGGL((k_pass<PREC, N>), dim3(L.grid), dim3(PASS_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob); break;
    PSD_CASE(1) PSD_CASE(2) PSD_CASE(3) PSD_CASE(4) PSD_CASE(5) PSD_CASE(6) PSD_CASE(7) PSD_CASE(8)
    PSD_CASE(9) PSD_CASE(10) PSD_CASE(11) PSD_CASE(12) PSD_CASE(13) PSD_CASE(14) PSD_CASE(15) PSD_CASE(16)
#undef PSD_CASE
    default: break;
  }
}

void launch_pass(const Launch& L, int prec, int ncb) {
  if (prec == F64) launch_pass_prec<F64>(L, ncb);
  else if (prec == F32) launch_pass_prec<F32>(L, ncb);
  else launch_pass_prec<B3>(L, ncb);
}

void launch_pass_reduce(const Launch& L) {
  hipLaunchKernelGGL(k_pass_reduce, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
