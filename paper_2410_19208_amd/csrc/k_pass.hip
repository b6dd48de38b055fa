// Passes over A: Y = M(Z) with M(Z) = A Z (Alg. 2) or (A Z + alpha Z)/alpha (Alg. 3, the
// scaled matrix B = (A + alpha I)/alpha applied without forming it).  Used for the sketch
// (Z = Omega), the power iterations (Z = Q) and the compression pass (Z = Q).
//
// Every pass streams A once from HBM; the n x r panel Z is re-read from L2 by every row tile.
// K is split into `split` chunks (at most 8); workgroups are dealt round-robin to the 8 XCDs
// and the tile index is chunk-minor, so with split = 8 every workgroup of one XCD works on the
// same K chunk and that XCD's L2 holds only its 1/8 of Z.  Partials are summed in a fixed
// order by k_pass_reduce, so results do not depend on scheduling.
//
// FP32 / BF16X3 (k_pass_lds): 8 waves own a 256-row tile and all r columns; each wave computes
// a 64-row x r/2 block (4 x r/32 MFMA tiles), which balances the LDS bytes read per MFMA
// between the A and Z operands.  Each K step of 32 moves the A slice (256 x 32 FP32) and the Z
// slice (32 x r) from global memory straight into LDS (global_load_lds_dwordx4, no VGPR
// round trip), double-buffered so the loads of step s+1 overlap the MFMAs of step s; one
// barrier per step.  Slots inside each 1 KB block are XOR-swizzled so every 16-lane LDS read
// of an MFMA operand touches 16 distinct 16-byte bank groups.
//   FP32   -> v_mfma_f32_16x16x4f32;
//   BF16X3 -> v_mfma_f32_16x16x32_bf16 on the splits x = hi + lo (hi = bf16(x),
//             lo = bf16(x - hi)), accumulating hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term,
//             ~2^-16 relative, is dropped).  A is split in registers after the LDS read; Z is
//             stored pre-split.
// FP64 (k_pass): 4 waves own a 64-row tile; A goes to registers in MFMA operand order, the
// Z slice through LDS; v_mfma_f64_16x16x4f64 (this path is MFMA bound).
#include "common.hpp"
#include "launch.hpp"

namespace psd {

// ---------------------------------------------------------------- FP64: register A, LDS Z
template <int NCB>
__global__ __launch_bounds__(PASS_THREADS, 2) void k_pass(const Prob* __restrict__ probs,
                                                         const int* __restrict__ tstart, int nprob) {
  constexpr int BM = PASS_BM_D, BK = PASS_BK_D, KPL = BK / 4, NC = NCB * 16;
  constexpr int CSTRIDE = BK * 8 + 16;   // bytes per LDS column (padded against bank conflicts)
  constexpr int CH = BK * 8 / 16;        // 16-byte chunks per column
  __shared__ __attribute__((aligned(16))) unsigned char lds[NC * CSTRIDE];

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
  const gmem<const double>* __restrict__ A = gp((const double*)p.A);
  const gmem<const double>* __restrict__ Zm = gp((const double*)p.zm);
  const int64_t lda = p.lda;

  f64x4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = f64x4{0, 0, 0, 0};

  const bool rows_full = (m0 + BM <= n) && p.avec;
  const int rowg = m0 + wave * 16 + lrow;

  for (int kk = kbeg; kk < kend; kk += BK) {
    // ---- A fragment: lane (row, kg) holds A[row][kk + kg*KPL .. + KPL)
    double a[KPL];
    const int c0 = kk + kg * KPL;
    if (rows_full && kk + BK <= n) {
      const gmem<const double>* src = A + (int64_t)rowg * lda + c0;
#pragma unroll
      for (int v = 0; v < KPL; v += 2) {
        f64x2 x = __builtin_nontemporal_load((const gmem<f64x2>*)(src + v));
        a[v] = x[0]; a[v + 1] = x[1];
      }
    } else {
#pragma unroll
      for (int v = 0; v < KPL; ++v) {
        const int col = c0 + v;
        a[v] = (rowg < n && col < n) ? A[(int64_t)rowg * lda + col] : 0.0;
      }
    }
    // ---- Z slice [kk, kk+BK) x [0, NC) into LDS (column-major, padded)
    for (int c = threadIdx.x; c < NC * CH; c += PASS_THREADS) {
      const int col = c / CH, ch = c - col * CH;
      const gmem<const u32x4>* src = (const gmem<const u32x4>*)(Zm + (int64_t)col * ld + kk) + ch;
      *(u32x4*)(lds + col * CSTRIDE + ch * 16) = *src;
    }
    __syncthreads();
#pragma unroll
    for (int t2 = 0; t2 < KPL; t2 += 2) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int col = cb * 16 + lrow;
        const double2 b = *(const double2*)(lds + col * CSTRIDE + (kg * KPL + t2) * 8);
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t2 + 0], b.x, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t2 + 1], b.y, acc[cb], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---- partial tile: lane holds rows acc_row(kg, v) of its 16-row block, column cb*16 + lrow
  double* __restrict__ out = (double*)p.part + (int64_t)s * p.rpad * ld;
  const int rbase = m0 + wave * 16;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    double* dst = out + (int64_t)(cb * 16 + lrow) * ld + rbase;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[acc_row<true>(kg, v)] = acc[cb][v];
  }
}

// ---------------------------------------------------------------- FP32 / BF16X3: LDS ring
constexpr int PL_THREADS = 512;                  // 8 waves: 4 row groups x 2 column halves
constexpr int PL_BM = PASS_BM_F;                 // 256 rows per tile (64 per row group)
constexpr int PL_BK = 32;                        // K per step
constexpr int PL_ABYTES = PL_BM * PL_BK * 4;     // A slice: 32 blocks of 1 KB (8 rows each)

// LDS bytes of one step: A slice + Z slice (2 KB per 16 columns: hi and lo, or FP32).
__host__ __device__ constexpr int pl_stage_bytes(int ncb) { return PL_ABYTES + ncb * 2048; }

// Operand pointers and sizes of one pass, held in registers (the descriptor is read once).
struct PlArgs {
  const float* A; int64_t lda;
  const void* z0; const void* z1;   // BF16X3: hi, lo; FP32: the panel (z1 unused)
  int n, ld, avec;
};

// Issue the loads of step k0 into `stage`.
//   A block b (rows 8b .. 8b+7 of the tile): row i at byte (i % 8) * 128, 16-byte slot s
//     holds the 4 floats of chunk s ^ ((i % 16) / 2), i.e. columns k0 + 4c .. +3.
//   Z, BF16X3: blocks 0..NCB-1 hold hi, NCB..2NCB-1 lo; block cb holds columns
//     16cb .. 16cb+15 at 64 bytes each; slot s of column j holds chunk s ^ ((j % 16) / 4)
//     (bf16 rows k0 + 8c .. +7).
//   Z, FP32: block b holds columns 8b .. 8b+7 at 128 bytes each; slot s of column j holds
//     chunk s ^ ((j % 16) / 2) (rows k0 + 4c .. +3).
// A rows past n are clamped to n - 1 (their outputs are never stored); A chunks starting at or
// past n read the row's first chunk instead and are zeroed after the LDS read.  Z rows in
// [n, ld) are zero in every panel.
template <int PREC, int NCB>
__device__ __forceinline__ void pl_issue(const PlArgs& g, unsigned char* stage, int m0, int k0, int wave,
                                         int lane) {
  const int n = g.n;
  if (g.avec) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int blk = wave * 4 + u;
      const int i = blk * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((i & 15) >> 1);
      const int row = min(m0 + i, n - 1);
      const int col = k0 + 4 * c;
      dma16(g.A + (int64_t)row * g.lda + (col < n ? col : 0), stage + blk * 1024);
    }
  } else {
    // rows not 16-byte aligned: element loads through VGPRs, same LDS layout
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int blk = wave * 4 + u;
      const int i = blk * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((i & 15) >> 1);
      const int row = min(m0 + i, n - 1);
      const int col = k0 + 4 * c;
      const gmem<const float>* src = gp(g.A) + (int64_t)row * g.lda;
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (col + e < n) ? src[col + e] : 0.0f;
      *(f32x4*)(stage + blk * 1024 + lane * 16) = v;
    }
  }
  unsigned char* zs = stage + PL_ABYTES;
#pragma unroll
  for (int u = 0; u < (2 * NCB + 7) / 8; ++u) {
    const int b = wave + 8 * u;
    if (b >= 2 * NCB) break;
    if constexpr (PREC == B3) {
      const bf16* z = (const bf16*)((b < NCB) ? g.z0 : g.z1);
      const int cb = (b < NCB) ? b : b - NCB;
      const int j = lane >> 2;
      const int c = (lane & 3) ^ (j >> 2);
      dma16(z + (int64_t)(cb * 16 + j) * g.ld + k0 + 8 * c, zs + b * 1024);
    } else {
      const float* z = (const float*)g.z0;
      const int col = b * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((col & 15) >> 1);
      dma16(z + (int64_t)col * g.ld + k0 + 4 * c, zs + b * 1024);
    }
  }
}

// MFMAs of one step.  Lane (li, kg) of an operand holds K indices 8kg .. 8kg+7 of the step.
template <int PREC, int NCB>
__device__ __forceinline__ void pl_compute(const unsigned char* stage, int wr, int wc, int lane, int kvalid,
                                           f32x4 (&acc)[4][NCB / 2]) {
  constexpr int NCH = NCB / 2;
  const int li = lane & 15, kg = lane >> 4;
  const unsigned char* zs = stage + PL_ABYTES;
  // A fragments: rows wr*64 + rb*16 + li (so row % 16 == li)
  f32x4 a0[4], a1[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int i = wr * 64 + rb * 16 + li;
    const unsigned char* rowp = stage + (i >> 3) * 1024 + (i & 7) * 128;
    a0[rb] = *(const f32x4*)(rowp + (((2 * kg) ^ (li >> 1)) << 4));
    a1[rb] = *(const f32x4*)(rowp + (((2 * kg + 1) ^ (li >> 1)) << 4));
  }
  if (kvalid < PL_BK) {   // last step of a ragged K range: zero A past the end
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (8 * kg + e >= kvalid) a0[rb][e] = 0.0f;
        if (8 * kg + 4 + e >= kvalid) a1[rb][e] = 0.0f;
      }
  }
  if constexpr (PREC == B3) {
    bf16x8 ahi[4], alo[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = (e < 4) ? a0[rb][e] : a1[rb][e - 4];
        const bf16 h = (bf16)x;
        ahi[rb][e] = h;
        alo[rb][e] = (bf16)(x - (float)h);
      }
    const int zoff = li * 64 + ((kg ^ (li >> 2)) << 4);
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) {
      const int gcb = wc * NCH + cb;
      const bf16x8 bhi = *(const bf16x8*)(zs + gcb * 1024 + zoff);
      const bf16x8 blo = *(const bf16x8*)(zs + (NCB + gcb) * 1024 + zoff);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], bhi, acc[rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], blo, acc[rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[rb], bhi, acc[rb][cb], 0, 0, 0);
    }
  } else {
    const int zoff0 = (li & 7) * 128 + (((2 * kg) ^ (li >> 1)) << 4);
    const int zoff1 = (li & 7) * 128 + (((2 * kg + 1) ^ (li >> 1)) << 4);
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) {
      const int blk = 2 * (wc * NCH + cb) + (li >> 3);
      const f32x4 b0 = *(const f32x4*)(zs + blk * 1024 + zoff0);
      const f32x4 b1 = *(const f32x4*)(zs + blk * 1024 + zoff1);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[rb][e], b0[e], acc[rb][cb], 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[rb][e], b1[e], acc[rb][cb], 0, 0, 0);
    }
  }
}

template <int PREC, int NCB>
__global__ __launch_bounds__(PL_THREADS, 1) void k_pass_lds(const Prob* __restrict__ probs,
                                                           const int* __restrict__ tstart, int nprob) {
  static_assert(NCB % 2 == 0, "panel widths are multiples of 32 columns");
  constexpr int NCH = NCB / 2;
  constexpr int SB = pl_stage_bytes(NCB);
  extern __shared__ __attribute__((aligned(1024))) unsigned char smem[];

  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (t >= p.npass_tiles) return;
  const int s = t % p.split;
  const int m0 = (t / p.split) * PL_BM;
  const int n = p.n, ld = p.ld;
  const int kbeg = s * p.kchunk;
  const int kend = min(n, kbeg + p.kchunk);
  const int nsteps = (kend - kbeg + PL_BK - 1) / PL_BK;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int wr = wave & 3, wc = wave >> 2;

  f32x4 acc[4][NCH];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) acc[rb][cb] = f32x4{0, 0, 0, 0};

  PlArgs g;
  g.A = (const float*)p.A; g.lda = p.lda;
  g.z0 = (PREC == B3) ? (const void*)p.zhi : p.zm;
  g.z1 = (PREC == B3) ? (const void*)p.zlo : p.zm;
  g.n = n; g.ld = ld; g.avec = p.avec;
  float* __restrict__ out = (float*)p.part + (int64_t)s * p.rpad * ld;

  pl_issue<PREC, NCB>(g, smem, m0, kbeg, wave, lane);
  for (int st = 0; st < nsteps; ++st) {
    // this wave's loads of step st have landed; the barrier publishes everyone's, and also
    // ends every wave's reads of the other buffer (step st - 1), which step st + 1 overwrites
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    const int k0 = kbeg + st * PL_BK;
    if (st + 1 < nsteps) pl_issue<PREC, NCB>(g, smem + ((st + 1) & 1) * SB, m0, k0 + PL_BK, wave, lane);
    pl_compute<PREC, NCB>(smem + (st & 1) * SB, wr, wc, lane, kend - k0, acc);
  }

  // ---- partial tile: lane (li, kg) holds rows 4kg .. 4kg+3 of block (rb, cb), column li
  const int li = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int rbase = m0 + wr * 64 + rb * 16;
    if (rbase >= n) break;
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) {
      float* dst = out + (int64_t)((wc * NCH + cb) * 16 + li) * ld + rbase + 4 * kg;
      *(f32x4*)dst = acc[rb][cb];
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

#define PSD_NCB_EVEN(X) X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16)

void launch_pass(const Launch& L, int prec, int ncb) {
  if (prec == F64) {
    switch (ncb) {
#define PSD_CASE(N) case N: hipLaunchKernelGGL((k_pass<N>), dim3(L.grid), dim3(PASS_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob); break;
      PSD_NCB_EVEN(PSD_CASE)
#undef PSD_CASE
      default: break;
    }
    return;
  }
  switch (ncb) {
#define PSD_CASE(N)                                                                                              \
  case N:                                                                                                        \
    if (prec == F32)                                                                                             \
      hipLaunchKernelGGL((k_pass_lds<F32, N>), dim3(L.grid), dim3(PL_THREADS), 2 * pl_stage_bytes(N), L.stream, \
                         L.probs, L.tstart, L.nprob);                                                            \
    else                                                                                                         \
      hipLaunchKernelGGL((k_pass_lds<B3, N>), dim3(L.grid), dim3(PL_THREADS), 2 * pl_stage_bytes(N), L.stream,  \
                         L.probs, L.tstart, L.nprob);                                                            \
    break;
    PSD_NCB_EVEN(PSD_CASE)
#undef PSD_CASE
    default: break;
  }
}

// Opt the LDS-ring pass kernels into more than 64 KB of dynamic LDS.
void pass_init() {
#define PSD_ATTR(N)                                                                                    \
  hipFuncSetAttribute((const void*)k_pass_lds<F32, N>, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                      2 * pl_stage_bytes(N));                                                          \
  hipFuncSetAttribute((const void*)k_pass_lds<B3, N>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                      2 * pl_stage_bytes(N));
  PSD_NCB_EVEN(PSD_ATTR)
#undef PSD_ATTR
}

void launch_pass_reduce(const Launch& L) {
  hipLaunchKernelGGL(k_pass_reduce, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
