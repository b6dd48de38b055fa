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
// BF16X3 (k_pass_b3): v_mfma_f32_16x16x32_bf16 on the splits x = hi + lo (hi = bf16(x),
// lo = bf16(x - hi)), accumulating hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term, ~2^-16
// relative, is dropped).  A is symmetric, so a tile's K slice is read as whole rows of A
// (coalesced 1 KB rows); Z is stored pre-split and its slices stream into LDS by DMA (no VGPR
// round trip).  8 waves x 32 rows x all r columns.  Widths 10 .. 14 on 16-byte aligned rows
// (pass_b3l_tile): A slices also reach LDS by DMA and are split from there, and the registers
// this frees prefetch the MFMA B operands; other widths (pass_b3_tile) load A straight into
// registers in MFMA operand order, two steps ahead.
// FP32 (k_pass_f32): 8 waves own a 256-row tile and all r columns; each wave computes a
// 64-row x r/2 block (4 x r/32 MFMA tiles).  Each K step of 32 moves the A slice (256 x 32)
// and the Z slice (32 x r) from global memory straight into LDS, double-buffered, one
// barrier per step; v_mfma_f32_16x16x4f32 (this path is MFMA bound).  Slots inside each
// 1 KB LDS block are XOR-swizzled so the 16-lane reads of an MFMA operand spread over the
// banks.
// FP64 (k_pass): 4 waves own a 64-row tile; A goes to registers in MFMA operand order, the
// Z slice through LDS; v_mfma_f64_16x16x4f64 (this path is MFMA bound).
#include <type_traits>

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

// ---------------------------------------------------------------- FP32: LDS ring
constexpr int PL_THREADS = 512;                  // 8 waves: 4 row groups x 2 column halves
constexpr int PL_BM = PASS_BM_F;                 // 256 rows per tile (64 per row group)
constexpr int PL_BK = 32;                        // K per step
constexpr int PL_ABYTES = PL_BM * PL_BK * 4;     // A slice: 32 blocks of 1 KB (8 rows each)

// LDS bytes of one step: A slice + Z slice (2 KB per 16 columns).
__host__ __device__ constexpr int pl_stage_bytes(int ncb) { return PL_ABYTES + ncb * 2048; }

// Operand pointers and sizes of one pass, held in registers (the descriptor is read once).
struct PlArgs {
  const float* A; int64_t lda;
  const float* z;
  int n, ld, avec;
};

// Issue the loads of step k0 into `stage`.
//   A block b (rows 8b .. 8b+7 of the tile): row i at byte (i % 8) * 128, 16-byte slot s
//     holds the 4 floats of chunk s ^ ((i % 16) / 2), i.e. columns k0 + 4c .. +3.
//   Z: block b holds columns 8b .. 8b+7 at 128 bytes each; slot s of column j holds chunk
//     s ^ ((j % 16) / 2) (rows k0 + 4c .. +3).
// A rows past n are clamped to n - 1 (their outputs are never stored); A chunks starting at or
// past n read the row's first chunk instead and are zeroed after the LDS read.  Z rows in
// [n, ld) are zero in every panel, and ld >= n + 32.
template <int NCB>
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
    const int col = b * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((col & 15) >> 1);
    dma16(g.z + (int64_t)col * g.ld + k0 + 4 * c, zs + b * 1024);
  }
}

// MFMAs of one step.  Lane (li, kg) of an operand holds K indices 8kg .. 8kg+7 of the step.
template <int NCB>
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
  {
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

template <int NCB>
__global__ __launch_bounds__(PL_THREADS, 1) void k_pass_f32(const Prob* __restrict__ probs,
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
  g.z = (const float*)p.zm;
  g.n = n; g.ld = ld; g.avec = p.avec;
  float* __restrict__ out = (float*)p.part + (int64_t)s * p.rpad * ld;

  pl_issue<NCB>(g, smem, m0, kbeg, wave, lane);
  for (int st = 0; st < nsteps; ++st) {
    // this wave's loads of step st have landed; the barrier publishes everyone's, and also
    // ends every wave's reads of the other buffer (step st - 1), which step st + 1 overwrites
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    const int k0 = kbeg + st * PL_BK;
    if (st + 1 < nsteps) pl_issue<NCB>(g, smem + ((st + 1) & 1) * SB, m0, k0 + PL_BK, wave, lane);
    pl_compute<NCB>(smem + (st & 1) * SB, wr, wc, lane, kend - k0, acc);
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

// ---------------------------------------------------------------- BF16X3: A read transposed
// A is symmetric, so a tile's K slice of A can be read as whole rows of A: the 256 output rows
// m0 .. m0+255 of the tile are 256 consecutive columns of A, and step k0 reads rows
// k0 .. k0+31 of A over those columns (1 KB per row; reading 128 bytes from each of 256 rows
// instead streams markedly slower).  Wave w owns output rows m0 + 32w .. +31 and every column
// of the panel.  Lane (li, kg) loads, for e = 0..7, the two floats of row k0 + 8kg + e at
// columns m0 + 32w + 2li, +1: for v = 0, 1 the eight values of column m0 + 32w + 2li + v are
// the MFMA A operand (K = 8kg .. 8kg+7) of row li of "virtual" row block v, whose 16 rows are
// m0 + 32w + 2i + v.  So A never passes through LDS: it is loaded PB_DIST steps ahead into a
// register ring, and only the Z slices (shared by the 8 waves) stream through a ring of
// PB_DIST + 1 LDS slices.
// VB = 2 virtual row blocks per wave (8 waves, two per SIMD).  Four (4 waves, one per SIMD,
// halving the LDS reads of Z) would need more than the register file with a 3-slot ring.
constexpr int PB_VB = 2;
constexpr int PB_BK = 32;
constexpr int PB_DIST = 2;                       // steps in flight ahead of the one computed
constexpr int PB_RING = PB_DIST + 1;
static_assert(PASS_BK_F % PB_BK == 0, "K chunks must be whole pass steps");
__host__ __device__ constexpr int pb_slice_bytes(int ncb) { return ncb * 2048; }   // hi + lo
__host__ __device__ constexpr int pb_lds_bytes(int ncb) { return PB_RING * pb_slice_bytes(ncb); }
// Z blocks (1 KB) per wave and step: wave w issues blocks w, w + 8, ... mod 2 ncb, so every
// wave issues the same number of loads (a repeated block rewrites the same bytes)
__host__ __device__ constexpr int pb_zpw(int ncb) { return (2 * ncb + 7) / 8; }

// Z slice layout: block b (1 KB) holds columns 16cb .. 16cb+15 of hi (b = cb) or lo
// (b = NCB + cb) for the step's 32 K rows, copied whole from one tile of the split panel
// (zsplit_index): chunk c (K rows 8c .. 8c+7) of column jj at byte 256 c + 16 jj.  Lane (li, kg)
// of an MFMA operand read takes chunk kg of column li, byte 16 x lane: 64 consecutive 16-byte
// pieces, which a ds_read_b128 serves without bank conflicts (64 bytes per column instead,
// swizzled or not, costs about 1.6x as long per read).

// s_waitcnt with vmcnt = N (0..63), lgkmcnt = 0, expcnt unchanged
#define PB_VMCNT(N) (0x0070 | ((N) & 15) | (((N) >> 4) << 14))

template <int VB> struct PbVec;
template <> struct PbVec<2> { using T = f32x2; };
template <> struct PbVec<4> { using T = f32x4; };

// One tile, VB virtual row blocks per wave (256 / (16 VB) waves).  AVEC: 16-byte aligned rows
// and n % 4 == 0 (A as VB-float loads; such a group of columns is wholly inside or wholly
// past column n); otherwise element loads at clamped addresses, and every step waits for all
// of its loads.
template <int NCB, int VB, bool AVEC>
__device__ __forceinline__ void pass_b3_tile(const Prob& p, int t, unsigned char* smem) {
  using VT = typename PbVec<VB>::T;
  constexpr int NW = PASS_BM_F / (16 * VB);       // waves
  constexpr int SB = pb_slice_bytes(NCB);
  constexpr int ZPW = (2 * NCB + NW - 1) / NW;    // Z blocks per wave and step
  constexpr int LPS = AVEC ? 8 + ZPW : 0;         // loads per wave and step
  const int s = t % p.split;
  const int m0 = (t / p.split) * PASS_BM_F;
  const int n = p.n, ld = p.ld;
  const int kbeg = s * p.kchunk;
  // 16-byte path: whole steps only (rows from ktail, n rounded down to a multiple of the step,
  // up to n are added by k_pass_reduce)
  const int kend = max(kbeg, min(AVEC ? p.ktail : n, kbeg + p.kchunk));
  const int nsteps = (kend - kbeg + PB_BK - 1) / PB_BK;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int li = lane & 15, kg = lane >> 4;
  const gmem<const bf16>* __restrict__ zhi = gp((const bf16*)p.zhi);
  const gmem<const bf16>* __restrict__ zlo = gp((const bf16*)p.zlo);
  const gmem<const float>* __restrict__ A = gp((const float*)p.A);
  const int64_t lda = p.lda;
  // first of this lane's VB columns (a group past n reads column 0 instead: its outputs are
  // rows past n, never stored)
  const int mc = m0 + 16 * VB * wave + VB * li;
  const int mcol = (mc < n) ? mc : 0;

  VT ar[PB_RING][8];         // A of the steps in flight: [ring slot][e]
  f32x4 acc[VB][NCB];
#pragma unroll
  for (int v = 0; v < VB; ++v)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[v][cb] = f32x4{0, 0, 0, 0};

  // 16-byte path: A read as a raw buffer whose range starts at row k0 of the step and ends at the
  // last element of row n - 1, so a row at or past n reads as zero without a per-lane clamp, and
  // every load is one scalar base plus this lane's fixed offset (row 8kg, column mcol) plus e rows.
  const int64_t lda4 = lda * 4;
  const uint32_t voff = (uint32_t)(((int64_t)8 * kg * lda + mcol) * 4);

  // loads of step st into ring slot S.  Steps past the last one load the last step again (a
  // slot nobody reads), so every step issues the same loads and the compiler's wait counts stay
  // exact.  Rows at or past the chunk end: the 16-byte path has none (its chunks are whole steps
  // and stop before ktail, so every row it reads is below n); the element path reads row kbeg
  // for them and zeroes them at use.
  auto issue = [&](auto S_, int st) {
    constexpr int S = decltype(S_)::value;
    const int k0 = kbeg + min(st, nsteps - 1) * PB_BK;
    if constexpr (AVEC) {
      const int64_t left = ((int64_t)(n - 1 - k0) * lda + n) * 4;   // bytes from row k0 to A's end
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)((const float*)p.A + (int64_t)k0 * lda), 0, (int)(uint32_t)min(left, (int64_t)0xffffffff),
          BUF_WORD3);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        ar[S][e] = __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, (int)(e * lda4), BUF_NT));
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * kg + e;
        const int64_t row = (int64_t)((k < kend) ? k : kbeg) * lda;
#pragma unroll
        for (int q = 0; q < VB; ++q) ar[S][e][q] = A[row + min(mc + q, n - 1)];
      }
    }
    unsigned char* zs = smem + S * SB;
#pragma unroll
    for (int u = 0; u < ZPW; ++u) {
      const int b = (wave + NW * u) % (2 * NCB);
      const gmem<const bf16>* z = (b < NCB) ? zhi : zlo;
      const int cb = (b < NCB) ? b : b - NCB;
      // tile (k0 / 32, cb) of the split panel starts at element (cb ld / 32 + k0 / 32) 512, which
      // is cb 16 ld + 16 k0 as k0 is a multiple of 32
      dma16((const void*)(z + (int64_t)cb * 16 * ld + 16 * k0 + 8 * lane), zs + b * 1024);
    }
  };

  // wait until this wave's loads of step st have landed (and its LDS reads of step st - 1 are
  // done): the only loads issued later are those of step st + 1.  Then a bare barrier: a
  // workgroup fence would also wait for the loads in flight for step st + 1 (LDS-DMA writes
  // count as vector memory operations).
  auto wait_step = [&]() {
    __builtin_amdgcn_s_waitcnt(PB_VMCNT(LPS));
    __asm__ volatile("s_barrier" ::: "memory");
    // nothing that uses the step's A registers may be scheduled above the wait (the wait
    // analysis would then drain every load in flight)
    __builtin_amdgcn_sched_barrier(0);
  };

  const int zoff = lane << 4;   // chunk kg of column li
  // hi/lo split of the A values of ring slot S (step st), done (up to width 14) one step ahead,
  // half-way through the previous step, so that its VALU work runs beside that step's MFMAs
  // instead of holding back the first MFMA of its own step
  bf16x8 ahi[PB_RING][VB], alo[PB_RING][VB];
  auto split = [&](auto S_, int st) {
    constexpr int S = decltype(S_)::value;
    const int kvalid = kend - (kbeg + st * PB_BK);
#pragma unroll
    for (int v = 0; v < VB; ++v)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float x = ar[S][e][v];
        // rows past the chunk end (element path only: the 16-byte path has whole steps)
        if (!AVEC && kvalid < PB_BK && 8 * kg + e >= kvalid) x = 0.0f;
        const bf16 hb = (bf16)x;
        ahi[S][v][e] = hb;
        alo[S][v][e] = (bf16)(x - (float)hb);
      }
  };

  // MFMAs of column-block pairs [cb0, cb1) of the step in ring slot S: 2 VB independent
  // accumulators between dependent MFMAs
  auto mfmas = [&](auto S_, auto CB0_, auto CB1_) {
    constexpr int S = decltype(S_)::value;
    const unsigned char* zs = smem + S * SB;
#pragma unroll
    for (int cb = decltype(CB0_)::value; cb < decltype(CB1_)::value; cb += 2) {
      const bf16x8 h0 = *(const bf16x8*)(zs + cb * 1024 + zoff);
      const bf16x8 h1 = *(const bf16x8*)(zs + (cb + 1) * 1024 + zoff);
      const bf16x8 l0 = *(const bf16x8*)(zs + (NCB + cb) * 1024 + zoff);
      const bf16x8 l1 = *(const bf16x8*)(zs + (NCB + cb + 1) * 1024 + zoff);
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[S][v], h0, acc[v][cb], 0, 0, 0);
        acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[S][v], h1, acc[v][cb + 1], 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[S][v], l0, acc[v][cb], 0, 0, 0);
        acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[S][v], l1, acc[v][cb + 1], 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[S][v], h0, acc[v][cb], 0, 0, 0);
        acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[S][v], h1, acc[v][cb + 1], 0, 0, 0);
      }
    }
  };

  // this wave's A loads of the step after the current one have landed: the only loads issued
  // after them are that step's Z slices and the loads of the step after it.  The scheduling
  // barrier keeps the split below the wait (a use hoisted above it would make the wait
  // analysis drain every load in flight).
  auto wait_next_a = [&]() {
    __builtin_amdgcn_s_waitcnt(PB_VMCNT(AVEC ? LPS + ZPW : 0));
    __builtin_amdgcn_sched_barrier(0);
  };

  // one step in ring slot S (= st mod PB_RING): its loads landed everywhere (the barrier also
  // ends every wave's reads of step st - 1, whose slot step st + PB_DIST overwrites), issue
  // step st + PB_DIST, compute step st, and half-way through split the A of step st + 1
  // (widths above 14 have no registers for two split steps: they split at the start of the step)
  constexpr bool AHEAD = NCB <= 14;
  constexpr int HALF = 2 * ((NCB / 2 + 1) / 2);   // column blocks before the split
  auto step = [&](auto S_, int st) {
    constexpr int S = decltype(S_)::value;
    wait_step();
    issue(std::integral_constant<int, (S + PB_DIST) % PB_RING>{}, st + PB_DIST);
    if constexpr (AHEAD) {
      mfmas(S_, std::integral_constant<int, 0>{}, std::integral_constant<int, HALF>{});
      wait_next_a();
      split(std::integral_constant<int, (S + 1) % PB_RING>{}, st + 1);
      mfmas(S_, std::integral_constant<int, HALF>{}, std::integral_constant<int, NCB>{});
    } else {
      split(S_, st);
      __builtin_amdgcn_sched_barrier(0);
      mfmas(S_, std::integral_constant<int, 0>{}, std::integral_constant<int, NCB>{});
    }
  };

  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  static_assert(PB_RING == 3, "the step loop below is unrolled for a ring of three");
  // a chunk that ktail leaves empty (nsteps = 0, kbeg >= 64 as n >= 32 on the 16-byte path)
  // loads the step before it, whose rows are below n, and writes a zero partial tile
  issue(S0{}, 0);
  issue(S1{}, 1);
  if constexpr (AHEAD) {
    wait_next_a();
    split(S0{}, 0);
  }
  int st = 0;
  for (; st + 3 <= nsteps; st += 3) {
    step(S0{}, st);
    step(S1{}, st + 1);
    step(S2{}, st + 2);
  }
  if (st < nsteps) step(S0{}, st);
  if (st + 1 < nsteps) step(S1{}, st + 1);
  // the repeated loads of the steps past the end must land before the workgroup's LDS is freed
  __builtin_amdgcn_s_waitcnt(PB_VMCNT(0));

  // ---- partial tile.  Lane (li, kg) of acc[v][cb] holds rows 4kg + r (r = 0..3) of virtual
  // block v, column li: output row m0 + 16 VB wave + VB (4 kg + r) + v, so the lane holds the
  // 4 VB consecutive rows from m0 + 16 VB wave + 4 VB kg (VB 16-byte stores per column).
  float* __restrict__ out = (float*)p.part + (int64_t)s * p.rpad * ld;
  const int rbase = m0 + 16 * VB * wave + 4 * VB * kg;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    float vals[4 * VB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int v = 0; v < VB; ++v) vals[VB * r + v] = acc[v][cb][r];
    float* col = out + (int64_t)(cb * 16 + li) * ld + rbase;
#pragma unroll
    for (int h = 0; h < VB; ++h)
      if (rbase + 4 * h < n) *(f32x4*)(col + 4 * h) = f32x4{vals[4 * h], vals[4 * h + 1], vals[4 * h + 2], vals[4 * h + 3]};
  }
}

// ---------------------------------------------------------------- BF16X3, A through LDS
// The same tile, product and virtual row blocks as pass_b3_tile on the 16-byte path, but the A
// slice of a step reaches LDS by DMA (1 KB rows) instead of through a ring of registers.  The
// registers that held A in flight prefetch the MFMA B operands one column-block pair ahead
// instead, and each step's barrier sits before its last pair, so the MFMAs of that pair run while
// the barrier clears and the next step's first operands are read.  A slices use a ring of 3 (rows
// padded to 1040 bytes, so the split's reads of rows 8 apart fall in other banks), Z slices a
// ring of 2; both are copied right after a step's barrier, by one wave per SIMD only, and must
// land by the next barrier.  The two rings take 157 KB at width 14 (width 16 does not fit).
// Used for widths 10 .. 14; measured at width 14, where the launch is about 7% shorter than with
// pass_b3_tile (copying A two steps ahead instead of one gained nothing).
// buffer range in bytes (a non-negative size), saturated to 32 bits
__device__ __forceinline__ int nrec32(int64_t bytes) {
  return (int)(((uint64_t)bytes >> 32) ? 0xffffffffu : (uint32_t)bytes);
}
constexpr int PBL_ROW = 1040;
constexpr int PBL_ASLOT = PB_BK * PBL_ROW;
__host__ __device__ constexpr bool pbl_used(int ncb) { return ncb >= 10 && ncb <= 14; }
__host__ __device__ constexpr int pbl_lds_bytes(int ncb) { return 3 * PBL_ASLOT + 2 * pb_slice_bytes(ncb); }
static_assert(pbl_lds_bytes(14) <= 160 * 1024, "both rings must fit the LDS of one CU");

template <int NCB>
__device__ __forceinline__ void pass_b3l_tile(const Prob& p, int t, unsigned char* smem) {
  constexpr int VB = 2;                           // 8 waves of 32 rows
  constexpr int SB = pb_slice_bytes(NCB);
  // Only waves 0 .. 3, one per SIMD, copy slices: a wave that issues a burst of copies stalls
  // until the vector memory unit has taken them (about 1 KB per instruction), so with the
  // copies in one wave of each SIMD the other wave keeps the matrix core busy meanwhile.
  constexpr int DW = 4;                           // copying waves
  constexpr int ZPC = 2 * NCB / DW;               // Z blocks per copying wave and step
  constexpr int APC = PB_BK / DW;                 // A rows per copying wave and step
  static_assert((2 * NCB) % DW == 0, "Z blocks split evenly over the copying waves");
  const int s = t % p.split;
  const int m0 = (t / p.split) * PASS_BM_F;
  const int n = p.n, ld = p.ld;
  const int kbeg = s * p.kchunk;
  const int kend = max(kbeg, min(p.ktail, kbeg + p.kchunk));   // whole steps, all rows below n
  const int nsteps = (kend - kbeg + PB_BK - 1) / PB_BK;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int li = lane & 15, kg = lane >> 4;
  const bool copier = wave < DW;
  const int64_t lda = p.lda;
  unsigned char* const aring = smem;
  unsigned char* const zring = smem + 3 * PBL_ASLOT;

  f32x4 acc[VB][NCB];
#pragma unroll
  for (int v = 0; v < VB; ++v)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[v][cb] = f32x4{0, 0, 0, 0};

  // copy of one A row: lane l copies columns m0 + 4l .. +3 (a group at or past n copies
  // column 0 instead: its outputs are rows past n, never stored); the buffer starts at row k0
  // and ends at A's last element, as in pass_b3_tile
  const int ca = m0 + 4 * lane;
  const uint32_t voff = (uint32_t)((ca < n ? ca : 0) * 4);
  // A's base stays in scalar registers (otherwise the compiler reloads it from the descriptor
  // every step, and the wait for that load also waits for the operand reads in flight)
  const float* Ab = (const float*)p.A;
  __asm__ volatile("" : "+s"(Ab));
  const int lda4 = (int)(lda * 4);
  // steps past the last one copy the last step again (into a slot nobody reads), so every step
  // issues the same loads and the wait counts below stay exact
  auto issue_a = [&](int slot, int st) {
    if (!copier) return;
    const int k0 = kbeg + min(st, nsteps - 1) * PB_BK;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Ab + (int64_t)k0 * lda), 0, nrec32(((int64_t)(n - 1 - k0) * lda + n) * 4), BUF_WORD3);
    unsigned char* as = aring + slot * PBL_ASLOT;
#pragma unroll
    for (int u = 0; u < APC; ++u) {
      const int row = wave + DW * u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)(as + row * PBL_ROW), 16, voff, row * lda4, 0, BUF_NT);
    }
  };
  // Z tile (k0 / 32, cb) of a split panel starts at element cb 16 ld + 16 k0 (see pass_b3_tile).
  // One buffer covers both split panels (two regions of the same workspace): it starts at
  // element 16 k0 of the lower one, block b of a step is a fixed scalar offset (the panel's
  // distance from the base plus cb 16 ld elements), and every lane copies its 16 bytes at the
  // same lane offset.
  const uint32_t zvoff = (uint32_t)lane << 4;
  const char* const zbase = ((const char*)p.zhi < (const char*)p.zlo) ? (const char*)p.zhi : (const char*)p.zlo;
  const int64_t zspan = max((const char*)p.zhi, (const char*)p.zlo) - zbase + (int64_t)p.rpad * ld * 2;
  int zsoff[ZPC];
#pragma unroll
  for (int u = 0; u < ZPC; ++u) {
    const int b = wave % DW + DW * u;
    const char* panel = (b < NCB) ? (const char*)p.zhi : (const char*)p.zlo;
    zsoff[u] = (int)(panel - zbase) + ((b < NCB) ? b : b - NCB) * 32 * ld;
  }
  auto issue_z = [&](int slot, int st) {
    if (!copier) return;
    const int k0 = kbeg + min(st, nsteps - 1) * PB_BK;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(zbase + 32 * (int64_t)k0), 0, nrec32(zspan - 32 * (int64_t)k0), BUF_WORD3);
    unsigned char* zs = zring + slot * SB;
#pragma unroll
    for (int u = 0; u < ZPC; ++u) {
      const int b = wave + DW * u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)(zs + b * 1024), 16, zvoff, zsoff[u], 0, 0);
    }
  };

  // Step st runs in register set R = st mod 2 and reads Z slot R.  Its column-block pairs run
  // 12 MFMAs each while the B operands of the next pair are read.  With pair SP, the A values of
  // step st + 1 are read from LDS and split into the other register set.  Lane (li, kg) takes
  // rows 8kg .. 8kg+7 of the slice at columns 32 wave + 2 li, +1: virtual row blocks 0 and 1.
  // The step's barrier comes before its last pair.  By then the copies of the Z slice of step
  // st + 1 and the A slice of step st + 2 have landed (each copying wave waits for its own), and
  // every wave's reads of step st's Z slot and of A(st + 1) are done.  After the barrier waves
  // 0 .. 3 copy the Z slice of step st + 2 into slot R and the A slice of step st + 3 into the
  // slot of A(st).  Every wave then reads the first B operands of step st + 1 while the last
  // pair's MFMAs run, so no wave stands idle after the barrier.  The scheduling groups fix this order (the default schedule reads each pair's
  // operands just before its MFMAs and waits for them).
  constexpr int NP = NCB / 2;
  constexpr int SP = NP / 2 - 1;
  bf16x8 ahi[2][VB], alo[2][VB];
  bf16x8 b[2][4];
  const int aoff = 8 * kg * PBL_ROW + (32 * wave + 2 * li) * 4;
  const int zoff = lane << 4;
  auto bread = [&](bf16x8 (&d)[4], const unsigned char* zs, int cb) {
    d[0] = *(const bf16x8*)(zs + cb * 1024);
    d[1] = *(const bf16x8*)(zs + (cb + 1) * 1024);
    d[2] = *(const bf16x8*)(zs + (NCB + cb) * 1024);
    d[3] = *(const bf16x8*)(zs + (NCB + cb + 1) * 1024);
  };
  auto pair = [&](auto R_, const bf16x8 (&bb)[4], int cb) {
    constexpr int R = decltype(R_)::value;
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[R][v], bb[0], acc[v][cb], 0, 0, 0);
      acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[R][v], bb[1], acc[v][cb + 1], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[R][v], bb[2], acc[v][cb], 0, 0, 0);
      acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[R][v], bb[3], acc[v][cb + 1], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      acc[v][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[R][v], bb[0], acc[v][cb], 0, 0, 0);
      acc[v][cb + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[R][v], bb[1], acc[v][cb + 1], 0, 0, 0);
    }
  };
  // pair j of a step in register set R uses operand buffer (j + R NP) mod 2, so the first pair of
  // the next step never shares a buffer with the last pair of this one
  auto step = [&](auto R_, int st, int a_issue, int a_next) {
    constexpr int R = decltype(R_)::value;
    const unsigned char* zs = zring + R * SB + zoff;
    const unsigned char* as = aring + a_next * PBL_ASLOT + aoff;
    f32x2 xa[8];
#pragma unroll
    for (int j = 0; j < NP - 1; ++j) {
      const int c = (j + R * NP) & 1;
      bread(b[c ^ 1], zs, 2 * j + 2);
      __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
      if (j == SP) {
#pragma unroll
        for (int e = 0; e < 8; ++e) xa[e] = *(const f32x2*)(as + e * PBL_ROW);
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
      }
      pair(R_, b[c], 2 * j);
      __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
      if (j == SP) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int v = 0; v < VB; ++v) {
            const bf16 hb = (bf16)xa[e][v];
            ahi[1 - R][v][e] = hb;
            alo[1 - R][v][e] = (bf16)(xa[e][v] - (float)hb);
          }
      }
    }
    __builtin_amdgcn_s_waitcnt(PB_VMCNT(0));
    __asm__ volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    issue_z(R, st + 2);
    issue_a(a_issue, st + 3);
    constexpr int cl = (NP - 1 + R * NP) & 1;
    bread(b[cl ^ 1], zring + (1 - R) * SB + zoff, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 1);
    pair(R_, b[cl], 2 * (NP - 1));
    __builtin_amdgcn_sched_group_barrier(0x008, 12, 1);
  };

  using R0 = std::integral_constant<int, 0>;
  using R1 = std::integral_constant<int, 1>;
  // a chunk that ktail leaves empty (nsteps = 0) copies the step before it, whose rows are below
  // n (kbeg >= 64), and writes a zero partial tile
  issue_a(0, 0);
  issue_a(1, 1);
  issue_a(2, 2);
  issue_z(0, 0);
  issue_z(1, 1);
  __builtin_amdgcn_s_waitcnt(PB_VMCNT(0));
  __asm__ volatile("s_barrier" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
  {
    const unsigned char* as = aring + aoff;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const f32x2 x = *(const f32x2*)(as + e * PBL_ROW);
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        const bf16 hb = (bf16)x[v];
        ahi[0][v][e] = hb;
        alo[0][v][e] = (bf16)(x[v] - (float)hb);
      }
    }
    bread(b[0], zring + zoff, 0);
  }
  int st = 0, a0 = 0;   // a0 = st mod 3: the A slot of step st
  for (; st + 2 <= nsteps; st += 2) {
    const int a1 = (a0 == 2) ? 0 : a0 + 1, a2 = (a1 == 2) ? 0 : a1 + 1;
    step(R0{}, st, a0, a1);
    step(R1{}, st + 1, a1, a2);
    a0 = a2;
  }
  if (st < nsteps) step(R0{}, st, a0, (a0 == 2) ? 0 : a0 + 1);
  // the copies of the steps past the end must land before the workgroup's LDS is freed
  __builtin_amdgcn_s_waitcnt(PB_VMCNT(0));

  // ---- partial tile (same lane layout as pass_b3_tile)
  float* __restrict__ out = (float*)p.part + (int64_t)s * p.rpad * ld;
  const int rbase = m0 + 16 * VB * wave + 4 * VB * kg;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    float vals[4 * VB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int v = 0; v < VB; ++v) vals[VB * r + v] = acc[v][cb][r];
    float* col = out + (int64_t)(cb * 16 + li) * ld + rbase;
#pragma unroll
    for (int h = 0; h < VB; ++h)
      if (rbase + 4 * h < n) *(f32x4*)(col + 4 * h) = f32x4{vals[4 * h], vals[4 * h + 1], vals[4 * h + 2], vals[4 * h + 3]};
  }
}

__host__ __device__ constexpr int pb_kernel_lds(int ncb) {
  return (pbl_used(ncb) && pbl_lds_bytes(ncb) > pb_lds_bytes(ncb)) ? pbl_lds_bytes(ncb) : pb_lds_bytes(ncb);
}

template <int NCB, int VB>
__global__ __launch_bounds__(PASS_BM_F / (16 * VB) * 64, 1)
void k_pass_b3(const Prob* __restrict__ probs, const int* __restrict__ tstart, int nprob) {
  static_assert(NCB % 2 == 0, "panel widths are multiples of 32 columns");
  extern __shared__ __attribute__((aligned(1024))) unsigned char smem[];
  int pi, t;
  if (nprob == 2 && probs[0].A == probs[1].A && probs[0].lda == probs[1].lda && probs[0].n == probs[1].n &&
      probs[0].split == probs[1].split && tstart[0] == 0 && tstart[1] == tstart[2] - tstart[1]) {
    // Two problems streaming the same A with the same tiling: tile t of both runs on the same
    // XCD (workgroup b runs on XCD b mod 8) one group of 8 workgroups apart, so the two reads
    // of each A slice meet in that XCD's L2 and HBM serves one.
    const int b = blockIdx.x, g = b >> 4, w = b & 15;
    pi = w >> 3;
    t = 8 * g + (w & 7);
  } else {
    pi = find_prob(tstart, nprob, blockIdx.x);
    t = blockIdx.x - tstart[pi];
  }
  const Prob& p = probs[pi];
  if (t >= p.npass_tiles) return;
  if (p.avec) {
    if constexpr (pbl_used(NCB) && VB == 2) pass_b3l_tile<NCB>(p, t, smem);
    else pass_b3_tile<NCB, VB, true>(p, t, smem);
  } else {
    pass_b3_tile<NCB, VB, false>(p, t, smem);
  }
}

// Y = sum_s part[s] in fixed order; scaled: Y = (Y + alpha Z) / alpha.  Zero outside n x r.
// One thread per 16-byte vector of a panel column (ld is a multiple of 128, so vectors never
// straddle columns), RD_VEC vectors per thread.
constexpr int RD_THREADS = 256;
constexpr int RD_VEC = 2;
template <typename T>
__device__ __forceinline__ void reduce_body(const Prob& p, int64_t vbase) {
  constexpr int VW = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VW)));
  const int64_t P = (int64_t)p.rpad * p.ld;
  const gmem<const T>* __restrict__ part = gp((const T*)p.part);
  const gmem<const T>* __restrict__ z = gp((const T*)p.zm);
  gmem<T>* __restrict__ y = gp((T*)p.y);
  const bool scaled = (p.variant == PSDPROJ_SCALED);
  const T alpha = (T)p.scal[S_ALPHA];
  const int split = p.split;
#pragma unroll
  for (int u = 0; u < RD_VEC; ++u) {
    const int64_t idx = (vbase + (int64_t)u * RD_THREADS + threadIdx.x) * VW;
    if (idx >= P) break;
    const int col = (int)(idx / p.ld), row = (int)(idx - (int64_t)col * p.ld);
    V v = {};
    if (col < p.r && row < p.n) {
      for (int s = 0; s < split; ++s) v += *(const gmem<V>*)(part + (int64_t)s * P + idx);
      if constexpr (sizeof(T) == 4) {
        // rows ktail .. n-1 of the K range, which the 16-byte BF16X3 pass leaves out (fewer
        // than 32): FP32 products added in K order, A[k][row .. row+VW-1] read as one vector (A
        // is symmetric; rows of A are 16-byte aligned and n % 4 == 0 on that path)
        const gmem<const T>* __restrict__ A = gp((const T*)p.A);
        for (int k = p.ktail; k < p.n; ++k)
          v += *(const gmem<V>*)(A + (int64_t)k * p.lda + row) * z[(int64_t)col * p.ld + k];
      }
      if (scaled) v = (v + alpha * *(const gmem<V>*)(z + idx)) / alpha;
#pragma unroll
      for (int q = 0; q < VW; ++q)
        if (row + q >= p.n) v[q] = 0;
    }
    *(gmem<V>*)(y + idx) = v;
  }
}

__global__ __launch_bounds__(RD_THREADS) void k_pass_reduce(const Prob* __restrict__ probs,
                                                            const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int64_t vbase = (int64_t)(blockIdx.x - tstart[pi]) * RD_THREADS * RD_VEC;
  if (p.prec == F64) reduce_body<double>(p, vbase);
  else reduce_body<float>(p, vbase);
}

// ---------------------------------------------------------------- tile counts and launchers
int tiles_pass(const Prob& p) {
  if (p.csr) return (p.n + 31) / 32;   // k_spmm: 32 rows per workgroup
  const int bm = (p.prec == F64) ? PASS_BM_D : PASS_BM_F;
  return ((p.n + bm - 1) / bm) * p.split;
}
int tiles_reduce(const Prob& p) {
  const int64_t vecs = (int64_t)p.rpad * p.ld * (p.prec == F64 ? 8 : 4) / 16;
  return (int)((vecs + RD_THREADS * RD_VEC - 1) / (RD_THREADS * RD_VEC));
}

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
      hipLaunchKernelGGL((k_pass_f32<N>), dim3(L.grid), dim3(PL_THREADS), 2 * pl_stage_bytes(N), L.stream, \
                         L.probs, L.tstart, L.nprob);                                                            \
    else                                                                                                         \
      hipLaunchKernelGGL((k_pass_b3<N, PB_VB>), dim3(L.grid), dim3(PASS_BM_F / (16 * PB_VB) * 64),               \
                         pb_kernel_lds(N), L.stream,                                                             \
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
  hipFuncSetAttribute((const void*)k_pass_f32<N>, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                      2 * pl_stage_bytes(N));                                                          \
  hipFuncSetAttribute((const void*)k_pass_b3<N, PB_VB>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                      pb_kernel_lds(N));
  PSD_NCB_EVEN(PSD_ATTR)
#undef PSD_ATTR
}

void launch_pass_reduce(const Launch& L) {
  hipLaunchKernelGGL(k_pass_reduce, dim3(L.grid), dim3(RD_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
