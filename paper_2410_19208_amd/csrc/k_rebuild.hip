// Rebuild of the projection (Alg. 2 line 3, Alg. 3 line 4):
//   P = Q V max(D,0) V^T Q^T = W W^T,  W = Q V_keep diag(sqrt(w)),  n x r_plus.
// The clamp leaves only the r_plus columns with positive weight (r_plus is data dependent and
// read on the device), so the contraction depth is r_plus, not r.
//
// One workgroup computes one 128 x 128 tile P_IJ with I >= J (lower triangle) on MFMA and
// writes both P_IJ and P_JI = P_IJ^T through a half-tile LDS stage (coalesced rows); the LDS
// footprint stays near 32 KB, so several workgroups share a CU and one's stores overlap
// another's MFMAs.  Diagonal tiles write their lower half and its mirror, so P is exactly
// symmetric.  W is row-major so each lane's MFMA operand is a contiguous run of one row.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int RB_THREADS = 256;

template <int PREC> struct RbCfg;
template <> struct RbCfg<F64> { typedef double T; typedef f64x4 Acc; static constexpr int KS = 4; };
template <> struct RbCfg<F32> { typedef float T; typedef f32x4 Acc; static constexpr int KS = 16; };
template <> struct RbCfg<B3> { typedef float T; typedef f32x4 Acc; static constexpr int KS = 32; };

// XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on
// XCD b mod 8, and each problem's tiles start at a multiple of 8), so XCD x runs tiles
// x, x+8, x+16, ...  The lower triangle of nb x nb tiles is cut into super-tiles of RB_SUPER x
// RB_SUPER tiles (lower triangle, row by row), super-tile s goes to XCD s mod 8, and each XCD
// runs its super-tiles' tiles in order: the W rows one super-tile touches (2 x RB_SUPER row
// blocks, under 2 MB) stay in that XCD's L2 while it works through them, instead of every
// XCD re-reading every block of W for every row of tiles.
// Used from RB_XCD_MIN row blocks on (W of a smaller problem fits in one L2 anyway, and the
// super-tiles would leave most XCDs idle); below, the tiles run row by row.
constexpr int RB_SUPER = 8;
constexpr int RB_XCD_MIN = 48;

// tiles of super-tile (SI, SJ), SJ <= SI, for nb row blocks
__host__ __device__ inline int rb_super_tiles(int SI, int SJ, int nb) {
  const int mi = min(RB_SUPER, nb - SI * RB_SUPER), mj = min(RB_SUPER, nb - SJ * RB_SUPER);
  return (SI == SJ) ? mi * (mi + 1) / 2 : mi * mj;
}

// number of tiles XCD x runs
__host__ __device__ inline int rb_xcd_tiles(int x, int nb) {
  const int ns = (nb + RB_SUPER - 1) / RB_SUPER;
  int cnt = 0, s = 0;
  for (int SI = 0; SI < ns; ++SI)
    for (int SJ = 0; SJ <= SI; ++SJ, ++s)
      if ((s & 7) == x) cnt += rb_super_tiles(SI, SJ, nb);
  return cnt;
}

// tile t of the launch -> (I, J), I >= J; false for padding
__device__ __forceinline__ bool tile_ij(int t, int nb, int& I, int& J) {
  if (nb < RB_XCD_MIN) {   // row by row: (0,0), (1,0), (1,1), (2,0), ...
    if (t >= nb * (nb + 1) / 2) return false;
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
    return true;
  }
  const int x = t & 7;
  int k = t >> 3;
  const int ns = (nb + RB_SUPER - 1) / RB_SUPER;
  int s = 0;
  for (int SI = 0; SI < ns; ++SI)
    for (int SJ = 0; SJ <= SI; ++SJ, ++s) {
      if ((s & 7) != x) continue;
      const int cnt = rb_super_tiles(SI, SJ, nb);
      if (k >= cnt) { k -= cnt; continue; }
      const int mj = min(RB_SUPER, nb - SJ * RB_SUPER);
      int i, j;
      if (SI == SJ) {   // lower triangle of the super-tile, row by row
        i = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= k) ++i;
        while (i * (i + 1) / 2 > k) --i;
        j = k - i * (i + 1) / 2;
      } else {
        i = k / mj;
        j = k - i * mj;
      }
      I = SI * RB_SUPER + i;
      J = SJ * RB_SUPER + j;
      return true;
    }
  return false;
}

template <int PREC>
__device__ void rebuild_tile(const Prob& p, int I, int J) {
  typedef typename RbCfg<PREC>::T T;
  typedef typename RbCfg<PREC>::Acc Acc;
  constexpr int TS = RB_TILE;                       // 128
  extern __shared__ __attribute__((aligned(1024))) unsigned char smem[];

  const int n = p.n;
  const int I0 = I * TS, J0 = J * TS;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int l16 = lane & 15, kg = lane >> 4;
  const int rplus = min(max(p.iscal[I_RPLUS], 0), p.rpad);
  const int kw = p.rwpad;
  const gmem<const bf16>* __restrict__ whi = gp((const bf16*)p.whi);
  const gmem<const bf16>* __restrict__ wlo = gp((const bf16*)p.wlo);
  Acc acc[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  // wave owns rows I0 + wave*32 + [0,32), all 128 columns
  const int ra0 = I0 + wave * 32 + l16;
  const int ra1 = ra0 + 16;
  constexpr int KS = RbCfg<PREC>::KS;
  if constexpr (PREC == F64) {
    const gmem<const double>* W = gp((const double*)p.wf);
    for (int k0 = 0; k0 < rplus; k0 += KS) {
      const int kk = k0 + kg;
      const double a0 = W[(int64_t)ra0 * kw + kk];
      const double a1 = W[(int64_t)ra1 * kw + kk];
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const double b = W[(int64_t)(J0 + cb * 16 + l16) * kw + kk];
        acc[0][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][cb], 0, 0, 0);
        acc[1][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][cb], 0, 0, 0);
      }
    }
  } else {
    // The K-slice of W_J (rows J0 .. J0+127, 64 bytes of K each: 32 bf16 or 16 floats) is
    // shared by the four waves: it goes global -> LDS by direct loads into a two-slice ring
    // (block cb holds rows 16cb .. 16cb+15 at 64 bytes each, 16-byte slot s of row j holding
    // chunk s ^ ((j % 16) / 4), so each 16-lane read hits 16 distinct bank groups; BF16X3
    // keeps hi in blocks 0..7 and lo in 8..15).  Each wave's own rows of W_I are prefetched
    // into registers one slice ahead.
    constexpr int NBLK = (PREC == B3) ? 16 : 8;
    constexpr int SLICE = NBLK * 1024;
    const int nks = (rplus + KS - 1) / KS;
    const gmem<const float>* Wf = gp((const float*)p.wf);
    auto issue = [&](int ks) {
      unsigned char* dst = smem + (ks & 1) * SLICE;
      const int k0 = ks * KS;
      const int j = lane >> 2, c = (lane & 3) ^ (j >> 2);
#pragma unroll
      for (int u = 0; u < NBLK / 4; ++u) {
        const int b = wave + 4 * u;
        const int cb = b & 7;
        const int64_t row = J0 + cb * 16 + j;
        if constexpr (PREC == B3) dma16((const void*)(((b < 8) ? whi : wlo) + row * kw + k0 + 8 * c), dst + b * 1024);
        else dma16((const void*)(Wf + row * kw + k0 + 4 * c), dst + b * 1024);
      }
    };
    typedef typename std::conditional<PREC == B3, bf16x8, f32x4>::type Frag;
    Frag an[4];   // B3: hi rows ra0, ra1 then lo rows ra0, ra1; F32: rows ra0, ra1
    auto load_a = [&](int ks) {
      const int k0 = ks * KS;
      if constexpr (PREC == B3) {
        const int kk = k0 + kg * 8;
        an[0] = *(const gmem<bf16x8>*)(whi + (int64_t)ra0 * kw + kk);
        an[1] = *(const gmem<bf16x8>*)(whi + (int64_t)ra1 * kw + kk);
        an[2] = *(const gmem<bf16x8>*)(wlo + (int64_t)ra0 * kw + kk);
        an[3] = *(const gmem<bf16x8>*)(wlo + (int64_t)ra1 * kw + kk);
      } else {
        const int kk = k0 + kg * 4;
        an[0] = *(const gmem<f32x4>*)(Wf + (int64_t)ra0 * kw + kk);
        an[1] = *(const gmem<f32x4>*)(Wf + (int64_t)ra1 * kw + kk);
      }
    };
    if (nks > 0) {
      issue(0);
      load_a(0);
    }
    const int boff = l16 * 64 + ((kg ^ (l16 >> 2)) << 4);
    for (int ks = 0; ks < nks; ++ks) {
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's slice loads and A rows
      lds_barrier();                        // everyone's slice; reads of the other slice done
      Frag a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = an[q];
      if (ks + 1 < nks) {
        issue(ks + 1);
        load_a(ks + 1);
      }
      const unsigned char* sl = smem + (ks & 1) * SLICE;
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        if constexpr (PREC == B3) {
          const bf16x8 bhi = *(const bf16x8*)(sl + cb * 1024 + boff);
          const bf16x8 blo = *(const bf16x8*)(sl + (8 + cb) * 1024 + boff);
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], bhi, acc[r][cb], 0, 0, 0);
            acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], blo, acc[r][cb], 0, 0, 0);
            acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2 + r], bhi, acc[r][cb], 0, 0, 0);
          }
        } else {
          const f32x4 b = *(const f32x4*)(sl + cb * 1024 + boff);
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][e], b[e], acc[r][cb], 0, 0, 0);
        }
      }
    }
  }
  // Store through LDS in two halves of 64 rows (the waves 2h, 2h+1 own half h), so the LDS
  // never holds more than the W_J ring or a half tile and three workgroups share a CU: one's
  // stores overlap another's MFMAs.  Half h of P_IJ goes out as whole 512-byte rows, its
  // transpose as 256-byte row pieces of P_JI.  Diagonal tiles write element (i, j) with
  // i >= j to P_II and, for i > j, to its mirror, so P is exactly symmetric.
  constexpr int LDT = TS + 1;
  T* half = (T*)smem;                               // [64][LDT]
  gmem<T>* P = gp((T*)p.P);
  const int64_t ldp = p.ldp;
  const bool diag = (I == J);
  if constexpr (PREC != F64) lds_barrier();         // every wave is done with the W_J ring
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if ((wave >> 1) == h) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            half[((wave & 1) * 32 + a * 16 + acc_row<PREC == F64>(kg, v)) * LDT + cb * 16 + l16] = (T)acc[a][cb][v];
    }
    lds_barrier();
    const int R0 = I0 + 64 * h;                     // first row of P_IJ in this half
    // P_IJ rows R0 .. R0+63: thread e covers 4 consecutive columns of one row
#pragma unroll 2
    for (int e = threadIdx.x; e < 64 * TS / 4; e += RB_THREADS) {
      const int i = e / (TS / 4), c = 4 * (e % (TS / 4));
      if (R0 + i >= n) continue;
      const T* src = half + i * LDT + c;
      if (!diag && J0 + c + 3 < n && sizeof(T) == 4) {
        __builtin_nontemporal_store(f32x4{(float)src[0], (float)src[1], (float)src[2], (float)src[3]},
                                    (gmem<f32x4>*)(P + (int64_t)(R0 + i) * ldp + J0 + c));
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (J0 + c + q < n && (!diag || 64 * h + i >= c + q)) P[(int64_t)(R0 + i) * ldp + J0 + c + q] = src[q];
      }
    }
    // P_JI: row J0 + j, columns R0 .. R0+63; thread e covers 4 consecutive columns
#pragma unroll 2
    for (int e = threadIdx.x; e < 64 * TS / 4; e += RB_THREADS) {
      const int j = e / 16, i = 4 * (e % 16);
      if (J0 + j >= n) continue;
      const T x[4] = {half[i * LDT + j], half[(i + 1) * LDT + j], half[(i + 2) * LDT + j], half[(i + 3) * LDT + j]};
      if (!diag && R0 + i + 3 < n && sizeof(T) == 4) {
        __builtin_nontemporal_store(f32x4{(float)x[0], (float)x[1], (float)x[2], (float)x[3]},
                                    (gmem<f32x4>*)(P + (int64_t)(J0 + j) * ldp + R0 + i));
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (R0 + i + q < n && (!diag || 64 * h + i + q > j)) P[(int64_t)(J0 + j) * ldp + R0 + i + q] = x[q];
      }
    }
    if (h == 0) lds_barrier();                      // the second half overwrites the first
  }
}

template <int PREC>
__global__ __launch_bounds__(RB_THREADS) void k_rebuild(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                        int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  const int G = tstart[pi + 1] - tstart[pi];   // this problem's workgroups, a multiple of 8
  const int nb = (p.n + RB_TILE - 1) / RB_TILE;
  for (int u = t; u < p.rb_tiles; u += G) {
    int I, J;
    if (!tile_ij(u, nb, I, J)) continue;
    rebuild_tile<PREC>(p, I, J);
    if (u + G < p.rb_tiles) lds_barrier();     // the next tile rewrites the LDS stage
  }
}

// A multiple of 8, so the next problem's tiles start on XCD 0: the lower tiles rounded up, or
// for the XCD order 8 x the longest XCD tile list.
int rebuild_tile_count(const Prob& p) {
  const int nb = (p.n + RB_TILE - 1) / RB_TILE;
  if (nb < RB_XCD_MIN) return (nb * (nb + 1) / 2 + 7) / 8 * 8;
  int mx = 0;
  for (int x = 0; x < 8; ++x) mx = std::max(mx, rb_xcd_tiles(x, nb));
  return 8 * mx;
}
int tiles_rebuild(const Prob& p) {
  const int per_xcd = rebuild_tile_count(p) / 8;
  return 8 * ((per_xcd + RB_PER_WG - 1) / RB_PER_WG);
}

// Dynamic LDS: the two-slice W_J ring, or later the half-tile stage (the larger of the two).
static constexpr int rb_lds(int prec) {
  return prec == F64 ? 64 * (RB_TILE + 1) * 8
                     : (64 * (RB_TILE + 1) * 4 > 2 * 16 * 1024 ? 64 * (RB_TILE + 1) * 4 : 2 * 16 * 1024);
}

void launch_rebuild(const Launch& L, int prec) {
  if (prec == F64)
    hipLaunchKernelGGL(k_rebuild<F64>, dim3(L.grid), dim3(RB_THREADS), rb_lds(F64), L.stream, L.probs, L.tstart,
                       L.nprob);
  else if (prec == F32)
    hipLaunchKernelGGL(k_rebuild<F32>, dim3(L.grid), dim3(RB_THREADS), rb_lds(F32), L.stream, L.probs, L.tstart,
                       L.nprob);
  else
    hipLaunchKernelGGL(k_rebuild<B3>, dim3(L.grid), dim3(RB_THREADS), rb_lds(B3), L.stream, L.probs, L.tstart,
                       L.nprob);
}

// Opt the FP64 rebuild (a 66 KB half-tile stage) into more than 64 KB of dynamic LDS.
void rebuild_init() {
  hipFuncSetAttribute((const void*)k_rebuild<F64>, hipFuncAttributeMaxDynamicSharedMemorySize, rb_lds(F64));
}

}  // namespace psd
