// Rebuild of the projection (Alg. 2 line 3, Alg. 3 line 4):
//   P = Q V max(D,0) V^T Q^T = W W^T,  W = Q V_keep diag(sqrt(w)),  n x r_plus.
// The clamp leaves only the r_plus columns with positive weight (r_plus is data dependent and
// read on the device), so the contraction depth is r_plus, not r.
//
// One workgroup computes one 128 x 128 tile P_IJ with I >= J (lower triangle) on MFMA, stages
// it in LDS, and writes both P_IJ and P_JI = P_IJ^T with row-contiguous stores; diagonal
// tiles take element (a, b) from max/min so P is exactly symmetric.  W is row-major so each
// lane's MFMA operand is a contiguous run of one row.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int RB_THREADS = 256;

template <int PREC> struct RbCfg;
template <> struct RbCfg<F64> { typedef double T; typedef f64x4 Acc; static constexpr int KS = 4; };
template <> struct RbCfg<F32> { typedef float T; typedef f32x4 Acc; static constexpr int KS = 16; };
template <> struct RbCfg<B3> { typedef float T; typedef f32x4 Acc; static constexpr int KS = 32; };

__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  // t enumerates lower tiles row by row: (0,0), (1,0), (1,1), (2,0), ...
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

template <int PREC>
__device__ void rebuild_tile(const Prob& p, int t) {
  typedef typename RbCfg<PREC>::T T;
  typedef typename RbCfg<PREC>::Acc Acc;
  constexpr int TS = RB_TILE;                       // 128
  constexpr int LDT = TS + 1;
  extern __shared__ __attribute__((aligned(1024))) unsigned char smem[];
  T* tile = (T*)smem;                               // [TS][LDT]

  int I, J;
  tile_ij(t, I, J);
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
    // into registers one slice ahead.  The staging tile below reuses the same LDS.
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
    lds_barrier();   // the staging tile overwrites the ring
  }
  // stage: lane holds rows acc_row(kg, v) of 16-row block a, column cb*16 + l16
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        tile[(wave * 32 + a * 16 + acc_row<PREC == F64>(kg, v)) * LDT + cb * 16 + l16] = (T)acc[a][cb][v];
  __syncthreads();
  gmem<T>* P = gp((T*)p.P);
  const int64_t ldp = p.ldp;
  if (I == J) {
    for (int e = threadIdx.x; e < TS * TS; e += RB_THREADS) {
      const int a = e / TS, b = e - a * TS;
      if (I0 + a < n && J0 + b < n) {
        const T v = (a >= b) ? tile[a * LDT + b] : tile[b * LDT + a];
        P[(int64_t)(I0 + a) * ldp + J0 + b] = v;
      }
    }
  } else {
    for (int e = threadIdx.x; e < TS * TS; e += RB_THREADS) {
      const int a = e / TS, b = e - a * TS;
      if (I0 + a < n && J0 + b < n) P[(int64_t)(I0 + a) * ldp + J0 + b] = tile[a * LDT + b];
      if (J0 + a < n && I0 + b < n) P[(int64_t)(J0 + a) * ldp + I0 + b] = tile[b * LDT + a];
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(RB_THREADS) void k_rebuild(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                        int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  const int nb = (p.n + RB_TILE - 1) / RB_TILE;
  if (t >= nb * (nb + 1) / 2) return;
  rebuild_tile<PREC>(p, t);
}

int tiles_rebuild(const Prob& p) {
  const int nb = (p.n + RB_TILE - 1) / RB_TILE;
  return nb * (nb + 1) / 2;
}

void launch_rebuild(const Launch& L, int prec) {
  if (prec == F64) {
    const size_t sh = (size_t)RB_TILE * (RB_TILE + 1) * sizeof(double);
    hipLaunchKernelGGL(k_rebuild<F64>, dim3(L.grid), dim3(RB_THREADS), sh, L.stream, L.probs, L.tstart, L.nprob);
  } else if (prec == F32) {
    const size_t sh = (size_t)RB_TILE * (RB_TILE + 1) * sizeof(float);
    hipLaunchKernelGGL(k_rebuild<F32>, dim3(L.grid), dim3(RB_THREADS), sh, L.stream, L.probs, L.tstart, L.nprob);
  } else {
    const size_t sh = (size_t)RB_TILE * (RB_TILE + 1) * sizeof(float);
    hipLaunchKernelGGL(k_rebuild<B3>, dim3(L.grid), dim3(RB_THREADS), sh, L.stream, L.probs, L.tstart, L.nprob);
  }
}

// Opt the FP64 rebuild into more than 64 KB of dynamic LDS.
void rebuild_init() {
  hipFuncSetAttribute((const void*)k_rebuild<F64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      RB_TILE * (RB_TILE + 1) * (int)sizeof(double));
  hipFuncSetAttribute((const void*)k_rebuild<F32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      RB_TILE * (RB_TILE + 1) * (int)sizeof(float));
  hipFuncSetAttribute((const void*)k_rebuild<B3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      RB_TILE * (RB_TILE + 1) * (int)sizeof(float));
}

}  // namespace psd
