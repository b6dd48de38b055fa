// Passes over a sparse A (CSR, both triangles of the symmetric matrix): Y = A Z for the sketch,
// the power steps and the compression of Alg. 1-3 when A is given as a sparse matrix (the paper's
// benchmark matrices are sparse, Sec. 4).  The dense passes stream every element of A; here the
// work is one row of Z per stored nonzero.
//   k_zt:   Z (column-major, ld) -> Zr (row-major, n x rpad), 64 x 64 tiles through LDS, so that
//           the sparse product reads each needed row of Z as one contiguous piece;
//   k_spmm: one workgroup per 32 rows of A; a wave takes one row at a time, its 64 lanes holding
//           4 columns of the panel each, and adds a_ij Zr[j, :] over the row's nonzeros in storage
//           order (FP64 for FP64 storage, FP32 otherwise: the split-BF16 products are not used for
//           a sparse A); the 32 x rpad result goes through LDS to the column-major partial
//           panel, which k_pass_reduce turns into Y (and the scaled operator).
// Column indices outside [0, n) and nonzero positions outside [0, nnz) are never followed; the
// first such index sets E_INVALID in the problem's status.  nnz travels in the descriptor's lda.
#include "common.hpp"
#include "launch.hpp"

namespace psd {

constexpr int ZT_TILE = 64;
constexpr int SP_ROWS = 32;
constexpr int SP_THREADS = 256;

template <typename T>
__device__ __forceinline__ void zt_tile(const Prob& p, int t) {
  __shared__ T tile[ZT_TILE][ZT_TILE + 1];
  const int nrb = (p.n + ZT_TILE - 1) / ZT_TILE;
  const int rb = t % nrb, cb = t / nrb;
  const int r0 = rb * ZT_TILE, c0 = cb * ZT_TILE;
  const gmem<const T>* z = gp((const T*)p.zm);
  gmem<T>* zr = gp((T*)p.zr);
  for (int e = threadIdx.x; e < ZT_TILE * ZT_TILE; e += SP_THREADS) {
    const int c = e / ZT_TILE, r = e % ZT_TILE;   // consecutive threads: consecutive rows of a column
    tile[c][r] = (r0 + r < p.n && c0 + c < p.rpad) ? z[(int64_t)(c0 + c) * p.ld + r0 + r] : (T)0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ZT_TILE * ZT_TILE; e += SP_THREADS) {
    const int r = e / ZT_TILE, c = e % ZT_TILE;   // consecutive threads: consecutive columns of a row
    if (r0 + r < p.n && c0 + c < p.rpad) zr[(int64_t)(r0 + r) * p.rpad + c0 + c] = tile[c][r];
  }
}

__global__ __launch_bounds__(SP_THREADS) void k_zt(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                   int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (p.prec == F64) zt_tile<double>(p, t);
  else zt_tile<float>(p, t);
}

template <typename T>
__device__ __forceinline__ void spmm_block(const Prob& p, int t, unsigned char* smem) {
  typedef T V4 __attribute__((ext_vector_type(4)));
  T* out = (T*)smem;   // [SP_ROWS][rpad]
  const int n = p.n, rpad = p.rpad;
  const int64_t nnz = p.lda;
  const int i0 = t * SP_ROWS;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const gmem<const int32_t>* rowptr = gp(p.rowptr);
  const gmem<const int32_t>* colidx = gp(p.colidx);
  const gmem<const T>* vals = gp((const T*)p.A);
  const gmem<const T>* zr = gp((const T*)p.zr);
  const int c = 4 * lane;   // this lane's 4 columns
  bool bad = false;
  for (int rr = wave; rr < SP_ROWS; rr += SP_THREADS / WAVE) {
    const int i = i0 + rr;
    V4 acc = {0, 0, 0, 0};
    if (i < n) {
      const int64_t k0 = max((int64_t)rowptr[i], (int64_t)0), k1 = min((int64_t)rowptr[i + 1], nnz);
      for (int64_t k = k0; k < k1; ++k) {
        const int j = colidx[k];
        if ((unsigned)j >= (unsigned)n) { bad = true; continue; }
        const T a = vals[k];
        if (c < rpad) acc += a * *(const gmem<V4>*)(zr + (int64_t)j * rpad + c);
      }
    }
    if (c < rpad) *(V4*)(out + rr * rpad + c) = acc;
  }
  if (bad) set_status(p, PSDPROJ_E_INVALID);
  __syncthreads();
  // column-major partial panel: column col, rows i0 .. i0 + 31 (zero past n)
  gmem<T>* part = gp((T*)p.part);
  for (int e = threadIdx.x; e < SP_ROWS * rpad; e += SP_THREADS) {
    const int col = e / SP_ROWS, r = e % SP_ROWS;
    if (i0 + r < p.ld) part[(int64_t)col * p.ld + i0 + r] = out[r * rpad + col];
  }
}

__global__ __launch_bounds__(SP_THREADS) void k_spmm(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int t = blockIdx.x - tstart[pi];
  if (p.prec == F64) spmm_block<double>(p, t, smem);
  else spmm_block<float>(p, t, smem);
}

int tiles_zt(const Prob& p) {
  return ((p.n + ZT_TILE - 1) / ZT_TILE) * ((p.rpad + ZT_TILE - 1) / ZT_TILE);
}

void launch_zt(const Launch& L) {
  hipLaunchKernelGGL(k_zt, dim3(L.grid), dim3(SP_THREADS), 0, L.stream, L.probs, L.tstart, L.nprob);
}

void launch_spmm(const Launch& L) {
  // LDS: SP_ROWS rows of the widest panel in the launch, in the widest element (double)
  const size_t lds = (size_t)SP_ROWS * (size_t)L.maxnb * 16 * sizeof(double);
  hipLaunchKernelGGL(k_spmm, dim3(L.grid), dim3(SP_THREADS), lds, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
