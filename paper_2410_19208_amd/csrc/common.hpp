// Internal types shared by the HIP kernels and the host runtime of libpsdproj.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "psdproj.h"

namespace psd {

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(2))) double f64x2;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

enum Prec : int { F64 = 0, F32 = 1, B3 = 2 };

// Global-memory pointers.  Pointers read from the problem descriptor are generic, so accesses
// through them compile to FLAT instructions, which also count against the LDS wait counter:
// every wait for an LDS read would then wait for all global loads and stores in flight.
// Kernels convert descriptor pointers with gp() so that they use global instructions.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ gmem<T>* gp(T* ptr) { return (gmem<T>*)ptr; }

// Tiling constants.  The pass kernels use 16x16 MFMA tiles; a wave owns RB row blocks of 16
// rows and every column block of the panel.
constexpr int WAVE = 64;
constexpr int PASS_THREADS = 256;             // FP64 pass: 4 waves
constexpr int PASS_BM_F = 256;                // rows per tile, FP32 / BF16X3 (8 waves)
constexpr int PASS_BM_D = 64;                 // rows per tile, FP64 (16 per wave)
constexpr int PASS_BK_F = 64;                 // K chunk granularity, FP32 / BF16X3
constexpr int PASS_BK_D = 32;                 // K per LDS stage, FP64
constexpr int PANEL_TAIL = 32;                // zero rows past n in every panel: a pass step of K
                                              // rows that starts before n stays inside the column
constexpr int RPAD = 32;                      // panel column padding multiple
constexpr int GRAM_TILE = 32;                 // Gram output tile
constexpr int GRAM_CHUNK = 1024;              // rows per Gram partial
constexpr int RB_TILE = 128;                  // rebuild output tile (P)
constexpr int APPLY_ROWS = 64;                // rows per apply/formw tile
constexpr int GEMV_TILE = 256;                // GEMV tile edge (upper-triangle tiles of A)
constexpr int MAX_SPLIT = 16;               // pass split-K factors 1 .. MAX_SPLIT
// Tiles per workgroup of the streaming GEMV and rebuild kernels: a workgroup loops over its
// problem's tiles with the stride of the problem's workgroup count (a multiple of 8 for the
// rebuild, so every tile keeps its XCD), amortising launch, prologue and epilogue.
constexpr int GV_PER_WG = 1;
constexpr int RB_PER_WG = 1;
constexpr int NSCAL = 16;
constexpr int NISCAL = 16;
// Alg. 5 with N <= PAIRED_MAX runs its two power iterations over one stream of two-vector
// products (the second run's iterates are rebuilt from a shifted Krylov basis); larger N
// runs them one after the other.
constexpr int PAIRED_MAX = 32;

// scal[] slots
enum { S_ALPHA = 0, S_SIGMA1 = 1, S_SIGMA2 = 2, S_NRM = 3, S_INV = 4, S_SHIFT = 5, S_TNORM = 6,
       S_THRESH = 7, S_GL = 8, S_GU = 9, S_PIVMIN = 10, S_INVB = 11, S_MU = 12, S_MU0 = 13 };
// iscal[] slots
enum { I_STATUS = 0, I_RPLUS = 1, I_NU = 2, I_COUNTER = 3, I_NEWTON = 4, I_NDROP = 5, I_PP = 6, I_WELL = 7 };

// Stage argument of the CholeskyQR2 kernels (Gram, its reduce, Cholesky, apply): the round
// (0 or 1) in the low 4 bits, and 16 (o + 1) with o the step's position in the problem's
// sequence of 1 + 2q orthonormalisations (0 when unknown).  Every step but the last only
// needs the range of its input: when the first round's Cholesky finds the input well
// conditioned (I_WELL), its Q = Y R^-1 is already orthonormal to far better than the pass
// precision and the second round is skipped.  The last step always runs both rounds.
constexpr int ORTH_ROUND_MASK = 15;

// Per-problem descriptor, resident in device memory (workspace header).
struct Prob {
  int32_t n, r, rpad, ld;          // order, sketch width, padded width, panel leading dim
  int32_t k, q, variant, prec;
  int32_t split, kchunk;           // pass split-K factor and chunk length
  int32_t ngchunk, alpha_iters;    // Gram row chunks, N of Alg. 4/5
  int32_t alpha_mode, rwpad;       // 0: alpha given (or plain), 1: estimate; rebuild-factor row stride
  int32_t npass_tiles, avec;       // avec: rows of A start and end 16-byte aligned (vector loads)
  int32_t ktail, sketch;           // BF16X3 16-byte path: K rows ktail .. n-1 (n mod 32 of them)
                                   // are added by the pass reduction, not the pass (else n);
                                   // sketch: 0 Gaussian test matrix, 1 structured (+-1 Hadamard)
  int32_t gv_tiles, rb_tiles;       // tiles of the GEMV (Alg. 4 product) and of the rebuild
  int32_t srht_m, csr;             // structured sketch: transform size 2^srht_m >= n; csr: A is
                                   // sparse (CSR, both triangles), A points to its values
  int32_t paired, pad0;            // Alg. 5's two runs share one stream of products (N <= PAIRED_MAX)
  const int32_t* rowptr;           // CSR row starts (n + 1) and column indices
  const int32_t* colidx;
  void* zr;                        // CSR passes: the pass operand row-major (n x rpad)
  uint64_t seed;
  double alpha_in;
  const void* A; int64_t lda;
  void* P; int64_t ldp;
  // workspace pointers
  void* zm; bf16* zhi; bf16* zlo;  // pass operand: master (double/float) and BF16 split (tiled)
  void* y;                         // reduced pass output
  void* part;                      // split-K partials
  void* q1;                        // first-round CholQR panel
  void* wf; bf16* whi; bf16* wlo;  // rebuild factor, row-major n x rwpad
  double* gpart;                   // Gram partials ngchunk x rpad x rpad
  double* G; double* F; double* C; double* H; double* V;  // rpad x rpad, column-major
  double* evals; double* tau; double* td; double* te; double* wts; double* xt;  // eig scratch
  double* vec;                     // power vectors: 2 x ld
  double* vpart;                   // GEMV: sum of squares per block row (2 x nb when paired)
  double* gvp;                     // GEMV tile partials: nb x nb x GEMV_TILE (twice when paired)
  double* bh;                      // paired Alg. 5: Krylov basis b_0 .. b_{N+1}, (N + 2) x ld
  double* pw;                      // paired Alg. 5: rho_0 .. rho_{N+1}, then mu_0 .. mu_{N+1}
  double* scal;                    // NSCAL doubles
  int32_t* iscal;                  // NISCAL ints
  int32_t* drop;                   // rpad flags
  psdproj_result* res;
};

// Element (row i, column j) of the BF16 split copies of the pass operand (ld rows x rpad
// columns).  They are stored in 1 KB tiles of 32 rows x 16 columns, tile (i/32, j/16) at
// (j/16 * ld/32 + i/32) x 512 elements, and inside a tile chunk-major: rows 8c .. 8c+7 of
// column jj (one 16-byte chunk) at 128 c + 8 jj.  One K step of the pass then loads each
// column block as one contiguous 1 KB piece, straight into the LDS order its MFMA operand
// reads take without bank conflicts.
__host__ __device__ __forceinline__ int64_t zsplit_index(int i, int j, int ld) {
  return ((int64_t)(j >> 4) * (ld >> 5) + (i >> 5)) * 512 + ((i >> 3) & 3) * 128 + (j & 15) * 8 + (i & 7);
}

__device__ __forceinline__ bool orth_single(const Prob& p, int arg) {
  const int o = (arg >> 4) - 1;
  return o >= 0 && o < 2 * p.q && p.iscal[I_WELL] != 0;
}


// Row (within a 16x16 output block) of accumulator slot v held by a lane of group kg = lane/16:
// the FP32/BF16 16x16 MFMAs hold rows 4*kg + v, the FP64 16x16x4 MFMA holds rows 4*v + kg.
template <bool FP64_MFMA>
__device__ __forceinline__ int acc_row(int kg, int v) { return FP64_MFMA ? 4 * v + kg : 4 * kg + v; }

__device__ __forceinline__ int find_prob(const int* __restrict__ tstart, int nprob, int b) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tstart[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void set_status(const Prob& p, int st) {
  // First error wins; integer atomic (status is not floating point).
  atomicCAS(&p.iscal[I_STATUS], 0, st);
}

// Wave index within the workgroup as a wave-uniform (scalar) value, so that branches and
// addresses derived from it stay scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

typedef __attribute__((address_space(3))) void lds_void;

// Raw buffer resources (stride 0): an access at or past num_records bytes reads zero and writes
// nothing.  Fourth descriptor word of the gfx9 family (32-bit data format), and the cache-policy
// bit that marks a buffer access non-temporal.
constexpr int BUF_WORD3 = 0x00020000;
constexpr int BUF_NT = 2;

// 16 bytes per lane from global memory into LDS at dst + 16 * lane (dst wave-uniform), without
// a VGPR round trip (global_load_lds_dwordx4); complete after this wave's vmcnt reaches 0.
__device__ __forceinline__ void dma16(const void* g, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds(g, (lds_void*)dst, 16, 0, 0);
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits for every
// outstanding global load and store of the wave (a round trip to L2 after a store); loops whose
// waves exchange data through LDS alone use this one.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders this wave's LDS accesses across its lanes (no other wave involved).
__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps (x finite, nonzero,
// normal); within an ulp or two of the IEEE quotient, with a short dependent chain.
__device__ __forceinline__ double rcp_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}

// Value of v in lane `src` (a constant or wave-uniform index), as a wave-uniform double.
__device__ __forceinline__ double bcast_f64(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Cross-lane move of a double by a DPP pattern (two 32-bit DPP moves).  Lanes whose row is
// masked out by ROWMASK, or whose source lane is invalid, receive 0.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
// The same for patterns where every lane has a valid source lane (quad permutations, row
// rotations): no old value to preserve, so no register initialisation before the moves.
template <int CTRL>
__device__ __forceinline__ double dpp_perm_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROR4 = 0x124;     // row_ror:4 (within 16-lane rows)
constexpr int DPP_ROR8 = 0x128;     // row_ror:8 (= lane ^ 8 within a row)
constexpr int DPP_BCAST15 = 0x142;  // row_bcast:15 (lane 15 of each row to the next row)
constexpr int DPP_BCAST31 = 0x143;  // row_bcast:31 (lane 31 to rows 2 and 3)

// Sum of a double over the wave with DPP moves (no LDS traffic), returned wave-uniform.  The
// addition order is fixed: quad sums, row sums (rotations by 4 and 8), then rows 0+1 and 2+3,
// then (0+1)+(2+3), read from lane 63.
__device__ __forceinline__ double wave_allsum(double v) {
  v += dpp_f64<DPP_XOR1>(v);
  v += dpp_f64<DPP_XOR2>(v);
  v += dpp_f64<DPP_ROR4>(v);
  v += dpp_f64<DPP_ROR8>(v);
  v += dpp_f64<DPP_BCAST15, 0xA>(v);
  v += dpp_f64<DPP_BCAST31, 0xC>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Tile t of the upper triangle of an nb x nb grid of 16x16 tiles, enumerated row by row:
// (0,0), (0,1), ..., (0,nb-1), (1,1), ...
__device__ __forceinline__ void upper_tile(int t, int nb, int& I, int& J) {
  int i = 0, rem = t;
  while (rem >= nb - i) { rem -= nb - i; ++i; }
  I = i;
  J = i + rem;
}

// Number of eigenvalues of T below x (Sturm sequence).
template <typename PD>
__device__ __forceinline__ int sturm_count(PD d, PD e2, int r, double x, double pivmin) {
  double q = d[0] - x;
  int c = q < 0.0;
  for (int i = 1; i < r; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d[i] - x) - e2[i - 1] / q;
    c += q < 0.0;
  }
  return c;
}

}  // namespace psd
