// Kernels of the exact projection X_+ = U max(D, 0) U^T (Thm 1) computed through the matrix sign
// function, X_+ = (X + X sign(X)) / 2 (the polar form (X + |X|)/2 with |X| = X sign(X)):
//   k_gemm64:      C = alpha A B + beta D, n x n, FP64 on v_mfma_f64_16x16x4f64 (128 x 128 tiles,
//                  4 waves of 64 x 64, K stages of 16 through two LDS buffers);
//   k_ex_sumsq / k_ex_finish: ||X||_F in FP64, fixed order;
//   k_ex_scale:    S = X / ||X||_F (FP64 copy), and X itself in FP64;
//   k_ex_poly:     W = 3 I - a^2 W, in place;
//   k_ex_final:    P = (Q + Q^T) / 2 in the storage precision (Q = (X + X S) / 2), exactly
//                  symmetric; k_ex_trace: Tr(S) for the count of positive eigenvalues.
#include <atomic>

#include "common.hpp"
#include "exact_kernels.hpp"

namespace psd {

constexpr int GM_T = 256;      // threads per GEMM workgroup (4 waves)
constexpr int GM_B = 128;      // output tile edge; each wave computes 64 x 64
constexpr int GM_K = 16;       // K per LDS stage
constexpr int GM_PAD = 2;      // doubles of padding per LDS row
constexpr int GM_LD = GM_B + GM_PAD;

// A, B, C, D column-major with leading dimensions; element (i, j) of A at A[j * lda + i].
// Tile 128 x 128 per workgroup, 4 waves of 64 x 64 (4 x 4 blocks of v_mfma_f64_16x16x4f64).  The
// A and B slices of a K stage (16 columns of A's 128 rows, 16 rows of B's 128 columns) go
// through two LDS buffers: the next stage's global loads are issued into registers before the
// current stage's products and stored to the other buffer after them, one barrier per stage.
// Interior stages with even leading dimensions load 16 bytes per thread and access; other stages
// load element by element with zeros outside n x n.
__global__ __launch_bounds__(GM_T, 2) void k_gemm64(int n, const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                                    int64_t ldc, double alpha, const double* __restrict__ D,
                                                    int64_t ldd, double beta) {
  extern __shared__ __attribute__((aligned(16))) double gsm[];
  double* sA = gsm;                       // [2][GM_K][GM_LD]: sA[b][k][i] = A(i0 + i, k0 + k)
  double* sB = gsm + 2 * GM_K * GM_LD;    // [2][GM_K][GM_LD]: sB[b][k][j] = B(k0 + k, j0 + j)
  const int i0 = blockIdx.x * GM_B, j0 = blockIdx.y * GM_B;
  const int tid = threadIdx.x, wave = wave_id(), lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1, li = lane & 15, kg = lane >> 4;
  const gmem<const double>* Ag = gp(A);
  const gmem<const double>* Bg = gp(B);
  const bool vec = ((lda | ldb) & 1) == 0;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0, 0, 0, 0};

  // thread's share of a stage: 4 pairs of A (rows 2 ia, 2 ia + 1 of column ka) and 4 pairs of B
  // (rows 2 kb, 2 kb + 1 of column jb)
  f64x2 ra[4], rb[4];
  auto load = [&](int k0) {
    const bool inner = vec && i0 + GM_B <= n && j0 + GM_B <= n && k0 + GM_K <= n;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + GM_T * u;
      const int ka = e >> 6, ia = e & 63;          // A: 64 pairs of rows per column
      const int jb = e >> 3, kb = e & 7;           // B: 8 pairs of rows per column
      const int gi = i0 + 2 * ia, gka = k0 + ka;
      const int gj = j0 + jb, gkb = k0 + 2 * kb;
      if (inner) {
        ra[u] = *(const gmem<f64x2>*)(Ag + (int64_t)gka * lda + gi);
        rb[u] = *(const gmem<f64x2>*)(Bg + (int64_t)gj * ldb + gkb);
      } else {
        ra[u][0] = (gi < n && gka < n) ? Ag[(int64_t)gka * lda + gi] : 0.0;
        ra[u][1] = (gi + 1 < n && gka < n) ? Ag[(int64_t)gka * lda + gi + 1] : 0.0;
        rb[u][0] = (gj < n && gkb < n) ? Bg[(int64_t)gj * ldb + gkb] : 0.0;
        rb[u][1] = (gj < n && gkb + 1 < n) ? Bg[(int64_t)gj * ldb + gkb + 1] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
    double* a = sA + buf * GM_K * GM_LD;
    double* b = sB + buf * GM_K * GM_LD;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + GM_T * u;
      const int ka = e >> 6, ia = e & 63;
      const int jb = e >> 3, kb = e & 7;
      *(f64x2*)(a + ka * GM_LD + 2 * ia) = ra[u];
      b[(2 * kb) * GM_LD + jb] = rb[u][0];
      b[(2 * kb + 1) * GM_LD + jb] = rb[u][1];
    }
  };

  const int nst = (n + GM_K - 1) / GM_K;
  load(0);
  store(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) load((st + 1) * GM_K);
    const double* a = sA + cur * GM_K * GM_LD;
    const double* b = sB + cur * GM_K * GM_LD;
#pragma unroll
    for (int kk = 0; kk < GM_K; kk += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = a[(kk + kg) * GM_LD + 64 * wr + 16 * t + li];
        bv[t] = b[(kk + kg) * GM_LD + 64 * wc + 16 * t + li];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    if (st + 1 < nst) store(cur ^ 1);   // the other buffer: its last readers passed the previous barrier
    __syncthreads();
  }
  // lane (li, kg) of acc[x][y] holds rows acc_row<true>(kg, v) of block (x, y), column li
  gmem<double>* Cg = gp(C);
  const gmem<const double>* Dg = gp(D);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gj = j0 + 64 * wc + 16 * y + li;
      if (gj >= n) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + 64 * wr + 16 * x + acc_row<true>(kg, v);
        if (gi >= n) continue;
        double r = alpha * acc[x][y][v];
        if (beta != 0.0) r = fma(beta, Dg[(int64_t)gj * ldd + gi], r);
        Cg[(int64_t)gj * ldc + gi] = r;
      }
    }
}

// partial sums of squares of X (T, row stride ldx), one per block of rows; then the finish
// kernel adds them in block order.
constexpr int EX_T = 256;
template <typename T>
__global__ __launch_bounds__(EX_T) void k_ex_sumsq(int n, const T* __restrict__ X, int64_t ldx, int rows,
                                                   double* __restrict__ part) {
  __shared__ double red[EX_T / WAVE];
  const int r0 = blockIdx.x * rows, r1 = min(n, r0 + rows);
  double s = 0.0;
  for (int i = r0; i < r1; ++i)
    for (int j = threadIdx.x; j < n; j += EX_T) {
      const double v = (double)gp(X)[(int64_t)i * ldx + j];
      s = fma(v, v, s);
    }
  const double w = wave_allsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < EX_T / WAVE; ++k) t += red[k];
    part[blockIdx.x] = t;
  }
}

// out[0] = ||X||_F, out[1] = 1 / ||X||_F (0 when X = 0); status NONFINITE when not finite
__global__ __launch_bounds__(64) void k_ex_finish(const double* __restrict__ part, int nblk, double* __restrict__ out,
                                                  psdproj_result* __restrict__ res) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[k];
  const double f = sqrt(s);
  out[0] = f;
  out[1] = (f > 0.0 && isfinite(f)) ? 1.0 / f : 0.0;
  psdproj_result r;
  r.status = isfinite(f) ? PSDPROJ_OK : PSDPROJ_E_NONFINITE;
  r.r_plus = 0;
  r.alpha_used = 0.0;
  r.sigma1 = 0.0;
  r.sigma2 = 0.0;
  *res = r;
}

// X64 = X (FP64 copy, column-major ld n; X symmetric so its row-major layout is the same matrix)
// and S = X / ||X||_F
template <typename T>
__global__ __launch_bounds__(EX_T) void k_ex_scale(int n, const T* __restrict__ X, int64_t ldx,
                                                   const double* __restrict__ out, double* __restrict__ X64,
                                                   double* __restrict__ S) {
  const int i = blockIdx.y, j = blockIdx.x * EX_T + threadIdx.x;
  if (j >= n) return;
  const double v = (double)gp(X)[(int64_t)i * ldx + j];
  X64[(int64_t)i * n + j] = v;
  S[(int64_t)i * n + j] = v * out[1];
}

__global__ __launch_bounds__(EX_T) void k_ex_poly(int n, double* __restrict__ W, double a2) {
  const int i = blockIdx.y, j = blockIdx.x * EX_T + threadIdx.x;
  if (j >= n) return;
  const int64_t e = (int64_t)i * n + j;
  W[e] = (i == j ? 3.0 : 0.0) - a2 * W[e];
}

template <typename T>
__global__ __launch_bounds__(EX_T) void k_ex_final(int n, const double* __restrict__ Q, T* __restrict__ P,
                                                   int64_t ldp) {
  const int i = blockIdx.y, j = blockIdx.x * EX_T + threadIdx.x;
  if (j >= n) return;
  gp(P)[(int64_t)i * ldp + j] = (T)(0.5 * (Q[(int64_t)i * n + j] + Q[(int64_t)j * n + i]));
}

// r_plus = round(Tr((I + S) / 2)), the number of positive eigenvalues once S = sign(X)
__global__ __launch_bounds__(EX_T) void k_ex_trace(int n, const double* __restrict__ S, psdproj_result* __restrict__ res) {
  __shared__ double red[EX_T / WAVE];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += EX_T) s += S[(int64_t)i * n + i];
  const double w = wave_allsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < EX_T / WAVE; ++k) t += red[k];
    res->r_plus = (int)floor(0.5 * (n + t) + 0.5);
  }
}

int exact_sumsq_blocks(int n, int* rows) {
  const int R = max(1, (n + 1023) / 1024);
  *rows = R;
  return (n + R - 1) / R;
}

static constexpr size_t gemm64_lds() { return (size_t)4 * GM_K * GM_LD * sizeof(double); }

// Opt the GEMM into more than 64 KB of dynamic LDS (two buffers of A and B slices).
void gemm64_init() {
  hipFuncSetAttribute((const void*)k_gemm64, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm64_lds());
}

void launch_gemm64(int n, const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                   double alpha, const double* D, int64_t ldd, double beta, hipStream_t s) {
  static std::atomic<unsigned> ready{0};   // one bit per device: the LDS attribute is set
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 32 && !(ready.load() & (1u << dev))) {
    gemm64_init();
    ready.fetch_or(1u << dev);
  }
  const int nt = (n + GM_B - 1) / GM_B;
  hipLaunchKernelGGL(k_gemm64, dim3(nt, nt), dim3(GM_T), gemm64_lds(), s, n, A, lda, B, ldb, C, ldc, alpha, D, ldd,
                     beta);
}

void launch_ex_norm(int n, bool fp64, const void* X, int64_t ldx, double* part, double* out, psdproj_result* res,
                    hipStream_t s) {
  int R = 1;
  const int nb = exact_sumsq_blocks(n, &R);
  if (fp64)
    hipLaunchKernelGGL(k_ex_sumsq<double>, dim3(nb), dim3(EX_T), 0, s, n, (const double*)X, ldx, R, part);
  else
    hipLaunchKernelGGL(k_ex_sumsq<float>, dim3(nb), dim3(EX_T), 0, s, n, (const float*)X, ldx, R, part);
  hipLaunchKernelGGL(k_ex_finish, dim3(1), dim3(64), 0, s, part, nb, out, res);
}

void launch_ex_scale(int n, bool fp64, const void* X, int64_t ldx, const double* out, double* X64, double* S,
                     hipStream_t s) {
  const dim3 g((n + EX_T - 1) / EX_T, n);
  if (fp64) hipLaunchKernelGGL(k_ex_scale<double>, g, dim3(EX_T), 0, s, n, (const double*)X, ldx, out, X64, S);
  else hipLaunchKernelGGL(k_ex_scale<float>, g, dim3(EX_T), 0, s, n, (const float*)X, ldx, out, X64, S);
}

void launch_ex_poly(int n, double* W, double a2, hipStream_t s) {
  hipLaunchKernelGGL(k_ex_poly, dim3((n + EX_T - 1) / EX_T, n), dim3(EX_T), 0, s, n, W, a2);
}

void launch_ex_final(int n, bool fp64, const double* Q, void* P, int64_t ldp, hipStream_t s) {
  const dim3 g((n + EX_T - 1) / EX_T, n);
  if (fp64) hipLaunchKernelGGL(k_ex_final<double>, g, dim3(EX_T), 0, s, n, Q, (double*)P, ldp);
  else hipLaunchKernelGGL(k_ex_final<float>, g, dim3(EX_T), 0, s, n, Q, (float*)P, ldp);
}

void launch_ex_trace(int n, const double* S, psdproj_result* res, hipStream_t s) {
  hipLaunchKernelGGL(k_ex_trace, dim3(1), dim3(EX_T), 0, s, n, S, res);
}

}  // namespace psd
