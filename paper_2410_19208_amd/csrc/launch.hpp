// Host-side launchers of the grouped kernels.  Every kernel's grid covers the tiles of all
// problems of a launch: tstart[i] is the first block of problem i (tstart[nprob] = grid).
#pragma once
#include "common.hpp"

namespace psd {

struct Launch {
  unsigned grid;          // total blocks
  const Prob* probs;      // device array
  const int* tstart;      // device array, nprob + 1 entries
  int nprob;
  hipStream_t stream;
  int maxnb;              // largest r_pad / 16 among the launch's problems
};

// Tile counts per problem, shared by host planning and the kernels' tile decoding.
int tiles_omega(const Prob& p);
int tiles_vec(const Prob& p);
int tiles_pass(const Prob& p);
int tiles_reduce(const Prob& p);
int tiles_gram(const Prob& p, bool full);
int tiles_small(const Prob& p);       // one block per problem
int tiles_apply(const Prob& p);
int tiles_gemv(const Prob& p);       // workgroups (GV_PER_WG tiles each)
int gemv_tile_count(const Prob& p);
int tiles_gemv_rows(const Prob& p);  // one block per 256-row block row
int tiles_bisect(const Prob& p);
int tiles_invit(const Prob& p);
int tiles_rebuild(const Prob& p);    // workgroups (RB_PER_WG tiles each, a multiple of 8)
int rebuild_tile_count(const Prob& p);

void launch_omega(const Launch& L);
void launch_power_init(const Launch& L, int which);
void launch_power_init2(const Launch& L);
void launch_words(uint64_t seed, uint32_t stream_id, uint64_t c0, int64_t count, uint32_t* out, hipStream_t s);
void launch_gauss(uint64_t seed, uint32_t stream_id, uint64_t start, int64_t count, double* out, hipStream_t s);
void launch_srht(uint64_t seed, int n, int r, double* out, hipStream_t s);

// Passes over A: part[s] = A[:, chunk s] * Z[chunk s, :]; reduce: Y = sum_s part[s]
// (+ scaled epilogue (Y + alpha Z)/alpha).
void launch_pass(const Launch& L, int prec, int ncb);
void launch_pass_reduce(const Launch& L);
// CSR operand: Z to row-major (k_zt), then the sparse pass (k_spmm, one partial, no split)
int tiles_zt(const Prob& p);
void launch_zt(const Launch& L);
void launch_spmm(const Launch& L);
void pass_init();                     // dynamic-LDS attributes of the pass kernels

// Gram X^T Y (mode 0: Y^T Y of the pass output, upper tiles; 1: Q1^T Q1; 2: Q^T Y full,
// symmetrised) and its deterministic reduction.
void launch_gram(const Launch& L, int mode);
void launch_gram_reduce(const Launch& L, int mode);

// Orthonormalisation factors (one block per problem) and panel products.
void launch_chol(const Launch& L, int round);
void launch_apply(const Launch& L, int round);
void apply_init();

// Eigensolver of the compressed matrix and the rebuild.
void launch_tridiag(const Launch& L);
void launch_bisect(const Launch& L);
void launch_invit(const Launch& L);
void launch_backxf(const Launch& L);
void launch_formw(const Launch& L);
void launch_rebuild(const Launch& L, int prec);
void rebuild_init();
void launch_setup(const Launch& L);
void launch_finalize(const Launch& L);

// Alg. 4/5 matrix-vector products.
void launch_gemv(const Launch& L, int last);
void launch_gemv_finish(const Launch& L, int last);
void launch_alpha(const Launch& L);
void launch_gemv2(const Launch& L, int j);
void launch_gemv2_finish(const Launch& L, int j);
void launch_alpha2(const Launch& L);

}  // namespace psd
