// Host-side planning structures of libpsdproj.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

namespace psd {

enum Kind {
  K_SETUP, K_OMEGA, K_PINIT, K_GEMV, K_ALPHA, K_PASS, K_PRED, K_GRAM_SYM, K_GRAM_FULL, K_GRED,
  K_CHOL, K_APPLY, K_TRIDIAG, K_BISECT, K_INVIT, K_REBUILD, K_FINAL, K_GEMV_FIN, K_FACTOR, K_BACKXF, K_ZT,
  K_SDLS_FORM, K_SDLS_TRACE, K_SDLS_UPDATE, K_GEMM64, K_EXACT_MISC, K_PINIT2, K_GEMV2, K_GEMV2_FIN,
  K_ALPHA2, K_NKINDS
};
// Which problems take part in a stage: all; those estimating alpha with the two runs one after
// the other (N > PAIRED_MAX) or sharing products (N <= PAIRED_MAX), at every iteration or only
// below their N (sequential) or N + 1 (paired); those with q > iter.
enum When { W_ALL, W_SEQ, W_SEQ_ITER, W_PAIRED, W_PAIRED_ITER, W_POWER };

struct Stage { int kind, arg, when, iter; };

struct LaunchRec {
  int kind, arg, first, count, prec, ncb, toff, maxnb;
  unsigned grid;
};

struct Group { int first, count, prec, ncb; };

struct Schedule {
  std::vector<int> order;          // problem order on the device (sorted by kernel key)
  std::vector<Group> groups;
  std::vector<LaunchRec> launches;
  std::vector<int> tdata;          // all tile-start tables
  size_t prob_bytes = 0, header_bytes = 0;
};

// An immutable, validated problem description with its tiling and workspace layout.
struct Plan {
  psdproj_desc d;
  int r, rpad, ld, prec, es, ncb, alpha_mode, csr, paired;
  int split, kchunk, ngchunk, rwpad;
  size_t region;          // workspace bytes of the problem's own buffers
  size_t header_single;   // header bytes of a single run
  size_t o_zm, o_zhi, o_zlo, o_y, o_part, o_q1, o_wf, o_whi, o_wlo, o_gpart;
  size_t o_G, o_F, o_C, o_H, o_V, o_xt, o_evals, o_tau, o_td, o_te, o_wts;
  size_t o_vec, o_vpart, o_gvp, o_scal, o_iscal, o_drop, o_zr, o_bh, o_pw;
  Schedule single;        // launch schedule of a single run (header_single bytes of header)
};

psdproj_status make_plan(const psdproj_desc* d, Plan& pl);
// A sparse operand (CSR, both triangles of the symmetric matrix): row starts and column indices
struct Csr { const int32_t* rowptr; const int32_t* colidx; };
Prob make_prob(const Plan& pl, unsigned char* region, const void* A, int64_t lda, void* P, int64_t ldp,
               psdproj_result* res, const Csr* csr = nullptr);
void build_schedule(const Plan* const* plans, int count, Schedule& s);
psdproj_status upload(void* dst, const void* src, size_t bytes, hipStream_t stream);
psdproj_status enqueue(const Schedule& s, unsigned char* hdr, hipStream_t stream, bool allow_timing = true);
// Kernel timing of a launch made outside a schedule (the SDLS and exact-projection kernels):
// while timing is enabled for `kind`, the scope brackets the launches it encloses with events.
struct ProfScope {
  ProfScope(int kind, hipStream_t stream);
  ~ProfScope();
  int kind;
  hipStream_t stream;
  hipEvent_t a = nullptr, b = nullptr;
};
psdproj_status check_operands(const Plan& pl, const void* A, int64_t lda, const void* P, int64_t ldp);
psdproj_status run_group(int count, const Plan* const* plans, const void* const* A, const int64_t* lda,
                         void* const* P, const int64_t* ldp, unsigned char* ws, size_t ws_bytes,
                         psdproj_result* results, hipStream_t stream, const Csr* csr = nullptr);

}  // namespace psd
