// Host-side planning structures of libpsdproj.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

namespace psd {

enum Kind {
  K_SETUP, K_OMEGA, K_PINIT, K_GEMV, K_ALPHA, K_PASS, K_PRED, K_GRAM_SYM, K_GRAM_FULL, K_GRED,
  K_CHOL, K_APPLY, K_TRIDIAG, K_BISECT, K_INVIT, K_REBUILD, K_FINAL, K_GEMV_FIN, K_FACTOR, K_BACKXF, K_NKINDS
};
enum When { W_ALL, W_ALPHA, W_ALPHA_ITER, W_POWER };

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
  int r, rpad, ld, prec, es, ncb, alpha_mode;
  int split, kchunk, ngchunk, rwpad;
  size_t region;          // workspace bytes of the problem's own buffers
  size_t header_single;   // header bytes of a single run
  size_t o_zm, o_zhi, o_zlo, o_y, o_part, o_q1, o_wf, o_whi, o_wlo, o_gpart;
  size_t o_G, o_F, o_C, o_H, o_V, o_xt, o_evals, o_tau, o_td, o_te, o_wts;
  size_t o_vec, o_vpart, o_gvp, o_scal, o_iscal, o_drop;
  Schedule single;        // launch schedule of a single run (header_single bytes of header)
};

psdproj_status make_plan(const psdproj_desc* d, Plan& pl);
Prob make_prob(const Plan& pl, unsigned char* region, const void* A, int64_t lda, void* P, int64_t ldp,
               psdproj_result* res);
void build_schedule(const Plan* const* plans, int count, Schedule& s);
psdproj_status upload(void* dst, const void* src, size_t bytes, hipStream_t stream);
psdproj_status enqueue(const Schedule& s, unsigned char* hdr, hipStream_t stream, bool allow_timing = true);
psdproj_status check_operands(const Plan& pl, const void* A, int64_t lda, const void* P, int64_t ldp);
psdproj_status run_group(int count, const Plan* const* plans, const void* const* A, const int64_t* lda,
                         void* const* P, const int64_t* ldp, unsigned char* ws, size_t ws_bytes,
                         psdproj_result* results, hipStream_t stream);

}  // namespace psd
