// Dual gradient descent for the SDLS problem (Alg. 6): the host loop of psdproj_sdls_solve.
// Each iteration forms X = C/rho + sum y_i A_i on the device, projects it in place with the
// library's grouped launch sequence (Alg. 2, or Alg. 3 with alpha by Alg. 5; the exact projection
// of Thm 1 for scal = -1), forms g_i = Tr(A_i^T Xhat_+) - b_i and updates y, all on the device;
// the host reads ||g|| (and the projection's status) to decide whether to stop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.hpp"
#include "exact.hpp"
#include "runtime.hpp"
#include "sdls.hpp"

namespace psd {
namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// the projection every iteration runs, as a plan (seed replaced per iteration)
psdproj_status sdls_plan(const psdproj_sdls_desc* d, Plan& pl) {
  psdproj_desc pd;
  std::memset(&pd, 0, sizeof(pd));
  pd.n = d->n;
  pd.k = d->k;
  pd.p = d->p;
  pd.q = d->q;
  pd.variant = (d->scal == 1) ? PSDPROJ_SCALED : PSDPROJ_PLAIN;
  pd.precision = d->precision;
  pd.seed = d->seed;
  pd.alpha = 0.0;   // Alg. 5 every iteration
  pd.alpha_iters = d->alpha_iters;
  pd.flags = 0;
  return make_plan(&pd, pl);
}

struct SdlsLayout {
  size_t proj = 0, part = 0, g = 0, out = 0, total = 0;
  size_t proj_bytes = 0;
  int nblk = 0;
};

psdproj_status sdls_layout(const psdproj_sdls_desc* d, SdlsLayout& L, Plan* pl_out) {
  if (!d) return PSDPROJ_E_INVALID;
  if (d->n < 1 || d->n > 65535 || d->m < 1 || d->m > (1 << 20)) return PSDPROJ_E_INVALID;
  if (d->scal < -1 || d->scal > 1) return PSDPROJ_E_INVALID;
  if (!(d->rho > 0.0) || !std::isfinite(d->rho) || !(d->beta > 0.0) || !std::isfinite(d->beta)) return PSDPROJ_E_INVALID;
  if (!(d->eps >= 0.0) || d->max_iters < 1) return PSDPROJ_E_INVALID;
  if (d->precision < PSDPROJ_FP64 || d->precision > PSDPROJ_BF16X3) return PSDPROJ_E_INVALID;
  if (d->flags != 0) return PSDPROJ_E_INVALID;
  if (d->scal == -1) {
    L.proj_bytes = exact_workspace_bytes((int)d->n, d->precision);
  } else {
    Plan pl;
    psdproj_status st = sdls_plan(d, pl);
    if (st != PSDPROJ_OK) return st;
    L.proj_bytes = pl.header_single + pl.region;
    if (pl_out) *pl_out = pl;
  }
  int R = 1;
  L.nblk = sdls_trace_blocks((int)d->n, &R);
  size_t o = 0;
  L.proj = o; o = al256(o + L.proj_bytes);
  L.part = o; o = al256(o + (size_t)d->m * L.nblk * 8);
  L.g = o; o = al256(o + (size_t)d->m * 8);
  L.out = o; o = al256(o + 64 + sizeof(psdproj_result));
  L.total = o;
  return PSDPROJ_OK;
}

}  // namespace
}  // namespace psd

using namespace psd;

extern "C" {

psdproj_status psdproj_sdls_workspace(const psdproj_sdls_desc* desc, size_t* bytes) {
  if (!bytes) return PSDPROJ_E_INVALID;
  SdlsLayout L;
  psdproj_status st = sdls_layout(desc, L, nullptr);
  if (st != PSDPROJ_OK) return st;
  *bytes = L.total;
  return PSDPROJ_OK;
}

psdproj_status psdproj_sdls_solve(const psdproj_sdls_desc* desc, const void* C, int64_t ldc, const void* A,
                                  int64_t lda, int64_t a_stride, const double* b_dev, double* y_dev, void* X,
                                  int64_t ldx, void* workspace, size_t workspace_bytes, psdproj_sdls_info* info,
                                  psdproj_stream_t stream) {
  SdlsLayout L;
  Plan base;
  psdproj_status st = sdls_layout(desc, L, &base);
  if (st != PSDPROJ_OK) return st;
  const int n = (int)desc->n, m = desc->m;
  if (!C || !A || !b_dev || !y_dev || !X || !workspace || !info) return PSDPROJ_E_INVALID;
  if (ldc < n || lda < n || ldx < n || a_stride < (int64_t)n * lda) return PSDPROJ_E_INVALID;
  if ((uintptr_t)workspace & 255) return PSDPROJ_E_INVALID;
  if (workspace_bytes < L.total) return PSDPROJ_E_NOMEM;
  const bool fp64 = desc->precision == PSDPROJ_FP64;
  if (desc->scal != -1) {
    st = check_operands(base, X, ldx, X, ldx);
    if (st != PSDPROJ_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  unsigned char* ws = (unsigned char*)workspace;
  double* part = (double*)(ws + L.part);
  double* g = (double*)(ws + L.g);
  double* out = (double*)(ws + L.out);
  psdproj_result* res = (psdproj_result*)(ws + L.out + 64);
  info->status = PSDPROJ_OK;
  info->iters = 0;
  info->grad_norm = 0.0;
  for (int it = 1; it <= desc->max_iters; ++it) {
    {
      ProfScope t(K_SDLS_FORM, s);
      launch_sdls_form(fp64, C, ldc, A, lda, a_stride, m, y_dev, 1.0 / desc->rho, X, ldx, n, s);
    }
    if (hipGetLastError() != hipSuccess) return PSDPROJ_E_DEVICE;
    if (desc->scal == -1) {
      st = exact_projection(n, desc->precision, X, ldx, X, ldx, ws + L.proj, L.proj_bytes, res, s);
    } else {
      Plan pl = base;
      pl.d.seed = desc->seed + (uint64_t)(it - 1);   // iteration it draws from key seed + it - 1
      const Plan* pp = &pl;
      const void* Ap = X;
      void* Pp = X;
      st = run_group(1, &pp, &Ap, &ldx, &Pp, &ldx, ws + L.proj, L.proj_bytes, res, s);
    }
    if (st != PSDPROJ_OK) return st;
    {
      ProfScope t(K_SDLS_TRACE, s);
      launch_sdls_trace(fp64, A, lda, a_stride, m, X, ldx, n, part, s);
    }
    {
      ProfScope t(K_SDLS_UPDATE, s);
      launch_sdls_update(part, L.nblk, m, b_dev, desc->beta, y_dev, g, out, s);
    }
    if (hipGetLastError() != hipSuccess) return PSDPROJ_E_DEVICE;
    struct { double gnorm; char pad[56]; psdproj_result r; } host;
    static_assert(sizeof(host) >= 64 + sizeof(psdproj_result), "read-back layout");
    if (hipMemcpyAsync(&host, out, 64 + sizeof(psdproj_result), hipMemcpyDeviceToHost, s) != hipSuccess)
      return PSDPROJ_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PSDPROJ_E_DEVICE;
    info->iters = it;
    info->grad_norm = host.gnorm;
    if (host.r.status != PSDPROJ_OK) {
      info->status = host.r.status;
      break;
    }
    if (!std::isfinite(host.gnorm)) { info->status = PSDPROJ_E_NONFINITE; break; }
    if (!(host.gnorm > desc->eps)) break;
  }
  return PSDPROJ_OK;
}

}  // extern "C"
