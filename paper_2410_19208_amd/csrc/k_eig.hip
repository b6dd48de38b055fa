// Symmetric eigensolve of the r x r compressed matrix C (Alg. 2 line 2, Alg. 3 line 3) and
// the clamp (Alg. 2 line 3: max(D, 0); Alg. 3 line 4: alpha (max(D, 1) - I)), in FP64.
//
//  k_tridiag : Householder reduction C = Q_H T Q_H^T (one workgroup per problem); also the
//              Gershgorin interval of T and the Sturm count nu of eigenvalues below the clamp
//              threshold (0 plain, 1 scaled), so only the r - nu kept eigenpairs get vectors.
//  k_bisect  : every eigenvalue of T by multisection of Sturm counts, one wave per eigenvalue
//              (64 trial points per round).
//  k_invit   : eigenvectors of T for the kept eigenvalues by inverse iteration (tridiagonal LU
//              with partial pivoting), Gram-Schmidt within clusters of close eigenvalues, and
//              the clamped weights; the vectors of T go to xt.
//  k_backxf  : back-transformation of each by the Householder reflectors, one wave per
//              eigenvector.  Writes V (column c = c-th largest kept eigenvalue, column-major)
//              and F = V diag(sqrt(w)) (row-major).
#include "common.hpp"
#include "launch.hpp"

namespace psd {



// Sturm counts (eigenvalues of T below x) at two points at once: two independent recurrences
// interleaved, and 1/q as a hardware reciprocal refined by two Newton steps instead of an
// IEEE division, so the dependent chain per step is a few fused multiply-adds.
__device__ __forceinline__ void sturm_count2(const double* d, const double* e2, int r, double x0, double x1,
                                             double pivmin, int& c0, int& c1) {
  double q0 = d[0] - x0, q1 = d[0] - x1;
  c0 = q0 < 0.0;
  c1 = q1 < 0.0;
  for (int i = 1; i < r; ++i) {
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    double r0 = __builtin_amdgcn_rcp(q0), r1 = __builtin_amdgcn_rcp(q1);
    r0 = fma(r0, fma(-q0, r0, 1.0), r0);
    r1 = fma(r1, fma(-q1, r1, 1.0), r1);
    r0 = fma(r0, fma(-q0, r0, 1.0), r0);
    r1 = fma(r1, fma(-q1, r1, 1.0), r1);
    const double di = d[i], ei = e2[i - 1];
    q0 = (di - x0) - ei * r0;
    q1 = (di - x1) - ei * r1;
    c0 += q0 < 0.0;
    c1 += q1 < 0.0;
  }
}

// One wave per eigenvalue index j (ascending); lane l tests x = lo + (hi - lo)(m+1)/129 at
// m = l and m = l + 64 (128-way multisection).
__global__ __launch_bounds__(256) void k_bisect(const Prob* __restrict__ probs, const int* __restrict__ tstart,
                                                int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int j = (blockIdx.x - tstart[pi]) * 4 + wave_id();
  const int lane = threadIdx.x & 63;
  const int r = p.r;
  if (j >= r) return;
  const gmem<const double>* d = gp((const double*)p.td);
  const gmem<const double>* e2 = gp((const double*)p.evals + PSDPROJ_MAX_RANK);
  const double pivmin = p.scal[S_PIVMIN];
  double lo = p.scal[S_GL], hi = p.scal[S_GU];
  if (!(isfinite(lo) && isfinite(hi))) {
    if (lane == 0) p.evals[j] = __builtin_nan("");
    return;
  }
  __shared__ double dl[4][PSDPROJ_MAX_RANK], el[4][PSDPROJ_MAX_RANK];   // per wave: T's d and e^2
  const int w = wave_id();
  for (int i = lane; i < r; i += WAVE) {
    dl[w][i] = d[i];
    el[w][i] = (i + 1 < r) ? e2[i] : 0.0;
  }
  lds_wave_sync();
  for (int round = 0; round < 24; ++round) {
    const double width = hi - lo;
    const double tol = 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin;
    if (!(width > 2.0 * tol)) break;
    const double x0 = lo + width * (double)(lane + 1) / 129.0;
    const double x1 = lo + width * (double)(lane + 65) / 129.0;
    int c0, c1;
    sturm_count2(dl[w], el[w], r, x0, x1, pivmin, c0, c1);
    // the first point (in increasing order) whose count exceeds j bounds the eigenvalue above
    const unsigned long long m0 = __ballot(c0 > j), m1 = __ballot(c1 > j);
    double nlo = lo, nhi = hi;
    if (m0) {
      const int f = __ffsll((long long)m0) - 1;
      nhi = __shfl(x0, f, 64);
      if (f > 0) nlo = __shfl(x0, f - 1, 64);
    } else if (m1) {
      const int f = __ffsll((long long)m1) - 1;
      nhi = __shfl(x1, f, 64);
      nlo = (f > 0) ? __shfl(x1, f - 1, 64) : __shfl(x0, 63, 64);
    } else {
      nlo = __shfl(x1, 63, 64);
    }
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) p.evals[j] = 0.5 * (lo + hi);
}

// Deterministic start vector for inverse iteration (a fixed hash, independent of the seed).
__device__ __forceinline__ double start_component(int j, int i) {
  uint32_t h = (uint32_t)(j * 2654435761u) ^ (uint32_t)(i * 2246822519u) ^ 0x9E3779B9u;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)h + 0.5) * (1.0 / 4294967296.0) - 0.5;
}

// One wave per block: every block owns one candidate cluster leader, so block-wide barriers
// are wave barriers and early exits are block-uniform.
__global__ __launch_bounds__(WAVE) void k_invit(const Prob* __restrict__ probs,
                                                const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int lane = threadIdx.x;
  const int r = p.r, rp = p.rpad;
  const int nu = p.iscal[I_NU];
  const int j0 = nu + (blockIdx.x - tstart[pi]);
  const double tnorm = p.scal[S_TNORM];
  const double thr = p.scal[S_THRESH];
  const bool scaled = (p.variant == PSDPROJ_SCALED);
  const double alpha = p.scal[S_ALPHA];

  // weights and r_plus (the first wave of each problem; read by later kernels): weight c is
  // that of eigenvalue r-1-c, and r_plus counts the leading positive finite weights down to
  // eigenvalue nu.  Lanes take 64 weights at a time; a ballot finds the first that fails.
  if (blockIdx.x == tstart[pi]) {
    int rplus = rp;
    double wv[(PSDPROJ_MAX_RANK + WAVE - 1) / WAVE];
#pragma unroll
    for (int c0 = 0, u = 0; c0 < PSDPROJ_MAX_RANK; c0 += WAVE, ++u) {
      const int c = c0 + lane, jj = r - 1 - c;
      double wgt = 0.0;
      bool ok = false;
      if (c < rp && jj >= nu) {
        const double lam = p.evals[jj];
        wgt = scaled ? alpha * (fmax(lam, 1.0) - 1.0) : fmax(lam, 0.0);
        ok = wgt > 0.0 && isfinite(wgt);
      }
      wv[u] = wgt;
      const unsigned long long bad = __ballot(!ok);
      if (bad != 0ull) rplus = min(rplus, c0 + __ffsll((long long)bad) - 1);
    }
#pragma unroll
    for (int c0 = 0, u = 0; c0 < PSDPROJ_MAX_RANK; c0 += WAVE, ++u) {
      const int c = c0 + lane;
      if (c < rp) p.wts[c] = (c < rplus) ? wv[u] : 0.0;
    }
    if (lane == 0) p.iscal[I_RPLUS] = rplus;
  }
  if (j0 >= r) return;
  const double gtol = 1e-5 * tnorm;
  // only cluster leaders work; a cluster is a run of kept eigenvalues closer than gtol
  if (j0 > nu && p.evals[j0] - p.evals[j0 - 1] <= gtol) return;

  __shared__ double U0[PSDPROJ_MAX_RANK], U1[PSDPROJ_MAX_RANK], U2[PSDPROJ_MAX_RANK];
  __shared__ double Lm[PSDPROJ_MAX_RANK], x[PSDPROJ_MAX_RANK], b[PSDPROJ_MAX_RANK], iu0[PSDPROJ_MAX_RANK];
  __shared__ int piv[PSDPROJ_MAX_RANK];
  __shared__ double dl[PSDPROJ_MAX_RANK], el[PSDPROJ_MAX_RANK];
  const gmem<const double>* d = gp((const double*)p.td);
  const gmem<const double>* e = gp((const double*)p.te);
  gmem<double>* xt = gp(p.xt);
  const double tiny = 2.220446049250313e-16 * fmax(tnorm, 1e-300);

  // T's diagonal and off-diagonal into LDS once: the LU recurrence below then waits on LDS
  // reads rather than on global loads at every step
  for (int i = lane; i < r; i += WAVE) {
    dl[i] = d[i];
    el[i] = (i + 1 < r) ? e[i] : 0.0;
  }
  __syncthreads();
  int jc = j0;
  do {
    const double lam = p.evals[jc];
    // --- LU of T - lam I with partial pivoting (all lanes compute the same values; lane 0
    // stores them).  Branch-free step: the pivot is chosen by a compare and selects, and
    // 1/pivot is the refined hardware reciprocal (IEEE division only for a pivot below the
    // normal range, the same in all lanes).
    {
      double cd = dl[0] - lam, cs = (r > 1) ? el[0] : 0.0;
      for (int i = 0; i + 1 < r; ++i) {
        const double nd = dl[i + 1] - lam;
        const double ns = (i + 2 < r) ? el[i + 1] : 0.0;
        const double sb = el[i];
        const bool keep = fabs(cd) >= fabs(sb);
        const double pv = keep ? ((cd == 0.0) ? tiny : cd) : sb;
        const double num = keep ? sb : cd;
        double m;
        if (fabs(pv) >= 2.2250738585072014e-308) m = num * rcp_f64(pv);
        else m = num / pv;
        if (lane == 0) {   // one lane stores (64 lanes writing one address serialise)
          U0[i] = pv;
          U1[i] = keep ? cs : nd;
          U2[i] = keep ? 0.0 : ns;
          Lm[i] = m;
          piv[i] = keep ? 0 : 1;
        }
        const double ncd = keep ? nd - m * cs : cs - m * nd;
        cs = keep ? ns : -m * ns;
        cd = ncd;
      }
      if (cd == 0.0) cd = tiny;
      if (lane == 0) U0[r - 1] = cd;
    }
    __syncthreads();
    for (int i = lane; i < r; i += WAVE) {
      b[i] = start_component(jc, i);
      iu0[i] = 1.0 / U0[i];   // the substitutions multiply by these
    }
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      // --- solve (T - lam I) x = b: forward with row swaps, then back substitution (lane 0).
      // The running entries stay in registers; the LDS operands are read in chunks of SC
      // steps ahead of the chain, so each step waits only on its multiply-add.
      if (lane == 0) {
        constexpr int SC = 8;
        double cur = b[0];
        for (int i0 = 0; i0 + 1 < r; i0 += SC) {
          double bn[SC], lm[SC];
          int pw[SC];
#pragma unroll
          for (int k = 0; k < SC; ++k) {
            const int i = min(i0 + k, r - 2);
            bn[k] = b[i + 1];
            lm[k] = Lm[i];
            pw[k] = piv[i];
          }
#pragma unroll
          for (int k = 0; k < SC; ++k) {
            const int i = i0 + k;
            if (i + 1 < r) {
              double nxt = bn[k];
              if (pw[k]) { const double t = cur; cur = nxt; nxt = t; }
              nxt -= lm[k] * cur;
              b[i] = cur;
              cur = nxt;
            }
          }
        }
        b[r - 1] = cur;
        double x1 = b[r - 1] * iu0[r - 1], x2 = 0.0;
        x[r - 1] = x1;
        if (r >= 2) {
          const double x0 = (b[r - 2] - U1[r - 2] * x1) * iu0[r - 2];
          x[r - 2] = x0;
          x2 = x1;
          x1 = x0;
        }
        for (int i0 = r - 3; i0 >= 0; i0 -= SC) {
          double bb[SC], u1[SC], u2[SC], iu[SC];
#pragma unroll
          for (int k = 0; k < SC; ++k) {
            const int i = max(i0 - k, 0);
            bb[k] = b[i];
            u1[k] = U1[i];
            u2[k] = U2[i];
            iu[k] = iu0[i];
          }
#pragma unroll
          for (int k = 0; k < SC; ++k) {
            const int i = i0 - k;
            if (i >= 0) {
              const double x0 = (bb[k] - u1[k] * x1 - u2[k] * x2) * iu[k];
              x[i] = x0;
              x2 = x1;
              x1 = x0;
            }
          }
        }
      }
      __syncthreads();
      // --- Gram-Schmidt against earlier members of the cluster (stored in xt)
      for (int m = j0; m < jc; ++m) {
        const gmem<double>* xm = xt + (int64_t)(m - nu) * rp;
        double s = 0.0;
        for (int i = lane; i < r; i += WAVE) s += xm[i] * x[i];
        s = wave_sum(s);
        for (int i = lane; i < r; i += WAVE) x[i] -= s * xm[i];
        __syncthreads();
      }
      // --- normalise: b = x / ||x|| (scaled first against overflow)
      double mx = 0.0;
      for (int i = lane; i < r; i += WAVE) mx = fmax(mx, fabs(x[i]));
      for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
      const double inv_mx = (mx > 0.0) ? 1.0 / mx : 0.0;
      double s2 = 0.0;
      for (int i = lane; i < r; i += WAVE) { const double t = x[i] * inv_mx; s2 += t * t; }
      s2 = wave_sum(s2);
      const double sc = (s2 > 0.0) ? inv_mx / sqrt(s2) : 0.0;
      for (int i = lane; i < r; i += WAVE) b[i] = x[i] * sc;
      __syncthreads();
    }
    // b holds the unit eigenvector of T: kept for later cluster members and for k_backxf
    gmem<double>* xs = xt + (int64_t)(jc - nu) * rp;
    for (int i = lane; i < r; i += WAVE) xs[i] = b[i];
    __syncthreads();
    ++jc;
  } while (jc < r && p.evals[jc] - p.evals[jc - 1] <= gtol);
  (void)thr;
}

// Back-transformation u = H_0 H_1 ... H_{r-3} y of every kept eigenvector y of T (left in xt
// by k_invit), one wave per eigenvector, so the members of a cluster, found one after another
// by their leader, are transformed side by side.  Lane l holds entries l + 64 q (q < 4) in
// registers; the next reflector's column is loaded while the current one is applied.  Writes
// column c = r-1-j of V (column-major) and row-major F = V diag(sqrt(w)).
__global__ __launch_bounds__(WAVE) void k_backxf(const Prob* __restrict__ probs,
                                                 const int* __restrict__ tstart, int nprob) {
  const int pi = find_prob(tstart, nprob, blockIdx.x);
  const Prob& p = probs[pi];
  const int lane = threadIdx.x;
  const int r = p.r, rp = p.rpad;
  const int nu = p.iscal[I_NU];
  const int jc = nu + (blockIdx.x - tstart[pi]);
  if (jc >= r) return;
  const bool scaled = (p.variant == PSDPROJ_SCALED);
  const double alpha = p.scal[S_ALPHA];
  const double lam = p.evals[jc];
  const gmem<const double>* xs = gp((const double*)p.xt) + (int64_t)(jc - nu) * rp;
  double bv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) bv[q] = (lane + 64 * q < r) ? xs[lane + 64 * q] : 0.0;
  // Reflector columns (and their tau) stream through a ring of BX register slots: slot k is
  // refilled with the reflector BX steps further on as soon as it has been applied, so a
  // column's load has BX reflectors' worth of work to hide behind.
  constexpr int BX = 8;
  const gmem<const double>* Hc = gp((const double*)p.H);
  const gmem<const double>* Tc = gp((const double*)p.tau);
  double hr[BX][4], tr[BX];
  auto hload = [&](int jh, double (&h)[4], double& t) {
    jh = max(jh, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = Hc[(int64_t)jh * rp + min(lane + 64 * q, rp - 1)];
    t = Tc[jh];
  };
#pragma unroll
  for (int k = 0; k < BX; ++k) hload(r - 3 - k, hr[k], tr[k]);
  for (int base = r - 3; base >= 0; base -= BX) {
#pragma unroll
    for (int k = 0; k < BX; ++k) {
      const int jh = base - k;
      if (jh >= 0) {
        const double tau = tr[k];
        double v[4], sdot = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = lane + 64 * q;
          v[q] = (i == jh + 1) ? 1.0 : ((i > jh + 1 && i < r) ? hr[k][q] : 0.0);
          sdot += v[q] * bv[q];
        }
        sdot = wave_allsum(sdot) * tau;   // tau = 0: identity reflector
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] -= sdot * v[q];
      }
      hload(base - k - BX, hr[k], tr[k]);
    }
  }
  // column c = r-1-jc (descending eigenvalue order)
  const int c = r - 1 - jc;
  const double wgt = scaled ? alpha * (fmax(lam, 1.0) - 1.0) : fmax(lam, 0.0);
  const double sw = (wgt > 0.0 && isfinite(wgt)) ? sqrt(wgt) : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    if (i < rp) {
      const double u = (i < r) ? bv[q] : 0.0;
      p.V[(int64_t)c * rp + i] = u;
      p.F[(int64_t)i * rp + c] = u * sw;   // row-major (read by the factor apply)
    }
  }
}

int tiles_bisect(const Prob& p) { return (p.r + 3) / 4; }
int tiles_invit(const Prob& p) { return p.r; }

void launch_bisect(const Launch& L) {
  hipLaunchKernelGGL(k_bisect, dim3(L.grid), dim3(256), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_invit(const Launch& L) {
  hipLaunchKernelGGL(k_invit, dim3(L.grid), dim3(WAVE), 0, L.stream, L.probs, L.tstart, L.nprob);
}
void launch_backxf(const Launch& L) {
  hipLaunchKernelGGL(k_backxf, dim3(L.grid), dim3(WAVE), 0, L.stream, L.probs, L.tstart, L.nprob);
}

}  // namespace psd
