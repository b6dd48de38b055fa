// Host runtime of libpsdproj: plans, workspace layout, the grouped launch schedule and the
// C ABI of psdproj.h (single runs and batches; the request server lives in server.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace psd {

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
static int rup(int x, int m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------------------ tile table
// Split-K of the passes per (precision, n bucket, padded width), chosen by the tuner
// (paper_2410_19208_amd/tune.py, which times every candidate on the GPU and writes
// tile_table.inc).  Bucket b holds 2^b <= n < 2^(b+1) (b clamped to [6, 14]); a missing entry
// keeps the built-in rule.  An override (psdproj_tile_override) takes precedence, for the tuner's
// own measurements.
namespace {
struct TileEntry { int prec, nlog2, rpad, split; };
const TileEntry TILE_TABLE[] = {
#include "tile_table.inc"
};
std::mutex tile_mu;
int tile_override[3] = {0, 0, 0};

int n_bucket(int64_t n) {
  int b = 0;
  while (b < 62 && (int64_t(1) << (b + 1)) <= n) ++b;
  return std::min(14, std::max(6, b));
}

int tuned_split(int prec, int64_t n, int rpad) {
  {
    std::lock_guard<std::mutex> g(tile_mu);
    if (tile_override[prec] > 0) return tile_override[prec];
  }
  const int b = n_bucket(n);
  for (const TileEntry& e : TILE_TABLE)
    if (e.prec == prec && e.nlog2 == b && e.rpad == rpad) return e.split;
  return 0;
}
}  // namespace

// ------------------------------------------------------------------------------ planning
psdproj_status make_plan(const psdproj_desc* d, Plan& pl) {
  if (!d) return PSDPROJ_E_INVALID;
  if (d->n < 1 || d->n > (1 << 20)) return PSDPROJ_E_INVALID;
  if (d->k < 1 || d->p < 0) return PSDPROJ_E_INVALID;
  const int64_t r = (int64_t)d->k + d->p;
  if (r > d->n || r > PSDPROJ_MAX_RANK) return PSDPROJ_E_INVALID;
  if (d->q < 0 || d->q > 16) return PSDPROJ_E_INVALID;
  if (d->variant != PSDPROJ_PLAIN && d->variant != PSDPROJ_SCALED) return PSDPROJ_E_INVALID;
  if (d->precision < PSDPROJ_FP64 || d->precision > PSDPROJ_BF16X3) return PSDPROJ_E_INVALID;
  if ((d->flags & ~(uint32_t)(PSDPROJ_FLAG_SRHT | PSDPROJ_FLAG_CSR)) != 0) return PSDPROJ_E_INVALID;
  int alpha_mode = 0;
  if (d->variant == PSDPROJ_SCALED) {
    if (std::isnan(d->alpha) || std::isinf(d->alpha)) return PSDPROJ_E_INVALID;
    if (d->alpha <= 0.0) {
      if (d->alpha_iters < 1 || d->alpha_iters > 1000) return PSDPROJ_E_INVALID;
      alpha_mode = 1;
    }
  }
  pl.d = *d;
  const int n = (int)d->n;
  pl.r = (int)r;
  pl.rpad = rup(pl.r, RPAD);
  pl.ld = rup(n + PANEL_TAIL, 128);
  pl.prec = d->precision;
  pl.es = (pl.prec == F64) ? 8 : 4;
  pl.ncb = pl.rpad / 16;
  pl.alpha_mode = alpha_mode;
  pl.paired = (alpha_mode == 1 && d->alpha_iters <= PAIRED_MAX) ? 1 : 0;
  pl.csr = (d->flags & PSDPROJ_FLAG_CSR) ? 1 : 0;
  // split-K, at most 8 (one K chunk per XCD).  FP64: enough workgroups to fill 256 CUs twice.
  // FP32 / BF16X3 (one 8-wave workgroup per CU): 8 chunks of at least 64 columns, so each
  // XCD's L2 holds one chunk of the panel.
  const int bm = (pl.prec == F64) ? PASS_BM_D : PASS_BM_F;
  const int bk = (pl.prec == F64) ? PASS_BK_D : PASS_BK_F;
  const int mt = (n + bm - 1) / bm;
  int split = (pl.prec == F64) ? std::min(8, std::max(1, (512 + mt - 1) / mt))
                               : std::min(8, std::max(1, (n + 63) / 64));
  const int tuned = tuned_split(pl.prec, n, pl.rpad);
  if (tuned > 0) split = std::min(tuned, MAX_SPLIT);
  if (pl.csr) split = 1;   // the sparse pass has no K chunks
  int kchunk = rup((n + split - 1) / split, bk);
  split = (n + kchunk - 1) / kchunk;
  pl.split = split;
  pl.kchunk = kchunk;
  pl.ngchunk = (pl.ld + GRAM_CHUNK - 1) / GRAM_CHUNK;
  pl.rwpad = pl.rpad;

  // workspace region of one problem
  const size_t P = (size_t)pl.rpad * pl.ld;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = al256(o + bytes); return at; };
  pl.o_zm = take(P * pl.es);
  pl.o_zhi = (pl.prec == B3) ? take(P * 2) : 0;
  pl.o_zlo = (pl.prec == B3) ? take(P * 2) : 0;
  pl.o_y = take(P * pl.es);
  pl.o_part = take((size_t)split * P * pl.es);
  pl.o_q1 = take(P * pl.es);
  pl.o_wf = take((size_t)pl.ld * pl.rwpad * pl.es);
  pl.o_whi = (pl.prec == B3) ? take((size_t)pl.ld * pl.rwpad * 2) : 0;
  pl.o_wlo = (pl.prec == B3) ? take((size_t)pl.ld * pl.rwpad * 2) : 0;
  const size_t RR = (size_t)pl.rpad * pl.rpad * 8;
  pl.o_gpart = take((size_t)pl.ngchunk * RR);
  pl.o_G = take(RR);
  pl.o_F = take(RR);
  pl.o_C = take(RR);
  pl.o_H = take(RR);
  pl.o_V = take(RR);
  pl.o_xt = take(RR);
  pl.o_evals = take(2 * PSDPROJ_MAX_RANK * 8);
  pl.o_tau = take(PSDPROJ_MAX_RANK * 8);
  pl.o_td = take(PSDPROJ_MAX_RANK * 8);
  pl.o_te = take(PSDPROJ_MAX_RANK * 8);
  pl.o_wts = take(PSDPROJ_MAX_RANK * 8);
  pl.o_vec = take((size_t)2 * pl.ld * 8);
  const size_t gnb = (size_t)(n + GEMV_TILE - 1) / GEMV_TILE;
  const size_t nvec = pl.paired ? 2 : 1;   // vectors per product
  pl.o_vpart = take(nvec * gnb * 8);
  pl.o_gvp = take(nvec * gnb * gnb * GEMV_TILE * 8);
  pl.o_bh = pl.paired ? take((size_t)(d->alpha_iters + 2) * pl.ld * 8) : 0;
  pl.o_pw = pl.paired ? take((size_t)2 * (PAIRED_MAX + 2) * 8) : 0;
  pl.o_scal = take(NSCAL * 8);
  pl.o_iscal = take(NISCAL * 4);
  pl.o_drop = take(PSDPROJ_MAX_RANK * 4);
  pl.o_zr = pl.csr ? take((size_t)n * pl.rpad * pl.es) : 0;
  pl.region = o;
  // schedule and header of a single run
  const Plan* one = &pl;
  build_schedule(&one, 1, pl.single);
  pl.header_single = pl.single.header_bytes;
  return PSDPROJ_OK;
}

Prob make_prob(const Plan& pl, unsigned char* region, const void* A, int64_t lda, void* P, int64_t ldp,
               psdproj_result* res, const Csr* csr) {
  Prob p;
  std::memset(&p, 0, sizeof(p));
  const psdproj_desc& d = pl.d;
  p.n = (int)d.n; p.r = pl.r; p.rpad = pl.rpad; p.ld = pl.ld;
  p.k = d.k; p.q = d.q; p.variant = d.variant; p.prec = pl.prec;
  p.split = pl.split; p.kchunk = pl.kchunk; p.ngchunk = pl.ngchunk;
  p.alpha_iters = d.alpha_iters; p.alpha_mode = pl.alpha_mode; p.rwpad = pl.rwpad;
  p.seed = d.seed; p.alpha_in = d.alpha;
  p.A = A; p.lda = lda; p.P = P; p.ldp = ldp;
  // 16-byte loads of A: rows start 16-byte aligned and end on a 16-byte boundary, so an
  // aligned 16-byte chunk of a row lies wholly inside or wholly past column n
  p.avec = ((lda * pl.es) % 16 == 0 && (d.n * pl.es) % 16 == 0) ? 1 : 0;
  // the 16-byte BF16X3 pass reads whole 32-row steps of A, all below n; the partial step's rows
  // are added by the pass reduction (n < 32: the element path)
  if (pl.prec == B3 && d.n < 32) p.avec = 0;
  // the 16-byte paths address up to 32 rows of A by 32-bit byte offsets from a per-step base;
  // longer rows take the element paths (64-bit addresses)
  if (lda > (int64_t(1) << 24)) p.avec = 0;
  p.ktail = (pl.prec == B3 && p.avec) ? (int)(d.n - d.n % 32) : (int)d.n;
  p.sketch = (d.flags & PSDPROJ_FLAG_SRHT) ? 1 : 0;
  p.csr = pl.csr;
  if (pl.csr) {
    p.avec = 0;
    p.ktail = (int)d.n;
    p.rowptr = csr ? csr->rowptr : nullptr;
    p.colidx = csr ? csr->colidx : nullptr;
    p.zr = region ? (void*)(region + pl.o_zr) : nullptr;
  }
  p.srht_m = 1;
  while ((int64_t(1) << p.srht_m) < d.n) ++p.srht_m;
  auto at = [&](size_t off) { return (void*)(region + off); };
  p.zm = at(pl.o_zm);
  p.zhi = (bf16*)(pl.prec == B3 ? at(pl.o_zhi) : nullptr);
  p.zlo = (bf16*)(pl.prec == B3 ? at(pl.o_zlo) : nullptr);
  p.y = at(pl.o_y); p.part = at(pl.o_part); p.q1 = at(pl.o_q1);
  p.wf = at(pl.o_wf);
  p.whi = (bf16*)(pl.prec == B3 ? at(pl.o_whi) : nullptr);
  p.wlo = (bf16*)(pl.prec == B3 ? at(pl.o_wlo) : nullptr);
  p.gpart = (double*)at(pl.o_gpart);
  p.G = (double*)at(pl.o_G); p.F = (double*)at(pl.o_F); p.C = (double*)at(pl.o_C);
  p.H = (double*)at(pl.o_H); p.V = (double*)at(pl.o_V); p.xt = (double*)at(pl.o_xt);
  p.evals = (double*)at(pl.o_evals); p.tau = (double*)at(pl.o_tau);
  p.td = (double*)at(pl.o_td); p.te = (double*)at(pl.o_te); p.wts = (double*)at(pl.o_wts);
  p.vec = (double*)at(pl.o_vec); p.vpart = (double*)at(pl.o_vpart);
  p.gvp = (double*)at(pl.o_gvp);
  p.paired = pl.paired;
  p.bh = (double*)(pl.paired ? at(pl.o_bh) : nullptr);
  p.pw = (double*)(pl.paired ? at(pl.o_pw) : nullptr);
  p.scal = (double*)at(pl.o_scal); p.iscal = (int32_t*)at(pl.o_iscal); p.drop = (int32_t*)at(pl.o_drop);
  p.res = res;
  p.npass_tiles = tiles_pass(p);
  p.gv_tiles = gemv_tile_count(p);
  p.rb_tiles = rebuild_tile_count(p);
  return p;
}

// ------------------------------------------------------------------------------ schedule
// A problem's stage list; problems of a batch are aligned step by step, inactive ones get
// zero tiles.  Pass and rebuild kernels are templated on (precision, column blocks), so the
// problems are ordered by that key and those stages launch once per key group.
static bool active_in(const Plan& pl, const Stage& st) {
  switch (st.when) {
    case W_ALL: return true;
    case W_SEQ: return pl.alpha_mode == 1 && !pl.paired;
    case W_SEQ_ITER: return pl.alpha_mode == 1 && !pl.paired && st.iter < pl.d.alpha_iters;
    case W_PAIRED: return pl.paired;
    case W_PAIRED_ITER: return pl.paired && st.iter <= pl.d.alpha_iters;
    case W_POWER: return st.iter < pl.d.q;
  }
  return false;
}

static int stage_tiles(const Prob& p, int kind) {
  switch (kind) {
    case K_SETUP: case K_ALPHA: case K_CHOL: case K_TRIDIAG: case K_FINAL: return 1;
    case K_OMEGA: return tiles_omega(p);
    case K_PINIT: case K_PINIT2: case K_ALPHA2: return tiles_vec(p);
    case K_GEMV: case K_GEMV2: return tiles_gemv(p);
    case K_GEMV_FIN: case K_GEMV2_FIN: return tiles_gemv_rows(p);
    case K_PASS: return p.csr ? tiles_pass(p) : rup(tiles_pass(p), 8);
    case K_ZT: return p.csr ? tiles_zt(p) : 0;
    case K_PRED: return tiles_reduce(p);
    case K_GRAM_SYM: return tiles_gram(p, false);
    case K_GRAM_FULL: return tiles_gram(p, true);
    case K_GRED: return (int)(((int64_t)p.rpad * p.rpad + 255) / 256);
    case K_APPLY: case K_FACTOR: return tiles_apply(p);
    case K_BISECT: return tiles_bisect(p);
    case K_INVIT: case K_BACKXF: return tiles_invit(p);
    case K_REBUILD: return tiles_rebuild(p);
  }
  return 0;
}

// max_seq / max_paired: the largest N of Alg. 5 among the problems that run its two power
// iterations one after the other / over shared products (0: none).
static void stage_list(int max_seq, int max_paired, int max_q, std::vector<Stage>& out) {
  auto add = [&](int kind, int arg, int when, int iter) { out.push_back(Stage{kind, arg, when, iter}); };
  add(K_SETUP, 0, W_ALL, 0);
  add(K_OMEGA, 0, W_ALL, 0);
  if (max_paired > 0) {
    // products j = 0 .. N with [v_j, b_j], then the second run's iterates from the basis
    add(K_PINIT2, 0, W_PAIRED, 0);
    for (int j = 0; j <= max_paired; ++j) {
      add(K_GEMV2, j, W_PAIRED_ITER, j);
      add(K_GEMV2_FIN, j, W_PAIRED_ITER, j);
    }
    add(K_ALPHA2, 0, W_PAIRED, 0);
  }
  if (max_seq > 0) {
    for (int run = 0; run < 2; ++run) {
      add(K_PINIT, run, W_SEQ, 0);
      for (int it = 0; it < max_seq; ++it) {
        add(K_GEMV, 0, W_SEQ_ITER, it);
        add(K_GEMV_FIN, 0, W_SEQ_ITER, it);
      }
      add(K_GEMV, run + 1, W_SEQ, 0);
      add(K_GEMV_FIN, run + 1, W_SEQ, 0);
    }
    add(K_ALPHA, 0, W_SEQ, 0);
  }
  // o: position of the orthonormalisation in each problem's sequence (see orth_single)
  auto orth = [&](int when, int iter, int o) {
    const int a0 = 0 + 16 * (o + 1), a1 = 1 + 16 * (o + 1);
    add(K_ZT, 0, when, iter);
    add(K_PASS, 0, when, iter);
    add(K_PRED, 0, when, iter);
    add(K_GRAM_SYM, a0, when, iter);
    add(K_GRED, a0, when, iter);
    add(K_CHOL, a0, when, iter);
    add(K_APPLY, a0, when, iter);
    add(K_GRAM_SYM, a1, when, iter);
    add(K_GRED, a1, when, iter);
    add(K_CHOL, a1, when, iter);
    add(K_APPLY, a1, when, iter);
  };
  orth(W_ALL, 0, 0);
  for (int it = 0; it < max_q; ++it) {
    orth(W_POWER, it, 1 + 2 * it);
    orth(W_POWER, it, 2 + 2 * it);
  }
  add(K_ZT, 0, W_ALL, 0);
  add(K_PASS, 0, W_ALL, 0);
  add(K_PRED, 0, W_ALL, 0);
  add(K_GRAM_FULL, 2, W_ALL, 0);
  add(K_GRED, 2, W_ALL, 0);
  add(K_TRIDIAG, 0, W_ALL, 0);
  add(K_BISECT, 0, W_ALL, 0);
  add(K_INVIT, 0, W_ALL, 0);
  add(K_BACKXF, 0, W_ALL, 0);
  add(K_FACTOR, 2, W_ALL, 0);
  add(K_REBUILD, 0, W_ALL, 0);
  add(K_FINAL, 0, W_ALL, 0);
}

void build_schedule(const Plan* const* plans, int count, Schedule& s) {
  s.order.resize(count);
  for (int i = 0; i < count; ++i) s.order[i] = i;
  // pass and rebuild kernels are grouped by (precision, column blocks); a CSR operand takes
  // the sparse pass, so it is a key of its own (precision + 8)
  auto gkey = [&](int i) { return plans[i]->prec + 8 * plans[i]->csr; };
  std::stable_sort(s.order.begin(), s.order.end(), [&](int a, int b) {
    if (gkey(a) != gkey(b)) return gkey(a) < gkey(b);
    return plans[a]->ncb < plans[b]->ncb;
  });
  // groups of equal (key, ncb), as ranges of the sorted order
  s.groups.clear();
  for (int i = 0; i < count;) {
    int j = i;
    while (j < count && gkey(s.order[j]) == gkey(s.order[i]) && plans[s.order[j]]->ncb == plans[s.order[i]]->ncb) ++j;
    s.groups.push_back({i, j - i, gkey(s.order[i]), plans[s.order[i]]->ncb});
    i = j;
  }
  int max_seq = 0, max_paired = 0, max_q = 0;
  for (int i = 0; i < count; ++i) {
    if (plans[i]->paired) max_paired = std::max(max_paired, plans[i]->d.alpha_iters);
    else if (plans[i]->alpha_mode == 1) max_seq = std::max(max_seq, plans[i]->d.alpha_iters);
    max_q = std::max(max_q, plans[i]->d.q);
  }
  std::vector<Stage> stages;
  stage_list(max_seq, max_paired, max_q, stages);
  // tile counts need only the sizes, so a Prob without pointers is enough here
  std::vector<Prob> shape(count);
  for (int i = 0; i < count; ++i) shape[i] = make_prob(*plans[s.order[i]], nullptr, nullptr, 0, nullptr, 0, nullptr);
  s.launches.clear();
  s.tdata.clear();
  for (const Stage& st : stages) {
    const bool grouped = (st.kind == K_PASS || st.kind == K_REBUILD);
    const int ng = grouped ? (int)s.groups.size() : 1;
    for (int g = 0; g < ng; ++g) {
      const int first = grouped ? s.groups[g].first : 0;
      const int cnt = grouped ? s.groups[g].count : count;
      LaunchRec L;
      L.kind = st.kind; L.arg = st.arg; L.first = first; L.count = cnt;
      L.prec = grouped ? s.groups[g].prec : 0;
      L.ncb = grouped ? s.groups[g].ncb : 0;
      L.toff = (int)s.tdata.size();
      int tot = 0;
      L.maxnb = 1;
      s.tdata.push_back(0);
      for (int i = 0; i < cnt; ++i) {
        const Plan& pl = *plans[s.order[first + i]];
        if (active_in(pl, st)) {
          tot += stage_tiles(shape[first + i], st.kind);
          L.maxnb = std::max(L.maxnb, pl.rpad / 16);
        }
        s.tdata.push_back(tot);
      }
      L.grid = (unsigned)tot;
      if (tot > 0) s.launches.push_back(L);
      else s.tdata.resize(L.toff);
    }
  }
  s.prob_bytes = al256((size_t)count * sizeof(Prob));
  s.header_bytes = al256(s.prob_bytes + s.tdata.size() * sizeof(int));
}

// ------------------------------------------------------------------------------ upload ring
// Small host-to-device uploads (descriptors, tile tables) go through pinned slots; each slot
// is reused only after the event of its previous copy has completed.
namespace {
struct Slot { void* host = nullptr; size_t cap = 0; hipEvent_t ev = nullptr; bool used = false; };
struct Ring {
  std::mutex mu;
  std::vector<Slot> slots;
  size_t next = 0;
};
Ring& ring_for(int dev) {
  static std::mutex gmu;
  static std::vector<Ring*> rings;
  std::lock_guard<std::mutex> g(gmu);
  if ((int)rings.size() <= dev) rings.resize(dev + 1, nullptr);
  if (!rings[dev]) { rings[dev] = new Ring(); rings[dev]->slots.resize(16); }
  return *rings[dev];
}
}  // namespace

psdproj_status upload(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PSDPROJ_E_DEVICE;
  Ring& R = ring_for(dev);
  std::lock_guard<std::mutex> g(R.mu);
  Slot& s = R.slots[R.next];
  R.next = (R.next + 1) % R.slots.size();
  if (s.used && hipEventSynchronize(s.ev) != hipSuccess) return PSDPROJ_E_DEVICE;
  if (s.cap < bytes) {
    if (s.host) hipHostFree(s.host);
    s.host = nullptr;
    size_t cap = std::max(bytes, (size_t)65536);
    if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess) { s.cap = 0; return PSDPROJ_E_NOMEM; }
    s.cap = cap;
  }
  if (!s.ev && hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) return PSDPROJ_E_DEVICE;
  std::memcpy(s.host, src, bytes);
  if (hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return PSDPROJ_E_DEVICE;
  if (hipEventRecord(s.ev, stream) != hipSuccess) return PSDPROJ_E_DEVICE;
  s.used = true;
  return PSDPROJ_OK;
}

static void kernel_init_once() {
  static std::mutex mu;
  static std::vector<bool> done;
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, false);
  if (!done[dev]) { rebuild_init(); apply_init(); pass_init(); done[dev] = true; }
}

// ------------------------------------------------------------------------------ kernel timing
namespace {
struct Prof {
  std::mutex mu;
  bool on = false;
  uint64_t kinds = ~0ull;   // kinds timed while on (bit k: kind k)
  struct Pending { int kind; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[K_NKINDS] = {};
  int64_t count[K_NKINDS] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void resolve() {  // caller holds mu
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        total_ms[p.kind] += ms;
        count[p.kind] += 1;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};
Prof& prof() { static Prof P; return P; }
}  // namespace

ProfScope::ProfScope(int k, hipStream_t s) : kind(k), stream(s) {
  Prof& PR = prof();
  std::lock_guard<std::mutex> g(PR.mu);
  if (!PR.on || !((PR.kinds >> kind) & 1ull)) return;
  a = PR.get();
  b = PR.get();
  if (a) hipEventRecord(a, stream);
}

ProfScope::~ProfScope() {
  if (!a || !b) return;
  hipEventRecord(b, stream);
  Prof& PR = prof();
  std::lock_guard<std::mutex> g(PR.mu);
  PR.pending.push_back({kind, a, b});
}

// Enqueue every launch of a schedule whose header (Prob array + tile tables) is at `hdr`.
psdproj_status enqueue(const Schedule& s, unsigned char* hdr, hipStream_t stream, bool allow_timing) {
  kernel_init_once();
  const Prob* probs = (const Prob*)hdr;
  const int* tdev = (const int*)(hdr + s.prob_bytes);
  Prof& PR = prof();
  std::unique_lock<std::mutex> plock(PR.mu, std::defer_lock);
  bool timing_on = false;
  uint64_t timed_kinds = 0;
  if (allow_timing) {
    std::lock_guard<std::mutex> g(PR.mu);
    timing_on = PR.on;
    timed_kinds = PR.kinds;
  }
  for (const LaunchRec& R : s.launches) {
    Launch L{R.grid, probs + R.first, tdev + R.toff, R.count, stream, R.maxnb};
    hipEvent_t ea = nullptr, eb = nullptr;
    const bool timing = timing_on && ((timed_kinds >> R.kind) & 1ull);
    if (timing) {
      plock.lock();
      ea = PR.get();
      eb = PR.get();
      plock.unlock();
      if (ea) hipEventRecord(ea, stream);
    }
    switch (R.kind) {
      case K_SETUP: launch_setup(L); break;
      case K_OMEGA: launch_omega(L); break;
      case K_PINIT: launch_power_init(L, R.arg); break;
      case K_GEMV: launch_gemv(L, R.arg); break;
      case K_GEMV_FIN: launch_gemv_finish(L, R.arg); break;
      case K_ALPHA: launch_alpha(L); break;
      case K_PINIT2: launch_power_init2(L); break;
      case K_GEMV2: launch_gemv2(L, R.arg); break;
      case K_GEMV2_FIN: launch_gemv2_finish(L, R.arg); break;
      case K_ALPHA2: launch_alpha2(L); break;
      case K_PASS: (R.prec >= 8) ? launch_spmm(L) : launch_pass(L, R.prec, R.ncb); break;
      case K_ZT: launch_zt(L); break;
      case K_PRED: launch_pass_reduce(L); break;
      case K_GRAM_SYM: case K_GRAM_FULL: launch_gram(L, R.arg); break;
      case K_GRED: launch_gram_reduce(L, R.arg); break;
      case K_CHOL: launch_chol(L, R.arg); break;
      case K_APPLY: case K_FACTOR: launch_apply(L, R.arg); break;
      case K_TRIDIAG: launch_tridiag(L); break;
      case K_BISECT: launch_bisect(L); break;
      case K_INVIT: launch_invit(L); break;
      case K_BACKXF: launch_backxf(L); break;
      case K_REBUILD: launch_rebuild(L, R.prec & 7); break;
      case K_FINAL: launch_finalize(L); break;
    }
    if (hipGetLastError() != hipSuccess) return PSDPROJ_E_DEVICE;
    if (timing && ea && eb) {
      hipEventRecord(eb, stream);
      plock.lock();
      PR.pending.push_back({R.kind, ea, eb});
      plock.unlock();
    }
  }
  return PSDPROJ_OK;
}

static const char* const KIND_NAMES[K_NKINDS] = {
    "k_setup", "k_omega", "k_power_init", "k_gemv", "k_alpha", "k_pass", "k_pass_reduce", "k_gram",
    "k_gram_full", "k_gram_reduce", "k_chol", "k_apply", "k_tridiag", "k_bisect", "k_invit", "k_rebuild",
    "k_finalize", "k_gemv_finish", "k_apply_factor", "k_backxf", "k_zt", "k_sdls_form", "k_sdls_trace",
    "k_sdls_update", "k_gemm64", "k_exact_misc", "k_power_init2", "k_gemv2", "k_gemv2_finish", "k_alpha2"};

// ------------------------------------------------------------------------------ HIP graphs
// A schedule's launches reach the problems only through the header at `hdr` (each kernel
// takes a pointer to its problems' descriptors and tile table there), so one captured launch
// sequence serves every run with the same schedule and the same header address, whatever A, P
// and the results are: the header is rewritten before each replay.  The sequence holds kernel
// nodes only.
psdproj_status capture_schedule(const Schedule& s, unsigned char* hdr, hipGraph_t* graph, hipGraphExec_t* exec) {
  *graph = nullptr;
  *exec = nullptr;
  kernel_init_once();   // function attributes are set before the capture, not inside it
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return PSDPROJ_E_DEVICE;
  psdproj_status st = PSDPROJ_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(cs);
    return PSDPROJ_E_DEVICE;
  }
  st = enqueue(s, hdr, cs, /*allow_timing=*/false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  hipStreamDestroy(cs);
  if (st != PSDPROJ_OK || e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    return PSDPROJ_E_DEVICE;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x) {
    hipGraphDestroy(g);
    return PSDPROJ_E_DEVICE;
  }
  *graph = g;
  *exec = x;
  return PSDPROJ_OK;
}

namespace {
// Captured sequences of the runs issued through run_group (psdproj_run, psdproj_batch, the
// server), keyed by (device, header address, launch list).  A key is captured the second time it
// is seen, so one-off batches pay no instantiation; at most GRAPH_CACHE entries per process, the
// least recently used one evicted after its last replay has completed.
constexpr size_t GRAPH_CACHE = 64;
struct CachedGraph {
  std::vector<int64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;   // recorded after the latest replay
  uint64_t last = 0;
  int seen = 0;
};
struct GraphCache {
  std::mutex mu;
  std::vector<CachedGraph> entries;
  uint64_t clock = 0;
  int mode = -1;               // -1: not read yet; 0: off (PSDPROJ_GRAPHS=0); 1: on
  int64_t replays = 0, captures = 0;
};
GraphCache& graph_cache() { static GraphCache C; return C; }

std::vector<int64_t> schedule_key(const Schedule& s, const unsigned char* hdr) {
  int dev = 0;
  hipGetDevice(&dev);
  std::vector<int64_t> k;
  k.reserve(4 + 9 * s.launches.size());
  k.push_back(dev);
  k.push_back((int64_t)(uintptr_t)hdr);
  k.push_back((int64_t)s.prob_bytes);
  k.push_back((int64_t)s.launches.size());
  for (const LaunchRec& R : s.launches) {
    k.push_back(R.kind); k.push_back(R.arg); k.push_back(R.first); k.push_back(R.count); k.push_back(R.prec);
    k.push_back(R.ncb); k.push_back(R.toff); k.push_back(R.maxnb); k.push_back(R.grid);
  }
  return k;
}

void drop_entry(CachedGraph& e) {
  if (e.done) { hipEventSynchronize(e.done); hipEventDestroy(e.done); }
  if (e.exec) hipGraphExecDestroy(e.exec);
  if (e.graph) hipGraphDestroy(e.graph);
  e = CachedGraph();
}
}  // namespace

// Enqueue a schedule whose header is already at `hdr`: a replay of its captured sequence when
// there is one, otherwise the launches themselves (and a capture on the key's second run).
// Kernel timing, when enabled, needs the launches themselves.
psdproj_status launch_schedule(const Schedule& s, unsigned char* hdr, hipStream_t stream) {
  GraphCache& C = graph_cache();
  bool timing = false;
  {
    Prof& PR = prof();
    std::lock_guard<std::mutex> g(PR.mu);
    timing = PR.on;
  }
  std::unique_lock<std::mutex> lk(C.mu);
  if (C.mode < 0) {
    const char* env = std::getenv("PSDPROJ_GRAPHS");
    C.mode = (env && env[0] == '0') ? 0 : 1;
  }
  if (C.mode == 0 || timing || s.launches.empty()) {
    lk.unlock();
    return enqueue(s, hdr, stream);
  }
  const std::vector<int64_t> key = schedule_key(s, hdr);
  CachedGraph* hit = nullptr;
  for (auto& e : C.entries)
    if (e.key == key) { hit = &e; break; }
  if (!hit) {
    if (C.entries.size() >= GRAPH_CACHE) {
      auto lru = std::min_element(C.entries.begin(), C.entries.end(),
                                  [](const CachedGraph& a, const CachedGraph& b) { return a.last < b.last; });
      drop_entry(*lru);
      *lru = C.entries.back();
      C.entries.pop_back();
    }
    C.entries.push_back(CachedGraph());
    hit = &C.entries.back();
    hit->key = key;
  }
  hit->last = ++C.clock;
  hit->seen += 1;
  if (!hit->exec && hit->seen >= 2) {
    if (capture_schedule(s, hdr, &hit->graph, &hit->exec) == PSDPROJ_OK &&
        hipEventCreateWithFlags(&hit->done, hipEventDisableTiming) == hipSuccess) {
      C.captures += 1;
    } else {
      drop_entry(*hit);
      hit->key = key;
      hit->seen = -1000000;   // never captured again; launched directly
    }
  }
  if (!hit->exec) {
    lk.unlock();
    return enqueue(s, hdr, stream);
  }
  if (hipGraphLaunch(hit->exec, stream) != hipSuccess) return PSDPROJ_E_DEVICE;
  if (hipEventRecord(hit->done, stream) != hipSuccess) return PSDPROJ_E_DEVICE;
  C.replays += 1;
  return PSDPROJ_OK;
}

psdproj_status check_operands(const Plan& pl, const void* A, int64_t lda, const void* P, int64_t ldp) {
  const int64_t n = pl.d.n;
  if (pl.csr) return PSDPROJ_E_INVALID;   // a sparse operand goes through psdproj_run_csr
  if (!A || !P) return PSDPROJ_E_INVALID;
  if (lda < n || ldp < n) return PSDPROJ_E_INVALID;
  if (((uintptr_t)A & 15) || ((uintptr_t)P & 15)) return PSDPROJ_E_INVALID;
  const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (uintptr_t)(((n - 1) * lda + n) * pl.es);
  const uintptr_t p0 = (uintptr_t)P, p1 = p0 + (uintptr_t)(((n - 1) * ldp + n) * pl.es);
  const bool overlap = (a0 < p1) && (p0 < a1);
  if (overlap && !(A == P && lda == ldp)) return PSDPROJ_E_INVALID;
  return PSDPROJ_OK;
}

psdproj_status make_header(int count, const Plan* const* plans, const void* const* A, const int64_t* lda,
                           void* const* P, const int64_t* ldp, unsigned char* ws, size_t ws_bytes,
                           psdproj_result* results, Schedule& s, std::vector<unsigned char>& host,
                           const Csr* csr = nullptr) {
  build_schedule(plans, count, s);
  size_t need = s.header_bytes;
  for (int i = 0; i < count; ++i) need += plans[i]->region;
  if (ws_bytes < need) return PSDPROJ_E_NOMEM;
  host.assign(s.header_bytes, 0);
  Prob* hp = (Prob*)host.data();
  // regions follow the header in the caller's order
  std::vector<size_t> roff(count);
  size_t o = s.header_bytes;
  for (int i = 0; i < count; ++i) { roff[i] = o; o += plans[i]->region; }
  for (int k = 0; k < count; ++k) {
    const int i = s.order[k];
    hp[k] = make_prob(*plans[i], ws + roff[i], A[i], lda[i], P[i], ldp[i], results + i, csr ? csr + i : nullptr);
  }
  std::memcpy(host.data() + s.prob_bytes, s.tdata.data(), s.tdata.size() * sizeof(int));
  return PSDPROJ_OK;
}

psdproj_status run_group(int count, const Plan* const* plans, const void* const* A, const int64_t* lda,
                         void* const* P, const int64_t* ldp, unsigned char* ws, size_t ws_bytes,
                         psdproj_result* results, hipStream_t stream, const Csr* csr) {
  Schedule s;
  std::vector<unsigned char> host;
  psdproj_status st = make_header(count, plans, A, lda, P, ldp, ws, ws_bytes, results, s, host, csr);
  if (st != PSDPROJ_OK) return st;
  st = upload(ws, host.data(), s.header_bytes, stream);
  if (st != PSDPROJ_OK) return st;
  return launch_schedule(s, ws, stream);
}

// ------------------------------------------------------------------------------ static scratch
// Header words written by a kernel that carries them in its arguments: no host staging buffer,
// nothing allocated, an ordinary kernel on the stream.
constexpr int FILL_WORDS = 256;
struct FillChunk { uint32_t w[FILL_WORDS]; };

__global__ __launch_bounds__(FILL_WORDS) void k_fill_words(uint32_t* __restrict__ dst, FillChunk c, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.w[i];
}

static psdproj_status fill_by_kernel(unsigned char* dst, const void* src, size_t bytes, hipStream_t stream) {
  const unsigned char* s = (const unsigned char*)src;
  for (size_t o = 0; o < bytes; o += FILL_WORDS * 4) {
    FillChunk c;
    const size_t nb = std::min(bytes - o, (size_t)FILL_WORDS * 4);   // bytes is a multiple of 4
    std::memcpy(c.w, s + o, nb);
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(FILL_WORDS), 0, stream, (uint32_t*)(dst + o), c, (int)(nb / 4));
    if (hipGetLastError() != hipSuccess) return PSDPROJ_E_DEVICE;
  }
  return PSDPROJ_OK;
}

// The workspace of psdproj_run_static: one array per device, alive until the process ends.  In
// host code `scratch` names a host-side stand-in, not the device array: its device address comes
// from hipGetSymbolAddress, once per device with that device current, and only that address is
// ever handed to a kernel.
static_assert(PSDPROJ_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[PSDPROJ_STATIC_SCRATCH_BYTES];

static unsigned char* scratch_address() {
  static std::mutex mu;
  static std::vector<unsigned char*> addr;   // per device; null until looked up
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    addr[dev] = (unsigned char*)ptr;
  }
  return addr[dev];
}

psdproj_status run_static(const Plan& pl, const void* A, int64_t lda, void* P, int64_t ldp, psdproj_result* result,
                          hipStream_t stream) {
  if (pl.header_single + pl.region > (size_t)PSDPROJ_STATIC_SCRATCH_BYTES) return PSDPROJ_E_SCRATCH;
  unsigned char* ws = scratch_address();
  if (!ws) return PSDPROJ_E_DEVICE;
  // the kernels initialise every part of the workspace they read (counters in k_setup, whole
  // panels in k_omega), so the previous call's contents need no clearing
  const Prob pr = make_prob(pl, ws + pl.header_single, A, lda, P, ldp, result);
  static_assert(sizeof(Prob) % 4 == 0, "header words");
  psdproj_status st = fill_by_kernel(ws, &pr, sizeof(Prob), stream);
  if (st != PSDPROJ_OK) return st;
  st = fill_by_kernel(ws + pl.single.prob_bytes, pl.single.tdata.data(), pl.single.tdata.size() * sizeof(int), stream);
  if (st != PSDPROJ_OK) return st;
  return enqueue(pl.single, ws, stream, /*allow_timing=*/false);
}

}  // namespace psd

// ================================================================================ C ABI
using namespace psd;

extern "C" {

psdproj_status psdproj_plan(const psdproj_desc* desc, psdproj_plan_t* out, size_t* workspace_bytes) {
  if (!desc || !out) return PSDPROJ_E_INVALID;
  *out = nullptr;
  Plan* pl = new (std::nothrow) Plan();
  if (!pl) return PSDPROJ_E_NOMEM;
  psdproj_status st = make_plan(desc, *pl);
  if (st != PSDPROJ_OK) { delete pl; return st; }
  *out = (psdproj_plan_t)pl;
  if (workspace_bytes) *workspace_bytes = pl->header_single + pl->region;
  return PSDPROJ_OK;
}

void psdproj_plan_destroy(psdproj_plan_t plan) { delete (Plan*)plan; }

psdproj_status psdproj_plan_layout(psdproj_plan_t plan, psdproj_layout* out) {
  if (!plan || !out) return PSDPROJ_E_INVALID;
  const Plan& pl = *(const Plan*)plan;
  const size_t h = pl.header_single;
  out->r = pl.r; out->r_pad = pl.rpad; out->panel_ld = pl.ld; out->split_k = pl.split;
  out->panel_elem_bytes = pl.es;
  out->omega = h + pl.o_zm;       // holds Omega until the first orthonormalisation
  out->q_panel = h + pl.o_zm;     // holds Q after the last orthonormalisation
  out->compressed = h + pl.o_C;
  out->evals = h + pl.o_evals;
  out->weights = h + pl.o_wts;
  out->factor = h + pl.o_wf;
  out->power_vec = h + pl.o_vec;
  out->y_panel = h + pl.o_y;
  out->gram = h + pl.o_G;
  out->total = h + pl.region;
  return PSDPROJ_OK;
}

psdproj_status psdproj_run(psdproj_plan_t plan, const void* A, int64_t lda, void* P, int64_t ldp, void* workspace,
                           psdproj_result* result_dev, psdproj_stream_t stream) {
  if (!plan || !workspace || !result_dev) return PSDPROJ_E_INVALID;
  if ((uintptr_t)workspace & 255) return PSDPROJ_E_INVALID;
  const Plan* pl = (const Plan*)plan;
  psdproj_status st = check_operands(*pl, A, lda, P, ldp);
  if (st != PSDPROJ_OK) return st;
  return run_group(1, &pl, &A, &lda, &P, &ldp, (unsigned char*)workspace, pl->header_single + pl->region,
                   result_dev, (hipStream_t)stream);
}

psdproj_status psdproj_run_csr(psdproj_plan_t plan, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                               int64_t nnz, void* P, int64_t ldp, void* workspace, psdproj_result* result_dev,
                               psdproj_stream_t stream) {
  if (!plan || !row_ptr || !col_idx || !vals || !P || !workspace || !result_dev || nnz < 0) return PSDPROJ_E_INVALID;
  const Plan* pl = (const Plan*)plan;
  if (!pl->csr || ldp < pl->d.n || ((uintptr_t)P & 15) || ((uintptr_t)workspace & 255)) return PSDPROJ_E_INVALID;
  if (P == vals) return PSDPROJ_E_INVALID;
  const Csr c{row_ptr, col_idx};
  const void* Av = vals;
  void* Pv = P;
  const int64_t lda = nnz;   // the descriptor carries nnz in lda for a sparse operand
  return run_group(1, &pl, &Av, &lda, &Pv, &ldp, (unsigned char*)workspace, pl->header_single + pl->region,
                   result_dev, (hipStream_t)stream, &c);
}

psdproj_status psdproj_run_static(psdproj_plan_t plan, const void* A, int64_t lda, void* P, int64_t ldp,
                                  psdproj_result* result_dev, psdproj_stream_t stream) {
  if (!plan || !result_dev) return PSDPROJ_E_INVALID;
  const Plan* pl = (const Plan*)plan;
  psdproj_status st = check_operands(*pl, A, lda, P, ldp);
  if (st != PSDPROJ_OK) return st;
  return run_static(*pl, A, lda, P, ldp, result_dev, (hipStream_t)stream);
}

psdproj_status psdproj_static_scratch_bytes(psdproj_plan_t plan, size_t* needed, size_t* capacity) {
  if (!plan || !needed || !capacity) return PSDPROJ_E_INVALID;
  const Plan* pl = (const Plan*)plan;
  *needed = pl->header_single + pl->region;
  *capacity = PSDPROJ_STATIC_SCRATCH_BYTES;
  return PSDPROJ_OK;
}

psdproj_status psdproj_batch_workspace(int32_t count, const psdproj_plan_t* plans, size_t* bytes) {
  if (count < 1 || !plans || !bytes) return PSDPROJ_E_INVALID;
  std::vector<const Plan*> pls(count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return PSDPROJ_E_INVALID;
    pls[i] = (const Plan*)plans[i];
  }
  Schedule s;
  build_schedule(pls.data(), count, s);
  size_t need = s.header_bytes;
  for (int i = 0; i < count; ++i) need += pls[i]->region;
  *bytes = need;
  return PSDPROJ_OK;
}

psdproj_status psdproj_batch(int32_t count, const psdproj_plan_t* plans, const void* const* A, const int64_t* lda,
                             void* const* P, const int64_t* ldp, void* workspace, size_t workspace_bytes,
                             psdproj_result* results_dev, psdproj_stream_t stream) {
  if (count < 1 || !plans || !A || !lda || !P || !ldp || !workspace || !results_dev) return PSDPROJ_E_INVALID;
  if ((uintptr_t)workspace & 255) return PSDPROJ_E_INVALID;
  std::vector<const Plan*> pls(count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return PSDPROJ_E_INVALID;
    pls[i] = (const Plan*)plans[i];
    psdproj_status st = check_operands(*pls[i], A[i], lda[i], P[i], ldp[i]);
    if (st != PSDPROJ_OK) return st;
  }
  return run_group(count, pls.data(), A, lda, P, ldp, (unsigned char*)workspace, workspace_bytes, results_dev,
                   (hipStream_t)stream);
}

struct psdproj_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

psdproj_status psdproj_graph_create(int32_t count, const psdproj_plan_t* plans, const void* const* A,
                                    const int64_t* lda, void* const* P, const int64_t* ldp, void* workspace,
                                    size_t workspace_bytes, psdproj_result* results_dev, psdproj_graph_t* out) {
  if (!out) return PSDPROJ_E_INVALID;
  *out = nullptr;
  if (count < 1 || !plans || !A || !lda || !P || !ldp || !workspace || !results_dev) return PSDPROJ_E_INVALID;
  if ((uintptr_t)workspace & 255) return PSDPROJ_E_INVALID;
  std::vector<const Plan*> pls(count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return PSDPROJ_E_INVALID;
    pls[i] = (const Plan*)plans[i];
    psdproj_status st = check_operands(*pls[i], A[i], lda[i], P[i], ldp[i]);
    if (st != PSDPROJ_OK) return st;
  }
  Schedule s;
  std::vector<unsigned char> host;
  unsigned char* ws = (unsigned char*)workspace;
  psdproj_status st = make_header(count, pls.data(), A, lda, P, ldp, ws, workspace_bytes, results_dev, s, host);
  if (st != PSDPROJ_OK) return st;
  // the header is written once, now; the captured sequence only reads it
  if (hipMemcpy(ws, host.data(), s.header_bytes, hipMemcpyHostToDevice) != hipSuccess) return PSDPROJ_E_DEVICE;
  psdproj_graph_s* g = new (std::nothrow) psdproj_graph_s();
  if (!g) return PSDPROJ_E_NOMEM;
  st = capture_schedule(s, ws, &g->graph, &g->exec);
  if (st != PSDPROJ_OK) { delete g; return st; }
  *out = g;
  return PSDPROJ_OK;
}

psdproj_status psdproj_graph_launch(psdproj_graph_t graph, psdproj_stream_t stream) {
  if (!graph || !graph->exec) return PSDPROJ_E_INVALID;
  return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? PSDPROJ_OK : PSDPROJ_E_DEVICE;
}

void psdproj_graph_destroy(psdproj_graph_t graph) {
  if (!graph) return;
  if (graph->exec) hipGraphExecDestroy(graph->exec);
  if (graph->graph) hipGraphDestroy(graph->graph);
  delete graph;
}

psdproj_status psdproj_tile_override(int32_t precision, int32_t split) {
  if (precision < PSDPROJ_FP64 || precision > PSDPROJ_BF16X3 || split < 0 || split > MAX_SPLIT)
    return PSDPROJ_E_INVALID;
  std::lock_guard<std::mutex> g(tile_mu);
  tile_override[precision] = split;
  return PSDPROJ_OK;
}

psdproj_status psdproj_graph_stats(int64_t* captures, int64_t* replays) {
  if (!captures || !replays) return PSDPROJ_E_INVALID;
  GraphCache& C = graph_cache();
  std::lock_guard<std::mutex> g(C.mu);
  *captures = C.captures;
  *replays = C.replays;
  return PSDPROJ_OK;
}

psdproj_status psdproj_philox_words(uint64_t seed, uint32_t stream_id, uint64_t c0, int64_t count, uint32_t* out_dev,
                                    psdproj_stream_t stream) {
  if (count < 0 || (count > 0 && !out_dev)) return PSDPROJ_E_INVALID;
  launch_words(seed, stream_id, c0, count, out_dev, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_E_DEVICE;
}

psdproj_status psdproj_gaussian(uint64_t seed, uint32_t stream_id, uint64_t start, int64_t count, double* out_dev,
                                psdproj_stream_t stream) {
  if (count < 0 || (count > 0 && !out_dev)) return PSDPROJ_E_INVALID;
  launch_gauss(seed, stream_id, start, count, out_dev, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_E_DEVICE;
}

psdproj_status psdproj_srht_matrix(uint64_t seed, int64_t n, int32_t r, double* out_dev, psdproj_stream_t stream) {
  if (n < 1 || n > (1 << 20) || r < 1 || r > n || !out_dev) return PSDPROJ_E_INVALID;
  launch_srht(seed, (int)n, r, out_dev, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PSDPROJ_OK : PSDPROJ_E_DEVICE;
}

const char* psdproj_status_str(psdproj_status s) {
  switch (s) {
    case PSDPROJ_OK: return "ok";
    case PSDPROJ_E_INVALID: return "invalid argument";
    case PSDPROJ_E_ALPHA: return "estimated alpha is not positive and finite";
    case PSDPROJ_E_NONFINITE: return "non-finite value in a Gram or compressed matrix";
    case PSDPROJ_E_BREAKDOWN: return "reserved (never returned)";
    case PSDPROJ_E_NOMEM: return "workspace too small or allocation failed";
    case PSDPROJ_E_BUDGET: return "request exceeds the server HBM budget";
    case PSDPROJ_E_DEVICE: return "HIP runtime error";
    case PSDPROJ_E_PENDING: return "pending";
    case PSDPROJ_E_TIMEOUT: return "timed out";
    case PSDPROJ_E_SCRATCH: return "problem needs more workspace than the static scratch array holds";
  }
  return "unknown status";
}

int32_t psdproj_abi_version(void) { return PSDPROJ_ABI_VERSION; }

psdproj_status psdproj_profile_enable(int32_t enable) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = enable != 0;
  return PSDPROJ_OK;
}

psdproj_status psdproj_profile_select(uint64_t kinds) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.kinds = kinds;
  return PSDPROJ_OK;
}

psdproj_status psdproj_profile_reset(void) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.resolve();
  for (int k = 0; k < K_NKINDS; ++k) { P.total_ms[k] = 0.0; P.count[k] = 0; }
  return PSDPROJ_OK;
}

psdproj_status psdproj_profile_read(int32_t kind, double* total_ms, int64_t* launches) {
  if (kind < 0 || kind >= K_NKINDS || !total_ms || !launches) return PSDPROJ_E_INVALID;
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.resolve();
  *total_ms = P.total_ms[kind];
  *launches = P.count[kind];
  return PSDPROJ_OK;
}

int32_t psdproj_kernel_kinds(void) { return K_NKINDS; }

const char* psdproj_kernel_name(int32_t kind) {
  if (kind < 0 || kind >= K_NKINDS) return "";
  return KIND_NAMES[kind];
}

}  // extern "C"
