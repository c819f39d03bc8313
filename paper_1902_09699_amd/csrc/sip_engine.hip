// Host engine and C ABI of libsip: instance layout in a device arena, work
// tables, HIP-graph capture of iterations, admission / retirement of
// resident instances (the batched and served forms), results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "sip_internal.h"

// Device memory of sip_project_noalloc: every call on a GPU carves its
// descriptor, scalars, instance workspace, work tables and partial sums
// from this array (one copy per GPU, held until the process ends).
static constexpr long long kScratchBytes = 128ll << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace sip {

struct Tables;
// The kernels are built twice: FP64 accumulation (r64) and FP32 (r32).
namespace r64 {
template <typename T> void launch_iteration(hipStream_t st, const Tables& t, const Opts& o);
template <typename T> void launch_init(hipStream_t st, const InstDesc* D, int inst, int64_t N);
void launch_zero(hipStream_t st, uint32_t* a, int64_t n);
void launch_zero(hipStream_t st, double* a, int64_t n);
template <typename T> void launch_phase(hipStream_t st, const Tables& t, const Opts& o, int phase);
void launch_copy(hipStream_t st, void* dst, const void* src, int64_t n16);
}  // namespace r64
namespace r32 {
template <typename T> void launch_iteration(hipStream_t st, const Tables& t, const Opts& o);
template <typename T> void launch_phase(hipStream_t st, const Tables& t, const Opts& o, int phase);
}  // namespace r32
using r64::launch_init;
using r64::launch_zero;
using r64::launch_copy;
int32_t launch_dykstra(hipStream_t st, int p, const void* const* y, void* const* v, const double* w, void* x,
                       int64_t n, bool f64);
// level transfer of multilevel PARSDMM
template <typename T>
void launch_restrict(hipStream_t st, const T* src, const int64_t (&n)[3], T* dst, const int64_t (&c)[3]);
template <typename T>
void launch_prolong(hipStream_t st, const T* src, const int64_t (&s)[3], int64_t ssz, int64_t ssy, T* dst,
                    const int64_t (&f)[3], const int64_t (&d)[3], int64_t dsz, int64_t dsy, int stag);

namespace {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------- arena

// First-fit allocator over one device block (the batch's own allocation, or
// a borrowed block that it never frees); admission never calls the HIP
// allocator.
class Arena {
 public:
  bool init(int64_t bytes) {
    if (bytes <= 0) return false;
    if (hipMalloc(&base_, (size_t)bytes) != hipSuccess) { base_ = nullptr; return false; }
    owned_ = true;
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  bool borrow(char* base, int64_t bytes) {
    if (bytes <= 0 || !base) return false;
    base_ = base;
    owned_ = false;
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  ~Arena() { if (base_ && owned_) (void)hipFree(base_); }
  char* alloc(int64_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p) {
    const int64_t off = p - base_;
    auto u = used_.find(off);
    if (u == used_.end()) return;
    int64_t len = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) { len += nx->second; nx = free_.erase(nx); }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) { pv->second += len; return; }
    }
    free_[off] = len;
  }
  int64_t free_bytes() const { int64_t s = 0; for (auto& f : free_) s += f.second; return s; }

 private:
  char* base_ = nullptr;
  bool owned_ = false;
  int64_t size_ = 0;
  std::map<int64_t, int64_t> free_, used_;
};

// ------------------------------------------------------ set / grid helpers

struct OpInfo { int ncomp; int axis[3]; };

// Internal axes: 0 = z, 1 = y, 2 = x; a 2D grid has ny = 1.
bool op_info(int ndim, int op, OpInfo& oi) {
  oi.ncomp = 0;
  auto add = [&](int a) { oi.axis[oi.ncomp++] = a; };
  switch (op) {
    case SIP_OP_I: oi.ncomp = 1; oi.axis[0] = -1; return true;
    case SIP_OP_DZ: add(0); return true;
    case SIP_OP_DY: if (ndim != 3) return false; add(1); return true;
    case SIP_OP_DX: add(2); return true;
    case SIP_OP_GRAD: add(0); if (ndim == 3) add(1); add(2); return true;
    case SIP_OP_LAT: if (ndim == 3) add(1); add(2); return true;
    default: return false;
  }
}

void internal_dims(const sip_grid& g, int64_t n[3], double h[3]) {
  if (g.ndim == 3) {
    for (int a = 0; a < 3; ++a) { n[a] = g.n[a]; h[a] = g.h[a]; }
  } else {
    n[0] = g.n[0]; n[1] = 1; n[2] = g.n[1];
    h[0] = g.h[0]; h[1] = 1.0; h[2] = g.h[1];
  }
}

// Internal grid axis of a sip_line (internal form (z, y, x); 2D has y = 1).
int line_axis_of(int32_t line) { return line == SIP_LINE_Z ? 0 : (line == SIP_LINE_Y ? 1 : 2); }

int64_t rows_of(const sip_grid& g, const sip_set& s) {
  OpInfo oi;
  if (!op_info(g.ndim, s.op, oi)) return -1;
  int64_t n[3]; double h[3];
  internal_dims(g, n, h);
  const int64_t N = n[0] * n[1] * n[2];
  if (oi.axis[0] < 0) return N;
  int64_t rows = 0;
  for (int c = 0; c < oi.ncomp; ++c) rows += N / n[oi.axis[c]] * (n[oi.axis[c]] - 1);
  return rows;
}

int32_t validate(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o) {
  if (!g || !o || (nsets > 0 && !sets)) return SIP_EINVAL;
  if (g->ndim != 2 && g->ndim != 3) return SIP_EINVAL;
  if (nsets < 0 || nsets > SIP_MAX_SETS) return SIP_EINVAL;
  if (o->field != SIP_F32 && o->field != SIP_F64) return SIP_EINVAL;
  if (o->reduce != SIP_F64 && !(o->reduce == SIP_F32 && o->field == SIP_F32)) return SIP_EINVAL;
  int64_t N = 1;
  for (int a = 0; a < g->ndim; ++a) {
    if (g->n[a] < 1 || !(g->h[a] > 0.0) || !std::isfinite(g->h[a])) return SIP_EINVAL;
    N *= g->n[a];
    if (N >= (int64_t(1) << 31)) return SIP_EINVAL;
  }
  if (o->max_iter < 1 || o->cg_max < 0 || o->adapt_every < 0 || o->stop_every < 0) return SIP_EINVAL;
  if (o->stop_every > 0 && (o->evol_hist < 1 || o->evol_hist > kMaxHist - 1)) return SIP_EINVAL;
  if (!(o->rho0 > 0.0) || !(o->gamma0 >= 1.0 && o->gamma0 < 2.0)) return SIP_EINVAL;
  if (!(o->rho_ratio_max >= 1.0) || !(o->gamma_max >= 1.0 && o->gamma_max < 2.0)) return SIP_EINVAL;
  if (!(o->cg_rel > 0.0)) return SIP_EINVAL;
  int64_t n[3]; double h[3];
  internal_dims(*g, n, h);
  for (int i = 0; i < nsets; ++i) {
    const sip_set& s = sets[i];
    OpInfo oi;
    if (!op_info(g->ndim, s.op, oi)) return SIP_EINVAL;
    for (int c = 0; c < oi.ncomp; ++c)
      if (oi.axis[c] >= 0 && n[oi.axis[c]] < 2) return SIP_EINVAL;
    const int64_t M = rows_of(*g, s);
    if (s.line != SIP_LINE_NONE) {
      if (s.line != SIP_LINE_Z && s.line != SIP_LINE_Y && s.line != SIP_LINE_X) return SIP_EINVAL;
      if (s.line == SIP_LINE_Y && g->ndim != 3) return SIP_EINVAL;
      if (s.kind != SIP_SET_L1 && s.kind != SIP_SET_CARD && s.kind != SIP_SET_L2 && s.kind != SIP_SET_ANNULUS)
        return SIP_EINVAL;
      const int la = line_axis_of(s.line);
      const int64_t cap = o->field == SIP_F64 ? LineCap<double>::v : LineCap<float>::v;
      for (int c = 0; c < oi.ncomp; ++c)
        if (n[la] - (oi.axis[c] == la ? 1 : 0) > cap) return SIP_EUNSUPPORTED;
    }
    switch (s.kind) {
      case SIP_SET_BOUNDS:
        if (std::isnan(s.lo) || std::isnan(s.hi) || s.lo > s.hi) return SIP_EINVAL;
        break;
      case SIP_SET_L1:
        if (!(s.tau >= 0.0) || !std::isfinite(s.tau)) return SIP_EINVAL;
        break;
      case SIP_SET_CARD:
        if (s.k < 1 || (s.line == SIP_LINE_NONE && s.k > M)) return SIP_EINVAL;
        break;
      case SIP_SET_L2:
        if (!(s.tau >= 0.0) || !std::isfinite(s.tau)) return SIP_EINVAL;
        break;
      case SIP_SET_ANNULUS:
        if (!(s.lo >= 0.0) || !std::isfinite(s.lo) || std::isnan(s.hi) || s.lo > s.hi) return SIP_EINVAL;
        break;
      default:
        return SIP_EINVAL;
    }
    if ((s.lo_vec || s.hi_vec) && s.kind != SIP_SET_BOUNDS) return SIP_EINVAL;
  }
  return SIP_OK;
}

// Sets projected through the selection pipeline (a global reduction over
// the set's rows decides the projection).
bool is_thr(const sip_set& s) {
  return s.line == SIP_LINE_NONE &&
         (s.kind == SIP_SET_L1 || s.kind == SIP_SET_CARD || s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS);
}

// Byte layout of one instance's workspace.
struct Layout {
  int64_t total = 0;
  int64_t log = -1, m, r, p0, p1, cr[2], cp[2], yl, vl, vh0l = -1, v0l = -1, y0l = -1, xs0 = -1, xs1 = -1, ring = -1;
  struct SetL { int64_t y, v, vh0 = -1, v0 = -1, y0 = -1, lov = -1, hiv = -1; int64_t sel[2] = {-1, -1}, hc[2] = {-1, -1},
                hs[2] = {-1, -1}, cand[2] = {-1, -1}, cix = -1; } set[SIP_MAX_SETS];
};

Layout layout_of(const sip_grid& g, const sip_set* sets, int nsets, const sip_opts& o) {
  Layout L;
  int64_t n[3]; double h[3];
  internal_dims(g, n, h);
  const int64_t N = n[0] * n[1] * n[2];
  const int64_t esz = o.field == SIP_F64 ? 8 : 4;
  const int64_t vec = align_up(N * esz);
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t at = off; off += align_up(bytes); return at; };
  if (o.log_schedule) L.log = take((int64_t)o.max_iter * 2 * kMaxUnits * 8);
  L.m = take(vec); L.r = take(vec); L.p0 = take(vec); L.p1 = take(vec);
  for (int i = 0; i < 2; ++i) { L.cr[i] = take(vec); L.cp[i] = take(vec); }
  L.yl = take(vec); L.vl = take(vec);
  const bool adapt = o.adapt_every > 0, stop = o.stop_every > 0;
  if (adapt) { L.vh0l = take(vec); L.v0l = take(vec); L.y0l = take(vec); L.xs0 = take(vec); L.xs1 = take(vec); }
  if (stop) L.ring = take((int64_t)(o.evol_hist + 1) * vec);
  for (int i = 0; i < nsets; ++i) {
    OpInfo oi;
    op_info(g.ndim, sets[i].op, oi);
    const int64_t blk = oi.ncomp * vec;
    auto& S = L.set[i];
    S.y = take(blk); S.v = take(blk);
    if (adapt) { S.vh0 = take(blk); S.v0 = take(blk); S.y0 = take(blk); }
    if (sets[i].lo_vec) S.lov = take(blk);
    if (sets[i].hi_vec) S.hiv = take(blk);
    if (is_thr(sets[i])) {
      for (int src = 0; src < (stop ? 2 : 1); ++src) {
        S.sel[src] = take(sizeof(SelState));
        S.hc[src] = take(kNB * 4);
        S.hs[src] = take(kNB * 8);
        S.cand[src] = take((int64_t)oi.ncomp * N * esz);
      }
      if (sets[i].kind == SIP_SET_CARD) S.cix = take((int64_t)oi.ncomp * N * 4);
    }
  }
  L.total = align_up(off);
  return L;
}

Opts kernel_opts(const sip_opts& o) {
  Opts k;
  k.cg_max = o.cg_max; k.cg_fixed = o.cg_fixed; k.adapt_every = o.adapt_every; k.stop_every = o.stop_every;
  k.evol_hist = o.evol_hist; k.max_iter = o.max_iter; k.sel_fresh = o.sel_fresh ? 1 : 0;
  k.cg_rel2 = o.cg_rel * o.cg_rel; k.eps_corr = o.eps_corr; k.rho_ratio_max = o.rho_ratio_max;
  k.gamma_max = o.gamma_max; k.eps_evol = o.eps_evol; k.eps_feas = o.eps_feas;
  return k;
}

constexpr int64_t kTileQuantum = 256;  // item sizes are multiples of this

// Points per item: at least `base`, and few enough items that the
// per-instance partial reductions stay short.
int64_t tile_points(int64_t N, int64_t base, int64_t max_items) {
  int64_t t = std::max<int64_t>(base, (N + max_items - 1) / max_items);
  return (t + kTileQuantum - 1) / kTileQuantum * kTileQuantum;
}

}  // namespace

// ------------------------------------------------------------------ batch

struct Slot {
  bool used = false;
  sip_grid grid{};
  int nsets = 0;
  sip_set sets[SIP_MAX_SETS]{};
  char* ws = nullptr;
  Layout L;
  InstDesc desc{};
  void* x = nullptr;
  int64_t N = 0;
};

struct TileCfg {
  int64_t pt_base = 2048, pt_max_items = 512, thr_base = 2048, thr_max_items = 512;
  int pt_threads = 512;
  int cg_form = 0;
};

}  // namespace sip

struct sip_batch {
  sip_opts opts{};
  sip::Opts kopts{};
  int max_slots = 0;
  sip::Arena arena;
  std::vector<sip::Slot> slots;
  hipStream_t cap_stream = nullptr;
  // device
  sip::InstDesc* d_desc = nullptr;
  double* d_scal = nullptr;   // [max_slots][S_COUNT]
  double* h_scal = nullptr;   // pinned mirror
  // work tables (device, capacity-managed)
  sip::PtItem* d_pt = nullptr; int cap_pt = 0;
  sip::ThrItem* d_thr = nullptr; int cap_thr = 0;
  sip::SelItem* d_sel = nullptr; int cap_sel = 0;
  int32_t* d_inst = nullptr; int cap_inst = 0;
  double *d_xq = nullptr, *d_xq2 = nullptr;
  double *d_rr = nullptr, *d_pq = nullptr, *d_rr2 = nullptr, *d_pq2 = nullptr, *d_proj = nullptr, *d_thrw = nullptr, *d_thra = nullptr;
  uint32_t* d_tie = nullptr;
  uint32_t* d_h1c = nullptr; double* d_h1s = nullptr; int cap_h1 = 0;  // refine histograms, kNB per pipeline
  int cap_ppt = 0, cap_pthr = 0, cap_psp = 0;   // item capacity of the partial-sum buffers
  sip::PtItem* d_sp = nullptr; int cap_sp = 0;
  sip::LineItem* d_line = nullptr; int cap_line = 0;
  double* d_linep = nullptr; int cap_plinep = 0;
  sip::Tables tab{};
  int live_items = 0, live_inst = 0;
  bool dirty = true;
  int32_t live[4] = {0, 0, 0, 0};  // point, threshold, selection, instance items of the tables
  std::map<int, hipGraphExec_t> graphs;
  sip::TileCfg tiles;
  // Fixed-memory mode (a plan over a caller workspace, the allocation-free
  // entry point): every device buffer is carved once from
  // [fixed, fixed + fixed_size) and never freed.
  char* fixed = nullptr;
  int64_t fixed_size = 0, fixed_used = 0;
  bool no_graph = false;  // launch the iterations directly (no capture, no graph objects)
  bool pinned = true;     // h_scal from hipHostMalloc (else plain host memory)
};

struct sip_plan {
  sip_batch* b = nullptr;
  int32_t slot = 0;
  bool started = false;  // an m and x were given (sip_plan_start / sip_plan_project)
};

namespace sip {
namespace {

#define HIP_OK(expr)                                  \
  do {                                                \
    if ((expr) != hipSuccess) return SIP_EHIP;        \
  } while (0)

// Device memory of a batch: the HIP allocator, or in fixed-memory mode the
// next 256-byte aligned piece of the fixed block (SIP_EBUDGET when it is
// used up; pieces are never returned).
int32_t dev_alloc(sip_batch* b, void** p, int64_t bytes) {
  *p = nullptr;
  if (b->fixed) {
    const int64_t need = align_up(std::max<int64_t>(bytes, 1));
    if (b->fixed_used + need > b->fixed_size) return SIP_EBUDGET;
    *p = b->fixed + b->fixed_used;
    b->fixed_used += need;
    return SIP_OK;
  }
  HIP_OK(hipMalloc(p, (size_t)std::max<int64_t>(bytes, 1)));
  return SIP_OK;
}

int32_t dev_free(sip_batch* b, void* p) {
  if (!p || b->fixed) return SIP_OK;
  HIP_OK(hipFree(p));
  return SIP_OK;
}

// Capacity-managed device table: grows by doubling (fixed-memory mode: to
// exactly `need`, carved once per growth).
template <typename P>
int32_t ensure(sip_batch* b, P*& ptr, int& cap, int need, size_t elem_bytes) {
  if (need <= cap && ptr) return SIP_OK;
  int nc = b->fixed ? need : std::max(need, std::max(64, cap * 2));
  int32_t rc;
  if ((rc = dev_free(b, ptr))) return rc;
  ptr = nullptr;
  void* q = nullptr;
  if ((rc = dev_alloc(b, &q, (int64_t)nc * (int64_t)elem_bytes))) { cap = 0; return rc; }
  ptr = (P*)q;
  cap = nc;
  return SIP_OK;
}

// The item block b of a launch takes: block b runs on XCD b mod 8, and each
// XCD sweeps one contiguous slice of the n live items, which keeps the z/y
// neighbours a stencil reads in that XCD's L2.  A bijection on [0, n).
int xcd_item(int b, int n) {
  const int q = n >> 3, rem = n & 7, x = b & 7, j = b >> 3;
  return x * q + (x < rem ? x : rem) + j;
}

// A table in launch order: entry b is the item block b takes (idx = its
// index in the logical order), entries n .. cap - 1 are sentinels
// (inst = -1), so a block reads only its own entry to find its work.
template <typename Item>
std::vector<Item> launch_order(const std::vector<Item>& v, int cap, bool spread) {
  const int n = (int)v.size();
  std::vector<Item> out((size_t)std::max(cap, 0));
  for (int b = 0; b < cap; ++b) {
    if (b < n) {
      const int i = spread ? xcd_item(b, n) : b;
      out[b] = v[i];
      out[b].idx = i;
    } else {
      out[b] = Item{};
      out[b].inst = -1;
    }
  }
  return out;
}

void drop_graphs(sip_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Host form of a batch's work tables, in logical order, with their launch
// sizes (powers of two: a captured graph stays valid while the live items
// change below them; the rest of a launch is sentinel entries).
struct HostTables {
  std::vector<PtItem> pt, sp;
  std::vector<ThrItem> thr;
  std::vector<SelItem> sel;
  std::vector<LineItem> line;
  std::vector<int32_t> inst;
  int lpt = 0, lsp = 0, lthr = 0, lsel = 0, linst = 0, lline = 0;
};

// The work tables of the used slots; fills each slot's item ranges.
void build_host_tables(std::vector<Slot>& slots, const TileCfg& tiles, const sip_opts& o, HostTables& h) {
  for (int si = 0; si < (int)slots.size(); ++si) {
    Slot& s = slots[si];
    if (!s.used) continue;
    h.inst.push_back(si);
    const int N = (int)s.N;
    const int64_t tp = tile_points(N, tiles.pt_base, tiles.pt_max_items);
    s.desc.pt_begin = (int)h.pt.size();
    for (int64_t p0 = 0; p0 < N; p0 += tp)
      h.pt.push_back(PtItem{si, (int)p0, (int)std::min<int64_t>(tp, N - p0), 0});
    s.desc.pt_end = (int)h.pt.size();
    const int64_t tt = tile_points(N, tiles.thr_base, tiles.thr_max_items);
    s.desc.sp_begin = (int)h.sp.size();
    for (int64_t p0 = 0; p0 < N; p0 += tt)
      h.sp.push_back(PtItem{si, (int)p0, (int)std::min<int64_t>(tt, N - p0), 0});
    s.desc.sp_end = (int)h.sp.size();
    for (int k = 0; k < s.nsets; ++k) {
      SetDesc& sd = s.desc.sets[k];
      if (sd.thr < 0) continue;
      for (int src = 0; src < (o.stop_every > 0 ? 2 : 1); ++src) {
        h.sel.push_back(SelItem{si, k, src, 0});
        sd.item_begin[src] = (int)h.thr.size();
        for (int64_t p0 = 0; p0 < N; p0 += tt)
          h.thr.push_back(ThrItem{si, k, src, 0, (int)p0, (int)std::min<int64_t>(tt, N - p0), 0,
                                  (int)h.sel.size() - 1});
        sd.item_end[src] = (int)h.thr.size();
      }
    }
    for (int k = 0; k < s.nsets; ++k) {
      SetDesc& sd = s.desc.sets[k];
      if (sd.line_axis < 0) continue;
      sd.line_begin = (int)h.line.size();
      const int la = sd.line_axis;
      for (int c = 0; c < sd.ncomp; ++c) {
        int64_t dims[3] = {s.desc.n[0], s.desc.n[1], s.desc.n[2]};
        if (sd.axis[c] >= 0) dims[sd.axis[c]] -= 1;
        if (dims[la] <= 0) continue;
        const int64_t e0 = la == 0 ? 1 : dims[0], e1 = la == 1 ? 1 : dims[1], e2 = la == 2 ? 1 : dims[2];
        for (int64_t i0 = 0; i0 < e0; ++i0)
          for (int64_t i1 = 0; i1 < e1; ++i1)
            for (int64_t i2 = 0; i2 < e2; ++i2)
              h.line.push_back(LineItem{si, k, c, (int)dims[la],
                                        (int)(i0 * s.desc.stride[0] + i1 * s.desc.stride[1] + i2),
                                        (int)s.desc.stride[la], 0, 0});
      }
      sd.line_end = (int)h.line.size();
    }
  }
  auto pow2 = [](int n, int lo) { if (n <= 0) return 0; int c = lo; while (c < n) c <<= 1; return c; };
  h.lpt = pow2((int)h.pt.size(), 64);
  h.lthr = pow2((int)h.thr.size(), 64);
  h.lsel = pow2((int)h.sel.size(), 8);
  h.linst = pow2((int)h.inst.size(), 8);
  h.lsp = pow2((int)h.sp.size(), 64);
  h.lline = pow2((int)h.line.size(), 64);
}

// Device bytes of the work tables and partial-sum buffers at exactly the
// launch sizes of h: what fixed-memory mode carves, in rebuild_tables' order.
int64_t table_bytes(const HostTables& h) {
  auto A = [](int64_t b) { return align_up(std::max<int64_t>(b, 1)); };
  const int64_t pt = std::max(h.lpt, 1), sp = std::max(h.lsp, 1), thr = std::max(h.lthr, 1);
  const int64_t sel = std::max(h.lsel, 1), inst = std::max(h.linst, 1), line = std::max(h.lline, 1);
  return A(pt * (int64_t)sizeof(PtItem)) + A(sp * (int64_t)sizeof(PtItem)) + A(thr * (int64_t)sizeof(ThrItem)) +
         A(sel * (int64_t)sizeof(SelItem)) + A(inst * 4) + A(line * (int64_t)sizeof(LineItem)) + A(line * 64) +
         6 * A(pt * 8) + A(sp * kProjParts * 8) + A(sel * kNB * 4) + A(sel * kNB * 8) +
         2 * A(thr * kThrParts * 8) + A(thr * 12);
}

int32_t rebuild_tables(sip_batch* b, hipStream_t stream) {
  HostTables h;
  build_host_tables(b->slots, b->tiles, b->opts, h);
  const std::vector<PtItem>& pt = h.pt;
  const std::vector<ThrItem>& thr = h.thr;
  const std::vector<SelItem>& sel = h.sel;
  const std::vector<LineItem>& line = h.line;
  const std::vector<int32_t>& inst = h.inst;
  // nothing queued may still read the tables or partial buffers replaced below
  HIP_OK(hipStreamSynchronize(stream));
  const int lpt = h.lpt, lthr = h.lthr, lsel = h.lsel, linst = h.linst, lsp = h.lsp, lline = h.lline;
  const bool relaunch = lpt != b->tab.npt || lthr != b->tab.nthr || lsel != b->tab.nsel || linst != b->tab.ninst ||
                        lsp != b->tab.nsp || lline != b->tab.nline;
  int32_t rc;
  const int old_pt = b->cap_pt, old_thr = b->cap_thr, old_sel = b->cap_sel, old_inst = b->cap_inst;
  const int old_sp = b->cap_sp, old_line = b->cap_line;
  if ((rc = ensure(b, b->d_pt, b->cap_pt, std::max(lpt, 1), sizeof(PtItem)))) return rc;
  if ((rc = ensure(b, b->d_sp, b->cap_sp, std::max(lsp, 1), sizeof(PtItem)))) return rc;
  if ((rc = ensure(b, b->d_thr, b->cap_thr, std::max(lthr, 1), sizeof(ThrItem)))) return rc;
  if ((rc = ensure(b, b->d_sel, b->cap_sel, std::max(lsel, 1), sizeof(SelItem)))) return rc;
  if ((rc = ensure(b, b->d_inst, b->cap_inst, std::max(linst, 1), sizeof(int32_t)))) return rc;
  if ((rc = ensure(b, b->d_line, b->cap_line, std::max(lline, 1), sizeof(LineItem)))) return rc;
  bool moved = old_pt != b->cap_pt || old_thr != b->cap_thr || old_sel != b->cap_sel || old_inst != b->cap_inst ||
               old_sp != b->cap_sp || old_line != b->cap_line;
  auto regrow = [&](std::initializer_list<void**> ptrs, int64_t bytes) -> int32_t {
    for (void** q : ptrs) {
      int32_t r;
      if ((r = dev_free(b, *q))) return r;
      *q = nullptr;
    }
    for (void** q : ptrs) {
      int32_t r;
      if ((r = dev_alloc(b, q, bytes))) return r;
    }
    return SIP_OK;
  };
  if (b->cap_plinep < b->cap_line) {
    if ((rc = regrow({(void**)&b->d_linep}, (int64_t)b->cap_line * 8 * 8))) return rc;
    b->cap_plinep = b->cap_line;
    moved = true;
  }
  if (b->cap_ppt < b->cap_pt) {
    if ((rc = regrow({(void**)&b->d_rr, (void**)&b->d_pq, (void**)&b->d_rr2, (void**)&b->d_pq2, (void**)&b->d_xq,
                      (void**)&b->d_xq2},
                     (int64_t)b->cap_pt * 8)))
      return rc;
    b->cap_ppt = b->cap_pt;
    moved = true;
  }
  if (b->cap_psp < b->cap_sp) {
    if ((rc = regrow({(void**)&b->d_proj}, (int64_t)b->cap_sp * kProjParts * 8))) return rc;
    b->cap_psp = b->cap_sp;
    moved = true;
  }
  if (b->cap_h1 < b->cap_sel) {
    if ((rc = regrow({(void**)&b->d_h1c}, (int64_t)b->cap_sel * kNB * 4))) return rc;
    if ((rc = regrow({(void**)&b->d_h1s}, (int64_t)b->cap_sel * kNB * 8))) return rc;
    // the refine histograms start at zero (their consumers clear them after use)
    launch_zero(stream, b->d_h1c, (int64_t)b->cap_sel * kNB);
    launch_zero(stream, b->d_h1s, (int64_t)b->cap_sel * kNB);
    HIP_OK(hipGetLastError());
    b->cap_h1 = b->cap_sel;
    moved = true;
  }
  if (b->cap_pthr < b->cap_thr) {
    if ((rc = regrow({(void**)&b->d_thrw, (void**)&b->d_thra}, (int64_t)b->cap_thr * kThrParts * 8))) return rc;
    if ((rc = regrow({(void**)&b->d_tie}, (int64_t)b->cap_thr * 3 * 4))) return rc;
    b->cap_pthr = b->cap_thr;
    moved = true;
  }
  b->live[0] = (int32_t)pt.size();
  b->live[1] = (int32_t)thr.size();
  b->live[2] = (int32_t)sel.size();
  b->live[3] = (int32_t)inst.size();
  // every table is written up to its launch size (entries past the live
  // items are sentinels), in launch order
  const std::vector<PtItem> pt_l = launch_order(pt, lpt, true), sp_l = launch_order(h.sp, lsp, true);
  const std::vector<ThrItem> thr_l = launch_order(thr, lthr, true);
  const std::vector<LineItem> line_l = launch_order(line, lline, true);
  std::vector<SelItem> sel_l((size_t)lsel);
  for (int i = 0; i < lsel; ++i) {
    if (i < (int)sel.size()) sel_l[i] = sel[i];
    else { sel_l[i] = SelItem{}; sel_l[i].inst = -1; }
  }
  std::vector<int32_t> inst_l((size_t)linst, -1);
  std::copy(inst.begin(), inst.end(), inst_l.begin());
  if (lpt) HIP_OK(hipMemcpyAsync(b->d_pt, pt_l.data(), pt_l.size() * sizeof(PtItem), hipMemcpyHostToDevice, stream));
  if (lsp) HIP_OK(hipMemcpyAsync(b->d_sp, sp_l.data(), sp_l.size() * sizeof(PtItem), hipMemcpyHostToDevice, stream));
  if (lthr)
    HIP_OK(hipMemcpyAsync(b->d_thr, thr_l.data(), thr_l.size() * sizeof(ThrItem), hipMemcpyHostToDevice, stream));
  if (lsel)
    HIP_OK(hipMemcpyAsync(b->d_sel, sel_l.data(), sel_l.size() * sizeof(SelItem), hipMemcpyHostToDevice, stream));
  if (linst)
    HIP_OK(hipMemcpyAsync(b->d_inst, inst_l.data(), inst_l.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  if (lline)
    HIP_OK(hipMemcpyAsync(b->d_line, line_l.data(), line_l.size() * sizeof(LineItem), hipMemcpyHostToDevice, stream));
  // The LDS-staged CG form runs the steps of each instance without a y axis
  // whose items fit a block's LDS with one row before and two after (p) and
  // one row after (r) in 60 KiB (the rest of 64 KiB holds the block sums);
  // the batch's other instances run the two-launch steps beside them.
  // Whether an instance qualifies depends on its own grid and the tile
  // settings only.
  int form = b->tiles.cg_form, cap2 = 0, capr2 = 0, rest2 = 0;
  if (form == 2) {
    const int64_t W = b->opts.field == SIP_F64 ? 2 : 4, esz = b->opts.field == SIP_F64 ? 8 : 4;
    std::vector<int64_t> len((size_t)b->max_slots, 0);
    for (const PtItem& q : pt) len[q.inst] = std::max<int64_t>(len[q.inst], q.len);
    int64_t cp = 0, cr = 0;
    for (int si = 0; si < b->max_slots; ++si) {
      Slot& sl = b->slots[si];
      if (!sl.used) continue;
      const int64_t nx = sl.desc.n[2];
      const int64_t p = (len[si] + 3 * nx + 2 * W + W - 1) / W * W, r = (len[si] + nx + W + W - 1) / W * W;
      sl.desc.cg2 = (sl.desc.n[1] == 1 && len[si] > 0 && (p + r) * esz <= 61440) ? 1 : 0;
      if (sl.desc.cg2) { cp = std::max(cp, p); cr = std::max(cr, r); }
      else rest2 = 1;
    }
    if (cp == 0) form = 0;
    cap2 = (int)cp;
    capr2 = (int)cr;
  } else {
    for (int si = 0; si < b->max_slots; ++si) b->slots[si].desc.cg2 = 0;
  }
  for (int si = 0; si < b->max_slots; ++si) {
    if (!b->slots[si].used) continue;
    HIP_OK(hipMemcpyAsync(b->d_desc + si, &b->slots[si].desc, sizeof(InstDesc), hipMemcpyHostToDevice, stream));
  }
  HIP_OK(hipStreamSynchronize(stream));
  Tables& t = b->tab;
  bool relaunch_cap = false;
  t.D = b->d_desc;
  t.pt = b->d_pt; t.npt = lpt;
  t.sp = b->d_sp; t.nsp = lsp;
  t.thr = b->d_thr; t.nthr = lthr;
  t.sel = b->d_sel; t.nsel = lsel;
  t.inst = b->d_inst; t.ninst = linst;
  t.rr_part = b->d_rr; t.pq_part = b->d_pq; t.proj_part = b->d_proj;
  t.rr2_part = b->d_rr2; t.pq2_part = b->d_pq2; t.xq_part = b->d_xq; t.xq2_part = b->d_xq2;
  t.line = b->d_line; t.nline = lline; t.line_part = b->d_linep;
  int cap = 2;
  for (const LineItem& li : line) while (cap < li.len) cap <<= 1;
  if (cap != t.line_cap) relaunch_cap = true;
  t.line_cap = cap;
  int units = 2;
  for (int si = 0; si < b->max_slots; ++si)
    if (b->slots[si].used) units = std::max(units, b->slots[si].nsets + 2);
  if (units != t.proj_units) relaunch_cap = true;
  t.proj_units = units;
  t.thrw_part = b->d_thrw; t.thra_part = b->d_thra; t.tie_part = b->d_tie;
  t.h1c = b->d_h1c; t.h1s = b->d_h1s;
  int64_t pipe_rows = 0;
  for (int si = 0; si < b->max_slots; ++si) {
    const Slot& sl = b->slots[si];
    if (!sl.used) continue;
    for (int k = 0; k < sl.nsets; ++k)
      if (sl.desc.sets[k].thr >= 0) pipe_rows = std::max<int64_t>(pipe_rows, sl.desc.sets[k].rows);
  }
  const int passes = pipe_rows <= kOnePassRows ? 1 : 2;
  if (passes != t.sel_passes) relaunch_cap = true;
  t.sel_passes = passes;
  int64_t points = 0;
  for (int si = 0; si < b->max_slots; ++si)
    if (b->slots[si].used) points += b->slots[si].N;
  const int fuse = points <= kFuseSetsPoints ? 1 : 0;
  if (fuse != t.fuse_sets) relaunch_cap = true;
  t.fuse_sets = fuse;
  const int sfuse = (passes == 1 && (int)thr.size() <= kFuseSelItems) ? 1 : 0;
  if (sfuse != t.sel_fused) relaunch_cap = true;
  t.sel_fused = sfuse;
  const bool threads_changed = t.pt_threads != (int)b->tiles.pt_threads || t.cg_form != form || t.cg2_cap != cap2 ||
                               t.cg2_capr != capr2 || t.cg2_rest != rest2;
  t.pt_threads = (int)b->tiles.pt_threads;
  t.cg_form = form;
  t.cg2_cap = cap2;
  t.cg2_capr = capr2;
  t.cg2_rest = form == 2 ? rest2 : 0;
  b->live_items = (int)pt.size() + (int)thr.size() + (int)line.size();
  b->live_inst = (int)inst.size();
  if (relaunch || moved || threads_changed || relaunch_cap) drop_graphs(b);
  b->dirty = false;
  return SIP_OK;
}

// Enqueue `iters` iterations of every kernel on `stream` (for capture, or
// launched directly).
void launch_iterations(sip_batch* b, hipStream_t stream, int iters) {
  for (int i = 0; i < iters; ++i) {
    if (b->opts.field == SIP_F64) r64::launch_iteration<double>(stream, b->tab, b->kopts);
    else if (b->opts.reduce == SIP_F32) r32::launch_iteration<float>(stream, b->tab, b->kopts);
    else r64::launch_iteration<float>(stream, b->tab, b->kopts);
  }
}

int32_t get_graph(sip_batch* b, int iters, hipGraphExec_t& out) {
  auto it = b->graphs.find(iters);
  if (it != b->graphs.end()) { out = it->second; return SIP_OK; }
  HIP_OK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  launch_iterations(b, b->cap_stream, iters);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(b->cap_stream, &g) != hipSuccess || !g) return SIP_EHIP;
  hipGraphExec_t ge = nullptr;
  const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return SIP_EHIP;
  b->graphs[iters] = ge;
  out = ge;
  return SIP_OK;
}

void initial_scalars(const sip_batch* b, const Slot& s, double* S) {
  for (int i = 0; i < S_COUNT; ++i) S[i] = 0.0;
  const sip_opts& o = b->opts;
  for (int u = 0; u <= s.nsets; ++u) { S[S_RHO + u] = o.rho0; S[S_GAMMA + u] = o.gamma0; }
  double c0 = o.rho0, ca[3] = {0, 0, 0};
  for (int u = 0; u < s.nsets; ++u) {
    const SetDesc& sd = s.desc.sets[u];
    if (sd.op == SIP_OP_I) c0 += o.rho0;
    else for (int c = 0; c < sd.ncomp; ++c) ca[sd.axis[c]] += o.rho0;
  }
  S[S_C0] = c0;
  for (int a = 0; a < 3; ++a) S[S_CAX + a] = ca[a] * s.desc.h2inv[a];
  S[S_K] = 1.0;
  S[S_REVOL] = -1.0;
  for (int i = 0; i < SIP_MAX_SETS; ++i) S[S_RFEAS + i] = -1.0;
}

void fill_result(const Slot& s, const double* S, sip_result* r) {
  std::memset(r, 0, sizeof(*r));
  r->status = (int32_t)S[S_ERR];
  r->iters = (int32_t)S[S_ITERS];
  r->cg_steps = (int32_t)S[S_CGTOT];
  r->converged = S[S_STATE] == 1.0 ? 1 : 0;
  r->nsets = s.nsets;
  r->sel_reused = (int32_t)S[S_REUSE];
  r->r_evol = S[S_REVOL];
  for (int i = 0; i < SIP_MAX_SETS; ++i) r->r_feas[i] = i < s.nsets ? S[S_RFEAS + i] : -1.0;
  for (int u = 0; u <= s.nsets; ++u) { r->rho[u] = S[S_RHO + u]; r->gamma[u] = S[S_GAMMA + u]; }
}

// A batch whose device buffers come from the HIP allocator (mem = null) or
// are all carved from the block [mem, mem + mem_bytes) (fixed-memory mode:
// descriptors, scalars, the arena, then the work tables at the first run).
// no_graph: iterations are launched directly and the host mirror of the
// scalars is plain memory, so the batch makes no HIP allocation at all.
int32_t create_batch(sip_batch** out, int32_t max_slots, int64_t arena_bytes, const sip_opts* o, char* mem,
                     int64_t mem_bytes, bool no_graph) {
  if (!out || !o || max_slots < 1 || arena_bytes <= 0) return SIP_EINVAL;
  *out = nullptr;
  sip_opts probe = *o;
  sip_grid g{}; g.ndim = 2; g.n[0] = 2; g.n[1] = 2; g.h[0] = g.h[1] = 1.0;
  if (validate(&g, nullptr, 0, &probe) != SIP_OK) return SIP_EINVAL;
  sip_batch* b = new (std::nothrow) sip_batch();
  if (!b) return SIP_ENOMEM;
  b->opts = *o;
  b->kopts = kernel_opts(*o);
  b->max_slots = max_slots;
  b->slots.resize(max_slots);
  b->fixed = mem;
  b->fixed_size = mem ? mem_bytes : 0;
  b->no_graph = no_graph;
  b->pinned = !no_graph;
  int32_t rc = SIP_OK;
  void* q = nullptr;
  if ((rc = dev_alloc(b, &q, (int64_t)sizeof(InstDesc) * max_slots)) != SIP_OK) { sip_batch_destroy(b); return rc; }
  b->d_desc = (InstDesc*)q;
  if ((rc = dev_alloc(b, &q, (int64_t)sizeof(double) * S_COUNT * max_slots)) != SIP_OK) {
    sip_batch_destroy(b);
    return rc;
  }
  b->d_scal = (double*)q;
  if (mem) {
    if ((rc = dev_alloc(b, &q, arena_bytes)) != SIP_OK || !b->arena.borrow((char*)q, align_up(arena_bytes))) {
      sip_batch_destroy(b);
      return rc != SIP_OK ? rc : SIP_EINVAL;
    }
  } else if (!b->arena.init(arena_bytes)) {
    sip_batch_destroy(b);
    return SIP_ENOMEM;
  }
  if (!no_graph && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    sip_batch_destroy(b);
    return SIP_EHIP;
  }
  const size_t hbytes = sizeof(double) * S_COUNT * max_slots;
  if (b->pinned) {
    if (hipHostMalloc((void**)&b->h_scal, hbytes, 0) != hipSuccess) {
      b->h_scal = nullptr;
      sip_batch_destroy(b);
      return SIP_ENOMEM;
    }
  } else {
    b->h_scal = new (std::nothrow) double[(size_t)S_COUNT * max_slots];
    if (!b->h_scal) { sip_batch_destroy(b); return SIP_ENOMEM; }
  }
  std::memset(b->h_scal, 0, hbytes);
  if (hipMemcpy(b->d_scal, b->h_scal, hbytes, hipMemcpyHostToDevice) != hipSuccess) {
    sip_batch_destroy(b);
    return SIP_EHIP;
  }
  *out = b;
  return SIP_OK;
}

// A slot's descriptor: grid, sets, operator components, the state arrays
// of the workspace at ws (null: sizes only) and the iterate x_dev.
void describe_slot(Slot& s, const sip_grid& g, const sip_set* sets, int nsets, const sip_opts& o, char* ws,
                   void* x_dev, double* scal) {
  s.used = true;
  s.grid = g;
  s.nsets = nsets;
  for (int i = 0; i < nsets; ++i) s.sets[i] = sets[i];
  s.L = layout_of(g, sets, nsets, o);
  s.ws = ws;
  s.x = x_dev;
  int64_t n[3]; double h[3];
  internal_dims(g, n, h);
  s.N = n[0] * n[1] * n[2];
  InstDesc& d = s.desc;
  std::memset(&d, 0, sizeof(d));
  d.ndim = g.ndim; d.nsets = nsets; d.active = 1;
  for (int a = 0; a < 3; ++a) { d.n[a] = n[a]; d.hinv[a] = 1.0 / h[a]; d.h2inv[a] = 1.0 / (h[a] * h[a]); }
  d.N = s.N;
  const int64_t esz = o.field == SIP_F64 ? 8 : 4;
  d.cs = align_up(s.N * esz) / esz;
  d.stride[2] = 1; d.stride[1] = n[2]; d.stride[0] = n[1] * n[2];
  d.div_x = make_fastdiv((uint32_t)n[2]);
  const int64_t grp = 16 / esz;
  d.vec_ok = ((uintptr_t)x_dev % 16 == 0) ? 1 : 0;
  d.vec_nb = (n[2] % grp == 0) ? 1 : 0;  // then both row strides (nx, ny*nx) are multiples
  d.div_y = make_fastdiv((uint32_t)n[1]);
  const Layout& L = s.L;
  auto at = [&](int64_t off) -> void* { return (off >= 0 && ws) ? (void*)(ws + off) : nullptr; };
  d.m = at(L.m); d.x = x_dev; d.r = at(L.r); d.p[0] = at(L.p0); d.p[1] = at(L.p1);
  for (int i = 0; i < 2; ++i) { d.cr[i] = at(L.cr[i]); d.cp[i] = at(L.cp[i]); }
  d.xs[0] = at(L.xs0); d.xs[1] = at(L.xs1); d.ring = at(L.ring);
  d.yl = at(L.yl); d.vl = at(L.vl); d.vh0l = at(L.vh0l); d.v0l = at(L.v0l); d.y0l = at(L.y0l);
  d.scal = scal;
  d.log = (double*)at(L.log);
  d.log_cap = o.log_schedule ? o.max_iter : 0;
  int nthr = 0;
  for (int i = 0; i < nsets; ++i) {
    SetDesc& sd = d.sets[i];
    OpInfo oi;
    op_info(g.ndim, sets[i].op, oi);
    sd.kind = sets[i].kind; sd.op = sets[i].op; sd.ncomp = oi.ncomp;
    for (int c = 0; c < 3; ++c) sd.axis[c] = c < oi.ncomp ? oi.axis[c] : -1;
    sd.thr = is_thr(sets[i]) ? nthr++ : -1;
    sd.line_axis = sets[i].line != SIP_LINE_NONE ? line_axis_of(sets[i].line) : -1;
    sd.lo = sets[i].lo; sd.hi = sets[i].hi; sd.tau = sets[i].tau; sd.k = sets[i].k;
    sd.rows = rows_of(g, sets[i]);
    const auto& SL = L.set[i];
    sd.y = at(SL.y); sd.v = at(SL.v); sd.vh0 = at(SL.vh0); sd.v0 = at(SL.v0); sd.y0 = at(SL.y0);
    sd.lov = at(SL.lov); sd.hiv = at(SL.hiv);
    for (int src = 0; src < 2; ++src) {
      sd.sel[src] = (SelState*)at(SL.sel[src]);
      sd.hcnt[src] = (uint32_t*)at(SL.hc[src]);
      sd.hsum[src] = (double*)at(SL.hs[src]);
      sd.cand[src] = at(SL.cand[src]);
    }
    sd.cand_ix = (uint32_t*)at(SL.cix);
  }
}

// Carve slot si's workspace from the arena, describe it and copy the
// per-row bound vectors into it (waited for, so the caller may release
// them on return).
int32_t place_slot(sip_batch* b, int si, const sip_grid& g, const sip_set* sets, int nsets, void* x_dev,
                   hipStream_t stream) {
  Slot& s = b->slots[si];
  s = Slot();
  const Layout L = layout_of(g, sets, nsets, b->opts);
  char* ws = b->arena.alloc(L.total);
  if (!ws) return SIP_EBUDGET;
  describe_slot(s, g, sets, nsets, b->opts, ws, x_dev, b->d_scal + (size_t)si * S_COUNT);
  const InstDesc& d = s.desc;
  const size_t esz = b->opts.field == SIP_F64 ? 8 : 4;
  bool vec_bounds = false;
  for (int i = 0; i < nsets; ++i) {
    const SetDesc& sd = d.sets[i];
    const void* src[2] = {sets[i].lo_vec, sets[i].hi_vec};
    void* dst[2] = {sd.lov, sd.hiv};
    for (int q = 0; q < 2; ++q) {
      if (!src[q]) continue;
      vec_bounds = true;
      HIP_OK(hipMemcpy2DAsync(dst[q], (size_t)d.cs * esz, src[q], (size_t)s.N * esz, (size_t)s.N * esz,
                              (size_t)sd.ncomp, hipMemcpyDeviceToDevice, stream));
    }
  }
  if (vec_bounds) HIP_OK(hipStreamSynchronize(stream));
  return SIP_OK;
}

void initial_scalars(const sip_batch* b, const Slot& s, double* S);

// (Re)start slot si from m_dev: private copy of m, descriptor upload,
// initial scalars (rho0, gamma0, k = 1) and the init kernel (x = m,
// y_i = A_i m, v_i = 0, selection state cleared).  Waits for the stream
// (the host copies read stack memory).
int32_t start_slot(sip_batch* b, int si, const void* m_dev, hipStream_t stream) {
  Slot& s = b->slots[si];
  const size_t esz = b->opts.field == SIP_F64 ? 8 : 4;
  double S[S_COUNT];
  initial_scalars(b, s, S);
  HIP_OK(hipMemcpyAsync(s.desc.m, m_dev, (size_t)s.N * esz, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(b->d_desc + si, &s.desc, sizeof(InstDesc), hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(s.desc.scal, S, sizeof(S), hipMemcpyHostToDevice, stream));
  if (b->opts.field == SIP_F64) launch_init<double>(stream, b->d_desc, si, s.N);
  else launch_init<float>(stream, b->d_desc, si, s.N);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(stream));
  return SIP_OK;
}

bool tiles_from(const sip_tiles& t, TileCfg& tc) {
  if (t.pt_points < kTileQuantum || t.thr_points < kTileQuantum || t.pt_points % kTileQuantum ||
      t.thr_points % kTileQuantum || t.pt_max_items < 1 || t.thr_max_items < 1 ||
      (t.pt_threads != 256 && t.pt_threads != 512) || (t.cg_form < 0 || t.cg_form > 2))
    return false;
  tc.pt_base = t.pt_points; tc.pt_max_items = t.pt_max_items;
  tc.thr_base = t.thr_points; tc.thr_max_items = t.thr_max_items;
  tc.pt_threads = t.pt_threads; tc.cg_form = t.cg_form;
  return true;
}

// Device bytes of a one-instance batch in fixed-memory mode, in the order
// create_batch and rebuild_tables carve them: descriptor, scalars, the
// instance workspace, the work tables and partial-sum buffers.
int64_t plan_bytes_of(const sip_grid& g, const sip_set* sets, int nsets, const sip_opts& o, const TileCfg& tc) {
  std::vector<Slot> one(1);
  describe_slot(one[0], g, sets, nsets, o, nullptr, nullptr, nullptr);
  HostTables h;
  build_host_tables(one, tc, o, h);
  return align_up((int64_t)sizeof(InstDesc)) + align_up((int64_t)S_COUNT * 8) + one[0].L.total + table_bytes(h);
}

// Exported state of a plan: a header naming its layout, the scalar block,
// x, and the instance workspace (m, CG vectors, y_i, v_i, snapshots, x
// history, selection state, schedule log).
struct StateHeader {
  uint64_t magic;
  int64_t N, ws_total, n[3];
  int32_t ndim, nsets, field, reduce, adapt_every, stop_every, evol_hist, log;
  int32_t kinds[SIP_MAX_SETS], ops[SIP_MAX_SETS];
};
constexpr int64_t kStateScal = 256;                              // header in the first 256 bytes
constexpr int64_t kStateX = kStateScal + ((S_COUNT * 8 + 255) / 256) * 256;
static_assert(sizeof(StateHeader) <= kStateScal, "state header");

StateHeader state_header(const Slot& s, const sip_opts& o) {
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = 0x5349505354415445ull;  // "SIPSTATE"
  h.N = s.N;
  h.ws_total = s.L.total;
  for (int a = 0; a < 3; ++a) h.n[a] = s.desc.n[a];
  h.ndim = s.grid.ndim; h.nsets = s.nsets; h.field = o.field; h.reduce = o.reduce;
  h.adapt_every = o.adapt_every; h.stop_every = o.stop_every; h.evol_hist = o.evol_hist; h.log = o.log_schedule;
  for (int i = 0; i < s.nsets; ++i) { h.kinds[i] = s.sets[i].kind; h.ops[i] = s.sets[i].op; }
  return h;
}

int64_t state_bytes_of(const Slot& s, const sip_opts& o) {
  const int64_t esz = o.field == SIP_F64 ? 8 : 4;
  return kStateX + align_up(s.N * esz) + s.L.total;
}

// A plan's slot restarted from m with the iterate in x_dev (the descriptor
// is uploaded again, so x may change from call to call without new graphs).
int32_t restart_plan(sip_plan* p, const void* m_dev, void* x_dev, hipStream_t stream) {
  Slot& s = p->b->slots[p->slot];
  s.x = x_dev;
  s.desc.x = x_dev;
  s.desc.vec_ok = ((uintptr_t)x_dev % 16 == 0) ? 1 : 0;
  return start_slot(p->b, p->slot, m_dev, stream);
}

// The allocation-free entry point's device memory: a fixed array in every
// GPU's copy of the code object, found once per device by its symbol
// address (the array's name in host code is only a host-side stand-in).
constexpr int kMaxDevices = 64;
char* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

int32_t scratch_of_device(char** out) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SIP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SIP_EHIP;
    g_scratch[dev] = (char*)ptr;
  }
  *out = g_scratch[dev];
  return SIP_OK;
}

int32_t read_scal(sip_batch* b, hipStream_t stream) {
  HIP_OK(hipMemcpyAsync(b->h_scal, b->d_scal, (size_t)b->max_slots * S_COUNT * 8, hipMemcpyDeviceToHost, stream));
  HIP_OK(hipStreamSynchronize(stream));
  return SIP_OK;
}

}  // namespace
}  // namespace sip

using namespace sip;

// ==================================================================== C ABI

extern "C" {

const char* sip_strerror(int32_t st) {
  switch (st) {
    case SIP_OK: return "ok";
    case SIP_EINVAL: return "invalid argument";
    case SIP_ENOMEM: return "out of memory";
    case SIP_EHIP: return "HIP runtime error";
    case SIP_ENUMERIC: return "numerical failure (non-finite value or CG breakdown)";
    case SIP_EUNSUPPORTED: return "unsupported";
    case SIP_EBUDGET: return "batch full (slots or arena) or workspace too small";
    case SIP_ETOOLARGE: return "instance too large for the fixed device array of the allocation-free entry point";
    default: return "unknown status";
  }
}

int32_t sip_opts_default(sip_opts* o) {
  if (!o) return SIP_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->max_iter = 200; o->cg_max = 10; o->cg_fixed = 0; o->adapt_every = 2; o->stop_every = 0; o->evol_hist = 5;
  o->rho0 = 1.0; o->gamma0 = 1.0; o->eps_corr = 0.3; o->rho_ratio_max = 100.0; o->gamma_max = 1.999;
  o->eps_evol = 1e-2; o->eps_feas = 1e-3; o->cg_rel = 0.1; o->field = SIP_F32; o->reduce = SIP_F64; o->log_schedule = 0; o->sel_fresh = 0;
  return SIP_OK;
}

int64_t sip_set_rows(const sip_grid* g, const sip_set* s) {
  if (!g || !s || (g->ndim != 2 && g->ndim != 3)) return -1;
  return rows_of(*g, *s);
}

int32_t sip_validate(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o) {
  return validate(g, sets, nsets, o);
}

int64_t sip_workspace_bytes(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o) {
  if (validate(g, sets, nsets, o) != SIP_OK) return -1;
  return layout_of(*g, sets, nsets, *o).total;
}

int32_t sip_batch_create(sip_batch** out, int32_t max_slots, int64_t arena_bytes, const sip_opts* o) {
  return create_batch(out, max_slots, arena_bytes, o, nullptr, 0, false);
}

int32_t sip_batch_destroy(sip_batch* b) {
  if (!b) return SIP_OK;
  drop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  void* dev[] = {b->d_desc, b->d_scal, b->d_pt, b->d_thr, b->d_sel, b->d_inst, b->d_rr, b->d_pq,
                 b->d_rr2, b->d_pq2, b->d_xq, b->d_xq2, b->d_proj, b->d_thrw, b->d_thra, b->d_tie, b->d_sp,
                 b->d_line, b->d_linep, b->d_h1c, b->d_h1s};
  for (void* p : dev) (void)dev_free(b, p);
  if (b->h_scal) {
    if (b->pinned) (void)hipHostFree(b->h_scal);
    else delete[] b->h_scal;
  }
  delete b;
  return SIP_OK;
}

int32_t sip_batch_add(sip_batch* b, const sip_grid* g, const sip_set* sets, int32_t nsets, const void* m_dev,
                      void* x_dev, int32_t* slot_out, void* stream_) {
  if (!b || !m_dev || !x_dev) return SIP_EINVAL;
  const int32_t vr = validate(g, sets, nsets, &b->opts);
  if (vr != SIP_OK) return vr;
  hipStream_t stream = (hipStream_t)stream_;
  int si = -1;
  for (int i = 0; i < b->max_slots; ++i) if (!b->slots[i].used) { si = i; break; }
  if (si < 0) return SIP_EBUDGET;
  int32_t rc = place_slot(b, si, *g, sets, nsets, x_dev, stream);
  if (rc == SIP_OK) rc = start_slot(b, si, m_dev, stream);
  if (rc != SIP_OK) {
    if (b->slots[si].ws) b->arena.release(b->slots[si].ws);
    b->slots[si] = Slot();
    return rc;
  }
  b->dirty = true;
  if (slot_out) *slot_out = si;
  return SIP_OK;
}

int32_t sip_batch_run(sip_batch* b, int32_t iters, void* stream_) {
  if (!b || iters < 0) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (b->dirty) {
    const int32_t rc = rebuild_tables(b, stream);
    if (rc != SIP_OK) return rc;
  }
  if (b->live_inst == 0 || iters == 0) return SIP_OK;
  if (b->no_graph) {
    for (int i = 0; i < iters; ++i) launch_iterations(b, stream, 1);
    HIP_OK(hipGetLastError());
    return SIP_OK;
  }
  hipGraphExec_t ge;
  const int32_t rc = get_graph(b, iters, ge);
  if (rc != SIP_OK) return rc;
  HIP_OK(hipGraphLaunch(ge, stream));
  return SIP_OK;
}

int32_t sip_batch_poll(sip_batch* b, int32_t* done, void* stream_) {
  if (!b || !done) return SIP_EINVAL;
  const int32_t rc = read_scal(b, (hipStream_t)stream_);
  if (rc != SIP_OK) return rc;
  for (int i = 0; i < b->max_slots; ++i) {
    if (!b->slots[i].used) { done[i] = -1; continue; }
    const double* S = b->h_scal + (size_t)i * S_COUNT;
    done[i] = (S[S_STATE] != 0.0 || S[S_ERR] != 0.0) ? 1 : 0;
  }
  return SIP_OK;
}

int32_t sip_batch_result(sip_batch* b, int32_t slot, sip_result* res, void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used || !res) return SIP_EINVAL;
  const int32_t rc = read_scal(b, (hipStream_t)stream_);
  if (rc != SIP_OK) return rc;
  fill_result(b->slots[slot], b->h_scal + (size_t)slot * S_COUNT, res);
  return SIP_OK;
}

int32_t sip_batch_remove(sip_batch* b, int32_t slot, sip_result* res, void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return SIP_EINVAL;
  const int32_t rc = read_scal(b, (hipStream_t)stream_);
  if (rc != SIP_OK) return rc;
  if (res) fill_result(b->slots[slot], b->h_scal + (size_t)slot * S_COUNT, res);
  b->arena.release(b->slots[slot].ws);
  b->slots[slot] = Slot();
  b->dirty = true;
  return SIP_OK;
}

int32_t sip_batch_field(sip_batch* b, int32_t slot, int32_t which, int32_t set, void** ptr, int64_t* count,
                        int64_t* comp_stride) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used || !ptr || !count) return SIP_EINVAL;
  if (comp_stride) *comp_stride = b->slots[slot].desc.cs;
  const Slot& s = b->slots[slot];
  const InstDesc& d = s.desc;
  *ptr = nullptr;
  *count = 0;
  if (which <= 4) {
    if (set < 0 || set > s.nsets) return SIP_EINVAL;
    const bool ident = set == s.nsets;
    const int nc = ident ? 1 : d.sets[set].ncomp;
    void* p = nullptr;
    switch (which) {
      case 0: p = ident ? d.yl : d.sets[set].y; break;
      case 1: p = ident ? d.vl : d.sets[set].v; break;
      case 2: p = ident ? d.vh0l : d.sets[set].vh0; break;
      case 3: p = ident ? d.v0l : d.sets[set].v0; break;
      case 4: p = ident ? d.y0l : d.sets[set].y0; break;
    }
    if (!p) return SIP_EINVAL;
    *ptr = p;
    *count = nc * d.cs;
    return SIP_OK;
  }
  void* p = which == 5 ? d.r : which == 6 ? d.xs[0] : which == 7 ? d.xs[1] : nullptr;
  if (!p) return SIP_EINVAL;
  *ptr = p;
  *count = s.N;
  return SIP_OK;
}

int32_t sip_batch_get_params(sip_batch* b, int32_t slot, double* rho, double* gamma, int32_t* k, int32_t* have,
                             void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return SIP_EINVAL;
  const int32_t rc = read_scal(b, (hipStream_t)stream_);
  if (rc != SIP_OK) return rc;
  const double* S = b->h_scal + (size_t)slot * S_COUNT;
  const int p = b->slots[slot].nsets;
  for (int u = 0; u <= p; ++u) { if (rho) rho[u] = S[S_RHO + u]; if (gamma) gamma[u] = S[S_GAMMA + u]; }
  if (k) *k = (int32_t)S[S_K];
  if (have) *have = S[S_HAVE_SNAP] != 0.0;
  return SIP_OK;
}

int32_t sip_batch_set_params(sip_batch* b, int32_t slot, const double* rho, const double* gamma, int32_t k,
                             int32_t have, void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used || k < 1) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const int32_t rc = read_scal(b, stream);
  if (rc != SIP_OK) return rc;
  double* S = b->h_scal + (size_t)slot * S_COUNT;
  const Slot& s = b->slots[slot];
  const int p = s.nsets;
  for (int u = 0; u <= p; ++u) {
    if (rho) { if (!(rho[u] > 0.0)) return SIP_EINVAL; S[S_RHO + u] = rho[u]; }
    if (gamma) S[S_GAMMA + u] = gamma[u];
  }
  double c0 = S[S_RHO + p], ca[3] = {0, 0, 0};
  for (int u = 0; u < p; ++u) {
    const SetDesc& sd = s.desc.sets[u];
    if (sd.op == SIP_OP_I) c0 += S[S_RHO + u];
    else for (int c = 0; c < sd.ncomp; ++c) ca[sd.axis[c]] += S[S_RHO + u];
  }
  S[S_C0] = c0;
  for (int a = 0; a < 3; ++a) S[S_CAX + a] = ca[a] * s.desc.h2inv[a];
  S[S_K] = (double)k;
  S[S_HAVE_SNAP] = have ? 1.0 : 0.0;
  S[S_STATE] = (k > b->opts.max_iter) ? 2.0 : 0.0;
  HIP_OK(hipMemcpyAsync(b->d_scal + (size_t)slot * S_COUNT, S, sizeof(double) * S_COUNT, hipMemcpyHostToDevice, stream));
  HIP_OK(hipStreamSynchronize(stream));
  return SIP_OK;
}

int32_t sip_batch_schedule(sip_batch* b, int32_t slot, double* rho, double* gamma, int32_t max_n, int32_t* n,
                           void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used || !n) return SIP_EINVAL;
  const Slot& s = b->slots[slot];
  if (!s.desc.log) return SIP_EUNSUPPORTED;
  hipStream_t stream = (hipStream_t)stream_;
  int32_t rc = read_scal(b, stream);
  if (rc != SIP_OK) return rc;
  const double* S = b->h_scal + (size_t)slot * S_COUNT;
  int cnt = (int)S[S_K] - 1;
  if (S[S_STATE] == 1.0) cnt = (int)S[S_ITERS];
  cnt = std::min(cnt, std::min(max_n, s.desc.log_cap));
  *n = cnt;
  if (cnt <= 0) return SIP_OK;
  std::vector<double> buf((size_t)cnt * 2 * kMaxUnits);
  HIP_OK(hipMemcpyAsync(buf.data(), s.desc.log, buf.size() * 8, hipMemcpyDeviceToHost, stream));
  HIP_OK(hipStreamSynchronize(stream));
  const int p1 = s.nsets + 1;
  for (int i = 0; i < cnt; ++i)
    for (int u = 0; u < p1; ++u) {
      if (rho) rho[(size_t)i * p1 + u] = buf[(size_t)i * 2 * kMaxUnits + u];
      if (gamma) gamma[(size_t)i * p1 + u] = buf[(size_t)i * 2 * kMaxUnits + kMaxUnits + u];
    }
  return SIP_OK;
}

int32_t sip_batch_reset(sip_batch* b, int32_t slot, const void* m_dev, void* stream_) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used || !m_dev) return SIP_EINVAL;
  return start_slot(b, slot, m_dev, (hipStream_t)stream_);
}

int32_t sip_batch_time_kernel(sip_batch* b, int32_t kernel, int32_t reps, void* stream_, double* avg_ms) {
  if (!b || kernel < SIP_K_RHS || kernel > SIP_K_CG2_D0 || reps < 1 || !avg_ms) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (b->dirty) {
    const int32_t rc = rebuild_tables(b, stream);
    if (rc != SIP_OK) return rc;
  }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  for (int w = 0; w < 2; ++w) {  // warm the caches and the code object
    if (b->opts.field == SIP_F64) r64::launch_phase<double>(stream, b->tab, b->kopts, kernel);
    else if (b->opts.reduce == SIP_F32) r32::launch_phase<float>(stream, b->tab, b->kopts, kernel);
    else r64::launch_phase<float>(stream, b->tab, b->kopts, kernel);
  }
  HIP_OK(hipEventRecord(e0, stream));
  for (int i = 0; i < reps; ++i) {
    if (b->opts.field == SIP_F64) r64::launch_phase<double>(stream, b->tab, b->kopts, kernel);
    else if (b->opts.reduce == SIP_F32) r32::launch_phase<float>(stream, b->tab, b->kopts, kernel);
    else r64::launch_phase<float>(stream, b->tab, b->kopts, kernel);
  }
  HIP_OK(hipEventRecord(e1, stream));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return SIP_OK;
}

int32_t sip_stream_copy(void* dst, const void* src, int64_t bytes, void* stream_) {
  if (!dst || !src || bytes < 0 || bytes % 16) return SIP_EINVAL;
  launch_copy((hipStream_t)stream_, dst, src, bytes / 16);
  return hipGetLastError() == hipSuccess ? SIP_OK : SIP_EHIP;
}

int32_t sip_dykstra_update(int32_t p, const void* const* y, void* const* v, const double* w, void* x, int64_t n,
                           int32_t field, void* stream_) {
  if (p < 1 || p > SIP_MAX_SETS || !y || !v || !w || !x || n < 0 || (field != SIP_F32 && field != SIP_F64))
    return SIP_EINVAL;
  for (int i = 0; i < p; ++i)
    if (!y[i] || !v[i]) return SIP_EINVAL;
  if (n == 0) return SIP_OK;
  return launch_dykstra((hipStream_t)stream_, p, y, v, w, x, n, field == SIP_F64);
}

int32_t sip_batch_set_tiles(sip_batch* b, int32_t pt_points, int32_t pt_max_items, int32_t thr_points,
                            int32_t thr_max_items, int32_t pt_threads, int32_t cg_form) {
  if (!b || pt_points < kTileQuantum || thr_points < kTileQuantum || pt_points % kTileQuantum ||
      thr_points % kTileQuantum || pt_max_items < 1 || thr_max_items < 1 ||
      (pt_threads != 256 && pt_threads != 512) || (cg_form < 0 || cg_form > 2))
    return SIP_EINVAL;
  b->tiles.pt_threads = pt_threads;
  b->tiles.cg_form = cg_form;
  b->tiles.pt_base = pt_points;
  b->tiles.pt_max_items = pt_max_items;
  b->tiles.thr_base = thr_points;
  b->tiles.thr_max_items = thr_max_items;
  b->dirty = true;
  return SIP_OK;
}

int32_t sip_batch_items(sip_batch* b, int32_t* npt, int32_t* nthr, int32_t* nsel, int32_t* ninst) {
  if (!b) return SIP_EINVAL;
  if (npt) *npt = b->live[0];
  if (nthr) *nthr = b->live[1];
  if (nsel) *nsel = b->live[2];
  if (ninst) *ninst = b->live[3];
  return SIP_OK;
}

static int32_t run_to_end(sip_batch* b, int32_t chunk, hipStream_t stream) {
  const int total = b->opts.max_iter;
  std::vector<int32_t> done(b->max_slots);
  int ran = 0;
  while (ran < total) {
    const int n = std::min(chunk, total - ran);
    int32_t rc = sip_batch_run(b, n, stream);
    if (rc != SIP_OK) return rc;
    ran += n;
    if (b->opts.stop_every > 0 && ran < total) {
      rc = sip_batch_poll(b, done.data(), stream);
      if (rc != SIP_OK) return rc;
      bool all = true;
      for (int i = 0; i < b->max_slots; ++i) if (done[i] == 0) all = false;
      if (all) break;
    }
  }
  return hipStreamSynchronize(stream) == hipSuccess ? SIP_OK : SIP_EHIP;
}

int32_t sip_project(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o, const void* m_dev,
                    void* x_dev, sip_result* res, void* stream_) {
  const int32_t vr = validate(g, sets, nsets, o);
  if (vr != SIP_OK) return vr;
  hipStream_t stream = (hipStream_t)stream_;
  const int64_t ws = sip_workspace_bytes(g, sets, nsets, o);
  sip_batch* b = nullptr;
  int32_t rc = sip_batch_create(&b, 1, ws, o);
  if (rc != SIP_OK) return rc;
  int32_t slot = -1;
  rc = sip_batch_add(b, g, sets, nsets, m_dev, x_dev, &slot, stream);
  if (rc == SIP_OK) rc = run_to_end(b, std::min(o->max_iter, o->stop_every > 0 ? 5 * o->stop_every : 25), stream);
  sip_result r{};
  if (rc == SIP_OK) rc = sip_batch_remove(b, slot, &r, stream);
  sip_batch_destroy(b);
  if (rc != SIP_OK) return rc;
  if (res) *res = r;
  return r.status;
}

int32_t sip_project_batched(int32_t B, const sip_grid* grids, const sip_set* sets_flat, const int32_t* nsets,
                            const sip_opts* o, const void* const* m_dev, void* const* x_dev, sip_result* res,
                            int32_t graph_iters, void* stream_) {
  if (B < 1 || !grids || !nsets || !o || !m_dev || !x_dev) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  int64_t total = 0;
  int64_t off = 0;
  for (int i = 0; i < B; ++i) {
    const int64_t ws = sip_workspace_bytes(&grids[i], sets_flat + off, nsets[i], o);
    if (ws < 0) return SIP_EINVAL;
    total += ws;
    off += nsets[i];
  }
  sip_batch* b = nullptr;
  int32_t rc = sip_batch_create(&b, B, total, o);
  if (rc != SIP_OK) return rc;
  std::vector<int32_t> slots(B, -1);
  off = 0;
  for (int i = 0; i < B && rc == SIP_OK; ++i) {
    rc = sip_batch_add(b, &grids[i], sets_flat + off, nsets[i], m_dev[i], x_dev[i], &slots[i], stream);
    off += nsets[i];
  }
  if (rc == SIP_OK) rc = run_to_end(b, graph_iters > 0 ? graph_iters : 25, stream);
  int32_t first_bad = SIP_OK;
  if (rc == SIP_OK) {
    for (int i = 0; i < B; ++i) {
      sip_result r{};
      rc = sip_batch_result(b, slots[i], &r, stream);
      if (rc != SIP_OK) break;
      if (res) res[i] = r;
      if (r.status != SIP_OK && first_bad == SIP_OK) first_bad = r.status;
    }
  }
  sip_batch_destroy(b);
  return rc != SIP_OK ? rc : first_bad;
}

// ---------------------------------------------------------------- plans

int32_t sip_tiles_default(sip_tiles* t) {
  if (!t) return SIP_EINVAL;
  const TileCfg d;
  t->pt_points = (int32_t)d.pt_base; t->pt_max_items = (int32_t)d.pt_max_items;
  t->thr_points = (int32_t)d.thr_base; t->thr_max_items = (int32_t)d.thr_max_items;
  t->pt_threads = d.pt_threads; t->cg_form = d.cg_form;
  return SIP_OK;
}

int64_t sip_plan_bytes(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                       const sip_tiles* tiles) {
  if (validate(g, sets, nsets, o) != SIP_OK) return -1;
  TileCfg tc;
  if (tiles && !tiles_from(*tiles, tc)) return -1;
  return plan_bytes_of(*g, sets, nsets, *o, tc);
}

int32_t sip_plan_create(sip_plan** out, const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                        const sip_tiles* tiles, void* workspace, int64_t workspace_bytes, void* stream_) {
  if (!out) return SIP_EINVAL;
  *out = nullptr;
  const int32_t vr = validate(g, sets, nsets, o);
  if (vr != SIP_OK) return vr;
  TileCfg tc;
  if (tiles && !tiles_from(*tiles, tc)) return SIP_EINVAL;
  const int64_t need = plan_bytes_of(*g, sets, nsets, *o, tc);
  if (workspace && workspace_bytes < need) return SIP_EBUDGET;
  if (workspace && (uintptr_t)workspace % kAlign) return SIP_EINVAL;
  sip_plan* p = new (std::nothrow) sip_plan();
  if (!p) return SIP_ENOMEM;
  const int64_t ws = layout_of(*g, sets, nsets, *o).total;
  int32_t rc = create_batch(&p->b, 1, ws, o, (char*)workspace, workspace ? workspace_bytes : 0, false);
  if (rc == SIP_OK) {
    p->b->tiles = tc;
    rc = place_slot(p->b, 0, *g, sets, nsets, nullptr, (hipStream_t)stream_);
  }
  if (rc == SIP_OK) rc = rebuild_tables(p->b, (hipStream_t)stream_);
  if (rc != SIP_OK) {
    sip_plan_destroy(p);
    return rc;
  }
  *out = p;
  return SIP_OK;
}

int32_t sip_plan_destroy(sip_plan* p) {
  if (!p) return SIP_OK;
  if (p->b) sip_batch_destroy(p->b);
  delete p;
  return SIP_OK;
}

int32_t sip_plan_start(sip_plan* p, const void* m_dev, void* x_dev, void* stream_) {
  if (!p || !m_dev || !x_dev) return SIP_EINVAL;
  const int32_t rc = restart_plan(p, m_dev, x_dev, (hipStream_t)stream_);
  if (rc == SIP_OK) p->started = true;
  return rc;
}

int32_t sip_plan_iterate(sip_plan* p, int32_t iters, void* stream) {
  if (!p || !p->started || iters < 0) return SIP_EINVAL;
  return sip_batch_run(p->b, iters, stream);
}

int32_t sip_plan_result(sip_plan* p, sip_result* res, void* stream) {
  if (!p || !p->started || !res) return SIP_EINVAL;
  return sip_batch_result(p->b, p->slot, res, stream);
}

int32_t sip_plan_project(sip_plan* p, const void* m_dev, void* x_dev, sip_result* res, void* stream_) {
  if (!p || !m_dev || !x_dev) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  int32_t rc = sip_plan_start(p, m_dev, x_dev, stream_);
  const sip_opts& o = p->b->opts;
  if (rc == SIP_OK) rc = run_to_end(p->b, std::min(o.max_iter, o.stop_every > 0 ? 5 * o.stop_every : 25), stream);
  sip_result r{};
  if (rc == SIP_OK) rc = sip_batch_result(p->b, p->slot, &r, stream_);
  if (rc != SIP_OK) return rc;
  if (res) *res = r;
  return r.status;
}

int64_t sip_state_bytes(const sip_plan* p) {
  if (!p) return -1;
  return state_bytes_of(p->b->slots[p->slot], p->b->opts);
}

int32_t sip_state_export(sip_plan* p, void* dst_dev, void* stream_) {
  if (!p || !p->started || !dst_dev) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const Slot& s = p->b->slots[p->slot];
  const StateHeader hd = state_header(s, p->b->opts);
  const size_t esz = p->b->opts.field == SIP_F64 ? 8 : 4;
  char* dst = (char*)dst_dev;
  HIP_OK(hipMemcpyAsync(dst, &hd, sizeof(hd), hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(dst + kStateScal, s.desc.scal, S_COUNT * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(dst + kStateX, s.x, (size_t)s.N * esz, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(dst + kStateX + align_up(s.N * (int64_t)esz), s.ws, (size_t)s.L.total,
                        hipMemcpyDeviceToDevice, stream));
  // the header copy reads stack memory
  HIP_OK(hipStreamSynchronize(stream));
  return SIP_OK;
}

int32_t sip_state_import(sip_plan* p, const void* src_dev, void* stream_) {
  if (!p || !p->started || !src_dev) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const Slot& s = p->b->slots[p->slot];
  const StateHeader want = state_header(s, p->b->opts);
  StateHeader got;
  const char* src = (const char*)src_dev;
  HIP_OK(hipMemcpyAsync(&got, src, sizeof(got), hipMemcpyDeviceToHost, stream));
  HIP_OK(hipStreamSynchronize(stream));
  if (std::memcmp(&got, &want, sizeof(got)) != 0) return SIP_EINVAL;
  const size_t esz = p->b->opts.field == SIP_F64 ? 8 : 4;
  HIP_OK(hipMemcpyAsync(s.desc.scal, src + kStateScal, S_COUNT * 8, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(s.x, src + kStateX, (size_t)s.N * esz, hipMemcpyDeviceToDevice, stream));
  HIP_OK(hipMemcpyAsync(s.ws, src + kStateX + align_up(s.N * (int64_t)esz), (size_t)s.L.total,
                        hipMemcpyDeviceToDevice, stream));
  return SIP_OK;
}

// ----------------------------------------------- allocation-free projection

int32_t sip_project_noalloc(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                            const void* m_dev, void* x_dev, sip_result* res, void* stream_) {
  const int32_t vr = validate(g, sets, nsets, o);
  if (vr != SIP_OK) return vr;
  if (!m_dev || !x_dev) return SIP_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const TileCfg tc;
  if (plan_bytes_of(*g, sets, nsets, *o, tc) > kScratchBytes) return SIP_ETOOLARGE;
  char* base = nullptr;
  int32_t rc = scratch_of_device(&base);
  if (rc != SIP_OK) return rc;
  sip_batch* b = nullptr;
  rc = create_batch(&b, 1, layout_of(*g, sets, nsets, *o).total, o, base, kScratchBytes, true);
  if (rc != SIP_OK) return rc;
  rc = place_slot(b, 0, *g, sets, nsets, x_dev, stream);
  if (rc == SIP_OK) rc = start_slot(b, 0, m_dev, stream);
  if (rc == SIP_OK) rc = rebuild_tables(b, stream);
  if (rc == SIP_OK) rc = run_to_end(b, std::min(o->max_iter, o->stop_every > 0 ? 5 * o->stop_every : 25), stream);
  sip_result r{};
  if (rc == SIP_OK) rc = sip_batch_result(b, 0, &r, stream_);
  sip_batch_destroy(b);
  if (rc != SIP_OK) return rc;
  if (res) *res = r;
  return r.status;
}

}  // extern "C"

// ------------------------------------------------------------ multilevel

namespace {

// Grid and sets of level `level` (0 = the given grid): ceil(n / 2) points per
// axis and level, spacing doubled; l1 budgets and cardinalities scaled by
// the operator's row ratio (cardinality rounded half up, within [1, rows]).
void level_of(const sip_grid& g, const sip_set* sets, int nsets, int level, sip_grid& gl, sip_set* sl) {
  gl = g;
  for (int a = 0; a < g.ndim; ++a) {
    int64_t n = g.n[a];
    for (int l = 0; l < level; ++l) n = (n + 1) / 2;
    gl.n[a] = n;
    gl.h[a] = g.h[a] * std::ldexp(1.0, level);
  }
  for (int i = 0; i < nsets; ++i) {
    sl[i] = sets[i];
    const int64_t r0 = rows_of(g, sets[i]), rl = rows_of(gl, sets[i]);
    if (r0 <= 0 || rl <= 0) continue;  // rejected by validate()
    const double ratio = (double)rl / (double)r0;
    if (sets[i].kind == SIP_SET_L1) sl[i].tau = sets[i].tau * ratio;
    if (sets[i].kind == SIP_SET_L2) sl[i].tau = sets[i].tau * std::sqrt(ratio);
    if (sets[i].kind == SIP_SET_ANNULUS) { sl[i].lo = sets[i].lo * std::sqrt(ratio); sl[i].hi = sets[i].hi * std::sqrt(ratio); }
    if (sets[i].kind == SIP_SET_CARD) {
      int64_t k = (int64_t)std::floor((double)sets[i].k * ratio + 0.5);
      sl[i].k = std::min<int64_t>(rl, std::max<int64_t>(1, k));
    }
  }
}

template <typename T>
void prolong_state(hipStream_t st, const Slot& c, const Slot& f) {
  const InstDesc& dc = c.desc;
  const InstDesc& df = f.desc;
  const int64_t sc[3] = {dc.n[0], dc.n[1], dc.n[2]};
  const int64_t sf[3] = {df.n[0], df.n[1], df.n[2]};
  auto one = [&](const void* src, void* dst, int axis) {
    int64_t si[3] = {sc[0], sc[1], sc[2]}, di[3] = {sf[0], sf[1], sf[2]};
    if (axis >= 0) { si[axis] -= 1; di[axis] -= 1; }
    launch_prolong<T>(st, (const T*)src, si, sc[1] * sc[2], sc[2], (T*)dst, sf, di, sf[1] * sf[2], sf[2], axis);
  };
  one(dc.x, df.x, -1);
  if (df.ring) one(dc.x, df.ring, -1);  // history slot 0 = the initial x
  one(dc.yl, df.yl, -1);
  one(dc.vl, df.vl, -1);
  for (int i = 0; i < df.nsets; ++i) {
    const SetDesc& a = dc.sets[i];
    const SetDesc& b = df.sets[i];
    for (int k = 0; k < b.ncomp; ++k) {
      one((const T*)a.y + (size_t)k * dc.cs, (T*)b.y + (size_t)k * df.cs, b.axis[k]);
      one((const T*)a.v + (size_t)k * dc.cs, (T*)b.v + (size_t)k * df.cs, b.axis[k]);
    }
  }
}

}  // namespace

int32_t sip_level(const sip_grid* g, const sip_set* sets, int32_t nsets, int32_t level, sip_grid* g_out,
                  sip_set* sets_out) {
  if (!g || !g_out || level < 0 || (nsets > 0 && (!sets || !sets_out))) return SIP_EINVAL;
  if (nsets < 0 || nsets > SIP_MAX_SETS || (g->ndim != 2 && g->ndim != 3)) return SIP_EINVAL;
  sip_set tmp[SIP_MAX_SETS];
  level_of(*g, sets, nsets, level, *g_out, tmp);
  for (int i = 0; i < nsets; ++i) sets_out[i] = tmp[i];
  return SIP_OK;
}

int32_t sip_restrict(const sip_grid* g, int32_t dtype, const void* src_dev, void* dst_dev, void* stream_) {
  if (!g || !src_dev || !dst_dev || (g->ndim != 2 && g->ndim != 3)) return SIP_EINVAL;
  if (dtype != SIP_F32 && dtype != SIP_F64) return SIP_EINVAL;
  for (int a = 0; a < g->ndim; ++a)
    if (g->n[a] < 1) return SIP_EINVAL;
  sip_grid gc;
  level_of(*g, nullptr, 0, 1, gc, nullptr);
  int64_t n[3], c[3];
  double h[3];
  internal_dims(*g, n, h);
  internal_dims(gc, c, h);
  hipStream_t st = (hipStream_t)stream_;
  if (dtype == SIP_F64) launch_restrict<double>(st, (const double*)src_dev, n, (double*)dst_dev, c);
  else launch_restrict<float>(st, (const float*)src_dev, n, (float*)dst_dev, c);
  return hipGetLastError() == hipSuccess ? SIP_OK : SIP_EHIP;
}

int32_t sip_project_multilevel(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                               int32_t nlevels, const int32_t* level_iters, int32_t carry_params,
                               const void* m_dev, void* x_dev, sip_result* res, int32_t* level_iters_run,
                               void* stream_) {
  if (!g || !o || !level_iters || !m_dev || !x_dev || nlevels < 1 || nlevels > 16) return SIP_EINVAL;
  int32_t rc = validate(g, sets, nsets, o);
  if (rc != SIP_OK) return rc;
  for (int i = 0; i < nsets; ++i)
    if (sets[i].lo_vec || sets[i].hi_vec || sets[i].line != SIP_LINE_NONE) return SIP_EUNSUPPORTED;
  std::vector<sip_grid> grids(nlevels);
  std::vector<std::vector<sip_set>> lsets(nlevels, std::vector<sip_set>(std::max(nsets, 1)));
  for (int l = 0; l < nlevels; ++l) {
    if (level_iters[l] < 1) return SIP_EINVAL;
    level_of(*g, sets, nsets, l, grids[l], lsets[l].data());
    sip_opts ol = *o;
    ol.max_iter = level_iters[l];
    rc = validate(&grids[l], lsets[l].data(), nsets, &ol);
    if (rc != SIP_OK) return rc;  // e.g. too many levels for a difference axis
  }
  hipStream_t stream = (hipStream_t)stream_;
  const size_t esz = o->field == SIP_F64 ? 8 : 4;
  // coarse models and iterates (level 0 uses the caller's m and x)
  std::vector<void*> ms(nlevels, nullptr), xs(nlevels, nullptr);
  ms[0] = const_cast<void*>(m_dev);
  xs[0] = x_dev;
  auto cleanup = [&]() {
    for (int l = 1; l < nlevels; ++l) {
      if (ms[l]) (void)hipFree(ms[l]);
      if (xs[l]) (void)hipFree(xs[l]);
    }
  };
  for (int l = 1; l < nlevels; ++l) {
    int64_t n = 1;
    for (int a = 0; a < g->ndim; ++a) n *= grids[l].n[a];
    if (hipMalloc(&ms[l], (size_t)n * esz) != hipSuccess || hipMalloc(&xs[l], (size_t)n * esz) != hipSuccess) {
      cleanup();
      return SIP_ENOMEM;
    }
    rc = sip_restrict(&grids[l - 1], o->field, ms[l - 1], ms[l], stream);
    if (rc != SIP_OK) { cleanup(); return rc; }
  }
  sip_batch* prev = nullptr;
  sip_result r{};
  for (int l = nlevels - 1; l >= 0 && rc == SIP_OK; --l) {
    sip_opts ol = *o;
    ol.max_iter = level_iters[l];
    sip_batch* b = nullptr;
    rc = sip_batch_create(&b, 1, sip_workspace_bytes(&grids[l], lsets[l].data(), nsets, &ol), &ol);
    if (rc != SIP_OK) break;
    int32_t slot = -1;
    rc = sip_batch_add(b, &grids[l], lsets[l].data(), nsets, ms[l], xs[l], &slot, stream);
    if (rc == SIP_OK && prev) {
      if (o->field == SIP_F64) prolong_state<double>(stream, prev->slots[0], b->slots[slot]);
      else prolong_state<float>(stream, prev->slots[0], b->slots[slot]);
      if (hipGetLastError() != hipSuccess) rc = SIP_EHIP;
      if (rc == SIP_OK && carry_params) {
        // start from the coarser level's final (rho, gamma)
        double rho[SIP_MAX_SETS + 1], gam[SIP_MAX_SETS + 1];
        for (int i = 0; i <= nsets; ++i) { rho[i] = r.rho[i]; gam[i] = r.gamma[i]; }
        rc = sip_batch_set_params(b, slot, rho, gam, 1, 0, stream);
      }
    }
    if (rc == SIP_OK) rc = run_to_end(b, std::min(ol.max_iter, ol.stop_every > 0 ? 5 * ol.stop_every : 25), stream);
    if (prev) { sip_batch_destroy(prev); prev = nullptr; }
    if (rc == SIP_OK) rc = sip_batch_result(b, slot, &r, stream);
    if (rc == SIP_OK && level_iters_run) level_iters_run[l] = r.iters;
    if (rc == SIP_OK && r.status != SIP_OK) rc = r.status;
    prev = b;
  }
  if (prev) sip_batch_destroy(prev);
  if (hipStreamSynchronize(stream) != hipSuccess && rc == SIP_OK) rc = SIP_EHIP;
  cleanup();
  if (rc != SIP_OK) return rc;
  if (res) *res = r;
  return SIP_OK;
}
