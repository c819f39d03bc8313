// Internal layout shared by the gfx950 kernels and the host engine of
// libsip.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sip.h"

namespace sip {

constexpr int kBlock = 256;                 // threads per work-group (4 wave64)
constexpr int kMaxUnits = SIP_MAX_SETS + 1; // p sets + the identity block
constexpr int kNB = 2048;                   // buckets of a radix digit (11 bits)
constexpr int kMaxHist = 9;                 // x-history slots (evol_hist <= 8)
// Per point-item partial sums written by the projection kernel: 8 per unit
// (6 adapt dots + 2 feasibility sums) then the evolution sums.
constexpr int kUnitParts = 8;
constexpr int kEvolOff = kUnitParts * kMaxUnits;
constexpr int kProjParts = kEvolOff + 16;
constexpr int kThrParts = 8;                // per threshold item

// Scalar block of one instance (doubles).  Writers: the host at admission,
// k_finish at the end of an iteration, the designated leader block of the CG
// kernels (only slots no other block of the same launch reads).
enum Scal : int {
  S_RHO = 0,                    // [kMaxUnits]
  S_GAMMA = S_RHO + kMaxUnits,  // [kMaxUnits]
  S_C0 = S_GAMMA + kMaxUnits,   // stencil scalar of the identity part
  S_CAX,                        // [3] stencil scalars per axis (rho / h^2 sums)
  S_RR = S_CAX + 3,             // [2] r^T r of the current CG step, by step parity
  S_DONE = S_RR + 2,            // [2] CG finished flags, by step parity
  S_RR0 = S_DONE + 2,           // r^T r of the warm start
  S_CGTOT,                      // CG steps run so far
  S_K,                          // iteration counter k (1-based)
  S_STATE,                      // 0 running, 1 converged, 2 reached max_iter
  S_ERR,                        // 0 or a negative sip_status
  S_HAVE_SNAP,                  // adapt-rho-gamma holds a k0 snapshot
  S_REVOL,                      // last r_evol (-1: never evaluated)
  S_ITERS,                      // iterations completed
  S_ALPHA,                      // [2] CG step length by step parity (one-reduction form)
  S_RFEAS = S_ALPHA + 2,        // [SIP_MAX_SETS] last r_feas (-1: never)
  S_REUSE = S_RFEAS + SIP_MAX_SETS,  // selections that started from the w pass's list A
  S_PCP,                        // [2] p^T C p of the LDS-staged CG form, by step parity
  S_COUNT = S_RFEAS + SIP_MAX_SETS + 4
};

// SEL_POINT: an annulus at w = 0 (y = lo on the first row, 0 elsewhere).
enum SelMode : int { SEL_PROJECT = 0, SEL_INSIDE = 1, SEL_ZERO = 2, SEL_ALL = 3, SEL_POINT = 4 };

// Selection state of one pipeline (a threshold set's w = x-bar - v/rho, or
// on stopping-test iterations its s = A x).  Keys are the IEEE bit patterns
// of |value|; digits are resolved from the most significant end.
struct SelState {
  unsigned long long prefix;    // resolved high key bits (in place)
  unsigned long long c_above;   // elements with key above the resolved prefix range
  unsigned long long tkey;      // cardinality: key of the k-th largest magnitude
  unsigned long long keep_ties; // cardinality: how many entries equal to tkey to keep
  unsigned long long ties;      // cardinality: entries equal to tkey
  unsigned long long ncand;     // candidates appended by the refine pass
  double s_above;               // sum of the values above the resolved range
  double theta;                 // l1: the soft threshold
  double tk;                    // cardinality: value of the k-th largest magnitude
  int32_t digit;                // index of the next digit to resolve
  int32_t mode;                 // SelMode
  int32_t need_ties;            // cardinality: rank ties by linear index
  int32_t err;
  int32_t compact_next;         // the next refine pass also appends candidate keys
  int32_t final_;               // threshold known; later refine/select passes skip
  // Reuse of the previous iteration's first digit: the w pass gathers every
  // entry whose first-digit bucket is spec - 1 into the candidate buffer
  // from its start ("list A", nspec entries; spec 0: none).  When the first
  // selection stage picks that bucket and nspec equals its count, list A
  // holds the whole bucket (have_cand) and the refine passes read it instead
  // of every value; their candidates then follow it (from entry nspec).
  unsigned long long nspec;
  unsigned long long cnt0;      // entries in the first digit's chosen bucket
  int32_t spec;
  int32_t have_cand;
  unsigned long long pad_;
};

// A refine pass appends candidate keys only when the bucket it refines holds
// at most this many entries (a bigger bucket gets another histogram pass).
constexpr unsigned long long kCandCap = 16384;

struct SetDesc {
  int32_t kind, op, ncomp, thr;   // thr: index among threshold sets or -1
  int32_t axis[3];                // grid axis of each component (-1: identity)
  int32_t line_axis;              // line-wise set: grid axis of its lines; -1: whole vector
  double lo, hi, tau;
  int64_t k, rows;                // rows = M_i
  void* y; void* v;               // ncomp blocks of N
  void* vh0; void* v0; void* y0;  // adapt snapshots (ncomp blocks of N)
  void* lov; void* hiv;           // per-row bounds (ncomp blocks of N) or null
  // pipelines: [0] values w (every iteration), [1] values s (stopping test)
  SelState* sel[2];
  uint32_t* hcnt[2];
  double* hsum[2];
  void* cand[2];                  // candidate keys (u32 or u64), ncomp*N entries
  uint32_t* cand_ix;              // cardinality, pipeline 0: each candidate's item * 3 + component
  int32_t item_begin[2], item_end[2];  // threshold-item range of each pipeline
  int32_t line_begin, line_end;        // line-item range of a line-wise set
};

struct FastDiv {                  // n / d for 0 <= n < 2^31 (Granlund-Montgomery)
  uint32_t d, magic, shift;
};

struct InstDesc {
  int32_t ndim, nsets, active;
  int32_t vec_ok;                 // x and the workspace are 16-byte aligned: CG uses 128-bit groups
  int32_t vec_nb;                 // row strides are multiples of the group: 128-bit y/z neighbours
  int32_t cg2;                    // the batch runs this instance's CG steps in the LDS-staged form
  int64_t n[3];                   // axis sizes (3D: z, y, x; 2D: z, x, 1)
  int64_t N;
  int64_t cs;                     // element stride between operator components (N rounded up, 256-byte aligned)
  int64_t stride[3];              // element stride of each axis
  FastDiv div_x, div_y;           // point -> (row, x), row -> (z, y)
  double hinv[3], h2inv[3];
  void* m; void* x; void* r; void* p[2];
  void* cr[2]; void* cp[2];       // one-reduction CG: w = C r and s = C p, by step parity
  void* xs[2];                    // x snapshots of adapt-rho-gamma (alternating)
  void* ring;                     // x history for r_evol ((evol_hist + 1) blocks)
  void* yl; void* vl; void* vh0l; void* v0l; void* y0l;  // identity block p+1
  double* scal;                   // Scal block
  double* log;                    // schedule log or null
  int32_t pt_begin, pt_end;       // point-item range (RHS, CG)
  int32_t sp_begin, sp_end;       // projection-item range (finer tiles)
  int32_t log_cap, pad2_;
  SetDesc sets[SIP_MAX_SETS];
};

// Work items.  inst < 0 marks an entry past the live items of a launch;
// idx is the item's index in its table's logical order.
struct PtItem {                   // a range of grid points of one instance
  int32_t inst;
  int32_t begin, len;
  int32_t idx;
};

struct ThrItem {                  // a range of grid points of one pipeline
  int32_t inst, set, src, comp_parts;
  int32_t begin, len;
  int32_t idx, pipe;              // pipe: the pipeline's index in the selection table
};

struct SelItem {                  // one pipeline
  int32_t inst, set, src, pad_;
};

struct Opts {                     // options every kernel needs, by value
  int32_t cg_max, cg_fixed, adapt_every, stop_every, evol_hist, max_iter;
  int32_t sel_fresh;              // 1: no reuse of the previous first digit (SelState::spec stays 0)
  double cg_rel2, eps_corr, rho_ratio_max, gamma_max, eps_evol, eps_feas;
};

// One line of one component of a line-wise set: points start + t * stride,
// t = 0 .. len-1 (grid indexing of the component's block).
struct LineItem {
  int32_t inst, set, comp, len;
  int32_t start, stride;
  int32_t idx, pad_;
};

// Longest line a block sorts in LDS.
template <typename T> struct LineCap { static constexpr int v = sizeof(T) == 4 ? 4096 : 2048; };

// Device work tables and partial-sum buffers of one batch.  npt, nthr, nsel
// and ninst are the launch sizes (capacities); entries past the live items
// are sentinels (inst < 0).
struct Tables {
  const InstDesc* D;
  const PtItem* pt; int npt;
  const PtItem* sp; int nsp;
  const ThrItem* thr; int nthr;
  const SelItem* sel; int nsel;
  const int32_t* inst; int ninst;
  double* rr_part; double* pq_part; double* proj_part; double* thrw_part; double* thra_part;
  double* rr2_part; double* pq2_part;  // one-launch CG forms: odd-step partials
  double* xq_part; double* xq2_part;   // LDS-staged CG form: r^T s partials by step parity
  const LineItem* line; int nline;     // line items of line-wise sets
  int line_cap;                        // power of two >= the longest line (LDS entries per block)
  int proj_units;                      // projection blocks per item: max over instances of nsets + 2
  double* line_part;                   // 8 partial sums per line item
  uint32_t* tie_part;
  uint32_t* h1c; double* h1s;          // per pipeline (selection-table order): the refine histogram
                                       // when the first selection stage runs inside the refine pass
  int pt_threads;  // threads per block of the RHS and CG kernels (256 or 512)
  int cg_form;     // 0: two launches per CG step; 1: one (Chronopoulos-Gear); 2: one, LDS-staged (2D)
  int cg2_cap;     // form 2: LDS field values of p (longest item + 3 rows + 2 groups)
  int cg2_capr;    // form 2: LDS field values of r (longest item + 1 row + 1 group)
  int cg2_rest;    // form 2: some instances (3D, or rows too long for LDS) run the two-launch steps
  int sel_passes;  // refine + select passes after the first stage: 1 (it always compacts) or 2
  int fuse_sets;   // projection and w passes in one launch (small, latency-bound batches)
  int sel_fused;   // first selection stage done by every block of the (single) refine pass
};

// The first selection stage runs inside the refine pass (every block reads
// the 2048-bucket first-digit histogram) when the batch has one refine pass
// and at most this many threshold items.
constexpr int kFuseSelItems = 1024;

// The projection and w passes share a launch when the batch holds at most
// this many grid points (measured: one launch is faster up to a 4M-point
// grid, two launches for a 21M-point batch of 256 instances).
constexpr int64_t kFuseSetsPoints = 1 << 23;

// One refine pass (which then always appends candidates, and the select
// stage after it finishes over them) when every threshold pipeline of the
// batch has at most this many entries; two otherwise (the first appends only
// a bucket of at most kCandCap entries).
constexpr int64_t kOnePassRows = 1 << 19;

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.shift = s;
  // magic = floor(2^32 (2^s - d) / d) + 1; then n/d = (umulhi(n, magic) + n) >> s
  f.magic = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

__host__ __device__ inline uint32_t fastdiv(uint32_t n, const FastDiv& f) {
  const uint32_t t = (uint32_t)(((uint64_t)n * f.magic) >> 32);
  return (t + n) >> f.shift;
}

}  // namespace sip
