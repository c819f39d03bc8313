// gfx950 kernels of one PARSDMM iteration (PARSDMM listing; eq. SDMM_adaptive).
//
// Every kernel walks a work table: point items (a contiguous range of grid
// points of one instance), threshold items (a point range of one selection
// pipeline), selection items (one pipeline) or instances.  A table is stored
// in launch order, one entry per block of the launch: entry b is the item
// block b takes (with the item's index in the table's logical order, which
// orders its partial sums), and entries past the live items have inst < 0.
// The host orders the entries so that each of the 8 XCDs sweeps one
// contiguous slice of the logical table, which keeps the z/y neighbours a
// stencil reads in that XCD's L2; a block reads its entry with no other load
// before it.
//
// Reductions never use atomics on floating point across blocks except the
// histogram sums, which are exact for float keys (all values in one bucket
// share an exponent).  Each item writes its partial sums; the consumer
// (next launch) reduces an instance's partials in a fixed order, so results
// do not depend on which other instances share the launch.
#include <hip/hip_runtime.h>

#include "sip_internal.h"

// Accumulator type of every reduction (dot products, norms, histogram and
// prefix sums).  The library is built twice from this file: FP64
// accumulation (namespace r64, the default) and FP32 accumulation (r32, the
// precision ablation, selected by sip_opts.reduce).
#ifndef SIP_ACC
#define SIP_ACC double
#define SIP_KNS r64
#endif

namespace sip {
namespace SIP_KNS {

using acc_t = SIP_ACC;

// Threads per block of the set and threshold kernels: more registers per
// thread and no partial reduction at start, so smaller blocks let several
// stay resident per CU (latency hiding on many small items).
constexpr int kSB = 256;
constexpr int kSW = kSB / 64;
// The RHS and projection kernels are held to at most 96 registers, five
// waves per SIMD (the compiler's own choice, 97-113 registers and four
// waves, measured 2-4% slower on the 256-instance batch; six waves spill).
#define SIP_SETS_ATTR __attribute__((amdgpu_waves_per_eu(5)))
#define SIP_RHS_ATTR __attribute__((amdgpu_waves_per_eu(5)))

// Rounds of 16-byte groups a refine-pass thread loads before it bins any
// (the pass has no store to overlap with: without this each round is one
// memory round trip).
#ifndef SIP_REFINE_ROUNDS
#define SIP_REFINE_ROUNDS 2
#endif
constexpr int kRefineRounds = SIP_REFINE_ROUNDS;

// ---------------------------------------------------------------- helpers

// Data-parallel-primitive (DPP) moves: lane permutations inside the VALU,
// with no LDS round trip.  Rows not in ROW_MASK receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ int dpp_mov_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// The value of lane i - 1 (lane 0 gets 0) and of lane i + 1 (lane 63 gets
// 0): whole-wave shifts by one lane.
template <typename T>
__device__ __forceinline__ T lane_prev(T v) { return dpp_mov<0x138>(v); }
template <typename T>
__device__ __forceinline__ T lane_next(T v) { return dpp_mov<0x130>(v); }

__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }

// Sum over the 64 lanes, the same value in every lane: pairs, quads, the two
// halves of each 8, of each 16 (every lane of a group adds the same two
// partial sums, and IEEE addition commutes), then row 0 into row 1 and row 2
// into row 3, then rows 0-1 into rows 2-3; lane 63 holds the total.  The
// order is fixed, so every wave of every block gets the same bits.
template <typename A>
__device__ __forceinline__ A wave_sum(A v) {
  v += dpp_mov<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);       // row_half_mirror
  v += dpp_mov<0x140>(v);       // row_mirror
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

// Deterministic block sum of NV doubles over NT threads (a fixed butterfly in
// each wave, then the wave totals in order by one thread per value); every
// thread gets the totals.  lds needs lds_sum<NV, NT>() doubles.
template <int NV, int NT = kBlock>
constexpr int lds_sum() { return NV * (NT / 64 + 1); }

template <int NV, int NT = kBlock, typename A>
__device__ __forceinline__ void block_sum(A (&v)[NV], A* lds) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[i * NW + w] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    A t = 0;
    for (int q = 0; q < NW; ++q) t += lds[threadIdx.x * NW + q];
    lds[NV * NW + threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = lds[NV * NW + i];
  __syncthreads();
}

// Sum of parts[i * stride + off .. + NV) over items i in [begin, end).
template <int NV, int NT = kBlock, typename A>
__device__ __forceinline__ void reduce_range(const double* __restrict__ parts, int begin, int end, int stride,
                                             int off, A (&out)[NV], A* lds) {
#pragma unroll
  for (int j = 0; j < NV; ++j) out[j] = 0;
  for (int i = begin + (int)threadIdx.x; i < end; i += NT) {
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] += (A)parts[(size_t)i * stride + off + j];
  }
  block_sum<NV, NT>(out, lds);
}

// Sum of parts[begin .. end) computed by every wave on its own (lanes stride
// the range, then the butterfly): no LDS, no barrier, and the same order, so
// the same value, in every wave of every block.
// The first kPre partials of each lane are loaded by part_issue without any
// wait, so these loads fly together with a kernel's other first loads;
// part_finish adds them, then any further ones, in index order.
constexpr int kPre = 8;

__device__ __forceinline__ double ldgd(const double* p) {
  return *(__attribute__((address_space(1))) const double*)p;
}

// Requires end > begin (every instance has point items).  Loads only: no
// branch and no use of the values, so nothing here waits for them.
__device__ __forceinline__ void part_issue(const double* __restrict__ parts, int begin, int end,
                                           double (&pre)[kPre]) {
  // a lane past the range reads entry begin; part_finish drops that value
  const int i0 = begin + (int)(threadIdx.x & 63);
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int i = i0 + 64 * k;
    pre[k] = ldgd(parts + (i < end ? i : begin));
  }
}

__device__ __forceinline__ acc_t part_finish(const double* __restrict__ parts, int begin, int end,
                                             const double (&pre)[kPre]) {
  const int i0 = begin + (int)(threadIdx.x & 63);
  acc_t t = 0;
#pragma unroll
  for (int k = 0; k < kPre; ++k) t += i0 + 64 * k < end ? (acc_t)pre[k] : (acc_t)0;
  for (int i = i0 + 64 * kPre; i < end; i += 64) t += (acc_t)ldgd(parts + i);
  return wave_sum(t);
}

__device__ __forceinline__ acc_t wave_reduce(const double* __restrict__ parts, int begin, int end) {
  if (end <= begin) return 0;
  double pre[kPre];
  part_issue(parts, begin, end, pre);
  return part_finish(parts, begin, end, pre);
}

// Block total of one double, valid in thread 0 only (one barrier; lds must
// not be in use by other threads).
// Block totals of NV values, valid in thread 0 only, with one barrier (the
// same summation order as block_sum); lds needs NV * NT / 64 entries.
template <int NV, int NT, typename A>
__device__ __forceinline__ void block_total_n(A (&v)[NV], A* lds) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[i * NW + (threadIdx.x >> 6)] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      A t = 0;
      for (int q = 0; q < NW; ++q) t += lds[i * NW + q];
      v[i] = t;
    }
  }
}

// Block totals of two doubles with one barrier (thread 0 only); lds needs
// 2 * NT / 64 entries.
template <int NT, typename A>
__device__ __forceinline__ void block_total2(A& a, A& b, A* lds) {
  constexpr int NW = NT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) { lds[threadIdx.x >> 6] = a; lds[NW + (threadIdx.x >> 6)] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    A ta = 0, tb = 0;
    for (int q = 0; q < NW; ++q) { ta += lds[q]; tb += lds[NW + q]; }
    a = ta;
    b = tb;
  }
}

template <int NT, typename A>
__device__ __forceinline__ A block_total(A v, A* lds) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  A t = 0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < NW; ++q) t += lds[q];
  }
  return t;
}


template <typename T> struct KeyT;
template <> struct KeyT<float> {
  using K = uint32_t;
  static constexpr int bits = 31;
  static constexpr int ndig = 3;
  __device__ static int width(int d) { return d == 0 ? 11 : 10; }
  __device__ static K key(float v) { return __float_as_uint(v) & 0x7fffffffu; }
  __device__ static double value(K k) { return (double)__uint_as_float(k); }
  static constexpr K inf_key = 0x7f800000u;
};
template <> struct KeyT<double> {
  using K = unsigned long long;
  static constexpr int bits = 63;
  static constexpr int ndig = 6;
  __device__ static int width(int d) { return d < 3 ? 11 : 10; }
  __device__ static K key(double v) { return (K)__double_as_longlong(v) & 0x7fffffffffffffffull; }
  __device__ static double value(K k) { return __longlong_as_double((long long)k); }
  static constexpr K inf_key = 0x7ff0000000000000ull;
};

// bit position of the lowest bit of digit d
template <typename T> __device__ __forceinline__ int digit_shift(int d) {
  int s = KeyT<T>::bits;
  for (int i = 0; i <= d; ++i) s -= KeyT<T>::width(i);
  return s;
}

struct Geo {
  int nz, ny, nx, sy, sz, N, cs;
  FastDiv dx, dy;
  __device__ explicit Geo(const InstDesc& d)
      : nz((int)d.n[0]), ny((int)d.n[1]), nx((int)d.n[2]), sy((int)d.stride[1]), sz((int)d.stride[0]),
        N((int)d.N), cs((int)d.cs), dx(d.div_x), dy(d.div_y) {}
  __device__ __forceinline__ void coords(int P, int& iz, int& iy, int& ix) const {
    const uint32_t row = fastdiv((uint32_t)P, dx);
    ix = P - (int)row * nx;
    const uint32_t zz = fastdiv(row, dy);
    iy = (int)row - (int)zz * ny;
    iz = (int)zz;
  }
};

// (C f)(P) for C = c0 I + sum_a c_a L_a with L_a the 1D Neumann Laplacian
// along axis a (D_a^T D_a up to 1/h_a^2, folded into c_a).  f(Q) is a functor.
template <typename T, typename F>
__device__ __forceinline__ T apply_C(F f, T fc, int P, int iz, int iy, int ix, const Geo& g, T c0, T cz,
                                     T cy, T cx) {
  T lz = 0, ly = 0, lx = 0;
  if (iz > 0) lz += fc - f(P - g.sz);
  if (iz < g.nz - 1) lz += fc - f(P + g.sz);
  if (iy > 0) ly += fc - f(P - g.sy);
  if (iy < g.ny - 1) ly += fc - f(P + g.sy);
  if (ix > 0) lx += fc - f(P - 1);
  if (ix < g.nx - 1) lx += fc - f(P + 1);
  return c0 * fc + cz * lz + cy * ly + cx * lx;
}


// The scalars the RHS and CG kernels read, loaded together at kernel start
// (one round trip instead of one per use).
struct CgScal {
  double c0, cax[3], rr[2], done[2], rr0, state, err;
  __device__ __forceinline__ bool live() const { return state == 0.0 && err == 0.0; }
  // by step parity (selects, not an indexed access, so the block stays in registers)
  __device__ __forceinline__ double rr_at(int j) const { return (j & 1) ? rr[1] : rr[0]; }
  __device__ __forceinline__ double done_at(int j) const { return (j & 1) ? done[1] : done[0]; }
};

__device__ __forceinline__ CgScal cg_scal(const double* S) {
  CgScal q;
  q.c0 = ldgd(S + S_C0);
#pragma unroll
  for (int a = 0; a < 3; ++a) q.cax[a] = ldgd(S + S_CAX + a);
#pragma unroll
  for (int a = 0; a < 2; ++a) { q.rr[a] = ldgd(S + S_RR + a); q.done[a] = ldgd(S + S_DONE + a); }
  q.rr0 = ldgd(S + S_RR0);
  q.state = ldgd(S + S_STATE);
  q.err = ldgd(S + S_ERR);
  return q;
}

// The iteration scalars every set and selection kernel reads first, loaded
// together (one round trip instead of one per use).
struct ItScal {
  double state, err, k, have;
  __device__ __forceinline__ bool live() const { return state == 0.0 && err == 0.0; }
};

__device__ __forceinline__ ItScal it_scal(const double* S) {
  ItScal q;
  q.state = ldgd(S + S_STATE);
  q.err = ldgd(S + S_ERR);
  q.k = ldgd(S + S_K);
  q.have = ldgd(S + S_HAVE_SNAP);
  return q;
}

__device__ __forceinline__ bool is_adapt_iter(int k, const Opts& o) {
  return o.adapt_every > 0 && (k % o.adapt_every) == (1 % o.adapt_every);
}
__device__ __forceinline__ bool is_check_iter(int k, const Opts& o) {
  return o.stop_every > 0 && (k % o.stop_every) == 0 && k >= o.evol_hist;
}
__device__ __forceinline__ int adapt_call(int k, const Opts& o) { return (k - 1) / o.adapt_every + 1; }

// s = (A x) component along `axis` at P (forward difference), valid when the
// point is not on the last layer of that axis; axis < 0 is the identity.
template <typename T>
__device__ __forceinline__ bool comp_value(const T* x, int P, int axis, int iz, int iy, int ix, const Geo& g,
                                           const InstDesc& d, T& s) {
  if (axis < 0) { s = x[P]; return true; }
  if (axis == 0) { if (iz >= g.nz - 1) return false; s = (x[P + g.sz] - x[P]) * (T)d.hinv[0]; return true; }
  if (axis == 1) { if (iy >= g.ny - 1) return false; s = (x[P + g.sy] - x[P]) * (T)d.hinv[1]; return true; }
  if (ix >= g.nx - 1) return false;
  s = (x[P + 1] - x[P]) * (T)d.hinv[2];
  return true;
}

__device__ __forceinline__ bool comp_valid(int axis, int iz, int iy, int ix, const Geo& g) {
  if (axis < 0) return true;
  if (axis == 0) return iz < g.nz - 1;
  if (axis == 1) return iy < g.ny - 1;
  return ix < g.nx - 1;
}

// ------------------------------------------------------------ initialise

// Admission of one instance: x = m, y_i = A_i m, v_i = 0, y_{p+1} = m,
// v_{p+1} = 0, x-history slot 0 = m, clear selection histograms and states.
// d.m is the instance's private copy of m.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const InstDesc* __restrict__ D, int inst) {
  const InstDesc& d = D[inst];
  const Geo g(d);
  const T* m = (const T*)d.m;
  T* x = (T*)d.x;
  T* yl = (T*)d.yl;
  T* vl = (T*)d.vl;
  T* ring = (T*)d.ring;
  if (blockIdx.x == 0) {
    // the selection pipelines start from clear histograms and states
    for (int si = 0; si < d.nsets; ++si) {
      const SetDesc& s = d.sets[si];
      for (int src = 0; src < 2; ++src) {
        if (!s.hcnt[src]) continue;
        for (int b = threadIdx.x; b < kNB; b += kBlock) {
          s.hcnt[src][b] = 0u;
          s.hsum[src][b] = 0.0;
        }
        uint32_t* q = (uint32_t*)s.sel[src];
        for (int w = threadIdx.x; w < (int)(sizeof(SelState) / 4); w += kBlock) q[w] = 0u;
      }
    }
  }
  for (int P = blockIdx.x * kBlock + (int)threadIdx.x; P < g.N; P += gridDim.x * kBlock) {
    int iz, iy, ix;
    g.coords(P, iz, iy, ix);
    const T mv = m[P];
    x[P] = mv;
    yl[P] = mv;
    vl[P] = 0;
    if (ring) ring[P] = mv;
    for (int si = 0; si < d.nsets; ++si) {
      const SetDesc& s = d.sets[si];
      for (int c = 0; c < s.ncomp; ++c) {
        T val = 0;
        if (!comp_value<T>(m, P, s.axis[c], iz, iy, ix, g, d, val)) val = 0;
        ((T*)s.y)[(size_t)c * g.cs + P] = val;
        ((T*)s.v)[(size_t)c * g.cs + P] = 0;
      }
    }
  }
}

// ------------------------------------------------------- 16-byte groups

// 16-byte groups: a thread owns W = 16 / sizeof(T) consecutive points of an
// item and loads / stores them with one 128-bit global access.  Neighbours
// along x come from the adjacent lanes (shuffles; a lane whose neighbour lane
// has no group loads the value itself).  A neighbour window along y or z (the
// W values at P0 +- stride) starts (stride mod W) into an aligned group: the
// one or two aligned groups it covers are loaded and the window is picked
// out with the wave-uniform offset, so the loads of a round are all issued
// before any of them is waited for.  Every group address is aligned and
// starts in [0, N); an address outside is replaced by the lane's own group,
// whose values are then unused.  State arrays are padded to whole groups;
// the caller's x is not, so its last, partial group is read element by
// element (indexes clamped to N - 1) and written element by element.
template <typename T>
struct Grp {
  static constexpr int W = 16 / (int)sizeof(T);
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_cu32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

template <typename T>
__device__ __forceinline__ void ld16(const T* p, T (&o)[Grp<T>::W]) {
  const u32x4 u = *(g_cu32x4*)p;
  __builtin_memcpy(o, &u, 16);
}

template <typename T>
__device__ __forceinline__ void st16(T* p, const T (&o)[Grp<T>::W]) {
  u32x4 u;
  __builtin_memcpy(&u, o, 16);
  *(g_u32x4*)p = u;
}

// A streaming store (non-temporal hint): for arrays not read again before
// they would leave the caches (the projection and apply passes' y_i, v_i and
// snapshots; 0.3-0.5% on the 256-instance batch).
template <typename T>
__device__ __forceinline__ void st16nt(T* p, const T (&o)[Grp<T>::W]) {
  u32x4 u;
  __builtin_memcpy(&u, o, 16);
  __builtin_nontemporal_store(u, (g_u32x4*)p);
}

// The first W - 1 values of an aligned group (12 or 8 bytes).
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(1))) const u32x3 g_cu32x3;

template <typename T>
__device__ __forceinline__ void ld_head(const T* p, T (&o)[Grp<T>::W]) {
  if constexpr (sizeof(T) == 4) {
    const u32x3 u = *(g_cu32x3*)p;
    __builtin_memcpy(o, &u, 12);
    o[3] = (T)0;
  } else {
    o[0] = *(__attribute__((address_space(1))) const T*)p;
    o[1] = (T)0;
  }
}

template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(__attribute__((address_space(1))) const T*)p;
}

// Group loads that stay inside an unpadded array of N values (the values
// past N - 1 are copies of the last one and are never used).
template <typename T>
__device__ __forceinline__ void ld16p(const T* p, int G, int N, T (&o)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  if (G + W <= N) {
    ld16<T>(p + G, o);
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) o[e] = ldg(p + (G + e < N ? G + e : N - 1));
  }
}

template <typename T>
__device__ __forceinline__ void ld_headp(const T* p, int G, int N, T (&o)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  if (G + W - 1 <= N) {
    ld_head<T>(p + G, o);
  } else {
#pragma unroll
    for (int e = 0; e < W - 1; ++e) o[e] = ldg(p + (G + e < N ? G + e : N - 1));
    o[W - 1] = (T)0;
  }
}

// Store of the first cnt values of a group.
template <typename T>
__device__ __forceinline__ void st16p(T* p, int G, int cnt, const T (&o)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  if (cnt == W) {
    st16<T>(p + G, o);
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e)
      if (e < cnt) *(__attribute__((address_space(1))) T*)(p + G + e) = o[e];
  }
}

// o[e] = (A followed by B)[e + off] for a wave-uniform off in [0, W).
template <typename T>
__device__ __forceinline__ void pick(int off, const T (&A)[Grp<T>::W], const T (&B)[Grp<T>::W],
                                     T (&o)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    T v = A[e];
#pragma unroll
    for (int k = 1; k < W; ++k) {
      const T c = e + k < W ? A[(e + k) % W] : B[(e + k) % W];
      v = off == k ? c : v;
    }
    o[e] = v;
  }
}

// A stencil operand: value(Q) = a[0][Q] (NA = 1), a[0][Q] + beta a[1][Q]
// (NA = 2) or a[0][Q] + beta (a[1][Q] + beta2 a[2][Q]) (NA = 3).
template <typename T, int NA>
struct Src {
  const T* a[NA];
  T beta;
  T beta2;
};

template <typename T, int NA>
__device__ __forceinline__ T src_comb(const Src<T, NA>& f, T a0, T a1, T a2) {
  if constexpr (NA == 1) return a0;
  else if constexpr (NA == 2) return a0 + f.beta * a1;
  else return a0 + f.beta * (a1 + f.beta2 * a2);
}

// The operand at one point, by element loads.
template <typename T, int NA>
__device__ __forceinline__ T src_at(const Src<T, NA>& f, int Q) {
  return src_comb<T, NA>(f, f.a[0][Q], NA > 1 ? f.a[NA > 1 ? 1 : 0][Q] : (T)0, NA > 2 ? f.a[NA > 2 ? 2 : 0][Q] : (T)0);
}

template <typename T, int NA>
__device__ __forceinline__ void src_load(const Src<T, NA>& f, int G, int N, T (&R)[NA][Grp<T>::W]) {
#pragma unroll
  for (int q = 0; q < NA; ++q) ld16p<T>(f.a[q], G, N, R[q]);
}

template <typename T, int NA>
__device__ __forceinline__ void src_mix(const Src<T, NA>& f, const T (&R)[NA][Grp<T>::W], T (&o)[Grp<T>::W]) {
#pragma unroll
  for (int e = 0; e < Grp<T>::W; ++e)
    o[e] = src_comb<T, NA>(f, R[0][e], R[NA > 1 ? 1 : 0][e], R[NA > 2 ? 2 : 0][e]);
}

template <typename T, int NA>
__device__ __forceinline__ void src_load_head(const Src<T, NA>& f, int G, int N, T (&R)[NA][Grp<T>::W]) {
#pragma unroll
  for (int q = 0; q < NA; ++q) ld_headp<T>(f.a[q], G, N, R[q]);
}

template <typename T, int NA>
__device__ __forceinline__ T src_one(const Src<T, NA>& f, const T (&r)[NA]) {
  return src_comb<T, NA>(f, r[0], r[NA > 1 ? 1 : 0], r[NA > 2 ? 2 : 0]);
}

// Loads of the window at P0c + delta (off = (P0c + delta) mod W).  AL: the
// row strides are multiples of W, so off = 0 and one aligned group suffices.
template <typename T, int NA, bool AL>
__device__ __forceinline__ void win_load(const Src<T, NA>& f, int P0c, int delta, int off, int N,
                                         T (&A)[NA][Grp<T>::W], T (&B)[NA][Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  const int ga = P0c + delta - off, gb = ga + W;
  src_load<T, NA>(f, (unsigned)ga < (unsigned)N ? ga : P0c, N, A);
  if constexpr (!AL) src_load_head<T, NA>(f, (unsigned)gb < (unsigned)N ? gb : P0c, N, B);  // pick() reads B[0..W-2]
}

template <typename T, int NA, bool AL>
__device__ __forceinline__ void win_get(const Src<T, NA>& f, int off, const T (&A)[NA][Grp<T>::W],
                                        const T (&B)[NA][Grp<T>::W], T (&o)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  if constexpr (AL) {
    src_mix<T, NA>(f, A, o);
  } else {
    T a[W], b[W];
    src_mix<T, NA>(f, A, a);
    src_mix<T, NA>(f, B, b);
    pick<T>(off, a, b, o);
  }
}

// Window offsets of the four y/z directions.
struct Offs {
  int ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ Offs offs_of(const Geo& g) {
  constexpr int W = Grp<T>::W;
  Offs o;
  o.yp = g.sy & (W - 1);
  o.ym = (W - o.yp) & (W - 1);
  o.zp = g.sz & (W - 1);
  o.zm = (W - o.zp) & (W - 1);
  return o;
}

// Row strides are multiples of W (every window offset is 0).
template <typename T>
__device__ __forceinline__ bool rows_aligned(const Geo& g) {
  return (g.nx & (Grp<T>::W - 1)) == 0;
}

// Whether the instance uses the group path (its x buffer is 16-byte aligned).
__device__ __forceinline__ bool item_grouped(const InstDesc& d) { return d.vec_ok != 0; }

// One thread's group of one round.
struct GLane {
  int P0c;        // the group's first point (a safe aligned group if !vec)
  int cnt;        // points of the group inside the item (1..W if vec)
  bool vec;       // the group has points in the item
  bool next_vec;  // so has the next lane's
  int iz, iy, ix0;
  bool straddle;  // the group crosses the end of an x row
};

template <typename T>
__device__ __forceinline__ GLane glane(int P0, int begin, int end, const Geo& g) {
  constexpr int W = Grp<T>::W;
  GLane L;
  L.vec = P0 < end;
  L.cnt = end - P0 < W ? end - P0 : W;
  L.next_vec = dpp_mov_i<0x130>(L.vec ? 1 : 0) != 0;  // lane i + 1 (lane 63: none)
  L.P0c = L.vec ? P0 : begin;
  g.coords(L.P0c, L.iz, L.iy, L.ix0);
  L.straddle = L.ix0 + W > g.nx;
  return L;
}

// c = the operand at the lane's group, q = C c (all lanes of the wave call
// this; the result is meaningful where L.vec).  HY: the grid has a y axis
// (3D); z windows are always read (clamped and unused when nz = 1).
template <typename T, int NA, bool HY, bool AL>
__device__ __forceinline__ void group_C_v(const Src<T, NA>& f, const GLane& L, int lane, const Geo& g,
                                          const Offs& of, T (&R)[NA][Grp<T>::W], T (&c)[Grp<T>::W],
                                          T (&q)[Grp<T>::W], T c0, T cz, T cy, T cx) {
  constexpr int W = Grp<T>::W;
  const int N = g.N;
  T yma[NA][W], ymb[NA][W], ypa[NA][W], ypb[NA][W], zma[NA][W], zmb[NA][W], zpa[NA][W], zpb[NA][W];
  src_load<T, NA>(f, L.P0c, N, R);
  if constexpr (HY) {
    win_load<T, NA, AL>(f, L.P0c, -g.sy, of.ym, N, yma, ymb);
    win_load<T, NA, AL>(f, L.P0c, g.sy, of.yp, N, ypa, ypb);
  }
  win_load<T, NA, AL>(f, L.P0c, -g.sz, of.zm, N, zma, zmb);
  win_load<T, NA, AL>(f, L.P0c, g.sz, of.zp, N, zpa, zpb);
  T le[NA], re[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) { le[a] = 0; re[a] = 0; }
  const bool own_right = lane == 63 || !L.next_vec;
  if (lane == 0 && L.P0c > 0) {
#pragma unroll
    for (int a = 0; a < NA; ++a) le[a] = ldg(f.a[a] + L.P0c - 1);
  }
  if (own_right && L.P0c + W < g.N) {
#pragma unroll
    for (int a = 0; a < NA; ++a) re[a] = ldg(f.a[a] + L.P0c + W);
  }
  src_mix<T, NA>(f, R, c);
  T left = lane_prev(c[W - 1]);
  T right = lane_next(c[0]);
  if (lane == 0) left = src_one<T, NA>(f, le);
  if (own_right) right = src_one<T, NA>(f, re);
  T ym[W], yp[W], zm[W], zp[W];
  if constexpr (HY) {
    win_get<T, NA, AL>(f, of.ym, yma, ymb, ym);
    win_get<T, NA, AL>(f, of.yp, ypa, ypb, yp);
  }
  win_get<T, NA, AL>(f, of.zm, zma, zmb, zm);
  win_get<T, NA, AL>(f, of.zp, zpa, zpb, zp);
#pragma unroll
  for (int e = 0; e < W; ++e) {
    int ize = L.iz, iye = L.iy, ixe = L.ix0 + e;
    if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
    const T ce = c[e];
    const T lft = e > 0 ? c[e > 0 ? e - 1 : 0] : left;
    const T rgt = e < W - 1 ? c[e < W - 1 ? e + 1 : W - 1] : right;
    T lx = 0, ly = 0, lz = 0;
    if (ixe > 0) lx += ce - lft;
    if (ixe < g.nx - 1) lx += ce - rgt;
    if constexpr (HY) {
      if (iye > 0) ly += ce - ym[e];
      if (iye < g.ny - 1) ly += ce - yp[e];
    }
    if (ize > 0) lz += ce - zm[e];
    if (ize < g.nz - 1) lz += ce - zp[e];
    q[e] = c0 * ce + cz * lz + cy * ly + cx * lx;
  }
}

// R: the operand's own arrays at the group, as loaded.
template <typename T, int NA>
__device__ __forceinline__ void group_C_R(const Src<T, NA>& f, const GLane& L, int lane, const Geo& g,
                                          const Offs& of, T (&R)[NA][Grp<T>::W], T (&c)[Grp<T>::W],
                                          T (&q)[Grp<T>::W], T c0, T cz, T cy, T cx) {
  const bool al = rows_aligned<T>(g);
  if (g.ny > 1) {
    if (al) group_C_v<T, NA, true, true>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
    else group_C_v<T, NA, true, false>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
  } else {
    if (al) group_C_v<T, NA, false, true>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
    else group_C_v<T, NA, false, false>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
  }
}

template <typename T, int NA>
__device__ __forceinline__ void group_C(const Src<T, NA>& f, const GLane& L, int lane, const Geo& g, const Offs& of,
                                        T (&c)[Grp<T>::W], T (&q)[Grp<T>::W], T c0, T cz, T cy, T cx) {
  T R[NA][Grp<T>::W];
  group_C_R<T, NA>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
}

// (C f)(P) at one point, f given by a scalar fetch.
template <typename T, typename FS>
__device__ __forceinline__ T point_apply_C(int P, const Geo& g, FS f, T fc, T c0, T cz, T cy, T cx) {
  int iz, iy, ix;
  g.coords(P, iz, iy, ix);
  T lz = 0, ly = 0, lx = 0;
  if (iz > 0) lz += fc - f(P - g.sz);
  if (iz < g.nz - 1) lz += fc - f(P + g.sz);
  if (iy > 0) ly += fc - f(P - g.sy);
  if (iy < g.ny - 1) ly += fc - f(P + g.sy);
  if (ix > 0) lx += fc - f(P - 1);
  if (ix < g.nx - 1) lx += fc - f(P + 1);
  return c0 * fc + cz * lz + cy * ly + cx * lx;
}

// s = (A_axis f) at the lane's group (f itself for axis < 0); valid[e] false
// on the last layer along the axis (no such row; s = 0 there).  All lanes of
// the wave call this; the result is meaningful where L.vec.
template <typename T>
__device__ __forceinline__ void group_diff(const T* f, const GLane& L, int lane, const Geo& g, const InstDesc& d,
                                           const Offs& of, int axis, T (&s)[Grp<T>::W], bool (&valid)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
  const Src<T, 1> src{{f}, (T)0};
  T R[1][W], wa[1][W], wb[1][W];
  src_load<T, 1>(src, L.P0c, g.N, R);
  if (axis < 0) {
#pragma unroll
    for (int e = 0; e < W; ++e) { s[e] = R[0][e]; valid[e] = e < L.cnt; }
    return;
  }
  const T h = (T)d.hinv[axis];
  if (axis == 2) {
    const bool own_right = lane == 63 || !L.next_vec;
    T re = 0;
    if (own_right && L.P0c + W < g.N) re = ldg(f + L.P0c + W);
    T right = lane_next(R[0][0]);
    if (own_right) right = re;
#pragma unroll
    for (int e = 0; e < W; ++e) {
      int ize, iye, ixe = L.ix0 + e;
      if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
      valid[e] = e < L.cnt && ixe < g.nx - 1;
      const T nxt = e < W - 1 ? R[0][e < W - 1 ? e + 1 : W - 1] : right;
      s[e] = valid[e] ? (nxt - R[0][e]) * h : (T)0;
    }
    return;
  }
  const int st = axis == 0 ? g.sz : g.sy, off = axis == 0 ? of.zp : of.yp;
  T nb[W];
  if (rows_aligned<T>(g)) {
    win_load<T, 1, true>(src, L.P0c, st, off, g.N, wa, wb);
    win_get<T, 1, true>(src, off, wa, wb, nb);
  } else {
    win_load<T, 1, false>(src, L.P0c, st, off, g.N, wa, wb);
    win_get<T, 1, false>(src, off, wa, wb, nb);
  }
#pragma unroll
  for (int e = 0; e < W; ++e) {
    int ize = L.iz, iye = L.iy, ixe;
    if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
    valid[e] = e < L.cnt && (axis == 0 ? ize < g.nz - 1 : iye < g.ny - 1);
    s[e] = valid[e] ? (nb[e] - R[0][e]) * h : (T)0;
  }
}

// Coordinates-only validity of a component at the points of a group.
template <typename T>
__device__ __forceinline__ void group_valid(const GLane& L, const Geo& g, int axis, bool (&valid)[Grp<T>::W]) {
  constexpr int W = Grp<T>::W;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    int ize = L.iz, iye = L.iy, ixe = L.ix0 + e;
    if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
    valid[e] = e < L.cnt && comp_valid(axis, ize, iye, ixe, g);
  }
}

// Step j, first half: beta = rr_j / rr_{j-1}; p_j = r + beta p_{j-1} (p_0 = r);
// partial p_j^T C p_j.  With C = c0 I + sum_a c_a D_a^T D_a (unit forward
// differences), p^T C p = c0 |p|^2 + sum_a c_a |D_a p|^2: only the forward
// neighbours are read (half the windows of C p), and every term is a square.
template <typename T, int NA, bool HY, bool AL>
__device__ __forceinline__ acc_t group_pCp_v(const Src<T, NA>& f, const GLane& L, int lane, const Geo& g,
                                              const Offs& of, T (&c)[Grp<T>::W], const double (&cf)[4]) {
  constexpr int W = Grp<T>::W;
  const int N = g.N;
  T R[NA][W], ypa[NA][W], ypb[NA][W], zpa[NA][W], zpb[NA][W];
  src_load<T, NA>(f, L.P0c, N, R);
  if constexpr (HY) win_load<T, NA, AL>(f, L.P0c, g.sy, of.yp, N, ypa, ypb);
  win_load<T, NA, AL>(f, L.P0c, g.sz, of.zp, N, zpa, zpb);
  T re[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) re[a] = 0;
  const bool own_right = lane == 63 || !L.next_vec;
  if (own_right && L.P0c + W < N) {
#pragma unroll
    for (int a = 0; a < NA; ++a) re[a] = ldg(f.a[a] + L.P0c + W);
  }
  src_mix<T, NA>(f, R, c);
  T right = lane_next(c[0]);
  if (own_right) right = src_one<T, NA>(f, re);
  T yp[W], zp[W];
  if constexpr (HY) win_get<T, NA, AL>(f, of.yp, ypa, ypb, yp);
  win_get<T, NA, AL>(f, of.zp, zpa, zpb, zp);
  acc_t acc = 0;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    int ize = L.iz, iye = L.iy, ixe = L.ix0 + e;
    if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
    const acc_t ce = (acc_t)c[e];
    const acc_t rgt = (acc_t)(e < W - 1 ? c[e < W - 1 ? e + 1 : W - 1] : right);
    acc_t t = (acc_t)cf[0] * ce * ce;
    if (ixe < g.nx - 1) t += (acc_t)cf[3] * (rgt - ce) * (rgt - ce);
    if constexpr (HY) {
      if (iye < g.ny - 1) t += (acc_t)cf[2] * ((acc_t)yp[e] - ce) * ((acc_t)yp[e] - ce);
    }
    if (ize < g.nz - 1) t += (acc_t)cf[1] * ((acc_t)zp[e] - ce) * ((acc_t)zp[e] - ce);
    if (e < L.cnt) acc += t;
  }
  return acc;
}

template <typename T, int NA, int NT, bool ST = true>
__device__ __forceinline__ acc_t cg_dir_item(const InstDesc& d, const PtItem& it, const Geo& g, const Src<T, NA>& f,
                                              T* __restrict__ pout, const double (&cf)[4]) {
  constexpr int W = Grp<T>::W;
  const int lane = threadIdx.x & 63;
  const int end = it.begin + it.len;
  const bool grouped = item_grouped(d);
  const bool al = rows_aligned<T>(g);
  const bool hy = g.ny > 1;
  const Offs of = offs_of<T>(g);
  auto fs = [&](int Q) -> acc_t {
    if constexpr (NA == 1) return (acc_t)f.a[0][Q];
    else return (acc_t)(f.a[0][Q] + f.beta * f.a[1][Q]);
  };
  acc_t acc = 0;
  for (int base = it.begin; base < end; base += NT * W) {
    const int P0 = base + (int)threadIdx.x * W;
    bool vec = false;
    if (grouped) {
      const GLane L = glane<T>(P0, it.begin, end, g);
      T c[W];
      acc_t t;
      if (hy) t = al ? group_pCp_v<T, NA, true, true>(f, L, lane, g, of, c, cf)
                     : group_pCp_v<T, NA, true, false>(f, L, lane, g, of, c, cf);
      else t = al ? group_pCp_v<T, NA, false, true>(f, L, lane, g, of, c, cf)
                  : group_pCp_v<T, NA, false, false>(f, L, lane, g, of, c, cf);
      vec = L.vec;
      if (vec) {
        if constexpr (ST) st16<T>(pout + P0, c);
        acc += t;
      }
    }
    if (!vec) {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        int iz, iy, ix;
        g.coords(P, iz, iy, ix);
        const acc_t pc = fs(P);
        acc_t t = (acc_t)cf[0] * pc * pc;
        if (ix < g.nx - 1) { const acc_t dd = fs(P + 1) - pc; t += (acc_t)cf[3] * dd * dd; }
        if (iy < g.ny - 1) { const acc_t dd = fs(P + g.sy) - pc; t += (acc_t)cf[2] * dd * dd; }
        if (iz < g.nz - 1) { const acc_t dd = fs(P + g.sz) - pc; t += (acc_t)cf[1] * dd * dd; }
        if constexpr (ST) pout[P] = (T)pc;
        acc += t;
      }
    }
  }
  return acc;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_cg_dir(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, int j,
                                                const double* rr_part, double* pq_part, Opts o) {
  __shared__ acc_t lds[lds_sum<1, NT>()];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  if (d.cg2) return;  // its steps run in k_cg2_step
  double* S = d.scal;
  const CgScal q = cg_scal(S);
  double pre[kPre];
  part_issue(rr_part, d.pt_begin, d.pt_end, pre);
  // the sum comes before the state checks: a load whose only uses follow a
  // branch is moved below it by the compiler, one more round trip
  const double rr = part_finish(rr_part, d.pt_begin, d.pt_end, pre);
  if (!q.live()) return;
  bool done;
  double beta = 0.0;
  if (j == 0) {
    done = !(rr > 0.0);
  } else {
    done = q.done_at(j - 1) != 0.0 || !(rr > 0.0) || (!o.cg_fixed && rr < o.cg_rel2 * q.rr0);
    beta = rr / q.rr_at(j - 1);
  }
  const bool bad = !(rr <= 1.0e300) || rr != rr;  // non-finite residual
  if (iti == d.pt_begin && threadIdx.x == 0) {
    S[S_RR + (j & 1)] = rr;
    S[S_DONE + (j & 1)] = (done || bad) ? 1.0 : 0.0;
    if (j == 0) S[S_RR0] = rr;
    if (bad) S[S_ERR] = (double)SIP_ENUMERIC;
  }
  if (done || bad) return;
  const Geo g(d);
  const T* r = (const T*)d.r;
  const T* pin = (const T*)d.p[(j + 1) & 1];
  T* pout = (T*)d.p[j & 1];
  const double cf[4] = {q.c0, q.cax[0], q.cax[1], q.cax[2]};
  acc_t acc;
  if (j == 0) {
    const Src<T, 1> f{{r}, (T)0};
    acc = cg_dir_item<T, 1, NT>(d, it, g, f, pout, cf);
  } else {
    const Src<T, 2> f{{r, pin}, (T)beta};
    acc = cg_dir_item<T, 2, NT>(d, it, g, f, pout, cf);
  }
  acc = block_total<NT>(acc, lds);
  if (threadIdx.x == 0) pq_part[iti] = acc;
}

// Step j, second half: alpha = rr_j / p^T C p; x += alpha p; r -= alpha C p
// (C p recomputed from p); partial r^T r.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_cg_upd(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, int j,
                                                const double* pq_part, double* rr_part) {
  constexpr int W = Grp<T>::W;
  __shared__ acc_t lds[lds_sum<1, NT>()];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  if (d.cg2) return;  // its steps run in k_cg2_step
  double* S = d.scal;
  const CgScal qs = cg_scal(S);
  double pre[kPre];
  part_issue(pq_part, d.pt_begin, d.pt_end, pre);
  // summed before the state checks (stale when this step is skipped)
  const double pq = part_finish(pq_part, d.pt_begin, d.pt_end, pre);
  if (!qs.live()) return;
  if (qs.done_at(j) != 0.0) return;
  if (!(pq > 0.0) || !(pq <= 1.0e300)) {
    if (iti == d.pt_begin && threadIdx.x == 0) S[S_ERR] = (double)SIP_ENUMERIC;
    return;
  }
  const double alpha = qs.rr_at(j) / pq;
  if (iti == d.pt_begin && threadIdx.x == 0) S[S_CGTOT] += 1.0;
  const Geo g(d);
  T* x = (T*)d.x;
  T* r = (T*)d.r;
  const T* p = (const T*)d.p[j & 1];
  const T c0 = (T)qs.c0, cz = (T)qs.cax[0], cy = (T)qs.cax[1], cx = (T)qs.cax[2];
  const T al = (T)alpha;
  auto fs = [&](int Q) -> T { return p[Q]; };
  const Src<T, 1> f{{p}, (T)0};
  const int lane = threadIdx.x & 63;
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  acc_t acc[1] = {0};
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += NT * W) {
    const int P0 = base + (int)threadIdx.x * W;
    bool vec = false;
    if (grouped) {
      const GLane L = glane<T>(P0, it.begin, end, g);
      T xv[W], rv[W], c[W], q[W];
      ld16p<T>(x, L.P0c, g.N, xv);
      ld16<T>(r + L.P0c, rv);
      group_C<T, 1>(f, L, lane, g, of, c, q, c0, cz, cy, cx);
      vec = L.vec;
      if (vec) {
#pragma unroll
        for (int e = 0; e < W; ++e) {
          xv[e] = xv[e] + al * c[e];
          rv[e] = rv[e] - al * q[e];
          if (e < L.cnt) acc[0] += (acc_t)rv[e] * (acc_t)rv[e];
        }
        st16p<T>(x, P0, L.cnt, xv);
        st16<T>(r + P0, rv);
      }
    }
    if (!vec) {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        const T pc = p[P];
        const T qq = point_apply_C<T>(P, g, fs, pc, c0, cz, cy, cx);
        x[P] = x[P] + al * pc;
        const T rv = r[P] - al * qq;
        r[P] = rv;
        acc[0] += (acc_t)rv * (acc_t)rv;
      }
    }
  }
  const acc_t tot = block_total<NT>(acc[0], lds);
  if (threadIdx.x == 0) rr_part[iti] = tot;
}

// ------------------------------------------------- one-reduction CG form
//
// Chronopoulos and Gear's arrangement of CG: both inner products a step needs
// (gamma = r^T r and delta = r^T C r) are taken from the same vectors, so a
// step is one launch.  Entering step j: x_j, r_j, w_j = C r_j, p_{j-1},
// s_{j-1} = C p_{j-1} and the per-item partials of gamma_j and delta_j.
//   beta_j  = gamma_j / gamma_{j-1}                        (0 at j = 0)
//   alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1})
// (the denominator is p_j^T C p_j), then
//   p_j = r_j + beta_j p_{j-1},  s_j = w_j + beta_j s_{j-1},
//   x_{j+1} = x_j + alpha_j p_j,  r_{j+1} = r_j - alpha_j s_j,
//   w_{j+1} = C r_{j+1}, and the partials of gamma_{j+1}, delta_{j+1}.
// In exact arithmetic these are the iterates of the two-launch form.  r, w
// and s alternate between two buffers by step parity (neighbours' old values
// are read while other blocks write the new ones); x and p are updated in
// place.  r_{j+1} at a neighbour is formed from r_j, w_j and s_{j-1} there by
// the same expression as at the point that owns it.

// w_0 = C r_0 and the partials of delta_0 = r_0^T w_0 (r_0 from the RHS kernel).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_cg1_w0(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, double* dpart) {
  constexpr int W = Grp<T>::W;
  __shared__ acc_t lds[lds_sum<1, NT>()];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const CgScal qs = cg_scal(d.scal);
  if (!qs.live()) return;
  const Geo g(d);
  const T* r = (const T*)d.r;
  T* w = (T*)d.cr[0];
  const T c0 = (T)qs.c0, cz = (T)qs.cax[0], cy = (T)qs.cax[1], cx = (T)qs.cax[2];
  const Src<T, 1> f{{r}, (T)0, (T)0};
  auto fs = [&](int Q) -> T { return r[Q]; };
  const int lane = threadIdx.x & 63;
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  acc_t acc = 0;
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += NT * W) {
    const int P0 = base + (int)threadIdx.x * W;
    bool vec = false;
    if (grouped) {
      const GLane L = glane<T>(P0, it.begin, end, g);
      T c[W], q[W];
      group_C<T, 1>(f, L, lane, g, of, c, q, c0, cz, cy, cx);
      vec = L.vec;
      if (vec) {
#pragma unroll
        for (int e = 0; e < W; ++e)
          if (e < L.cnt) acc += (acc_t)c[e] * (acc_t)q[e];
        st16<T>(w + P0, q);
      }
    }
    if (!vec) {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        const T rc = r[P];
        const T qq = point_apply_C<T>(P, g, fs, rc, c0, cz, cy, cx);
        w[P] = qq;
        acc += (acc_t)rc * (acc_t)qq;
      }
    }
  }
  const acc_t tot = block_total<NT>(acc, lds);
  if (threadIdx.x == 0) dpart[iti] = tot;
}

// Step j (NA = 2 at j = 0, where p_0 = r_0 and s_0 = w_0; NA = 3 after).
template <typename T, int NT, int NA>
__global__ __launch_bounds__(NT) void k_cg1_step(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, int j, const double* gin,
                                                  const double* din, double* gout, double* dout, Opts o) {
  constexpr int W = Grp<T>::W;
  __shared__ acc_t lds_g[2 * (NT / 64)];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  double* S = d.scal;
  const CgScal qs = cg_scal(S);
  const double alpha_prev = ldgd(S + S_ALPHA + ((j + 1) & 1));
  double pg[kPre], pd[kPre];
  part_issue(gin, d.pt_begin, d.pt_end, pg);
  part_issue(din, d.pt_begin, d.pt_end, pd);
  // summed before the state checks, so the partials' loads stay with the
  // scalars' (the values are stale when the checks end the step)
  const double gam = part_finish(gin, d.pt_begin, d.pt_end, pg);
  const double del = part_finish(din, d.pt_begin, d.pt_end, pd);
  if (!qs.live()) return;
  const bool leader = iti == d.pt_begin && threadIdx.x == 0;
  if (j > 0 && qs.done_at(j - 1) != 0.0) {
    // finished at an earlier step (this step's partials were never written)
    if (leader) S[S_DONE + (j & 1)] = 1.0;
    return;
  }
  bool done = !(gam > 0.0);
  double beta = 0.0;
  if (j > 0) {
    done = done || (!o.cg_fixed && gam < o.cg_rel2 * qs.rr0);
    beta = gam / qs.rr_at(j - 1);
  }
  const bool bad = !(gam <= 1.0e300) || gam != gam;
  if (leader) {
    S[S_RR + (j & 1)] = gam;
    S[S_DONE + (j & 1)] = (done || bad) ? 1.0 : 0.0;
    if (j == 0) S[S_RR0] = gam;
    if (bad) S[S_ERR] = (double)SIP_ENUMERIC;
  }
  if (done || bad) return;
  const double pq = j == 0 ? del : del - beta * gam / alpha_prev;
  if (!(pq > 0.0) || !(pq <= 1.0e300)) {
    if (leader) S[S_ERR] = (double)SIP_ENUMERIC;
    return;
  }
  const double alpha = gam / pq;
  if (leader) {
    S[S_ALPHA + (j & 1)] = alpha;
    S[S_CGTOT] += 1.0;
  }
  const Geo g(d);
  T* x = (T*)d.x;
  T* p = (T*)d.p[0];
  const T* rj = (const T*)((j & 1) ? d.p[1] : d.r);
  T* rn = (T*)((j & 1) ? d.r : d.p[1]);
  const T* wj = (const T*)d.cr[j & 1];
  T* wn = (T*)d.cr[(j + 1) & 1];
  const T* sprev = (const T*)d.cp[(j + 1) & 1];
  T* sj = (T*)d.cp[j & 1];
  const T al = (T)alpha, be = (T)beta;
  const T c0 = (T)qs.c0, cz = (T)qs.cax[0], cy = (T)qs.cax[1], cx = (T)qs.cax[2];
  Src<T, NA> f;
  f.a[0] = rj;
  f.a[1] = wj;
  if constexpr (NA == 3) f.a[2] = sprev;
  f.beta = -al;
  f.beta2 = be;
  auto fs = [&](int Q) -> T { return src_at<T, NA>(f, Q); };
  const int lane = threadIdx.x & 63;
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  acc_t ag = 0, ad = 0;
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += NT * W) {
    const int P0 = base + (int)threadIdx.x * W;
    bool vec = false;
    if (grouped) {
      const GLane L = glane<T>(P0, it.begin, end, g);
      T xv[W], pv[W], R[NA][W], c[W], q[W];
      ld16p<T>(x, L.P0c, g.N, xv);
      if constexpr (NA == 3) ld16<T>(p + L.P0c, pv);
      group_C_R<T, NA>(f, L, lane, g, of, R, c, q, c0, cz, cy, cx);
      vec = L.vec;
      if (vec) {
        T pn[W], sn[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          if constexpr (NA == 3) {
            pn[e] = R[0][e] + be * pv[e];
            sn[e] = R[1][e] + be * R[2][e];
          } else {
            pn[e] = R[0][e];
            sn[e] = R[1][e];
          }
          xv[e] = xv[e] + al * pn[e];
          if (e < L.cnt) {
            ag += (acc_t)c[e] * (acc_t)c[e];
            ad += (acc_t)c[e] * (acc_t)q[e];
          }
        }
        st16p<T>(x, P0, L.cnt, xv);
        st16<T>(p + P0, pn);
        st16<T>(sj + P0, sn);
        st16<T>(rn + P0, c);
        st16<T>(wn + P0, q);
      }
    }
    if (!vec) {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        const T rc = fs(P);
        const T qq = point_apply_C<T>(P, g, fs, rc, c0, cz, cy, cx);
        T pn, sn;
        if constexpr (NA == 3) {
          pn = rj[P] + be * p[P];
          sn = wj[P] + be * sprev[P];
        } else {
          pn = rj[P];
          sn = wj[P];
        }
        x[P] = x[P] + al * pn;
        p[P] = pn;
        sj[P] = sn;
        rn[P] = rc;
        wn[P] = qq;
        ag += (acc_t)rc * (acc_t)rc;
        ad += (acc_t)rc * (acc_t)qq;
      }
    }
  }
  block_total2<NT>(ag, ad, lds_g);
  if (threadIdx.x == 0) {
    gout[iti] = ag;
    dout[iti] = ad;
  }
}

// ------------------------------------------ one-launch CG form, LDS-staged (2D)
//
// The two-launch form's iterates with one launch per step and no stored
// C-products, for grids without a y axis: a step reads x_j, r_j and p_{j-1}
// and writes x_{j+1}, r_{j+1} and p_j (6 vectors instead of 8).  Entering step
// j: the per-item partials of gamma_j = r_j^T r_j and, for j > 0, of
// Q_j = r_j^T C r_j and X_j = r_j^T s_{j-1} (s = C p); at j = 0 those of
// r_0^T C r_0 (a pass over r_0) in place of Q_0.
//   beta_j = gamma_j / gamma_{j-1}                            (0 at j = 0)
//   p_j^T C p_j = Q_j + 2 beta_j X_j + beta_j^2 p_{j-1}^T C p_{j-1}
// (p_j = r_j + beta_j p_{j-1} expanded; r_0^T C r_0 at j = 0) and
// alpha_j = gamma_j / p_j^T C p_j; then at every point
//   p_j = r_j + beta_j p_{j-1},  s_j = C p_j,
//   x_{j+1} = x_j + alpha_j p_j,  r_{j+1} = r_j - alpha_j s_j,
// and the partials of gamma_{j+1}, X_{j+1} = r_{j+1}^T s_j and
// Q_{j+1} = c0 |r_{j+1}|^2 + sum_a c_a |D_a r_{j+1}|^2 (unit forward
// differences, c_a folding 1/h_a^2 as in C).  A block stages p_j of its
// item and of one row before and two after it, and r_j of its item and the
// row after it, in LDS, forms s_j and r_{j+1} there for its points and the
// row after them (the forward neighbours of its last row), then the partial
// sums, and writes its points' x_{j+1}, p_j and r_{j+1}.  p_j, s_j, x_{j+1} and r_{j+1} are the two-launch
// form's expressions in the same order; only the double p_j^T C p_j is
// summed another way.  r and p alternate between two buffers by step parity
// (neighbours' old values are read while other blocks write the new ones); x
// is updated in place.

// (C f) at one point from its value and its six neighbours' (those outside
// the grid are not used), in the order of the other stencil kernels.
template <typename T, bool HY>
__device__ __forceinline__ T stencil7(T ce, T lft, T rgt, T ym, T yp, T zm, T zp, int iz, int iy, int ix,
                                      const Geo& g, T c0, T cz, T cy, T cx) {
  T lx = 0, ly = 0, lz = 0;
  if (ix > 0) lx += ce - lft;
  if (ix < g.nx - 1) lx += ce - rgt;
  if constexpr (HY) {
    if (iy > 0) ly += ce - ym;
    if (iy < g.ny - 1) ly += ce - yp;
  }
  if (iz > 0) lz += ce - zm;
  if (iz < g.nz - 1) lz += ce - zp;
  return c0 * ce + cz * lz + cy * ly + cx * lx;
}

// r_0^T C r_0 per item (the denominator of step 0), from r_0 of the RHS kernel.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_cg2_d0(const InstDesc* __restrict__ D, const PtItem* __restrict__ items,
                                                double* qpart) {
  __shared__ acc_t lds[lds_sum<1, NT>()];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const InstDesc& d = D[it.inst];
  if (!d.cg2) return;  // an instance of the two-launch form
  const CgScal q = cg_scal(d.scal);
  if (!q.live()) return;
  const Geo g(d);
  const double cf[4] = {q.c0, q.cax[0], q.cax[1], q.cax[2]};
  const Src<T, 1> f{{(const T*)d.r}, (T)0};
  acc_t acc = cg_dir_item<T, 1, NT, false>(d, it, g, f, nullptr, cf);
  acc = block_total<NT>(acc, lds);
  if (threadIdx.x == 0) qpart[it.idx] = acc;
}

// Step j (NA = 1 at j = 0, where p_0 = r_0; NA = 2 after).  Dynamic LDS: p
// over the staged range (`cap` >= the longest item + 3 rows + 2 W field
// values), then r over the item and the row after it (the rest).
template <typename T, int NT, int NA>
__global__ __launch_bounds__(NT) void k_cg2_step(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, int j,
                                                  const double* gin, const double* qin, const double* xin,
                                                  double* gout, double* qout, double* xout, Opts o, int cap) {
  constexpr int W = Grp<T>::W;
  extern __shared__ __align__(16) unsigned char cg2_dyn[];
  __shared__ acc_t lds[lds_sum<3, NT>()];
  T* lp = (T*)cg2_dyn;  // p_j at P - s0
  T* lr = lp + cap;     // r_j, then r_{j+1}, at P - b
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  if (!d.cg2) return;  // an instance of the two-launch form
  double* S = d.scal;
  const CgScal qs = cg_scal(S);
  const double pcp_prev = ldgd(S + S_PCP + ((j + 1) & 1));
  double pg[kPre], pq[kPre], px[kPre];
  part_issue(gin, d.pt_begin, d.pt_end, pg);
  part_issue(qin, d.pt_begin, d.pt_end, pq);
  if (NA == 2) part_issue(xin, d.pt_begin, d.pt_end, px);
  // summed before the state checks, so the partials' loads stay with the
  // scalars' (the values are stale when the checks end the step)
  const double gam = part_finish(gin, d.pt_begin, d.pt_end, pg);
  const double qq = part_finish(qin, d.pt_begin, d.pt_end, pq);
  const double xx = NA == 2 ? part_finish(xin, d.pt_begin, d.pt_end, px) : 0.0;
  if (!qs.live()) return;
  const bool leader = iti == d.pt_begin && threadIdx.x == 0;
  if (j > 0 && qs.done_at(j - 1) != 0.0) {
    // finished at an earlier step (this step's partials were never written)
    if (leader) S[S_DONE + (j & 1)] = 1.0;
    return;
  }
  bool done = !(gam > 0.0);
  double beta = 0.0;
  if (j > 0) {
    done = done || (!o.cg_fixed && gam < o.cg_rel2 * qs.rr0);
    beta = gam / qs.rr_at(j - 1);
  }
  const bool bad = !(gam <= 1.0e300) || gam != gam;
  if (leader) {
    S[S_RR + (j & 1)] = gam;
    S[S_DONE + (j & 1)] = (done || bad) ? 1.0 : 0.0;
    if (j == 0) S[S_RR0] = gam;
    if (bad) S[S_ERR] = (double)SIP_ENUMERIC;
  }
  if (done || bad) return;
  const double pcp = j == 0 ? qq : qq + 2.0 * beta * xx + beta * beta * pcp_prev;
  if (!(pcp > 0.0) || !(pcp <= 1.0e300)) {
    if (leader) S[S_ERR] = (double)SIP_ENUMERIC;
    return;
  }
  const double alpha = gam / pcp;
  if (leader) {
    S[S_PCP + (j & 1)] = pcp;
    S[S_CGTOT] += 1.0;
  }
  const Geo g(d);
  const int N = g.N, nx = g.nx, nz = g.nz;
  T* x = (T*)d.x;
  const T* rj = (const T*)((j & 1) ? d.p[1] : d.r);
  T* rnb = (T*)((j & 1) ? d.r : d.p[1]);
  T* pnb = (T*)((j & 1) ? d.cr[0] : d.p[0]);
  const T* pold = (const T*)((j & 1) ? d.p[0] : d.cr[0]);
  const T al = (T)alpha, be = (T)beta;
  const T c0 = (T)qs.c0, cz = (T)qs.cax[0], cy = (T)qs.cax[1], cx = (T)qs.cax[2];
  const double cf[4] = {qs.c0, qs.cax[0], qs.cax[1], qs.cax[2]};
  const int b = it.begin, e = it.begin + it.len;
  // staged range of p: one row before the item and two after it, whole
  // groups (the work arrays are padded to whole 256-byte blocks past N); r
  // over the item and the row after it
  const int s0 = (b - nx > 0 ? b - nx : 0) & ~(W - 1);
  const int hi = e + 2 * nx < N ? e + 2 * nx : N;
  const int s1 = (hi + W - 1) & ~(W - 1);
  const int pe = e + nx < N ? e + nx : N;
  // x of the thread's first UX groups of the item, loaded with the staging
  // (x by elements when the caller's x is not 16-byte aligned)
  constexpr int UX = 2, UA = 4;
  const bool xvec = item_grouped(d);
  T xpre[UX][W];
#pragma unroll
  for (int a = 0; a < UX; ++a) {
    const int G = b + (int)threadIdx.x * W + a * NT * W;
    const int cnt = e - G < W ? e - G : W;
    if (G >= e) continue;
    if (xvec) {
      ld16p<T>(x, G, N, xpre[a]);
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u) xpre[a][u] = u < cnt ? x[G + u] : (T)0;
    }
  }
  for (int G0 = s0 + (int)threadIdx.x * W; G0 < s1; G0 += UA * NT * W) {
    T rv[UA][W], pv[UA][W];
#pragma unroll
    for (int a = 0; a < UA; ++a) {
      const int G = G0 + a * NT * W;
      if (G >= s1) continue;
      ld16<T>(rj + G, rv[a]);
      if constexpr (NA == 2) ld16<T>(pold + G, pv[a]);
    }
#pragma unroll
    for (int a = 0; a < UA; ++a) {
      const int G = G0 + a * NT * W;
      if (G >= s1) continue;
#pragma unroll
      for (int u = 0; u < W; ++u) pv[a][u] = NA == 2 ? rv[a][u] + be * pv[a][u] : rv[a][u];
      u32x4 ra, pa;
      __builtin_memcpy(&ra, rv[a], 16);
      __builtin_memcpy(&pa, pv[a], 16);
      if (G >= b && G < pe) *(u32x4*)(lr + (G - b)) = ra;
      *(u32x4*)(lp + (G - s0)) = pa;
    }
  }
  __syncthreads();
  // The stencil and update phases read LDS by whole groups (16 bytes per
  // lane, consecutive lanes on consecutive groups: no bank conflicts), the
  // row neighbours too when the row length is a multiple of W (then a
  // group never straddles two rows), and single values only at a group's
  // two ends.  Values read for a point outside the grid or past the staged
  // rows are never used (the stencil's bounds checks drop them).
  const bool zvec = d.vec_nb != 0;
  auto ldg = [&](const T* base, int q, T (&o)[W]) {
    const u32x4 v4 = *(const u32x4*)(base + q);
    __builtin_memcpy(o, &v4, 16);
  };
  // s = C p at the W points of the group at G (its centre values into pc)
  auto s_group = [&](int G, int iz0, int ix0, T (&pc)[W], T (&sv)[W]) {
    const int q0 = G - s0;
    ldg(lp, q0, pc);
    const T pl = lp[q0 > 0 ? q0 - 1 : 0], pr = lp[q0 + W];
    T up[W], dn[W];
    if (zvec) {
      if (iz0 > 0) ldg(lp, q0 - nx, up);
      else {
#pragma unroll
        for (int u = 0; u < W; ++u) up[u] = (T)0;
      }
      if (iz0 < nz - 1) ldg(lp, q0 + nx, dn);
      else {
#pragma unroll
        for (int u = 0; u < W; ++u) dn[u] = (T)0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u) {
        const int qu = q0 + u - nx, qd = q0 + u + nx;
        up[u] = qu >= 0 ? lp[qu] : (T)0;
        dn[u] = lp[qd];
      }
    }
#pragma unroll
    for (int u = 0; u < W; ++u) {
      int izu = iz0, iyu = 0, ixu = ix0 + u;
      if (ixu >= nx) g.coords(G + u, izu, iyu, ixu);
      const T lft = u == 0 ? pl : pc[u > 0 ? u - 1 : 0];
      const T rgt = u == W - 1 ? pr : pc[u < W - 1 ? u + 1 : 0];
      sv[u] = stencil7<T, false>(pc[u], lft, rgt, (T)0, (T)0, up[u], dn[u], izu, 0, ixu, g, c0, cz, cy, cx);
    }
  };
  // r_{j+1} over the item and the row after it, in place of r_j (the last
  // group's values past the row after it are never read); a thread's first
  // UX groups are its first UX groups of the item too, so their p_j, s_j
  // and r_{j+1} stay in registers for the sums and stores below
  auto r_next = [&](int G, T (&pc)[W], T (&sv)[W], T (&rv)[W]) {
    int iz0, iy0, ix0;
    g.coords(G, iz0, iy0, ix0);
    s_group(G, iz0, ix0, pc, sv);
    ldg(lr, G - b, rv);
#pragma unroll
    for (int u = 0; u < W; ++u) rv[u] = rv[u] - al * sv[u];
    u32x4 v4;
    __builtin_memcpy(&v4, rv, 16);
    *(u32x4*)(lr + (G - b)) = v4;
  };
  T pk[UX][W], sk[UX][W], rk[UX][W];
#pragma unroll
  for (int a = 0; a < UX; ++a) {
    const int G = b + (int)threadIdx.x * W + a * NT * W;
    if (G < pe) r_next(G, pk[a], sk[a], rk[a]);
  }
  for (int G = b + (int)threadIdx.x * W + UX * NT * W; G < pe; G += NT * W) {
    T pc[W], sv[W], rv[W];
    r_next(G, pc, sv, rv);
  }
  __syncthreads();
  // the item's points: partial sums and stores (pn = p_j, sv = s_j and
  // rn = r_{j+1} of the group)
  acc_t acc[3] = {0, 0, 0};  // gamma, Q, X
  auto point_group = [&](int G, T (&xv)[W], const T (&pn)[W], const T (&sv)[W], const T (&rn)[W]) {
    int iz0, iy0, ix0;
    g.coords(G, iz0, iy0, ix0);
    const int cnt = e - G < W ? e - G : W;
    const int q = G - b;
    T rz[W];
    const T rx = lr[q + W];
    if (zvec) {
      if (iz0 < nz - 1) ldg(lr, q + nx, rz);
      else {
#pragma unroll
        for (int u = 0; u < W; ++u) rz[u] = (T)0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u) rz[u] = lr[q + u + nx];
    }
#pragma unroll
    for (int u = 0; u < W; ++u) {
      xv[u] = xv[u] + al * pn[u];
      if (u >= cnt) continue;
      int izu = iz0, iyu = 0, ixu = ix0 + u;
      if (ixu >= nx) g.coords(G + u, izu, iyu, ixu);
      const acc_t rc = (acc_t)rn[u];
      acc[0] += rc * rc;
      acc[2] += rc * (acc_t)sv[u];
      acc_t t = (acc_t)cf[0] * rc * rc;
      if (ixu < nx - 1) {
        const acc_t dd = (acc_t)(u < W - 1 ? rn[u < W - 1 ? u + 1 : 0] : rx) - rc;
        t += (acc_t)cf[3] * dd * dd;
      }
      if (izu < nz - 1) { const acc_t dd = (acc_t)rz[u] - rc; t += (acc_t)cf[1] * dd * dd; }
      acc[1] += t;
    }
    if (xvec) {
      st16p<T>(x, G, cnt, xv);
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u)
        if (u < cnt) x[G + u] = xv[u];
    }
    st16<T>(pnb + G, pn);
    st16<T>(rnb + G, rn);
  };
#pragma unroll
  for (int a = 0; a < UX; ++a) {
    const int G = b + (int)threadIdx.x * W + a * NT * W;
    if (G < e) point_group(G, xpre[a], pk[a], sk[a], rk[a]);
  }
  for (int G = b + (int)threadIdx.x * W + UX * NT * W; G < e; G += NT * W) {
    const int cnt = e - G < W ? e - G : W;
    T xv[W], pn[W], sv[W], rn[W];
    if (xvec) {
      ld16p<T>(x, G, N, xv);
    } else {
#pragma unroll
      for (int u = 0; u < W; ++u) xv[u] = u < cnt ? x[G + u] : (T)0;
    }
    int iz0, iy0, ix0;
    g.coords(G, iz0, iy0, ix0);
    s_group(G, iz0, ix0, pn, sv);
    ldg(lr, G - b, rn);
    point_group(G, xv, pn, sv, rn);
  }
  block_total_n<3, NT>(acc, lds);
  if (threadIdx.x == 0) {
    gout[iti] = acc[0];
    qout[iti] = acc[1];
    xout[iti] = acc[2];
  }
}

// -------------------------------------------------------- RHS + residual

// b = sum_{i<=p+1} A_i^T (rho_i y_i + v_i);  r = b - C x;  partial r^T r.
// A_i^T of a forward difference needs u = rho y + v one point back along the
// axis: the previous lane's last value for x, a window for y / z.
template <typename T, int NT>
__global__ __launch_bounds__(NT) SIP_RHS_ATTR void k_rhs(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, double* rr_part) {
  constexpr int W = Grp<T>::W;
  __shared__ acc_t lds[lds_sum<1, NT>()];
  const PtItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const CgScal qs = cg_scal(S);
  const T rl = (T)ldgd(S + S_RHO + d.nsets);
  if (!qs.live()) return;
  const Geo g(d);
  const T* x = (const T*)d.x;
  T* r = (T*)d.r;
  const T* yl = (const T*)d.yl;
  const T* vl = (const T*)d.vl;
  const T c0 = (T)qs.c0, cz = (T)qs.cax[0], cy = (T)qs.cax[1], cx = (T)qs.cax[2];
  const int lane = threadIdx.x & 63;
  auto fs = [&](int Q) -> T { return x[Q]; };
  const Src<T, 1> fx{{x}, (T)0};
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  const bool al = rows_aligned<T>(g);
  const int N = g.N;
  acc_t acc[1] = {0};
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += NT * W) {
    const int P0 = base + (int)threadIdx.x * W;
    bool vec = false;
    if (grouped) {
      const GLane L = glane<T>(P0, it.begin, end, g);
      T b[W];
      {
        T a0[W], a1[W];
        ld16<T>(yl + L.P0c, a0);
        ld16<T>(vl + L.P0c, a1);
#pragma unroll
        for (int e = 0; e < W; ++e) b[e] = rl * a0[e] + a1[e];
      }
      for (int si = 0; si < d.nsets; ++si) {
        const SetDesc& s = d.sets[si];
        const T rs = (T)ldgd(S + S_RHO + si);
        for (int c = 0; c < s.ncomp; ++c) {
          // u = v + rho y
          const Src<T, 2> fu{{(const T*)s.v + (size_t)c * g.cs, (const T*)s.y + (size_t)c * g.cs}, rs};
          const int a = s.axis[c];
          T R[2][W], wa[2][W], wb[2][W], u[W];
          src_load<T, 2>(fu, L.P0c, N, R);
          const int st = a == 0 ? g.sz : g.sy, off = a == 0 ? of.zm : of.ym;
          if (a == 0 || a == 1) {
            if (al) win_load<T, 2, true>(fu, L.P0c, -st, off, N, wa, wb);
            else win_load<T, 2, false>(fu, L.P0c, -st, off, N, wa, wb);
          }
          T le[2] = {(T)0, (T)0};
          if (a == 2 && lane == 0 && L.P0c > 0) {
            le[0] = ldg(fu.a[0] + L.P0c - 1);
            le[1] = ldg(fu.a[1] + L.P0c - 1);
          }
          src_mix<T, 2>(fu, R, u);
          if (a < 0) {
#pragma unroll
            for (int e = 0; e < W; ++e) b[e] += u[e];
            continue;
          }
          T prev[W];
          if (a == 2) {
            T left = lane_prev(u[W - 1]);
            if (lane == 0) left = src_one<T, 2>(fu, le);
#pragma unroll
            for (int e = 0; e < W; ++e) prev[e] = e > 0 ? u[e > 0 ? e - 1 : 0] : left;
          } else {
            if (al) win_get<T, 2, true>(fu, off, wa, wb, prev);
            else win_get<T, 2, false>(fu, off, wa, wb, prev);
          }
          const T h = (T)d.hinv[a];
          const int na = a == 0 ? g.nz : (a == 1 ? g.ny : g.nx);
#pragma unroll
          for (int e = 0; e < W; ++e) {
            int ize = L.iz, iye = L.iy, ixe = L.ix0 + e;
            if (L.straddle) g.coords(L.P0c + e, ize, iye, ixe);
            const int ia = a == 0 ? ize : (a == 1 ? iye : ixe);
            T t = 0;
            if (ia > 0) t += prev[e];
            if (ia < na - 1) t -= u[e];
            b[e] += t * h;
          }
        }
      }
      T cxv[W], xc[W];
      group_C<T, 1>(fx, L, lane, g, of, xc, cxv, c0, cz, cy, cx);
      vec = L.vec;
      if (vec) {
        T rv[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          rv[e] = b[e] - cxv[e];
          if (e < L.cnt) acc[0] += (acc_t)rv[e] * (acc_t)rv[e];
        }
        st16<T>(r + P0, rv);
      }
    }
    if (!vec) {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        int pz, py, px;
        g.coords(P, pz, py, px);
        T bb = rl * yl[P] + vl[P];
        for (int si = 0; si < d.nsets; ++si) {
          const SetDesc& s = d.sets[si];
          const T rs = (T)ldgd(S + S_RHO + si);
          for (int c = 0; c < s.ncomp; ++c) {
            const T* y = (const T*)s.y + (size_t)c * g.cs;
            const T* v = (const T*)s.v + (size_t)c * g.cs;
            const int a = s.axis[c];
            if (a < 0) {
              bb += v[P] + rs * y[P];
            } else {
              const int ia = a == 0 ? pz : (a == 1 ? py : px);
              const int na = a == 0 ? g.nz : (a == 1 ? g.ny : g.nx);
              const int st = a == 0 ? g.sz : (a == 1 ? g.sy : 1);
              T t = 0;
              if (ia > 0) t += v[P - st] + rs * y[P - st];
              if (ia < na - 1) t -= v[P] + rs * y[P];
              bb += t * (T)d.hinv[a];
            }
          }
        }
        const T xv = x[P];
        const T rv = bb - point_apply_C<T>(P, g, fs, xv, c0, cz, cy, cx);
        r[P] = rv;
        acc[0] += (acc_t)rv * (acc_t)rv;
      }
    }
  }
  const acc_t tot = block_total<NT>(acc[0], lds);
  if (threadIdx.x == 0) rr_part[iti] = tot;
}

// ------------------------------------------- clip-type sets + identity block

// For every bounds set and the identity block p+1 at the item's points:
// s = A_i x, x-bar = gamma s + (1 - gamma) y, w = x-bar - v/rho,
// y = clip(w) or (m + rho w)/(1 + rho), v += rho (y - x-bar); on adapt
// iterations the six adapt-rho-gamma dots against the k0 snapshot and the new
// snapshot; on stopping-test iterations the feasibility sums of s.  Then the
// x snapshot / x history writes and the r_evol sums.  Full 16-byte groups
// use 128-bit accesses; other points take the per-point path.
template <typename T>
struct ProjUnit {
  T rho, gam, one_m_g, irho, lo, hi, inv1p;
  bool ident;
};

// lo, hi: this row's bounds (the set's scalars or its per-row vectors).
template <typename T>
__device__ __forceinline__ void proj_point(const ProjUnit<T>& U, T sv, T yo, T vo, T mv, T lo, T hi, T& yn, T& vn,
                                           T& xb) {
  xb = U.gam * sv + U.one_m_g * yo;
  const T w = xb - vo * U.irho;
  if (U.ident) yn = (mv + U.rho * w) * U.inv1p;
  else yn = w < lo ? lo : (w > hi ? hi : w);
  vn = vo + U.rho * (yn - xb);
}

// One block of the projection pass: item bx, unit by.
template <typename T>
__device__ void proj_block(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, const Opts& o, double* parts, int bx, int by) {
  constexpr int W = Grp<T>::W;
  __shared__ acc_t lds[lds_sum<16, kSB>()];
  const PtItem it = items[bx];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const ItScal isc = it_scal(S);
  if (!isc.live()) return;
  const Geo g(d);
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  const int k = (int)isc.k;
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  const bool have = isc.have != 0.0;
  const bool dots = adapt && have;
  const int call = adapt ? adapt_call(k, o) : 0;
  const T* __restrict__ x = (const T*)d.x;
  const T* __restrict__ xr = (const T*)d.xs[(call & 1) ^ 1];
  const T* __restrict__ m = (const T*)d.m;
  const int end = it.begin + it.len;
  const int lane = threadIdx.x & 63;
  double* out = parts + (size_t)iti * kProjParts;

  // by: the unit (a bounds set or, at nsets, the identity block), or
  // at nsets + 1 the x snapshot / history part; units run in parallel blocks
  const int u = by;
  if (u <= d.nsets) {
    const bool ident = (u == d.nsets);
    const SetDesc* s = ident ? nullptr : &d.sets[u];
    if (!ident && (s->thr >= 0 || s->line_axis >= 0)) return;
    const double rho_d = ldgd(S + S_RHO + u), gam_d = ldgd(S + S_GAMMA + u);
    ProjUnit<T> U;
    U.rho = (T)rho_d; U.gam = (T)gam_d; U.irho = (T)(1.0 / rho_d);
    U.one_m_g = (T)(1.0 - gam_d);
    U.lo = ident ? (T)0 : (T)s->lo; U.hi = ident ? (T)0 : (T)s->hi;
    U.inv1p = (T)(1.0 / (1.0 + rho_d));
    U.ident = ident;
    const int ncomp = ident ? 1 : s->ncomp;
    acc_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < ncomp; ++c) {
      const int axis = ident ? -1 : s->axis[c];
      const size_t off = (size_t)c * g.cs;
      T* __restrict__ y = (T*)(ident ? d.yl : s->y) + off;
      T* __restrict__ v = (T*)(ident ? d.vl : s->v) + off;
      T* __restrict__ vh0 = (T*)(ident ? d.vh0l : s->vh0) + off;
      T* __restrict__ v0 = (T*)(ident ? d.v0l : s->v0) + off;
      T* __restrict__ y0 = (T*)(ident ? d.y0l : s->y0) + off;
      // per-row bound vectors (padded like y)
      const T* __restrict__ lov = (!ident && s->lov) ? (const T*)s->lov + off : nullptr;
      const T* __restrict__ hiv = (!ident && s->hiv) ? (const T*)s->hiv + off : nullptr;
      for (int base = it.begin; base < end; base += kSB * W) {
        const int P0 = base + (int)threadIdx.x * W;
        GLane L{};
        if (grouped) L = glane<T>(P0, it.begin, end, g);
        const bool full = grouped && L.vec;
        T sv[W], s0[W];
        bool ok[W], ok0[W];
        if (grouped) {
          group_diff<T>(x, L, lane, g, d, of, axis, sv, ok);
          if (dots) group_diff<T>(xr, L, lane, g, d, of, axis, s0, ok0);
        }
        if (full) {
          T yo[W], vo[W], yn[W], vn[W], mv[W], lb[W], ub[W];
          ld16<T>(y + P0, yo);
          ld16<T>(v + P0, vo);
          if (ident) ld16<T>(m + P0, mv);
          if (lov) ld16<T>(lov + P0, lb);
          else {
#pragma unroll
            for (int e = 0; e < W; ++e) lb[e] = U.lo;
          }
          if (hiv) ld16<T>(hiv + P0, ub);
          else {
#pragma unroll
            for (int e = 0; e < W; ++e) ub[e] = U.hi;
          }
          T xbv[W];
#pragma unroll
          for (int e = 0; e < W; ++e) {
            if (ok[e]) proj_point<T>(U, sv[e], yo[e], vo[e], ident ? mv[e] : (T)0, lb[e], ub[e], yn[e], vn[e], xbv[e]);
            else { yn[e] = yo[e]; vn[e] = vo[e]; xbv[e] = 0; }
          }
          st16nt<T>(y + P0, yn);
          st16nt<T>(v + P0, vn);
          if (adapt) {
            T vh[W];
#pragma unroll
            for (int e = 0; e < W; ++e) vh[e] = ok[e] ? vo[e] + U.rho * (yo[e] - sv[e]) : (T)0;
            if (have) {
              T a0[W], a1[W], a2[W];
              ld16<T>(vh0 + P0, a0);
              ld16<T>(y0 + P0, a1);
              ld16<T>(v0 + P0, a2);
#pragma unroll
              for (int e = 0; e < W; ++e) {
                if (!ok[e]) continue;
                const acc_t dh = (acc_t)sv[e] - (acc_t)s0[e];
                const acc_t dvh = (acc_t)vh[e] - (acc_t)a0[e];
                const acc_t dg = -((acc_t)yn[e] - (acc_t)a1[e]);
                const acc_t dv = (acc_t)vn[e] - (acc_t)a2[e];
                acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
                acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
              }
            }
            st16nt<T>(vh0 + P0, vh);
            st16nt<T>(v0 + P0, vn);
            st16nt<T>(y0 + P0, yn);
          }
          if (check && !ident) {
#pragma unroll
            for (int e = 0; e < W; ++e) {
              if (!ok[e]) continue;
              const T pc = sv[e] < lb[e] ? lb[e] : (sv[e] > ub[e] ? ub[e] : sv[e]);
              const acc_t ee = (acc_t)sv[e] - (acc_t)pc;
              acc[6] += ee * ee;
              acc[7] += (acc_t)sv[e] * (acc_t)sv[e];
            }
          }
        } else {
          for (int e = 0; e < W; ++e) {
            const int P = P0 + e;
            if (P >= end) break;
            int iz, iy, ix;
            g.coords(P, iz, iy, ix);
            T sp;
            if (!comp_value<T>(x, P, axis, iz, iy, ix, g, d, sp)) continue;
            const T yo = y[P], vo = v[P];
            const T lbp = lov ? lov[P] : U.lo, ubp = hiv ? hiv[P] : U.hi;
            T yn, vn, xb;
            proj_point<T>(U, sp, yo, vo, ident ? m[P] : (T)0, lbp, ubp, yn, vn, xb);
            y[P] = yn;
            v[P] = vn;
            if (adapt) {
              const T vh = vo + U.rho * (yo - sp);
              if (have) {
                T sq;
                comp_value<T>(xr, P, axis, iz, iy, ix, g, d, sq);
                const acc_t dh = (acc_t)sp - (acc_t)sq;
                const acc_t dvh = (acc_t)vh - (acc_t)vh0[P];
                const acc_t dg = -((acc_t)yn - (acc_t)y0[P]);
                const acc_t dv = (acc_t)vn - (acc_t)v0[P];
                acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
                acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
              }
              vh0[P] = vh;
              v0[P] = vn;
              y0[P] = yn;
            }
            if (check && !ident) {
              const T pc = sp < lbp ? lbp : (sp > ubp ? ubp : sp);
              const acc_t ee = (acc_t)sp - (acc_t)pc;
              acc[6] += ee * ee;
              acc[7] += (acc_t)sp * (acc_t)sp;
            }
          }
        }
      }
    }
    if (adapt || check) {
      block_total_n<8, kSB>(acc, lds);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[u * kUnitParts + q] = acc[q];
      }
    }
    return;
  }
  if (u != d.nsets + 1) return;

  // x snapshot for adapt-rho-gamma, x history and r_evol sums
  if (adapt || d.ring) {
    T* __restrict__ xw = (T*)d.xs[call & 1];
    T* __restrict__ ring = (T*)d.ring;
    const int H = o.evol_hist;
    acc_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    acc_t accx[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (grouped) {
      // 16-byte groups (the snapshot and history arrays are padded)
      for (int P0 = it.begin + (int)threadIdx.x * W; P0 < end; P0 += kSB * W) {
        const int cnt = end - P0 < W ? end - P0 : W;
        T xv[W];
        ld16p<T>(x, P0, g.N, xv);
        if (adapt) st16<T>(xw + P0, xv);
        if (ring) {
          st16<T>(ring + (size_t)(k % (H + 1)) * g.cs + P0, xv);
          if (check) {
#pragma unroll
            for (int e = 0; e < W; ++e)
              if (e < cnt) accx[0] += (acc_t)xv[e] * (acc_t)xv[e];
#pragma unroll
            for (int jj = 1; jj < kMaxHist; ++jj) {
              if (jj > H) break;
              T rv[W];
              ld16<T>(ring + (size_t)((k - jj) % (H + 1)) * g.cs + P0, rv);
              acc_t t = 0;
#pragma unroll
              for (int e = 0; e < W; ++e) {
                const acc_t df = (acc_t)xv[e] - (acc_t)rv[e];
                if (e < cnt) t += df * df;
              }
              if (jj <= 7) acc[jj] += t; else accx[jj - 7] += t;
            }
          }
        }
      }
    } else {
      for (int P = it.begin + (int)threadIdx.x; P < end; P += kSB) {
        const T xv = x[P];
        if (adapt) xw[P] = xv;
        if (ring) {
          ring[(size_t)(k % (H + 1)) * g.cs + P] = xv;
          if (check) {
            accx[0] += (acc_t)xv * (acc_t)xv;
#pragma unroll
            for (int jj = 1; jj < kMaxHist; ++jj) {
              if (jj > H) break;
              const acc_t e = (acc_t)xv - (acc_t)ring[(size_t)((k - jj) % (H + 1)) * g.cs + P];
              if (jj <= 7) acc[jj] += e * e; else accx[jj - 7] += e * e;
            }
          }
        }
      }
    }
    if (check) {
      acc_t all[16];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) { all[jj] = acc[jj]; all[8 + jj] = accx[jj]; }
      block_total_n<16, kSB>(all, lds);
      if (threadIdx.x == 0) {
        out[kEvolOff + 0] = all[8];
#pragma unroll
        for (int jj = 1; jj < 8; ++jj) out[kEvolOff + jj] = all[jj];
        out[kEvolOff + 8] = all[9];  // evol_hist <= 8
      }
    }
  }
}

// Block b of the projection launch -> (item, unit).  Workgroups are dealt
// to the 8 XCDs in turn, so blocks b, b + 8, b + 16, ... share an XCD and
// its L2: the units of one item (each reads the item's x and its stencil
// neighbours) go to consecutive blocks of one XCD, and table entry e goes
// to XCD e mod 8 (the host writes the table so that each XCD's entries are
// a contiguous run of items).  Units back to back cut the batch's re-reads
// of x by 80 MB per launch.  A launch has ceil(nsp / 8) * 8 * units blocks;
// the caller drops entries >= nsp.  The fused projection and w launch keeps
// the unit-major order, which measured faster there.
__device__ __forceinline__ void proj_map(int b, int units, int& item, int& unit) {
  const int grp = b / (8 * units), r = b - grp * 8 * units;
  unit = r >> 3;
  item = grp * 8 + (r & 7);
}

inline int proj_blocks(int nsp, int units) { return (nsp + 7) / 8 * 8 * units; }

template <typename T>
__global__ __launch_bounds__(kSB) SIP_SETS_ATTR void k_proj(const InstDesc* __restrict__ D, const PtItem* __restrict__ items, Opts o, double* parts,
                                               int nsp, int units) {
  int item, unit;
  proj_map((int)blockIdx.x, units, item, unit);
  if (item < nsp) proj_block<T>(D, items, o, parts, item, unit);
}

// --------------------------------------------- threshold sets: pass 1 (w)

// Pipeline 0 (every iteration): w = x-bar - v/rho for the set's components,
// stored over y (y's old value is used first for v-hat); adapt dots of the
// (dh, dvh) pair; radix histogram of the first key digit of |w|.
// Pipeline 1 (stopping-test iterations): histogram of |s| and ||s||^2.
// One block of the w pass: item bx.
// Entries of list A (see SelState) a w-pass block holds in LDS before it
// appends them with one atomic; a wave whose entries do not fit any more
// appends them at once (one atomic per wave and element).
template <typename T> struct StageCap { static constexpr int v = 4096 / (int)sizeof(typename KeyT<T>::K); };

template <typename T>
__device__ void thrw_block(const InstDesc* __restrict__ D, const ThrItem* __restrict__ items, const Opts& o, double* parts, int bx) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  constexpr int SC = StageCap<T>::v;
  __shared__ uint32_t hc[kNB];
  __shared__ acc_t hs[kNB];
  __shared__ acc_t lds[lds_sum<8, kSB>()];
  __shared__ K stk[SC];
  __shared__ uint8_t stc[SC];
  __shared__ uint32_t scnt;
  __shared__ unsigned long long sbase;
  const ThrItem it = items[bx];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const ItScal isc = it_scal(S);
  if (!isc.live()) return;
  const int k = (int)isc.k;
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  if (it.src == 1 && !check) return;
  const bool have = isc.have != 0.0;
  const int call = adapt ? adapt_call(k, o) : 0;
  const SetDesc& s = d.sets[it.set];
  const bool l1 = s.kind == SIP_SET_L1;
  // l2 ball / annulus: no histogram, ||w||^2 into slot 6 of the partials
  const bool l2k = s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS;
  // the first-digit bucket whose entries go to list A (-1: none)
  const int spec = l2k ? -1 : s.sel[it.src]->spec - 1;
  K* __restrict__ la = (K*)s.cand[it.src];
  uint32_t* __restrict__ lx = (it.src == 0 && s.cand_ix) ? s.cand_ix : nullptr;
  unsigned long long* nsp = &s.sel[it.src]->nspec;
  for (int b = threadIdx.x; b < kNB; b += kSB) { hc[b] = 0; hs[b] = 0; }
  if (threadIdx.x == 0) scnt = 0u;
  __syncthreads();
  const Geo g(d);
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  const T* x = (const T*)d.x;
  const T* xr = (const T*)d.xs[(call & 1) ^ 1];
  const int u = it.set;
  const double rho_d = ldgd(S + S_RHO + u), gam_d = ldgd(S + S_GAMMA + u);
  const T rho = (T)rho_d, gam = (T)gam_d, one_m_g = (T)(1.0 - gam_d);
  const T irho = (T)(1.0 / rho_d);
  const int sh0 = digit_shift<T>(0);
  constexpr int W = Grp<T>::W;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const bool dots = it.src == 0 && adapt && have;
  acc_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int end = it.begin + it.len;
  auto stage = [&](K key, int c) {
    const uint32_t q = atomicAdd(&scnt, 1u);
    if (q < (uint32_t)SC) {
      stk[q] = key;
      stc[q] = (uint8_t)c;
    } else {
      const unsigned long long at = atomicAdd(nsp, 1ull);
      la[at] = key;
      if (lx) lx[at] = (uint32_t)iti * 3u + (uint32_t)c;
    }
  };
  auto bin = [&](T val, int c) {
    if (l2k) {
      acc[6] += (acc_t)val * (acc_t)val;
      return;
    }
    const K key = KT::key(val);
    const int bkt = (int)(key >> sh0);
    atomicAdd(&hc[bkt], 1u);
    if (l1) atomicAdd(&hs[bkt], (acc_t)KT::value(key));
    if (bkt == spec) stage(key, c);
  };
  // a group's values, runs of equal buckets merged into one update (the
  // bucket sums of float keys are exact, so the merge changes no result)
  auto bin_group = [&](const T (&v)[W], const bool (&ok)[W], int c) {
    if (l2k) {
#pragma unroll
      for (int e = 0; e < W; ++e)
        if (ok[e]) acc[6] += (acc_t)v[e] * (acc_t)v[e];
      return;
    }
    K keys[W];
#pragma unroll
    for (int e = 0; e < W; ++e) keys[e] = KT::key(v[e]);
    if (spec >= 0) {
      // list A: the group's hits get consecutive LDS slots, one slot
      // reservation per wave (a wave prefix of the hit counts, 0..W)
      uint32_t hmask = 0u;
#pragma unroll
      for (int e = 0; e < W; ++e)
        if (ok[e] && (int)(keys[e] >> sh0) == spec) hmask |= 1u << e;
      const int nh = __popc(hmask);
      if (__ballot(nh != 0)) {
        uint32_t pre = 0u, tot = 0u;
#pragma unroll
        for (int bit = 0; bit < 3; ++bit) {
          const unsigned long long m = __ballot((nh >> bit) & 1);
          pre += (uint32_t)__popcll(m & below) << bit;
          tot += (uint32_t)__popcll(m) << bit;
        }
        const unsigned long long act = __ballot(true);
        const int lead = __ffsll((unsigned long long)act) - 1;
        uint32_t base = 0u;
        if (lane == lead) base = atomicAdd(&scnt, tot);
        base = __shfl(base, lead, 64);
        uint32_t q = base + pre;
        int nover = 0;
#pragma unroll
        for (int e = 0; e < W; ++e) {
          if (hmask & (1u << e)) {
            if (q < (uint32_t)SC) { stk[q] = keys[e]; stc[q] = (uint8_t)c; }
            else ++nover;
            ++q;
          }
        }
        if (__ballot(nover != 0)) {
          // the stage is full: the rest straight to list A
          uint32_t opre = 0u, otot = 0u;
#pragma unroll
          for (int bit = 0; bit < 3; ++bit) {
            const unsigned long long m = __ballot((nover >> bit) & 1);
            opre += (uint32_t)__popcll(m & below) << bit;
            otot += (uint32_t)__popcll(m) << bit;
          }
          unsigned long long gb = 0ull;
          if (lane == lead) gb = atomicAdd(nsp, (unsigned long long)otot);
          gb = __shfl(gb, lead, 64) + opre;
          int skip = nh - nover;  // this thread's staged hits come first
#pragma unroll
          for (int e = 0; e < W; ++e) {
            if (hmask & (1u << e)) {
              if (skip > 0) {
                --skip;
              } else {
                la[gb] = keys[e];
                if (lx) lx[gb] = (uint32_t)iti * 3u + (uint32_t)c;
                ++gb;
              }
            }
          }
        }
      }
    }
    int cur = -1;
    uint32_t n = 0;
    acc_t sum = 0;
#pragma unroll
    for (int e = 0; e < W; ++e) {
      if (!ok[e]) continue;
      const K key = keys[e];
      const int bkt = (int)(key >> sh0);
      if (bkt != cur) {
        if (n) {
          atomicAdd(&hc[cur], n);
          if (l1) atomicAdd(&hs[cur], sum);
        }
        cur = bkt;
        n = 0;
        sum = 0;
      }
      ++n;
      sum += (acc_t)KT::value(key);
    }
    if (n) {
      atomicAdd(&hc[cur], n);
      if (l1) atomicAdd(&hs[cur], sum);
    }
  };
  for (int c = 0; c < s.ncomp; ++c) {
    const int axis = s.axis[c];
    const size_t off = (size_t)c * g.cs;
    T* __restrict__ y = (T*)s.y + off;
    const T* __restrict__ v = (const T*)s.v + off;
    T* __restrict__ vh0 = (T*)s.vh0 + off;
    for (int base = it.begin; base < end; base += kSB * W) {
      const int P0 = base + (int)threadIdx.x * W;
      GLane L{};
      if (grouped) L = glane<T>(P0, it.begin, end, g);
      const bool full = grouped && L.vec;
      T sv[W], s0[W];
      bool ok[W], ok0[W];
      if (grouped) {
        group_diff<T>(x, L, lane, g, d, of, axis, sv, ok);
        if (dots) group_diff<T>(xr, L, lane, g, d, of, axis, s0, ok0);
      }
      if (full) {
        if (it.src == 0) {
          T yo[W], vo[W], wv[W];
          ld16<T>(y + P0, yo);
          ld16<T>(v + P0, vo);
#pragma unroll
          for (int e = 0; e < W; ++e) wv[e] = ok[e] ? gam * sv[e] + one_m_g * yo[e] - vo[e] * irho : yo[e];
          st16<T>(y + P0, wv);
          if (adapt) {
            T vh[W];
#pragma unroll
            for (int e = 0; e < W; ++e) vh[e] = ok[e] ? vo[e] + rho * (yo[e] - sv[e]) : (T)0;
            if (have) {
              T a0[W];
              ld16<T>(vh0 + P0, a0);
#pragma unroll
              for (int e = 0; e < W; ++e) {
                if (!ok[e]) continue;
                const acc_t dh = (acc_t)sv[e] - (acc_t)s0[e];
                const acc_t dvh = (acc_t)vh[e] - (acc_t)a0[e];
                acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
              }
            }
            st16<T>(vh0 + P0, vh);
          }
          bin_group(wv, ok, c);
        } else {
#pragma unroll
          for (int e = 0; e < W; ++e)
            if (ok[e]) acc[7] += (acc_t)sv[e] * (acc_t)sv[e];
          bin_group(sv, ok, c);
        }
        continue;
      }
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        int iz, iy, ix;
        g.coords(P, iz, iy, ix);
        T sp;
        if (!comp_value<T>(x, P, axis, iz, iy, ix, g, d, sp)) continue;
        T val;
        if (it.src == 0) {
          const T yo = y[P], vo = v[P];
          val = gam * sp + one_m_g * yo - vo * irho;
          y[P] = val;
          if (adapt) {
            const T vh = vo + rho * (yo - sp);
            if (have) {
              T sq;
              comp_value<T>(xr, P, axis, iz, iy, ix, g, d, sq);
              const acc_t dh = (acc_t)sp - (acc_t)sq;
              const acc_t dvh = (acc_t)vh - (acc_t)vh0[P];
              acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
            }
            vh0[P] = vh;
          }
        } else {
          val = sp;
          acc[7] += (acc_t)sp * (acc_t)sp;
        }
        bin(val, c);
      }
    }
  }
  __syncthreads();
  // the place of the block's staged list-A entries, asked for first: the
  // histogram flush and the block sums run while the atomic is in flight
  const uint32_t ns = scnt < (uint32_t)SC ? scnt : (uint32_t)SC;
  const bool app = spec >= 0 && ns > 0u;
  unsigned long long at = 0ull;
  if (app && threadIdx.x == 0) at = atomicAdd(nsp, (unsigned long long)ns);
  uint32_t* gc = s.hcnt[it.src];
  acc_t* gs = (acc_t*)s.hsum[it.src];
  for (int b = threadIdx.x; b < kNB; b += kSB) {
    const uint32_t cnt = hc[b];
    if (cnt) {
      atomicAdd(&gc[b], cnt);
      if (l1) atomicAdd(&gs[b], hs[b]);
    }
  }
  block_total_n<8, kSB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) parts[(size_t)iti * kThrParts + q] = acc[q];
    if (app) sbase = at;
  }
  if (app) {
    // the entries, with where they lie (cardinality ties)
    __syncthreads();
    for (int q = threadIdx.x; q < (int)ns; q += kSB) {
      la[sbase + q] = stk[q];
      if (lx) lx[sbase + q] = (uint32_t)iti * 3u + (uint32_t)stc[q];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kSB) SIP_SETS_ATTR void k_thr_w(const InstDesc* __restrict__ D, const ThrItem* __restrict__ items, Opts o, double* parts) {
  thrw_block<T>(D, items, o, parts, (int)blockIdx.x);
}

// The projection pass and the threshold sets' w pass in one launch: both read
// only x and their own sets' arrays, so they run side by side.  The w-pass
// blocks (the longer ones) come first, so they are dispatched in the first
// wave of resident blocks and the projection blocks fill in behind them.
template <typename T>
__global__ __launch_bounds__(kSB) SIP_SETS_ATTR void k_sets(const InstDesc* __restrict__ D, const PtItem* __restrict__ sp, const ThrItem* __restrict__ thr, Opts o,
                                              double* proj_parts, double* thrw_parts, int nsp, int units, int nthr) {
  const int b = (int)blockIdx.x;
  if (b < nthr) thrw_block<T>(D, thr, o, thrw_parts, b);
  else proj_block<T>(D, sp, o, proj_parts, (b - nthr) % nsp, (b - nthr) / nsp);
}

// ---------------------------------------------- selection (one block each)

// Move nb (<= kNB) buckets of a pipeline's global histogram into LDS and
// clear them there, in two halves: pull_issue loads all kNB buckets (the
// arrays always hold kNB, so it needs neither nb nor a wait and can be issued
// with a kernel's first loads); pull_finish stores the first nb to LDS and
// clears them in global memory.  Loads go through the global address space.
constexpr int kPull = kNB / kBlock;

__device__ __forceinline__ void pull_issue(const uint32_t* gc, const acc_t* gs, bool l1, uint32_t (&cv)[kPull],
                                           acc_t (&sv)[kPull]) {
#pragma unroll
  for (int r = 0; r < kPull; ++r) {
    const int b = (int)threadIdx.x + r * kBlock;
    cv[r] = *(__attribute__((address_space(1))) const uint32_t*)(gc + b);
    // unconditional load, then a select: a load behind a branch makes the
    // compiler wait for the loads before it
    const acc_t v = *(__attribute__((address_space(1))) const acc_t*)(gs + b);
    sv[r] = l1 ? v : (acc_t)0;
  }
}

__device__ __forceinline__ void pull_finish(uint32_t* gc, acc_t* gs, bool l1, int nb, const uint32_t (&cv)[kPull],
                                            const acc_t (&sv)[kPull], uint32_t* hc, acc_t* hs) {
#pragma unroll
  for (int r = 0; r < kPull; ++r) {
    const int b = (int)threadIdx.x + r * kBlock;
    if (b < nb) {
      hc[b] = cv[r];
      hs[b] = sv[r];
      *(__attribute__((address_space(1))) uint32_t*)(gc + b) = 0u;
      if (l1) *(__attribute__((address_space(1))) acc_t*)(gs + b) = (acc_t)0;
    }
  }
}

// pull_finish without the clearing (the histogram is read by several blocks).
__device__ __forceinline__ void pull_store(int nb, const uint32_t (&cv)[kPull], const acc_t (&sv)[kPull],
                                           uint32_t* hc, acc_t* hs) {
#pragma unroll
  for (int r = 0; r < kPull; ++r) {
    const int b = (int)threadIdx.x + r * kBlock;
    if (b < nb) {
      hc[b] = cv[r];
      hs[b] = sv[r];
    }
  }
}

// A selection state read by every block of a kernel (written by an earlier
// launch), loaded with 16-byte global loads issued together.
__device__ __forceinline__ SelState load_sel(const SelState* p) {
  static_assert(sizeof(SelState) % 16 == 0, "SelState is loaded in 16-byte pieces");
  constexpr int NQ = sizeof(SelState) / 16;
  u32x4 q[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = ((g_cu32x4*)p)[i];
  SelState st;
  __builtin_memcpy(&st, q, sizeof(SelState));
  return st;
}

// The state fields a block publishes while other blocks of the same launch
// may still append candidates (everything but the candidate count).
__device__ __forceinline__ void store_sel_but_ncand(SelState* g, const SelState& v) {
  g->prefix = v.prefix; g->c_above = v.c_above; g->tkey = v.tkey; g->keep_ties = v.keep_ties; g->ties = v.ties;
  g->s_above = v.s_above; g->theta = v.theta; g->tk = v.tk; g->digit = v.digit; g->mode = v.mode;
  g->need_ties = v.need_ties; g->err = v.err; g->compact_next = v.compact_next; g->final_ = v.final_;
  g->have_cand = v.have_cand; g->cnt0 = v.cnt0;
}

// Pick the bucket of the current digit.  l1: the largest bucket b whose lower
// edge L_b still has f(L_b) = sum_{u >= L_b} (u - L_b) >= tau (f decreases, so
// the soft threshold theta with f(theta) = tau lies in bucket b).  Cardinality:
// the largest b with at least k entries at or above L_b.  Updates the state:
// prefix gets digit b, everything in buckets above b moves to c_above/s_above.
// Returns the count of bucket b.
template <typename T>
__device__ unsigned long long select_digit(SelState& st, const uint32_t* hc, const acc_t* hs, int nb, int dig,
                                          const SetDesc& s, bool l1, unsigned long long* lc, acc_t* ls,
                                          int* lbest) {
  using KT = KeyT<T>;
  const int sh = digit_shift<T>(dig);
  const int per = nb / kBlock;  // nb is 1024 or 2048
  const int t = threadIdx.x;
  unsigned long long mc = 0;
  acc_t ms = 0;
  for (int i = 0; i < per; ++i) { mc += hc[t * per + i]; if (l1) ms += hs[t * per + i]; }
  // totals of the threads above this one (higher buckets), in a fixed order:
  // an inclusive suffix scan inside each wave, then the wave totals
  const int lane = t & 63, wv = t >> 6;
  unsigned long long ic = mc;
  acc_t is = ms;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long oc = __shfl_down(ic, off, 64);
    const acc_t os = __shfl_down(is, off, 64);
    if (lane + off < 64) { ic += oc; is += os; }
  }
  unsigned long long above_c = __shfl_down(ic, 1, 64);
  acc_t above_s = __shfl_down(is, 1, 64);
  if (lane == 63) { above_c = 0; above_s = 0; }
  if (lane == 0) { lc[wv] = ic; ls[wv] = is; }
  if (t == 0) *lbest = -1;
  __syncthreads();
  for (int q = kBlock / 64 - 1; q > wv; --q) { above_c += lc[q]; above_s += ls[q]; }
  __syncthreads();
  // walk own buckets from the top
  unsigned long long rc = st.c_above + above_c;
  acc_t rs = (acc_t)st.s_above + above_s;
  int best = -1;
  for (int i = per - 1; i >= 0; --i) {
    const int b = t * per + i;
    const unsigned long long cb = rc + hc[b];
    const acc_t sb = rs + (l1 ? hs[b] : (acc_t)0);
    bool ok;
    if (l1) {
      const acc_t L = (acc_t)KT::value((typename KT::K)(st.prefix | ((unsigned long long)b << sh)));
      ok = (sb - (acc_t)cb * L) >= (acc_t)s.tau;
    } else {
      ok = cb >= (unsigned long long)s.k;
    }
    if (ok) { best = b; break; }
    rc = cb;
    rs = sb;
  }
  if (best >= 0) atomicMax(lbest, best);
  __syncthreads();
  const int b = *lbest;
  __syncthreads();
  // the owner of b publishes the new above-sums
  unsigned long long bc = 0;
  if (b >= 0 && t == b / per) {
    unsigned long long cc = st.c_above + above_c;
    acc_t ss = (acc_t)st.s_above + above_s;
    for (int i = per - 1; i > b - t * per; --i) { cc += hc[t * per + i]; if (l1) ss += hs[t * per + i]; }
    lc[0] = cc;
    ls[0] = ss;
    lc[1] = hc[b];
  }
  __syncthreads();
  if (b >= 0) {
    bc = lc[1];
    if (t == 0) {
      st.c_above = lc[0];
      st.s_above = ls[0];
      st.prefix |= ((unsigned long long)b << sh);
    }
  } else if (t == 0) {
    st.err = SIP_ENUMERIC;
  }
  __syncthreads();
  return bc;
}

template <typename T>
__device__ void finish_selection(SelState& st, const SetDesc& s, unsigned long long last_count) {
  using KT = KeyT<T>;
  if (threadIdx.x != 0) return;
  if (s.kind == SIP_SET_L1) {
    st.theta = st.c_above > 0 ? (st.s_above - s.tau) / (double)st.c_above : 0.0;
    if (st.theta < 0.0) st.theta = 0.0;
  } else {
    st.tkey = st.prefix;
    st.tk = KT::value((typename KT::K)st.prefix);
    st.keep_ties = (unsigned long long)s.k - st.c_above;
    st.ties = last_count;
    st.need_ties = (st.ties > st.keep_ties && st.tkey != 0) ? 1 : 0;
  }
}

// The selection state of an l2 ball or annulus pipeline from ||w||^2 (the w
// pass's per-item partials in item order): the projection is a scaling (or,
// for an annulus at w = 0, a point).  Every thread calls this; the state is
// valid in thread 0.
__device__ __forceinline__ SelState l2_stage(const SetDesc& s, int src, const double* __restrict__ thrw_parts, acc_t* lds) {
  acc_t n2[1];
  reduce_range<1>(thrw_parts, s.item_begin[src], s.item_end[src], kThrParts, src == 0 ? 6 : 7, n2, lds);
  SelState q{};
  q.final_ = 1;
  q.mode = SEL_INSIDE;
  const double sq = (double)n2[0];
  if (!(sq <= 1.0e300)) q.err = SIP_ENUMERIC;
  const double nrm = sqrt(sq);
  if (src == 0 && !q.err) {
    if (s.kind == SIP_SET_L2) {
      if (nrm > s.tau) { q.mode = SEL_PROJECT; q.theta = s.tau / nrm; }
    } else if (nrm > s.hi) {
      q.mode = SEL_PROJECT; q.theta = s.hi / nrm;
    } else if (nrm < s.lo) {
      if (nrm > 0.0) { q.mode = SEL_PROJECT; q.theta = s.lo / nrm; }
      else q.mode = SEL_POINT;
    }
  }
  return q;
}

// The first selection stage over the first digit's histogram, already in
// LDS (hc, hs): totals, mode, non-finite keys, the first digit, and whether
// list A (prev: the state the w pass saw) holds that digit's whole bucket.
// passes: refine passes of the batch (with two, the second pass's
// candidates go after list A, so list A may fill at most half the buffer).
// Every thread calls this; st (LDS) holds the result.
template <typename T>
__device__ __forceinline__ void first_stage(SelState& st, const SetDesc& s, bool l1, const uint32_t* hc, const acc_t* hs,
                            unsigned long long* lc, acc_t* ls, int* lbest, acc_t* lds, const SelState& prev,
                            int passes) {
  using KT = KeyT<T>;
  acc_t tot[2] = {0, 0};
  for (int b = threadIdx.x; b < kNB; b += kBlock) {
    tot[0] += (acc_t)hc[b];
    tot[1] += hs[b];
  }
  block_total_n<2, kBlock>(tot, lds);
  if (threadIdx.x == 0) {
    st.prefix = 0; st.c_above = 0; st.s_above = 0.0; st.ncand = 0; st.err = 0; st.need_ties = 0;
    st.theta = 0.0; st.tkey = 0; st.tk = 0.0; st.keep_ties = 0; st.ties = 0; st.digit = 0;
    const int infb = (int)(KT::inf_key >> digit_shift<T>(0));
    unsigned long long nonfinite = 0;
    for (int b = infb; b < kNB; ++b) nonfinite += hc[b];
    if (nonfinite) st.err = SIP_ENUMERIC;
    if (l1) {
      if (!(s.tau > 0.0)) st.mode = SEL_ZERO;
      else if (tot[1] <= (acc_t)s.tau) st.mode = SEL_INSIDE;
      else st.mode = SEL_PROJECT;
    } else {
      st.mode = ((acc_t)s.k >= tot[0]) ? SEL_ALL : SEL_PROJECT;
    }
    st.final_ = 0;
    st.compact_next = 0;
    st.nspec = prev.nspec;
    st.spec = prev.spec;
    st.have_cand = 0;
    st.cnt0 = 0;
  }
  __syncthreads();
  if (st.mode == SEL_PROJECT && !st.err) {
    const unsigned long long cnt = select_digit<T>(st, hc, hs, kNB, 0, s, l1, lc, ls, lbest);
    if (threadIdx.x == 0) {
      st.digit = 1;
      st.compact_next = cnt <= kCandCap ? 1 : 0;
      st.cnt0 = cnt;
      // list A is the bucket when it was gathered for this bucket and holds
      // as many entries (every block appended its own); with two refine
      // passes at most half the candidate buffer, so that the second pass's
      // candidates fit after it
      const unsigned long long b0 = st.prefix >> digit_shift<T>(0);
      st.have_cand = (!st.err && prev.spec > 0 && (unsigned long long)(prev.spec - 1) == b0 &&
                      prev.nspec == cnt && (passes == 1 || 2ull * cnt <= (unsigned long long)s.rows)) ? 1 : 0;
    }
  }
  __syncthreads();
}

// Stage 1 in its own launch (one block per pipeline): clears the first
// digit's histogram once it is in LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sel1(const InstDesc* __restrict__ D, const SelItem* __restrict__ items, Opts o,
                                                 const double* __restrict__ thrw_parts, int passes) {
  __shared__ uint32_t hc[kNB];
  __shared__ acc_t hs[kNB];
  __shared__ unsigned long long lc[kBlock];
  __shared__ acc_t ls[kBlock];
  __shared__ int lbest;
  __shared__ acc_t lds[lds_sum<2>()];
  __shared__ SelState st;
  const SelItem si = items[blockIdx.x];
  if (si.inst < 0) return;
  const InstDesc& d = D[si.inst];
  const double* S = d.scal;
  const SetDesc& s = d.sets[si.set];
  const bool l1 = s.kind == SIP_SET_L1;
  uint32_t* gc = s.hcnt[si.src];
  acc_t* gs = (acc_t*)s.hsum[si.src];
  // the histogram (allocated for every selection item) travels with the
  // iteration scalars
  const ItScal isc = it_scal(S);
  uint32_t cv[kPull];
  acc_t sv[kPull];
  pull_issue(gc, gs, l1, cv, sv);
  if (!isc.live()) return;
  const int k = (int)isc.k;
  if (si.src == 1 && !is_check_iter(k, o)) return;
  if (s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS) {
    const SelState q = l2_stage(s, si.src, thrw_parts, lds);
    if (threadIdx.x == 0) *s.sel[si.src] = q;
    return;
  }
  const SelState prev = load_sel(s.sel[si.src]);
  pull_finish(gc, gs, l1, kNB, cv, sv, hc, hs);
  __syncthreads();
  first_stage<T>(st, s, l1, hc, hs, lc, ls, &lbest, lds, prev, passes);
  if (threadIdx.x == 0) {
    *s.sel[si.src] = st;
    if (st.have_cand) atomicAdd(d.scal + S_REUSE, 1.0);
  }
}

// Keys of list A one refine block reads (at least): list A goes to the
// pipeline's first ceil(nspec / kListChunk) blocks, the others have no work.
constexpr unsigned long long kListChunk = 2048;

// Whether refine pass `pass` (0 or 1; 1 is the last pass of the iteration)
// appends candidate keys: the first when digits remain after the one it
// histograms and the bucket it refines is small, the last always.  The
// threshold is therefore always final in a selection stage that holds the
// candidates, among them every entry equal to the k-th magnitude (so that
// stage also counts the cardinality ties).
template <typename T>
__device__ __forceinline__ bool pass_compacts(const SelState& st, int pass) {
  return pass == 1 || (st.compact_next && st.digit + 1 < KeyT<T>::ndig);
}

// Refine pass over all values: histogram of digit st.digit among entries
// whose higher digits match the resolved prefix; when the bucket is small
// (or on the last pass of a long key) their keys go to the candidate list,
// appended with one atomic per block round.
template <typename T, bool FIRST>
__global__ __launch_bounds__(kSB) void k_thr_refine(const InstDesc* __restrict__ D, const ThrItem* __restrict__ items, Opts o, int pass,
                                                       const double* __restrict__ thrw_parts, uint32_t* h1c, double* h1s) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ uint32_t hc[kNB];
  __shared__ acc_t hs[kNB];
  __shared__ uint32_t wcnt[kSW];
  __shared__ unsigned long long bbase;
  const ThrItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const SetDesc& s = d.sets[it.set];
  const bool l1 = s.kind == SIP_SET_L1;
  const ItScal isc = it_scal(S);
  SelState st = load_sel(s.sel[it.src]);  // with the iteration scalars
  uint32_t cv[kPull];
  acc_t sv[kPull];
  if constexpr (FIRST) pull_issue(s.hcnt[it.src], (const acc_t*)s.hsum[it.src], l1, cv, sv);
  if (!isc.live()) return;
  const int k = (int)isc.k;
  if (it.src == 1 && !is_check_iter(k, o)) return;
  if constexpr (FIRST) {
    __shared__ unsigned long long lc[kBlock];
    __shared__ acc_t ls[kBlock];
    __shared__ int lbest;
    __shared__ acc_t lds[lds_sum<2>()];
    __shared__ SelState sst;
    // the first selection stage, done by every block of the pipeline on its
    // own (the same arithmetic, so the same state); its first block
    // publishes the state (all but the candidate count, which other blocks
    // may already be raising)
    const bool lead = iti == s.item_begin[it.src];
    if (s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS) {
      const SelState q = l2_stage(s, it.src, thrw_parts, lds);
      if (lead && threadIdx.x == 0) *s.sel[it.src] = q;
      return;
    }
    pull_store(kNB, cv, sv, hc, hs);
    __syncthreads();
    first_stage<T>(sst, s, l1, hc, hs, lc, ls, &lbest, lds, st, 1);
    if (lead && threadIdx.x == 0) {
      store_sel_but_ncand(s.sel[it.src], sst);
      if (sst.have_cand) atomicAdd(d.scal + S_REUSE, 1.0);
    }
    st = sst;
    __syncthreads();  // hc, hs are reused below
  }
  if (st.mode != SEL_PROJECT || st.err || st.final_) return;
  const int dig = st.digit;
  // With list A holding the first digit's bucket, a pass that would append
  // that bucket appends nothing: list A is the candidate list.  A small one
  // (at most kCandCap entries) makes the pass needless: the select stage
  // after it resolves every remaining digit over list A.
  const bool compact0 = pass_compacts<T>(st, pass);
  const bool a_cand = st.have_cand && dig == 1 && compact0;
  if (a_cand && st.nspec <= kCandCap) return;
  const bool compact = compact0 && !a_cand;
  const int nb = 1 << KT::width(dig);
  for (int b = threadIdx.x; b < nb; b += kSB) { hc[b] = 0; hs[b] = 0; }
  __syncthreads();
  const int shp = digit_shift<T>(dig - 1), sh = digit_shift<T>(dig);
  const K want = (K)(st.prefix >> shp);
  const Geo g(d);
  const T* __restrict__ x = (const T*)d.x;
  K* __restrict__ cand = (K*)s.cand[it.src];
  uint32_t* __restrict__ cix = it.src == 0 ? s.cand_ix : nullptr;  // cardinality: where each candidate lies
  unsigned long long* ncand = &s.sel[it.src]->ncand;
  constexpr int W = Grp<T>::W;
  // bits of a per-thread hit count (0 .. kRefineRounds * W)
  constexpr int CB = kRefineRounds * W < 2 ? 1 : (kRefineRounds * W < 4 ? 2 : (kRefineRounds * W < 8 ? 3 :
                     (kRefineRounds * W < 16 ? 4 : (kRefineRounds * W < 32 ? 5 : 6))));
  static_assert(kRefineRounds * W <= 32, "hit mask bits");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int end = it.begin + it.len;
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  if (st.have_cand) {
    // list A instead of the values, in chunks of at least kListChunk keys to
    // the pipeline's first items (few blocks, so few histogram atomics); the
    // pass's candidates (a subset of list A) go after list A
    const unsigned long long na = st.nspec;
    const unsigned long long j = (unsigned long long)(iti - s.item_begin[it.src]);
    const unsigned long long nj = (unsigned long long)(s.item_end[it.src] - s.item_begin[it.src]);
    const unsigned long long ch = (na + nj - 1) / nj > kListChunk ? (na + nj - 1) / nj : kListChunk;
    const unsigned long long q0 = j * ch;
    if (q0 >= na) return;
    const unsigned long long q1 = q0 + ch < na ? q0 + ch : na;
    const K* __restrict__ la = cand;
    const uint32_t* __restrict__ lx = cix;
    K* __restrict__ lb = cand + na;
    uint32_t* __restrict__ lbx = cix ? cix + na : nullptr;
    constexpr int U = 16;  // keys per thread and round (a hit count of 0..16: 5 ballot bits)
    for (unsigned long long r0 = q0; r0 < q1; r0 += (unsigned long long)kSB * U) {
      K key[U];
      bool hit[U];
      int nh = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned long long q = r0 + (unsigned long long)(u * kSB) + threadIdx.x;
        key[u] = q < q1 ? *(__attribute__((address_space(1))) const K*)(la + q) : (K)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned long long q = r0 + (unsigned long long)(u * kSB) + threadIdx.x;
        hit[u] = q < q1 && (K)(key[u] >> shp) == want;
        if (hit[u]) {
          ++nh;
          const int bkt = (int)((key[u] >> sh) & (K)(nb - 1));
          atomicAdd(&hc[bkt], 1u);
          if (l1) atomicAdd(&hs[bkt], (acc_t)KT::value(key[u]));
        }
      }
      if (compact) {
        unsigned long long pre = 0, tot = 0;
#pragma unroll
        for (int bit = 0; bit < 5; ++bit) {
          const unsigned long long m = __ballot((nh >> bit) & 1);
          pre += (unsigned long long)__popcll(m & below) << bit;
          tot += (unsigned long long)__popcll(m) << bit;
        }
        if (lane == 0) wcnt[wv] = (uint32_t)tot;
        __syncthreads();
        if (threadIdx.x == 0) {
          unsigned long long t = 0;
          for (int w = 0; w < kSW; ++w) t += wcnt[w];
          bbase = t ? atomicAdd(ncand, t) : 0ull;
        }
        __syncthreads();
        if (nh) {
          unsigned long long off = bbase + pre;
          for (int w = 0; w < wv; ++w) off += wcnt[w];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (hit[u]) {
              if (lbx) lbx[off] = lx[r0 + (unsigned long long)(u * kSB) + threadIdx.x];
              lb[off++] = key[u];
            }
          }
        }
        __syncthreads();
      }
    }
  }
  // the components swept over the values (none when list A was read)
  const int ncomp_w = st.have_cand ? 0 : s.ncomp;
  for (int c = 0; c < ncomp_w; ++c) {
    const int axis = s.axis[c];
    const T* __restrict__ y = (const T*)s.y + (size_t)c * g.cs;
    for (int base0 = it.begin; base0 < end; base0 += kSB * W * kRefineRounds) {
    T valr[kRefineRounds][W];
    bool okr[kRefineRounds][W];
#pragma unroll
    for (int r = 0; r < kRefineRounds; ++r) {
      const int P0 = base0 + r * kSB * W + (int)threadIdx.x * W;
      T (&val)[W] = valr[r];
      bool (&ok)[W] = okr[r];
      if (grouped) {
        const GLane L = glane<T>(P0, it.begin, end, g);
        if (it.src == 1) {
          group_diff<T>(x, L, lane, g, d, of, axis, val, ok);
        } else {
          group_valid<T>(L, g, axis, ok);
          ld16<T>(y + L.P0c, val);
        }
        if (!L.vec) {
#pragma unroll
          for (int e = 0; e < W; ++e) ok[e] = false;
        }
      } else {
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const int P = P0 + e;
          ok[e] = false;
          val[e] = 0;
          if (P < end) {
            int iz, iy, ix;
            g.coords(P, iz, iy, ix);
            if (it.src == 0) {
              ok[e] = comp_valid(axis, iz, iy, ix, g);
              if (ok[e]) val[e] = y[P];
            } else {
              ok[e] = comp_value<T>(x, P, axis, iz, iy, ix, g, d, val[e]);
            }
          }
        }
      }
    }
    // keys, hits and the histogram of every round; the hits of all rounds
    // are appended with one block prefix and one global atomic
    K keyr[kRefineRounds][W];
    uint32_t hitm = 0;  // bit r * W + e: round r, element e is a hit
    int nhit = 0;
#pragma unroll
    for (int r = 0; r < kRefineRounds; ++r) {
      int cur = -1;
      uint32_t run = 0;
      acc_t rsum = 0;
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const K key = KT::key(valr[r][e]);
        keyr[r][e] = key;
        if (okr[r][e] && (K)(key >> shp) == want) {
          hitm |= 1u << (r * W + e);
          ++nhit;
          // runs of equal buckets merged into one update (exact sums for float keys)
          const int bkt = (int)((key >> sh) & (K)(nb - 1));
          if (bkt != cur) {
            if (run) {
              atomicAdd(&hc[cur], run);
              if (l1) atomicAdd(&hs[cur], rsum);
            }
            cur = bkt;
            run = 0;
            rsum = 0;
          }
          ++run;
          rsum += (acc_t)KT::value(key);
        }
      }
      if (run) {
        atomicAdd(&hc[cur], run);
        if (l1) atomicAdd(&hs[cur], rsum);
      }
    }
    if (compact) {
      // block-aggregated append: wave prefix of the per-thread hit counts
      // (one ballot per count bit), one atomic for the block
      unsigned long long pre = 0, tot = 0;
#pragma unroll
      for (int bit = 0; bit < CB; ++bit) {
        const unsigned long long m = __ballot((nhit >> bit) & 1);
        pre += (unsigned long long)__popcll(m & below) << bit;
        tot += (unsigned long long)__popcll(m) << bit;
      }
      if (lane == 0) wcnt[wv] = (uint32_t)tot;
      __syncthreads();
      if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < kSW; ++q) t += wcnt[q];
        bbase = t ? atomicAdd(ncand, t) : 0ull;
      }
      __syncthreads();
      if (nhit) {
        unsigned long long off = bbase + pre;
        for (int q = 0; q < wv; ++q) off += wcnt[q];
        const uint32_t code = (uint32_t)iti * 3u + (uint32_t)c;
#pragma unroll
        for (int r = 0; r < kRefineRounds; ++r) {
#pragma unroll
          for (int e = 0; e < W; ++e) {
            if (hitm & (1u << (r * W + e))) {
              if (cix) cix[off] = code;
              cand[off++] = keyr[r][e];
            }
          }
        }
      }
      __syncthreads();
    }
    }
  }
  __syncthreads();
  // the refine histogram: the first digit's buffer, cleared by the first
  // selection stage, unless every block is still reading that
  uint32_t* gc = FIRST ? h1c + (size_t)it.pipe * kNB : s.hcnt[it.src];
  acc_t* gs = (acc_t*)(FIRST ? h1s + (size_t)it.pipe * kNB : s.hsum[it.src]);
  for (int b = threadIdx.x; b < nb; b += kSB) {
    if (hc[b]) {
      atomicAdd(&gc[b], hc[b]);
      if (l1) atomicAdd(&gs[b], hs[b]);
    }
  }
}

// Select the digit the refine pass histogrammed (from the global histogram,
// which is cleared for the next pass).  If that pass appended candidates the
// remaining digits are resolved over them in LDS; if the digit was the last
// one the threshold is final; otherwise decide whether the next refine pass
// appends candidates.  Ends with theta (l1) or the k-th magnitude and the tie
// bookkeeping (cardinality) once final.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sel_next(const InstDesc* __restrict__ D, const SelItem* __restrict__ items, Opts o, int pass,
                                                     uint32_t* tie_part, int clear0, uint32_t* h1c, double* h1s) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ uint32_t hc[kNB];
  __shared__ acc_t hs[kNB];
  __shared__ unsigned long long lc[kBlock];
  __shared__ acc_t ls[kBlock];
  __shared__ int lbest;
  __shared__ SelState st;
  const SelItem si = items[blockIdx.x];
  if (si.inst < 0) return;
  const InstDesc& d = D[si.inst];
  const double* S = d.scal;
  const SetDesc& s = d.sets[si.set];
  // the state and the histogram (allocated for every selection item) are
  // loaded with the iteration scalars
  const ItScal isc = it_scal(S);
  const SelState st0 = load_sel(s.sel[si.src]);
  const bool l1 = s.kind == SIP_SET_L1;
  // the refine histogram: the pipeline's own in the batch table when the
  // first selection stage ran inside the refine pass
  uint32_t* gc = clear0 ? h1c + (size_t)blockIdx.x * kNB : s.hcnt[si.src];
  acc_t* gs = (acc_t*)(clear0 ? h1s + (size_t)blockIdx.x * kNB : s.hsum[si.src]);
  uint32_t cv[kPull];
  acc_t sv[kPull];
  pull_issue(gc, gs, l1, cv, sv);
  if (!isc.live()) return;
  const int k = (int)isc.k;
  if (si.src == 1 && !is_check_iter(k, o)) return;
  if (clear0) {
    // the first digit's histogram, read by every block of the refine pass
    uint32_t* g0 = s.hcnt[si.src];
    acc_t* s0 = (acc_t*)s.hsum[si.src];
    for (int b = threadIdx.x; b < kNB; b += kBlock) {
      g0[b] = 0u;
      if (l1) s0[b] = (acc_t)0;
    }
  }
  if (st0.mode != SEL_PROJECT || st0.err || st0.final_) return;
  if (threadIdx.x == 0) st = st0;  // first read after select_digit's barriers
  const bool compacted = pass_compacts<T>(st0, pass);
  // a_cand: list A (the first digit's bucket) is the candidate list; from_a:
  // the refine pass skipped it (small), so every digit from the second on is
  // resolved over it here.  Otherwise the pass's own candidates, after list A
  // if it was read.
  const bool a_cand = st0.have_cand && st0.digit == 1 && compacted;
  const bool from_a = a_cand && st0.nspec <= kCandCap;
  const unsigned long long cbase = (st0.have_cand && !a_cand) ? st0.nspec : 0ull;
  const K* cand = (const K*)s.cand[si.src] + cbase;
  const unsigned long long ncand = a_cand ? st0.nspec : (compacted ? st0.ncand : 0ull);
  int dig = st0.digit;
  int nb = 1 << KT::width(dig);
  pull_finish(gc, gs, l1, nb, cv, sv, hc, hs);
  __syncthreads();
  unsigned long long last = 0;
  if (!from_a) {
    last = select_digit<T>(st, hc, hs, nb, dig, s, l1, lc, ls, &lbest);
    ++dig;
  }
  if (compacted) {
    for (; dig < KT::ndig; ++dig) {
      if (st.err) break;
      nb = 1 << KT::width(dig);
      const int shp = digit_shift<T>(dig - 1), sh = digit_shift<T>(dig);
      const K want = (K)(st.prefix >> shp);
      for (int b = threadIdx.x; b < nb; b += kBlock) { hc[b] = 0; hs[b] = 0; }
      __syncthreads();
      // eight keys per thread in flight at a time (all of them loaded into
      // registers at once measured slower)
      constexpr int U = 8;
      for (unsigned long long i0 = threadIdx.x; i0 < ncand; i0 += (unsigned long long)kBlock * U) {
        K keys[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned long long i = i0 + (unsigned long long)u * kBlock;
          keys[u] = *(__attribute__((address_space(1))) const K*)(cand + (i < ncand ? i : 0));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const K key = keys[u];
          if (i0 + (unsigned long long)u * kBlock < ncand && (K)(key >> shp) == want) {
            const int bkt = (int)((key >> sh) & (K)(nb - 1));
            atomicAdd(&hc[bkt], 1u);
            if (l1) atomicAdd(&hs[bkt], (acc_t)KT::value(key));
          }
        }
      }
      __syncthreads();
      last = select_digit<T>(st, hc, hs, nb, dig, s, l1, lc, ls, &lbest);
    }
  }
  __syncthreads();
  if (dig >= KT::ndig) {
    if (!st.err) finish_selection<T>(st, s, last);
    if (threadIdx.x == 0) st.final_ = 1;
  } else if (threadIdx.x == 0) {
    st.digit = dig;
    st.compact_next = last <= kCandCap ? 1 : 0;
  }
  __syncthreads();
  if (st.final_ && st.need_ties && s.cand_ix && si.src == 0 && compacted) {
    // entries equal to the k-th magnitude per (item, component), for the
    // apply pass to rank them by linear index: every such entry is a
    // candidate, and the candidate's code says where it lies
    const int ib = s.item_begin[0], ie = s.item_end[0];
    for (int q = ib * 3 + (int)threadIdx.x; q < ie * 3; q += kBlock) tie_part[q] = 0u;
    __syncthreads();
    const K tk = (K)st.tkey;
    const uint32_t* __restrict__ cix = s.cand_ix + cbase;
    constexpr int U = 8;
    for (unsigned long long i0 = threadIdx.x; i0 < ncand; i0 += (unsigned long long)kBlock * U) {
      K keys[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned long long i = i0 + (unsigned long long)u * kBlock;
        keys[u] = *(__attribute__((address_space(1))) const K*)(cand + (i < ncand ? i : 0));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const unsigned long long i = i0 + (unsigned long long)u * kBlock;
        if (i < ncand && keys[u] == tk) atomicAdd(&tie_part[cix[i]], 1u);
      }
    }
  }
  if (threadIdx.x == 0) {
    st.ncand = 0;  // the candidates are used up; the next refine pass appends from 0
    *s.sel[si.src] = st;
  }
}

// Apply pass.  Pipeline 0: y = soft threshold of w (l1) or w on the kept
// support (cardinality); v = rho (y - w), which equals v + rho (y - x-bar);
// adapt dots of the (dg, dv) pair and the new y/v snapshots.  Pipeline 1:
// the feasibility distance ||s - P(s)||^2.
template <typename T>
__device__ void apply_item(const InstDesc* __restrict__ D, const ThrItem* __restrict__ items, const Opts& o, double* parts,
                           const uint32_t* tie_part, int bx) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ acc_t lds[lds_sum<8, kSB>()];
  __shared__ uint32_t wsum[kSW];
  __shared__ unsigned long long tie_base[3];
  const ThrItem it = items[bx];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const SetDesc& s = d.sets[it.set];
  const ItScal isc = it_scal(S);
  const SelState st = load_sel(s.sel[it.src]);  // with the iteration scalars
  if (!isc.live()) return;
  const int k = (int)isc.k;
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  if (it.src == 1 && !check) return;
  const bool have = isc.have != 0.0;
  if (st.err) return;
  const bool l1 = s.kind == SIP_SET_L1;
  // l2 ball / annulus: y = theta w, w, or the point lo e_0; their distance
  // on stopping-test iterations follows from ||s|| alone (k_finish)
  const bool l2k = s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS;
  if (l2k && it.src == 1) return;
  const int mode = st.mode;
  const Geo g(d);
  const bool grouped = item_grouped(d);
  const Offs of = offs_of<T>(g);
  const T* x = (const T*)d.x;
  const double rho_d = ldgd(S + S_RHO + it.set);
  const T rho = (T)rho_d;
  const T theta = (T)st.theta;
  const T lo_r = (T)s.lo;
  auto l2_prox = [&](T we, int P, int c) -> T {
    if (mode == SEL_PROJECT) return theta * we;
    if (mode == SEL_POINT) return (P == 0 && c == 0) ? lo_r : (T)0;
    return we;
  };
  const K tkey = (K)st.tkey;
  const bool rank_ties = (!l1) && mode == SEL_PROJECT && st.need_ties && it.src == 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (rank_ties) {
    // entries equal to the k-th magnitude before this item in linear order
    if (threadIdx.x < 3) {
      const int c = threadIdx.x;
      unsigned long long base = 0;
      if (c < s.ncomp) {
        for (int cc = 0; cc < c; ++cc)
          for (int q = s.item_begin[0]; q < s.item_end[0]; ++q) base += tie_part[(size_t)q * 3 + cc];
        for (int q = s.item_begin[0]; q < iti; ++q) base += tie_part[(size_t)q * 3 + c];
      }
      tie_base[c] = base;
    }
    __syncthreads();
  }
  acc_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int end = it.begin + it.len;
  for (int c = 0; c < s.ncomp; ++c) {
    const int axis = s.axis[c];
    const size_t off = (size_t)c * g.cs;
    T* y = (T*)s.y + off;
    T* v = (T*)s.v + off;
    T* y0 = (T*)s.y0 + off;
    T* v0 = (T*)s.v0 + off;
    unsigned long long run = rank_ties ? tie_base[c] : 0ull;
    if (!rank_ties) {
      // 16-byte groups (no index ranking needed); w of the thread's next
      // group is loaded while this one is processed (the arrays are padded
      // to whole groups)
      constexpr int W = Grp<T>::W;
      const bool pre = it.src == 0 && grouped;
      T wnext[W];
      if (pre && it.begin + (int)threadIdx.x * W < end) ld16<T>(y + it.begin + (int)threadIdx.x * W, wnext);
      int base = it.begin;
      for (; base < end; base += kSB * W) {
        const int P0 = base + (int)threadIdx.x * W;
        T wcur[W];
#pragma unroll
        for (int e = 0; e < W; ++e) wcur[e] = wnext[e];
        if (pre && P0 + kSB * W < end) ld16<T>(y + P0 + kSB * W, wnext);
        GLane L{};
        if (grouped) L = glane<T>(P0, it.begin, end, g);
        const bool full = grouped && L.vec;
        T sv[W];
        bool ok[W];
        if (grouped && it.src == 1) group_diff<T>(x, L, lane, g, d, of, axis, sv, ok);
        else if (full) group_valid<T>(L, g, axis, ok);
        if (full) {
          if (it.src == 1) {
#pragma unroll
            for (int e = 0; e < W; ++e) {
              if (!ok[e]) continue;
              const acc_t a = (acc_t)fabs((double)sv[e]);
              acc_t e2 = 0;
              if (l1) {
                if (mode == SEL_PROJECT) { const acc_t th = (acc_t)st.theta; const acc_t mn = a < th ? a : th; e2 = mn * mn; }
                else if (mode == SEL_ZERO) e2 = a * a;
              } else if (mode == SEL_PROJECT) {
                e2 = KT::key(sv[e]) < tkey ? a * a : (acc_t)0;
              }
              acc[6] += e2;
            }
            continue;
          }
          T yn[W], vn[W];
          const T (&w)[W] = wcur;
#pragma unroll
          for (int e = 0; e < W; ++e) {
            T r = w[e];
            if (ok[e]) {
              if (l2k) {
                r = l2_prox(w[e], P0 + e, c);
              } else if (l1) {
                if (mode == SEL_PROJECT) {
                  const T a = (w[e] < 0 ? -w[e] : w[e]) - theta;
                  r = a > 0 ? (w[e] < 0 ? -a : a) : (T)0;
                } else if (mode == SEL_ZERO) r = 0;
              } else if (mode == SEL_PROJECT) {
                const K key = KT::key(w[e]);
                r = (key > tkey || (key == tkey && (tkey == 0 || !st.need_ties))) ? w[e] : (T)0;
              }
            }
            yn[e] = r;
            vn[e] = ok[e] ? rho * (r - w[e]) : (T)0;
          }
          st16nt<T>(y + P0, yn);
          st16nt<T>(v + P0, vn);
          if (adapt) {
            if (have) {
              T a0[W], a1[W];
              ld16<T>(y0 + P0, a0);
              ld16<T>(v0 + P0, a1);
#pragma unroll
              for (int e = 0; e < W; ++e) {
                if (!ok[e]) continue;
                const acc_t dg = -((acc_t)yn[e] - (acc_t)a0[e]);
                const acc_t dv = (acc_t)vn[e] - (acc_t)a1[e];
                acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
              }
            }
            st16nt<T>(y0 + P0, yn);
            st16nt<T>(v0 + P0, vn);
          }
          continue;
        }
        for (int e = 0; e < W; ++e) {
          const int P = P0 + e;
          if (P >= end) break;
          int iz, iy, ix;
          g.coords(P, iz, iy, ix);
          T sp = 0;
          if (it.src == 1) {
            if (!comp_value<T>(x, P, axis, iz, iy, ix, g, d, sp)) continue;
            const acc_t a = (acc_t)fabs((double)sp);
            acc_t e2 = 0;
            if (l1) {
              if (mode == SEL_PROJECT) { const acc_t th = (acc_t)st.theta; const acc_t mn = a < th ? a : th; e2 = mn * mn; }
              else if (mode == SEL_ZERO) e2 = a * a;
            } else if (mode == SEL_PROJECT) {
              e2 = KT::key(sp) < tkey ? a * a : (acc_t)0;
            }
            acc[6] += e2;
            continue;
          }
          if (!comp_valid(axis, iz, iy, ix, g)) continue;
          const T we = y[P];
          T r = we;
          if (l2k) {
            r = l2_prox(we, P, c);
          } else if (l1) {
            if (mode == SEL_PROJECT) {
              const T a = (we < 0 ? -we : we) - theta;
              r = a > 0 ? (we < 0 ? -a : a) : (T)0;
            } else if (mode == SEL_ZERO) r = 0;
          } else if (mode == SEL_PROJECT) {
            const K key = KT::key(we);
            r = (key > tkey || (key == tkey && (tkey == 0 || !st.need_ties))) ? we : (T)0;
          }
          const T vv = rho * (r - we);
          y[P] = r;
          v[P] = vv;
          if (adapt) {
            if (have) {
              const acc_t dg = -((acc_t)r - (acc_t)y0[P]);
              const acc_t dv = (acc_t)vv - (acc_t)v0[P];
              acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
            }
            y0[P] = r;
            v0[P] = vv;
          }
        }
      }
      continue;
    }
    for (int base = it.begin; base < end; base += kSB) {
      const int P = base + (int)threadIdx.x;
      bool valid = false;
      T sv = 0;
      if (P < end) {
        int iz, iy, ix;
        g.coords(P, iz, iy, ix);
        if (it.src == 1) valid = comp_value<T>(x, P, axis, iz, iy, ix, g, d, sv);
        else valid = comp_valid(axis, iz, iy, ix, g);
      }
      if (it.src == 1) {
        if (valid) {
          acc_t e2;
          const acc_t a = (acc_t)fabs((double)sv);
          if (l1) {
            if (mode == SEL_PROJECT) { const acc_t th = (acc_t)st.theta; const acc_t mn = a < th ? a : th; e2 = mn * mn; }
            else if (mode == SEL_ZERO) e2 = a * a;
            else e2 = 0;
          } else {
            if (mode == SEL_PROJECT) {
              const K key = KT::key(sv);
              e2 = key < tkey ? a * a : (acc_t)0;
            } else e2 = 0;
          }
          acc[6] += e2;
        }
        continue;
      }
      const T w = valid ? y[P] : (T)0;
      const K key = KT::key(w);
      bool tie_keep = false;
      if (rank_ties) {
        const bool tie = valid && key == tkey;
        const unsigned long long mask = __ballot(tie);
        if (lane == 0) wsum[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        unsigned long long before = run;
        for (int q = 0; q < wv; ++q) before += wsum[q];
        const unsigned long long below = mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
        before += (unsigned long long)__popcll(below);
        tie_keep = tie && before < st.keep_ties;
        for (int q = 0; q < kSW; ++q) run += wsum[q];
        __syncthreads();
      }
      if (!valid) continue;
      T yn;
      if (l1) {
        if (mode == SEL_PROJECT) {
          const T a = (w < 0 ? -w : w) - theta;
          yn = a > 0 ? (w < 0 ? -a : a) : (T)0;
        } else if (mode == SEL_ZERO) yn = 0;
        else yn = w;
      } else {
        if (mode == SEL_PROJECT) {
          bool keep = key > tkey || (key == tkey && (tkey == 0 || !st.need_ties || tie_keep));
          yn = keep ? w : (T)0;
        } else yn = w;
      }
      const T vn = rho * (yn - w);
      y[P] = yn;
      v[P] = vn;
      if (adapt) {
        if (have) {
          const acc_t dg = -((acc_t)yn - (acc_t)y0[P]);
          const acc_t dv = (acc_t)vn - (acc_t)v0[P];
          acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
        }
        y0[P] = yn;
        v0[P] = vn;
      }
    }
  }
  block_total_n<8, kSB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) parts[(size_t)iti * kThrParts + q] = acc[q];
  }
}

// One block per item, written as a grid-stride loop over the item table:
// in the loop form the compiler keeps the apply body in 81 registers (113
// as a plain kernel body), five waves per SIMD instead of four (230 instead
// of 257 us on the 256-instance batch).
template <typename T>
__global__ __launch_bounds__(kSB) void k_thr_apply(const InstDesc* __restrict__ D, const ThrItem* __restrict__ items, Opts o, double* parts,
                                                      const uint32_t* tie_part, int nitems) {
  for (int b = blockIdx.x; b < nitems; b += gridDim.x) {
    apply_item<T>(D, items, o, parts, tie_part, b);
    __syncthreads();
  }
}

// ------------------------------------------------- line-wise threshold sets
//
// A set that acts on every line (row, column or fiber) of A x on its own:
// one block per line.  The line's w goes to LDS; the l1 ball and the
// cardinality set sort it there (a bitonic network on (|w|, index): larger
// magnitude first, ties to the lower index along the line), the l2 ball and
// the annulus only need the line's norm.  Lines are at most LineCap<T>::v
// long (longer ones are rejected at admission).

constexpr int kLB = 256;  // threads per line block

// How one line is projected.
enum LineMode : int { LM_KEEP = 0, LM_SOFT = 1, LM_ZERO = 2, LM_TOPK = 3, LM_SCALE = 4, LM_POINT = 5 };

template <typename T>
struct LineProj {
  int mode;
  T theta;                        // LM_SOFT: soft threshold; LM_SCALE: factor; LM_POINT: lo
  typename KeyT<T>::K tkey;       // LM_TOPK: the k-th (key, index)
  uint32_t tidx;
};

template <typename T>
__device__ __forceinline__ T line_apply(const LineProj<T>& q, T w, int e) {
  using KT = KeyT<T>;
  switch (q.mode) {
    case LM_SOFT: {
      const T a = (w < 0 ? -w : w) - q.theta;
      return a > 0 ? (w < 0 ? -a : a) : (T)0;
    }
    case LM_ZERO: return (T)0;
    case LM_TOPK: {
      const typename KT::K key = KT::key(w);
      return (key > q.tkey || (key == q.tkey && (uint32_t)e <= q.tidx)) ? w : (T)0;
    }
    case LM_SCALE: return q.theta * w;
    case LM_POINT: return e == 0 ? q.theta : (T)0;
    default: return w;
  }
}

// Block sum (every thread gets it) of one value per thread.
__device__ __forceinline__ acc_t line_sum(acc_t v, acc_t* lds) {
  acc_t a[1] = {v};
  block_sum<1, kLB>(a, lds);
  return a[0];
}

// Block maximum of one int per thread.
__device__ __forceinline__ int line_max(int v, int* ldi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) ldi[threadIdx.x >> 6] = v;
  __syncthreads();
  int m = ldi[0];
  for (int q = 1; q < kLB / 64; ++q) m = ldi[q] > m ? ldi[q] : m;
  return m;
}

// Sort lv[0..L) by (|value| descending, index ascending) into (lk, li).
template <typename T>
__device__ void line_sort(const T* lv, int L, typename KeyT<T>::K* lk, uint32_t* li) {
  using KT = KeyT<T>;
  int Lp = 2;
  while (Lp < L) Lp <<= 1;
  for (int i = threadIdx.x; i < Lp; i += kLB) {
    lk[i] = i < L ? KT::key(lv[i]) : (typename KT::K)0;
    li[i] = i < L ? (uint32_t)i : 0xffffffffu;
  }
  __syncthreads();
  for (int k2 = 2; k2 <= Lp; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < Lp; i += kLB) {
        const int ixj = i ^ j;
        if (ixj <= i) continue;
        const typename KT::K ka = lk[i], kb = lk[ixj];
        const uint32_t ia = li[i], ib = li[ixj];
        // a sorts before b: larger key, then smaller index
        const bool a_first = ka > kb || (ka == kb && ia < ib);
        const bool up = (i & k2) == 0;
        if (up ? !a_first : a_first) {
          lk[i] = kb; lk[ixj] = ka;
          li[i] = ib; li[ixj] = ia;
        }
      }
      __syncthreads();
    }
  }
}

// Cardinality with small k: the k-th entry of the line in the order
// (|value| descending, index ascending) by k rounds of a block-wide argmax,
// each over the entries after the previous round's pick.  Exact (keys and
// indices only), so the same entry as the sort finds.
constexpr int kTopkRounds = 32;

template <typename T>
__device__ void line_kth(const T* lv, int L, int k, typename KeyT<T>::K& tkey, uint32_t& tidx,
                         typename KeyT<T>::K* rk, uint32_t* ri) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  K pk = ~(K)0;            // previous pick: above every key
  uint32_t pi = 0;
  for (int round = 0; round < k; ++round) {
    K bk = 0;
    uint32_t bi = 0xffffffffu;
    for (int e = threadIdx.x; e < L; e += kLB) {
      const K key = KT::key(lv[e]);
      const bool after = key < pk || (key == pk && (uint32_t)e > pi);
      const bool first = key > bk || (key == bk && (uint32_t)e < bi);
      if (after && first) { bk = key; bi = (uint32_t)e; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const K ok = __shfl_xor(bk, o, 64);
      const uint32_t oi = __shfl_xor(bi, o, 64);
      if (ok > bk || (ok == bk && oi < bi)) { bk = ok; bi = oi; }
    }
    const int slot = (round & 1) * (kLB / 64);
    if ((threadIdx.x & 63) == 0) { rk[slot + (threadIdx.x >> 6)] = bk; ri[slot + (threadIdx.x >> 6)] = bi; }
    __syncthreads();
    for (int q = 0; q < kLB / 64; ++q) {
      const K ok = rk[slot + q];
      const uint32_t oi = ri[slot + q];
      if (ok > bk || (ok == bk && oi < bi)) { bk = ok; bi = oi; }
    }
    pk = bk;
    pi = bi;
  }
  tkey = pk;
  tidx = pi;
}

// The projection of the line lv[0..L) onto the set (l1 by the sorted
// prefix-sum rule of the whole-vector l1 projection; cardinality by the k-th
// sorted entry; l2 / annulus by the norm).
template <typename T>
__device__ LineProj<T> line_params(const SetDesc& s, int L, const T* lv, typename KeyT<T>::K* lk, uint32_t* li,
                                   acc_t* lds, int* ldi) {
  using KT = KeyT<T>;
  LineProj<T> q{LM_KEEP, (T)0, 0, 0};
  if (s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS) {
    acc_t t = 0;
    for (int e = threadIdx.x; e < L; e += kLB) t += (acc_t)lv[e] * (acc_t)lv[e];
    const double nrm = sqrt((double)line_sum(t, lds));
    if (s.kind == SIP_SET_L2) {
      if (nrm > s.tau) { q.mode = LM_SCALE; q.theta = (T)(s.tau / nrm); }
    } else if (nrm > s.hi) {
      q.mode = LM_SCALE; q.theta = (T)(s.hi / nrm);
    } else if (nrm < s.lo) {
      if (nrm > 0.0) { q.mode = LM_SCALE; q.theta = (T)(s.lo / nrm); }
      else { q.mode = LM_POINT; q.theta = (T)s.lo; }
    }
    return q;
  }
  if (s.kind == SIP_SET_CARD) {
    if (s.k >= L) return q;
    q.mode = LM_TOPK;
    if (s.k <= kTopkRounds) {
      __shared__ typename KT::K rk[2 * kLB / 64];
      __shared__ uint32_t ri[2 * kLB / 64];
      line_kth<T>(lv, L, (int)s.k, q.tkey, q.tidx, rk, ri);
      return q;
    }
    line_sort<T>(lv, L, lk, li);
    q.tkey = lk[s.k - 1];
    q.tidx = li[s.k - 1];
    return q;
  }
  // l1 ball
  if (!(s.tau > 0.0)) { q.mode = LM_ZERO; return q; }
  acc_t t = 0;
  for (int e = threadIdx.x; e < L; e += kLB) t += (acc_t)fabs((double)lv[e]);
  if (line_sum(t, lds) <= (acc_t)s.tau) return q;
  line_sort<T>(lv, L, lk, li);
  // running sums c_r over the sorted magnitudes: each thread owns a
  // contiguous chunk of positions; chunk totals are scanned in thread order
  const int chunk = (L + kLB - 1) / kLB;
  const int r0 = threadIdx.x * chunk, r1 = r0 + chunk < L ? r0 + chunk : L;
  acc_t own = 0;
  for (int r = r0; r < r1; ++r) own += (acc_t)KT::value(lk[r]);
  acc_t* scan = lds + lds_sum<1, kLB>();
  __syncthreads();
  scan[threadIdx.x] = own;
  __syncthreads();
  acc_t c = 0;
  for (int q2 = 0; q2 < (int)threadIdx.x; ++q2) c += scan[q2];
  // rho = the largest r + 1 with a_r - (c_r - tau) / (r + 1) > 0
  int best = 0;
  acc_t cc = c;
  for (int r = r0; r < r1; ++r) {
    const acc_t a = (acc_t)KT::value(lk[r]);
    cc += a;
    if (a - (cc - (acc_t)s.tau) / (acc_t)(r + 1) > 0) best = r + 1;
  }
  const int rho = line_max(best, ldi);
  __shared__ acc_t th_s;
  cc = c;
  for (int r = r0; r < r1; ++r) {
    cc += (acc_t)KT::value(lk[r]);
    if (r + 1 == rho) th_s = (cc - (acc_t)s.tau) / (acc_t)rho;
  }
  __syncthreads();
  q.mode = LM_SOFT;
  q.theta = (T)th_s;
  return q;
}

// One line: pass 1 computes s = (A x) on the line, x-bar, w = x-bar - v/rho
// into LDS and the v-hat snapshot with its adapt dots; the line projection;
// pass 2 writes y = P(w), v = rho (y - w) and the y / v snapshots with their
// dots; on stopping-test iterations the same projection of s gives the
// feasibility distance.  Partial sums as the projection kernel's units.
// Dynamic LDS: cap (a power of two >= the batch's longest line) values, keys
// and indices.
template <typename T>
constexpr size_t line_lds_per_entry() { return sizeof(T) + sizeof(typename KeyT<T>::K) + 4; }

template <typename T>
__global__ __launch_bounds__(kLB) void k_line(const InstDesc* __restrict__ D, const LineItem* __restrict__ items, Opts o, double* parts, int cap) {
  using KT = KeyT<T>;
  extern __shared__ __align__(16) unsigned char line_smem[];
  typename KT::K* lk = (typename KT::K*)line_smem;
  T* lv = (T*)(line_smem + (size_t)cap * sizeof(typename KT::K));
  uint32_t* li = (uint32_t*)(line_smem + (size_t)cap * (sizeof(typename KT::K) + sizeof(T)));
  __shared__ acc_t lds[lds_sum<8, kLB>() + kLB];
  __shared__ int ldi[kLB / 64];
  const LineItem it = items[blockIdx.x];
  if (it.inst < 0) return;
  const int iti = it.idx;
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  const ItScal isc = it_scal(S);
  if (!isc.live()) return;
  const int k = (int)isc.k;
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  const bool have = isc.have != 0.0;
  const int call = adapt ? adapt_call(k, o) : 0;
  const SetDesc& s = d.sets[it.set];
  const Geo g(d);
  const int axis = s.axis[it.comp];
  const size_t off = (size_t)it.comp * g.cs;
  T* y = (T*)s.y + off;
  T* v = (T*)s.v + off;
  T* vh0 = (T*)s.vh0 + off;
  T* v0 = (T*)s.v0 + off;
  T* y0 = (T*)s.y0 + off;
  const T* x = (const T*)d.x;
  const T* xr = (const T*)d.xs[(call & 1) ^ 1];
  const double rho_d = ldgd(S + S_RHO + it.set), gam_d = ldgd(S + S_GAMMA + it.set);
  const T rho = (T)rho_d, gam = (T)gam_d, one_m_g = (T)(1.0 - gam_d);
  const T irho = (T)(1.0 / rho_d);
  const int ast = axis == 0 ? g.sz : (axis == 1 ? g.sy : 1);
  const T h = axis >= 0 ? (T)d.hinv[axis] : (T)1;
  auto sval = [&](const T* f, int P) -> T { return axis < 0 ? f[P] : (f[P + ast] - f[P]) * h; };
  const int L = it.len;
  acc_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < L; e += kLB) {
    const int P = it.start + e * it.stride;
    const T sp = sval(x, P);
    const T yo = y[P], vo = v[P];
    lv[e] = gam * sp + one_m_g * yo - vo * irho;
    if (adapt) {
      const T vh = vo + rho * (yo - sp);
      if (have) {
        const acc_t dh = (acc_t)sp - (acc_t)sval(xr, P);
        const acc_t dvh = (acc_t)vh - (acc_t)vh0[P];
        acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
      }
      vh0[P] = vh;
    }
  }
  __syncthreads();
  const LineProj<T> qw = line_params<T>(s, L, lv, lk, li, lds, ldi);
  for (int e = threadIdx.x; e < L; e += kLB) {
    const int P = it.start + e * it.stride;
    const T w = lv[e];
    const T r = line_apply<T>(qw, w, e);
    const T vn = rho * (r - w);
    y[P] = r;
    v[P] = vn;
    if (adapt) {
      if (have) {
        const acc_t dg = -((acc_t)r - (acc_t)y0[P]);
        const acc_t dv = (acc_t)vn - (acc_t)v0[P];
        acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
      }
      y0[P] = r;
      v0[P] = vn;
    }
  }
  if (check) {
    __syncthreads();
    for (int e = threadIdx.x; e < L; e += kLB) {
      const T sp = sval(x, it.start + e * it.stride);
      lv[e] = sp;
      acc[7] += (acc_t)sp * (acc_t)sp;
    }
    __syncthreads();
    const LineProj<T> qs = line_params<T>(s, L, lv, lk, li, lds, ldi);
    for (int e = threadIdx.x; e < L; e += kLB) {
      const T sp = lv[e];
      const acc_t df = (acc_t)sp - (acc_t)line_apply<T>(qs, sp, e);
      acc[6] += df * df;
    }
  }
  block_total_n<8, kLB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) parts[(size_t)iti * 8 + q] = acc[q];
  }
}

// ----------------------------------------------------- end of iteration

__device__ bool spectral(double ab, double aa, double bb, double eps, double& est) {
  const double den = sqrt(aa) * sqrt(bb);
  if (!(den > 0.0)) return false;
  const double corr = ab / den;
  if (!(corr > eps)) return false;
  const double mg = ab / aa, sd = bb / ab;
  est = (2.0 * mg > sd) ? mg : sd - 0.5 * mg;
  return true;
}

// One block per instance: reduce the iteration's partial sums, run the
// stopping test (eqs. feas_stop, obj_stop, stopping_conditions), then
// adapt-rho-gamma for i = 1..p+1 with the gamma cap and rho-ratio guard,
// recompute the stencil scalars of C, and advance k.
// Eight waves, so the sums of an adapt iteration run in one round.
constexpr int kFB = 512;

template <typename T>
__global__ __launch_bounds__(kFB) void k_finish(const InstDesc* __restrict__ D, const int32_t* __restrict__ insts, Opts o,
                                                   const double* proj_parts, const double* thrw_parts,
                                                   const double* thra_parts, const double* line_parts) {
  __shared__ acc_t tout[4 * kMaxUnits + 2][8];
  __shared__ acc_t dots[kMaxUnits][8];
  __shared__ acc_t evol[16];
  const int inst = insts[blockIdx.x];
  if (inst < 0) return;
  const InstDesc& d = D[inst];
  double* S = d.scal;
  const ItScal isc = it_scal(S);
  if (isc.state != 0.0) return;
  if (isc.err != 0.0) {
    if (threadIdx.x == 0) S[S_STATE] = 3.0;
    return;
  }
  const int k = (int)isc.k;
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  const int p = d.nsets;
  // Every sum this kernel needs is a task: 8 consecutive per-item partial
  // values summed over an item range (a projection unit's dots; a threshold
  // set's w-pass and apply-pass dots, per pipeline; the evolution sums).
  // Each wave takes whole tasks (lanes stride the items, then a butterfly), so
  // all sums run at once with no barrier; the same order, so the same value,
  // as any other wave would produce.
  const int ntask_units = (adapt || check) ? p + 1 : 0;
  auto unit_tasks = [&](int u) -> int { return (u < p && d.sets[u].thr >= 0) ? (check ? 4 : 2) : 1; };
  int ntasks = 0;
  for (int u = 0; u < ntask_units; ++u) ntasks += unit_tasks(u);
  const bool evol_on = check && d.ring;
  if (evol_on) ntasks += 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // this thread's unit's (rho, gamma), loaded with the sums' partials
  const int uc = (int)threadIdx.x <= p ? (int)threadIdx.x : 0;
  const double rho_l = ldgd(S + S_RHO + uc), gam_l = ldgd(S + S_GAMMA + uc);
  for (int t = wv; t < ntasks; t += kFB / 64) {
    // locate task t
    const double* parts = proj_parts;
    int b = d.sp_begin, e = d.sp_end, stride = kProjParts, off = 0;
    int rem = t, u = 0;
    for (; u < ntask_units; ++u) {
      const int nt = unit_tasks(u);
      if (rem < nt) break;
      rem -= nt;
    }
    if (u < ntask_units) {
      if (u < p && d.sets[u].line_axis >= 0) {
        parts = line_parts;
        b = d.sets[u].line_begin;
        e = d.sets[u].line_end;
        stride = 8;
      } else if (unit_tasks(u) == 1 && !(u < p && d.sets[u].thr >= 0)) {
        off = u * kUnitParts;
      } else {
        const SetDesc& sd = d.sets[u];
        const int src = rem >> 1;
        parts = (rem & 1) ? thra_parts : thrw_parts;
        b = sd.item_begin[src];
        e = sd.item_end[src];
        stride = kThrParts;
      }
    } else {
      off = kEvolOff + 8 * rem;
    }
    acc_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // four items per lane in flight at a time, added in item order
    constexpr int U = 4;
    for (int i0 = b + lane; i0 < e; i0 += 64 * U) {
      double q[U][8];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int i = i0 + 64 * r < e ? i0 + 64 * r : i0;
#pragma unroll
        for (int j = 0; j < 8; ++j) q[r][j] = ldgd(parts + (size_t)i * stride + off + j);
      }
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (i0 + 64 * r < e) {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] += (acc_t)q[r][j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) tout[t][j] = v[j];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int u = 0; u < ntask_units; ++u) {
      if (!(u < p && d.sets[u].thr >= 0)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) dots[u][j] = tout[t][j];
        t += 1;
      } else {
        // w pass: dh dots in 0..2, ||s||^2 in 7 (pipeline 1); apply pass:
        // dg/dv dots in 3..5, the feasibility distance in 6 (pipeline 1)
        for (int j = 0; j < 3; ++j) { dots[u][j] = tout[t][j]; dots[u][3 + j] = tout[t + 1][3 + j]; }
        dots[u][6] = check ? tout[t + 3][6] : (acc_t)0;
        dots[u][7] = check ? tout[t + 2][7] : (acc_t)0;
        t += check ? 4 : 2;
      }
    }
    if (evol_on) {
#pragma unroll
      for (int j = 0; j < 8; ++j) { evol[j] = tout[t][j]; evol[8 + j] = tout[t + 1][j]; }
    }
  }
  // The per-set work runs in parallel, thread u for unit u (p + 1 <= 256):
  // selection errors, the schedule log, r_feas, the new (rho, gamma); thread 0
  // combines.  Every value is computed as a single thread would.
  __shared__ int s_err, s_bad, s_conv;
  __shared__ double s_rho[kMaxUnits], s_gam[kMaxUnits];
  const int u = (int)threadIdx.x;
  if (u == 0) { s_err = 0; s_bad = 0; s_conv = 0; }
  __syncthreads();
  if (u < p && d.sets[u].thr >= 0) {
    const int e0 = d.sets[u].sel[0]->err;
    const int e1 = check ? d.sets[u].sel[1]->err : 0;
    if (e0 || e1) s_err = e1 ? e1 : e0;  // every selection error is SIP_ENUMERIC
  }
  __syncthreads();
  if (s_err) {
    if (u == 0) { S[S_ERR] = (double)s_err; S[S_STATE] = 3.0; }
    return;
  }
  if (u < p && d.sets[u].thr >= 0 && (d.sets[u].kind == SIP_SET_L1 || d.sets[u].kind == SIP_SET_CARD)) {
    // the next w pass gathers the entries of this iteration's first-digit
    // bucket (list A) when the selection went through the radix digits
    // and the bucket is small enough to be of use: on average at most a
    // w-pass block's LDS stage per item (a block whose stage fills appends
    // the rest with a global atomic per wave and group)
    const SetDesc& sd = d.sets[u];
    for (int src = 0; src < (check ? 2 : 1); ++src) {
      SelState* q = sd.sel[src];
      const unsigned long long nit = (unsigned long long)(sd.item_end[src] - sd.item_begin[src]);
      const bool radix = q->mode == SEL_PROJECT && q->final_ && !q->err && !o.sel_fresh &&
                         q->cnt0 <= nit * (unsigned long long)StageCap<T>::v;
      q->spec = radix ? (int)(q->prefix >> digit_shift<T>(0)) + 1 : 0;
      q->nspec = 0ull;
    }
  }
  const double rho_u = u <= p ? rho_l : 0.0, gam_u = u <= p ? gam_l : 0.0;
  if (d.log && k <= d.log_cap && u <= p) {
    double* row = d.log + (size_t)(k - 1) * 2 * kMaxUnits;
    row[u] = rho_u;
    row[kMaxUnits + u] = gam_u;
  }
  if (check) {
    if (u < p) {
      double num = dots[u][6];
      const double den = dots[u][7];
      const SetDesc& s = d.sets[u];
      if ((s.kind == SIP_SET_L2 || s.kind == SIP_SET_ANNULUS) && s.line_axis < 0) {
        // distance of s to the ball / shell from ||s|| (= sqrt(den)) alone
        const double nrm = sqrt(den);
        const double lo = s.kind == SIP_SET_L2 ? 0.0 : s.lo, hi = s.kind == SIP_SET_L2 ? s.tau : s.hi;
        const double t = nrm < lo ? lo : (nrm > hi ? hi : nrm);
        num = (nrm - t) * (nrm - t);
      }
      if (s.thr >= 0 && s.kind == SIP_SET_CARD && s.sel[1]->mode == SEL_PROJECT) {
        // the dropped entries equal to the k-th magnitude all have that magnitude
        const SelState& q = *s.sel[1];
        num += (double)(q.ties - q.keep_ties) * q.tk * q.tk;
      }
      double rf;
      if (den > 0.0) rf = sqrt(num) / sqrt(den);
      else rf = (num > 0.0) ? INFINITY : 0.0;
      S[S_RFEAS + u] = rf;
      if (!(rf < o.eps_feas)) s_bad = 1;
    }
    __syncthreads();
    if (u == 0) {
      double worst = 0.0;
      for (int j = 1; j <= o.evol_hist; ++j) worst = evol[j] > worst ? evol[j] : worst;
      const double xn = evol[0];
      double re;
      if (xn > 0.0) re = sqrt(worst) / sqrt(xn);
      else re = worst > 0.0 ? INFINITY : 0.0;
      S[S_REVOL] = re;
      if (re < o.eps_evol && !s_bad) {
        S[S_STATE] = 1.0;
        S[S_ITERS] = (double)k;
        s_conv = 1;
      }
    }
    __syncthreads();
    if (s_conv) return;
  }
  if (adapt) {
    if (isc.have != 0.0) {
      if (u <= p) {
        double a = 0.0, b = 0.0, rn, gn;
        const bool oa = spectral(dots[u][0], dots[u][1], dots[u][2], o.eps_corr, a);
        const bool ob = spectral(dots[u][3], dots[u][4], dots[u][5], o.eps_corr, b);
        if (oa && ob) { const double gm = sqrt(a * b); rn = gm; gn = 1.0 + 2.0 * gm / (a + b); }
        else if (oa) { rn = a; gn = 1.9; }
        else if (ob) { rn = b; gn = 1.1; }
        else { rn = rho_u; gn = 1.5; }
        if (gn > o.gamma_max) gn = o.gamma_max;
        s_rho[u] = rn;
        s_gam[u] = gn;
      }
      __syncthreads();
      if (u < p) {
        const double rl = s_rho[p];
        const double lo = rl / o.rho_ratio_max, hi = rl * o.rho_ratio_max;
        const double r = s_rho[u];
        s_rho[u] = r < lo ? lo : (r > hi ? hi : r);
      }
      __syncthreads();
      if (u <= p) { S[S_RHO + u] = s_rho[u]; S[S_GAMMA + u] = s_gam[u]; }
    } else {
      if (u <= p) s_rho[u] = rho_u;
      __syncthreads();
    }
    if (u == 0) {
      S[S_HAVE_SNAP] = 1.0;
      double c0 = s_rho[p], ca[3] = {0.0, 0.0, 0.0};
      for (int q = 0; q < p; ++q) {
        const SetDesc& s = d.sets[q];
        if (s.op == SIP_OP_I) c0 += s_rho[q];
        else for (int c = 0; c < s.ncomp; ++c) ca[s.axis[c]] += s_rho[q];
      }
      S[S_C0] = c0;
      for (int a = 0; a < 3; ++a) S[S_CAX + a] = ca[a] * d.h2inv[a];
    }
  }
  if (u == 0) {
    S[S_ITERS] = (double)k;
    S[S_K] = (double)(k + 1);
    if (k + 1 > o.max_iter) S[S_STATE] = 2.0;
  }
}

// Clears a pipeline's histogram (used at admission; graph-safe, no memset).
__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = 0;
}
__global__ __launch_bounds__(kBlock) void k_zero_f64(double* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = 0.0;
}

// ------------------------------------------------------ host-side launchers

template <typename T>
void launch_init(hipStream_t st, const InstDesc* __restrict__ D, int inst, int64_t N) {
  const int64_t nb = (N + kBlock - 1) / kBlock;
  k_init<T><<<(int)(nb < 2048 ? nb : 2048), kBlock, 0, st>>>(D, inst);
}

// RHS and the CG steps with NT threads per block.
template <typename T, int NT>
void launch_cg(hipStream_t st, const Tables& t, const Opts& o) {
  k_rhs<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.rr_part);
  if (t.cg_form == 2) {
    k_cg2_d0<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.pq_part);
    double* g[2] = {t.rr_part, t.rr2_part};
    double* q[2] = {t.pq_part, t.pq2_part};
    double* x[2] = {t.xq_part, t.xq2_part};
    const size_t lb = (size_t)(t.cg2_cap + t.cg2_capr) * sizeof(T);
    for (int j = 0; j < o.cg_max; ++j) {
      const int a = j & 1, b = (j + 1) & 1;
      if (j == 0)
        k_cg2_step<T, NT, 1><<<t.npt, NT, lb, st>>>(t.D, t.pt, j, g[a], q[a], x[a], g[b], q[b], x[b], o, t.cg2_cap);
      else
        k_cg2_step<T, NT, 2><<<t.npt, NT, lb, st>>>(t.D, t.pt, j, g[a], q[a], x[a], g[b], q[b], x[b], o, t.cg2_cap);
      if (t.cg2_rest) {
        // the other instances' steps (their items' partials only)
        k_cg_dir<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, t.rr_part, t.pq_part, o);
        k_cg_upd<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, t.pq_part, t.rr_part);
      }
    }
    return;
  }
  if (t.cg_form == 1) {
    k_cg1_w0<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.pq_part);
    for (int j = 0; j < o.cg_max; ++j) {
      double* g[2] = {t.rr_part, t.rr2_part};
      double* dd[2] = {t.pq_part, t.pq2_part};
      if (j == 0)
        k_cg1_step<T, NT, 2><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, g[0], dd[0], g[1], dd[1], o);
      else
        k_cg1_step<T, NT, 3><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, g[j & 1], dd[j & 1], g[(j + 1) & 1],
                                                    dd[(j + 1) & 1], o);
    }
    return;
  }
  for (int j = 0; j < o.cg_max; ++j) {
    k_cg_dir<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, t.rr_part, t.pq_part, o);
    k_cg_upd<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, j, t.pq_part, t.rr_part);
  }
}

template <typename T, int NT>
void launch_point_phase(hipStream_t st, const Tables& t, const Opts& o, int phase) {
  if (!t.npt) return;
  if (phase == 0) k_rhs<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.rr_part);
  if (phase == 1) k_cg_dir<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, 1, t.rr_part, t.pq_part, o);
  if (phase == 2) k_cg_upd<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, 1, t.pq_part, t.rr_part);
  if (phase == 6)
    k_cg1_step<T, NT, 3><<<t.npt, NT, 0, st>>>(t.D, t.pt, 1, t.rr2_part, t.pq2_part, t.rr_part, t.pq_part, o);
  if (phase == 7) k_cg1_w0<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.pq_part);
  if (phase == 9 && t.cg_form == 2)
    k_cg2_step<T, NT, 2><<<t.npt, NT, (size_t)(t.cg2_cap + t.cg2_capr) * sizeof(T), st>>>(
        t.D, t.pt, 1, t.rr2_part, t.pq2_part, t.xq2_part, t.rr_part, t.pq_part, t.xq_part, o, t.cg2_cap);
  if (phase == 10) k_cg2_d0<T, NT><<<t.npt, NT, 0, st>>>(t.D, t.pt, t.pq_part);
}

template <typename T>
void launch_iteration(hipStream_t st, const Tables& t, const Opts& o) {
  if (t.npt > 0) {
    if (t.pt_threads == 256) launch_cg<T, 256>(st, t, o);
    else launch_cg<T, 512>(st, t, o);
  }
  const bool proj = t.npt > 0 && t.nsp > 0;
  if (proj && t.nthr > 0 && t.fuse_sets) {
    k_sets<T><<<t.nsp * t.proj_units + t.nthr, kSB, 0, st>>>(t.D, t.sp, t.thr, o, t.proj_part, t.thrw_part,
                                                              t.nsp, t.proj_units, t.nthr);
  } else {
    if (proj)
      k_proj<T><<<proj_blocks(t.nsp, t.proj_units), kSB, 0, st>>>(t.D, t.sp, o, t.proj_part, t.nsp, t.proj_units);
    if (t.nthr > 0) k_thr_w<T><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, t.thrw_part);
  }
  if (t.nthr > 0) {
    if (t.sel_fused) {
      // one refine pass that also does the first selection stage
      k_thr_refine<T, true><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, 1, t.thrw_part, t.h1c, t.h1s);
      k_sel_next<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.sel, o, 1, t.tie_part, 1, t.h1c, t.h1s);
    } else {
      k_sel1<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.sel, o, t.thrw_part, t.sel_passes);
      if (t.sel_passes == 2) {
        k_thr_refine<T, false><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, 0, t.thrw_part, t.h1c, t.h1s);
        k_sel_next<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.sel, o, 0, t.tie_part, 0, t.h1c, t.h1s);
      }
      // the last pass always appends candidates, so its select stage is final
      k_thr_refine<T, false><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, 1, t.thrw_part, t.h1c, t.h1s);
      k_sel_next<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.sel, o, 1, t.tie_part, 0, t.h1c, t.h1s);
    }
    k_thr_apply<T><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, t.thra_part, t.tie_part, t.nthr);
  }
  if (t.nline > 0)
    k_line<T><<<t.nline, kLB, t.line_cap * line_lds_per_entry<T>(), st>>>(t.D, t.line, o, t.line_part,
                                                                         t.line_cap);
  if (t.ninst > 0)
    k_finish<T><<<t.ninst, kFB, 0, st>>>(t.D, t.inst, o, t.proj_part, t.thrw_part, t.thra_part,
                                            t.line_part);
}

// One kernel of the iteration on its own (timing); CG kernels use step 1.
// 0 rhs, 1 cg_dir, 2 cg_upd, 3 proj, 4 thr_w, 5 thr_apply, 6 one-reduction
// CG step, 7 its w_0 = C r_0 pass, 8 line-wise sets, 9 LDS-staged CG step
// (only where the batch runs that form), 10 its r_0^T C r_0 pass.
template <typename T>
void launch_phase(hipStream_t st, const Tables& t, const Opts& o, int phase) {
  switch (phase) {
    case 0:
    case 1:
    case 2:
    case 6:
    case 7:
    case 9:
    case 10:
      if (t.pt_threads == 256) launch_point_phase<T, 256>(st, t, o, phase);
      else launch_point_phase<T, 512>(st, t, o, phase);
      break;
    case 3:
      if (t.nsp)
        k_proj<T><<<proj_blocks(t.nsp, t.proj_units), kSB, 0, st>>>(t.D, t.sp, o, t.proj_part, t.nsp, t.proj_units);
      break;
    case 4: if (t.nthr) k_thr_w<T><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, t.thrw_part); break;
    case 5: if (t.nthr) k_thr_apply<T><<<t.nthr, kSB, 0, st>>>(t.D, t.thr, o, t.thra_part, t.tie_part, t.nthr); break;
    case 8:
      if (t.nline)
        k_line<T><<<t.nline, kLB, t.line_cap * line_lds_per_entry<T>(), st>>>(t.D, t.line, o, t.line_part,
                                                                             t.line_cap);
      break;
    default: break;
  }
}

// Streaming copy, 16 bytes per lane per step: the bandwidth reference.
__global__ __launch_bounds__(kBlock) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) dst[i] = src[i];
}

void launch_copy(hipStream_t st, void* dst, const void* src, int64_t n16) {
  if (n16 > 0) k_copy<<<2048, kBlock, 0, st>>>((const uint4*)src, (uint4*)dst, n16);
}

template void launch_phase<float>(hipStream_t, const Tables&, const Opts&, int);
template void launch_phase<double>(hipStream_t, const Tables&, const Opts&, int);
template void launch_iteration<float>(hipStream_t, const Tables&, const Opts&);
template void launch_iteration<double>(hipStream_t, const Tables&, const Opts&);
template void launch_init<float>(hipStream_t, const InstDesc*, int, int64_t);
template void launch_init<double>(hipStream_t, const InstDesc*, int, int64_t);

void launch_zero(hipStream_t st, uint32_t* a, int64_t n) {
  if (n > 0) k_zero_u32<<<(int)((n + kBlock - 1) / kBlock < 1024 ? (n + kBlock - 1) / kBlock : 1024), kBlock, 0, st>>>(a, n);
}
void launch_zero(hipStream_t st, double* a, int64_t n) {
  if (n > 0) k_zero_f64<<<(int)((n + kBlock - 1) / kBlock < 1024 ? (n + kBlock - 1) / kBlock : 1024), kBlock, 0, st>>>(a, n);
}

}  // namespace SIP_KNS
}  // namespace sip
