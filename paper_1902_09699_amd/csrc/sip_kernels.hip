// gfx950 kernels of one PARSDMM iteration (PARSDMM listing; eq. SDMM_adaptive).
//
// Every kernel walks a work table: point items (a contiguous range of grid
// points of one instance), threshold items (a point range of one selection
// pipeline), selection items (one pipeline) or instances.  Blocks are mapped
// to items so that each of the 8 XCDs sweeps one contiguous slice of the
// table, which keeps the z/y neighbours a stencil reads in that XCD's L2.
//
// Reductions never use atomics on floating point across blocks except the
// histogram sums, which are exact for float keys (all values in one bucket
// share an exponent).  Each item writes its partial sums; the consumer
// (next launch) reduces an instance's partials in a fixed order, so results
// do not depend on which other instances share the launch.
#include <hip/hip_runtime.h>

#include "sip_internal.h"

namespace sip {

constexpr int kPB = 1024;  // threads per block of the CG and RHS kernels
// Threads per block of the set and threshold kernels: more registers per
// thread and no partial reduction at start, so smaller blocks let several
// stay resident per CU (latency hiding on many small items).
constexpr int kSB = 256;
constexpr int kSW = kSB / 64;

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int xcd_item(int b, int G) {
  const int q = G >> 3, rem = G & 7, x = b & 7, j = b >> 3;
  return x * q + (x < rem ? x : rem) + j;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum of NV doubles over NT threads (a fixed butterfly in
// each wave, then the wave totals in order by one thread per value); every
// thread gets the totals.  lds needs lds_sum<NV, NT>() doubles.
template <int NV, int NT = kBlock>
constexpr int lds_sum() { return NV * (NT / 64 + 1); }

template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
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
    double t = 0.0;
    for (int q = 0; q < NW; ++q) t += lds[threadIdx.x * NW + q];
    lds[NV * NW + threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = lds[NV * NW + i];
  __syncthreads();
}

// Sum of parts[i * stride + off .. + NV) over items i in [begin, end).
template <int NV, int NT = kBlock>
__device__ __forceinline__ void reduce_range(const double* __restrict__ parts, int begin, int end, int stride,
                                             int off, double (&out)[NV], double* lds) {
#pragma unroll
  for (int j = 0; j < NV; ++j) out[j] = 0.0;
  for (int i = begin + (int)threadIdx.x; i < end; i += NT) {
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] += parts[(size_t)i * stride + off + j];
  }
  block_sum<NV, NT>(out, lds);
}

template <int NT>
__device__ __forceinline__ double reduce_one(const double* __restrict__ parts, int begin, int end, double* lds) {
  double a[1];
  reduce_range<1, NT>(parts, begin, end, 1, 0, a, lds);
  return a[0];
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
  int nz, ny, nx, sy, sz, N;
  FastDiv dx, dy;
  __device__ explicit Geo(const InstDesc& d)
      : nz((int)d.n[0]), ny((int)d.n[1]), nx((int)d.n[2]), sy((int)d.stride[1]), sz((int)d.stride[0]),
        N((int)d.N), dx(d.div_x), dy(d.div_y) {}
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

__device__ __forceinline__ bool inst_live(const double* S) { return S[S_STATE] == 0.0 && S[S_ERR] == 0.0; }

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
// v_{p+1} = 0, x-history slot 0 = m.  d.m is the instance's private copy of m.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const InstDesc* D, int inst) {
  const InstDesc& d = D[inst];
  const Geo g(d);
  const T* m = (const T*)d.m;
  T* x = (T*)d.x;
  T* yl = (T*)d.yl;
  T* vl = (T*)d.vl;
  T* ring = (T*)d.ring;
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
        ((T*)s.y)[(size_t)c * g.N + P] = val;
        ((T*)s.v)[(size_t)c * g.N + P] = 0;
      }
    }
  }
}

// -------------------------------------------------------- RHS + residual

// Items are processed in rounds of kPB * U points; the U points of a thread
// are independent, so their loads are issued together (memory-level
// parallelism), and __restrict__ lets stores trail loads.
constexpr int kUset = 2;

// b = sum_{i<=p+1} A_i^T (rho_i y_i + v_i);  r = b - C x;  partial r^T r.
template <typename T>
__global__ __launch_bounds__(kPB) void k_rhs(const InstDesc* D, const Counts* cnt, const PtItem* items, double* rr_part) {
  __shared__ double lds[lds_sum<1, kPB>()];
  if ((int)blockIdx.x >= cnt->npt) return;
  const int iti = xcd_item(blockIdx.x, cnt->npt);
  const PtItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const Geo g(d);
  const T* __restrict__ x = (const T*)d.x;
  T* __restrict__ r = (T*)d.r;
  const T* __restrict__ yl = (const T*)d.yl;
  const T* __restrict__ vl = (const T*)d.vl;
  const T rl = (T)S[S_RHO + d.nsets];
  const T c0 = (T)S[S_C0], cz = (T)S[S_CAX + 0], cy = (T)S[S_CAX + 1], cx = (T)S[S_CAX + 2];
  double acc[1] = {0.0};
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += kPB * kUset) {
    int Pu[kUset], iz[kUset], iy[kUset], ix[kUset];
    T b[kUset];
#pragma unroll
    for (int u = 0; u < kUset; ++u) {
      Pu[u] = base + u * kPB + (int)threadIdx.x;
      const int P = Pu[u] < end ? Pu[u] : end - 1;
      g.coords(P, iz[u], iy[u], ix[u]);
      b[u] = rl * yl[P] + vl[P];
    }
    for (int si = 0; si < d.nsets; ++si) {
      const SetDesc& s = d.sets[si];
      const T rs = (T)S[S_RHO + si];
      for (int c = 0; c < s.ncomp; ++c) {
        const T* __restrict__ y = (const T*)s.y + (size_t)c * g.N;
        const T* __restrict__ v = (const T*)s.v + (size_t)c * g.N;
        const int a = s.axis[c];
        const T hi = (T)d.hinv[a < 0 ? 0 : a];
#pragma unroll
        for (int u = 0; u < kUset; ++u) {
          const int P = Pu[u] < end ? Pu[u] : end - 1;
          if (a < 0) {
            b[u] += rs * y[P] + v[P];
          } else {
            const int ia = a == 0 ? iz[u] : (a == 1 ? iy[u] : ix[u]);
            const int na = a == 0 ? g.nz : (a == 1 ? g.ny : g.nx);
            const int st = a == 0 ? g.sz : (a == 1 ? g.sy : 1);
            T t = 0;
            if (ia > 0) t += rs * y[P - st] + v[P - st];
            if (ia < na - 1) t -= rs * y[P] + v[P];
            b[u] += t * hi;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kUset; ++u) {
      if (Pu[u] >= end) continue;
      const int P = Pu[u];
      const T xc = x[P];
      T lz = 0, ly = 0, lx = 0;
      if (iz[u] > 0) lz += xc - x[P - g.sz];
      if (iz[u] < g.nz - 1) lz += xc - x[P + g.sz];
      if (iy[u] > 0) ly += xc - x[P - g.sy];
      if (iy[u] < g.ny - 1) ly += xc - x[P + g.sy];
      if (ix[u] > 0) lx += xc - x[P - 1];
      if (ix[u] < g.nx - 1) lx += xc - x[P + 1];
      const T rv = b[u] - (c0 * xc + cz * lz + cy * ly + cx * lx);
      r[P] = rv;
      acc[0] += (double)rv * (double)rv;
    }
  }
  block_sum<1, kPB>(acc, lds);
  if (threadIdx.x == 0) rr_part[iti] = acc[0];
}

// ---------------------------------------------------------------- CG

// 16-byte groups: a thread owns W = 16 / sizeof(T) consecutive points, loads
// and stores them with one 128-bit access, takes its x-neighbours from the
// adjacent lanes (shuffles) and its y/z neighbours with 128-bit loads when
// the row stride is a multiple of W.  Groups cut by the item end, and
// instances whose x buffer is not 16-byte aligned, take a per-point path.
template <typename T>
struct Grp {
  static constexpr int W = 16 / (int)sizeof(T);
};

template <typename T>
__device__ __forceinline__ void ld16(const T* __restrict__ p, T (&o)[Grp<T>::W]) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  __builtin_memcpy(o, &u, 16);
}

template <typename T>
__device__ __forceinline__ void st16(T* __restrict__ p, const T (&o)[Grp<T>::W]) {
  uint4 u;
  __builtin_memcpy(&u, o, 16);
  *reinterpret_cast<uint4*>(p) = u;
}

// For the group of W points at P0 (all threads of the wave call this, for the
// shuffles): c = values at the group (fetchv / fetchs give the value a
// stencil sees), q = C c.  Returns whether the group was handled as a whole;
// otherwise the caller runs the per-point path.
template <typename T, typename FV, typename FS>
__device__ __forceinline__ bool group_apply_C(int P0, bool full, int lane, const Geo& g, bool vec_nb, FV fetchv,
                                              FS fetchs, T (&c)[Grp<T>::W], T (&q)[Grp<T>::W], T c0, T cz, T cy,
                                              T cx) {
  constexpr int W = Grp<T>::W;
  if (full) {
    fetchv(P0, c);
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) c[e] = 0;
  }
  T left = __shfl_up(c[W - 1], 1, 64);
  T right = __shfl_down(c[0], 1, 64);
  const int next_full = __shfl_down(full ? 1 : 0, 1, 64);
  if (!full) return false;
  int iz, iy, ix0;
  g.coords(P0, iz, iy, ix0);
  const bool straddle = ix0 + W > g.nx;
  if (lane == 0) left = P0 > 0 ? fetchs(P0 - 1) : (T)0;
  if (lane == 63 || !next_full) right = P0 + W < g.N ? fetchs(P0 + W) : (T)0;
  T ym[W], yp[W], zm[W], zp[W];
  const bool vnb = vec_nb && !straddle;
  if (vnb) {
    if (iy > 0) fetchv(P0 - g.sy, ym);
    if (iy < g.ny - 1) fetchv(P0 + g.sy, yp);
    if (iz > 0) fetchv(P0 - g.sz, zm);
    if (iz < g.nz - 1) fetchv(P0 + g.sz, zp);
  }
#pragma unroll
  for (int e = 0; e < W; ++e) {
    int ize = iz, iye = iy, ixe = ix0 + e;
    if (straddle) g.coords(P0 + e, ize, iye, ixe);
    const T ce = c[e];
    const T lft = e > 0 ? c[e > 0 ? e - 1 : 0] : left;
    const T rgt = e < W - 1 ? c[e < W - 1 ? e + 1 : W - 1] : right;
    T lx = 0, ly = 0, lz = 0;
    if (ixe > 0) lx += ce - lft;
    if (ixe < g.nx - 1) lx += ce - rgt;
    if (vnb) {
      if (iye > 0) ly += ce - ym[e];
      if (iye < g.ny - 1) ly += ce - yp[e];
      if (ize > 0) lz += ce - zm[e];
      if (ize < g.nz - 1) lz += ce - zp[e];
    } else {
      const int P = P0 + e;
      if (iye > 0) ly += ce - fetchs(P - g.sy);
      if (iye < g.ny - 1) ly += ce - fetchs(P + g.sy);
      if (ize > 0) lz += ce - fetchs(P - g.sz);
      if (ize < g.nz - 1) lz += ce - fetchs(P + g.sz);
    }
    q[e] = c0 * ce + cz * lz + cy * ly + cx * lx;
  }
  return true;
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

// Step j, first half: beta = rr_j / rr_{j-1}; p_j = r + beta p_{j-1} (p_0 = r);
// partial p_j^T C p_j with C p_j evaluated on the fly (never stored).
template <typename T>
__global__ __launch_bounds__(kPB) void k_cg_dir(const InstDesc* D, const Counts* cnt, const PtItem* items, int j,
                                                const double* rr_part, double* pq_part, Opts o) {
  constexpr int W = Grp<T>::W;
  __shared__ double lds[lds_sum<1, kPB>()];
  if ((int)blockIdx.x >= cnt->npt) return;
  const int iti = xcd_item(blockIdx.x, cnt->npt);
  const PtItem it = items[iti];
  const InstDesc& d = D[it.inst];
  double* S = d.scal;
  if (!inst_live(S)) return;
  const double rr = reduce_one<kPB>(rr_part, d.pt_begin, d.pt_end, lds);
  bool done;
  double beta = 0.0;
  if (j == 0) {
    done = !(rr > 0.0);
  } else {
    done = S[S_DONE + ((j - 1) & 1)] != 0.0 || !(rr > 0.0) || (!o.cg_fixed && rr < o.cg_rel2 * S[S_RR0]);
    beta = rr / S[S_RR + ((j - 1) & 1)];
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
  const T* __restrict__ r = (const T*)d.r;
  const T* __restrict__ pin = (const T*)d.p[(j + 1) & 1];
  T* __restrict__ pout = (T*)d.p[j & 1];
  const T c0 = (T)S[S_C0], cz = (T)S[S_CAX + 0], cy = (T)S[S_CAX + 1], cx = (T)S[S_CAX + 2];
  const T bt = (T)beta;
  const bool first = j == 0;
  auto fs = [&](int Q) -> T { return first ? r[Q] : r[Q] + bt * pin[Q]; };
  auto fv = [&](int Q, T (&o)[W]) {
    ld16<T>(r + Q, o);
    if (!first) {
      T b[W];
      ld16<T>(pin + Q, b);
#pragma unroll
      for (int e = 0; e < W; ++e) o[e] += bt * b[e];
    }
  };
  const int lane = threadIdx.x & 63;
  double acc[1] = {0.0};
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += kPB * W) {
    const int P0 = base + (int)threadIdx.x * W;
    const bool full = d.vec_ok && P0 + W <= end;
    T c[W], q[W];
    if (group_apply_C<T>(P0, full, lane, g, d.vec_nb, fv, fs, c, q, c0, cz, cy, cx)) {
      st16<T>(pout + P0, c);
#pragma unroll
      for (int e = 0; e < W; ++e) acc[0] += (double)c[e] * (double)q[e];
    } else {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        const T pc = fs(P);
        const T qq = point_apply_C<T>(P, g, fs, pc, c0, cz, cy, cx);
        pout[P] = pc;
        acc[0] += (double)pc * (double)qq;
      }
    }
  }
  block_sum<1, kPB>(acc, lds);
  if (threadIdx.x == 0) pq_part[iti] = acc[0];
}

// Step j, second half: alpha = rr_j / p^T C p; x += alpha p; r -= alpha C p
// (C p recomputed from p); partial r^T r.
template <typename T>
__global__ __launch_bounds__(kPB) void k_cg_upd(const InstDesc* D, const Counts* cnt, const PtItem* items, int j,
                                                const double* pq_part, double* rr_part) {
  constexpr int W = Grp<T>::W;
  __shared__ double lds[lds_sum<1, kPB>()];
  if ((int)blockIdx.x >= cnt->npt) return;
  const int iti = xcd_item(blockIdx.x, cnt->npt);
  const PtItem it = items[iti];
  const InstDesc& d = D[it.inst];
  double* S = d.scal;
  if (!inst_live(S)) return;
  if (S[S_DONE + (j & 1)] != 0.0) return;
  const double pq = reduce_one<kPB>(pq_part, d.pt_begin, d.pt_end, lds);
  if (!(pq > 0.0) || !(pq <= 1.0e300)) {
    if (iti == d.pt_begin && threadIdx.x == 0) S[S_ERR] = (double)SIP_ENUMERIC;
    return;
  }
  const double alpha = S[S_RR + (j & 1)] / pq;
  if (iti == d.pt_begin && threadIdx.x == 0) S[S_CGTOT] += 1.0;
  const Geo g(d);
  T* __restrict__ x = (T*)d.x;
  T* __restrict__ r = (T*)d.r;
  const T* __restrict__ p = (const T*)d.p[j & 1];
  const T c0 = (T)S[S_C0], cz = (T)S[S_CAX + 0], cy = (T)S[S_CAX + 1], cx = (T)S[S_CAX + 2];
  const T al = (T)alpha;
  auto fs = [&](int Q) -> T { return p[Q]; };
  auto fv = [&](int Q, T (&o)[W]) { ld16<T>(p + Q, o); };
  const int lane = threadIdx.x & 63;
  double acc[1] = {0.0};
  const int end = it.begin + it.len;
  for (int base = it.begin; base < end; base += kPB * W) {
    const int P0 = base + (int)threadIdx.x * W;
    const bool full = d.vec_ok && P0 + W <= end;
    T c[W], q[W];
    if (group_apply_C<T>(P0, full, lane, g, d.vec_nb, fv, fs, c, q, c0, cz, cy, cx)) {
      T xv[W], rv[W];
      ld16<T>(x + P0, xv);
      ld16<T>(r + P0, rv);
#pragma unroll
      for (int e = 0; e < W; ++e) {
        xv[e] = xv[e] + al * c[e];
        rv[e] = rv[e] - al * q[e];
        acc[0] += (double)rv[e] * (double)rv[e];
      }
      st16<T>(x + P0, xv);
      st16<T>(r + P0, rv);
    } else {
      for (int e = 0; e < W; ++e) {
        const int P = P0 + e;
        if (P >= end) break;
        const T pc = p[P];
        const T qq = point_apply_C<T>(P, g, fs, pc, c0, cz, cy, cx);
        x[P] = x[P] + al * pc;
        const T rv = r[P] - al * qq;
        r[P] = rv;
        acc[0] += (double)rv * (double)rv;
      }
    }
  }
  block_sum<1, kPB>(acc, lds);
  if (threadIdx.x == 0) rr_part[iti] = acc[0];
}

// ------------------------------------------- clip-type sets + identity block

// For every bounds set and the identity block p+1 at the item's points:
// s = A_i x, x-bar = gamma s + (1 - gamma) y, w = x-bar - v/rho,
// y = clip(w) or (m + rho w)/(1 + rho), v += rho (y - x-bar); on adapt
// iterations the six adapt-rho-gamma dots against the k0 snapshot and the new
// snapshot; on stopping-test iterations the feasibility sums of s.  Then the
// x snapshot / x history writes and the r_evol sums.
template <typename T>
__global__ __launch_bounds__(kSB) void k_proj(const InstDesc* D, const Counts* cnt, const PtItem* items, Opts o, double* parts) {
  __shared__ double lds[lds_sum<8, kSB>()];
  if ((int)blockIdx.x >= cnt->nsp) return;
  const int iti = xcd_item(blockIdx.x, cnt->nsp);
  const PtItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const Geo g(d);
  const int k = (int)S[S_K];
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  const bool have = S[S_HAVE_SNAP] != 0.0;
  const int call = adapt ? adapt_call(k, o) : 0;
  const T* __restrict__ x = (const T*)d.x;
  const T* __restrict__ xr = (const T*)d.xs[(call & 1) ^ 1];
  const T* __restrict__ m = (const T*)d.m;
  const int end = it.begin + it.len;
  double* out = parts + (size_t)iti * kProjParts;

  for (int u = 0; u <= d.nsets; ++u) {
    const bool ident = (u == d.nsets);
    const SetDesc* s = ident ? nullptr : &d.sets[u];
    if (!ident && s->thr >= 0) continue;
    const double rho_d = S[S_RHO + u];
    const T rho = (T)rho_d, gam = (T)S[S_GAMMA + u], irho = (T)(1.0 / rho_d);
    const T one_m_g = (T)(1.0 - S[S_GAMMA + u]);
    const T lo = ident ? (T)0 : (T)s->lo, hi = ident ? (T)0 : (T)s->hi;
    const T inv1p = (T)(1.0 / (1.0 + rho_d));
    const int ncomp = ident ? 1 : s->ncomp;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < ncomp; ++c) {
      const int axis = ident ? -1 : s->axis[c];
      const size_t off = (size_t)c * g.N;
      T* __restrict__ y = (T*)(ident ? d.yl : s->y) + off;
      T* __restrict__ v = (T*)(ident ? d.vl : s->v) + off;
      T* __restrict__ vh0 = (T*)(ident ? d.vh0l : s->vh0) + off;
      T* __restrict__ v0 = (T*)(ident ? d.v0l : s->v0) + off;
      T* __restrict__ y0 = (T*)(ident ? d.y0l : s->y0) + off;
      for (int base = it.begin; base < end; base += kSB * kUset) {
#pragma unroll
        for (int uu = 0; uu < kUset; ++uu) {
          const int P = base + uu * kSB + (int)threadIdx.x;
          if (P >= end) continue;
          int iz, iy, ix;
          g.coords(P, iz, iy, ix);
          T sv;
          if (!comp_value<T>(x, P, axis, iz, iy, ix, g, d, sv)) continue;
          const T yo = y[P], vo = v[P];
          const T xb = gam * sv + one_m_g * yo;
          const T w = xb - vo * irho;
          T yn;
          if (ident) yn = (m[P] + rho * w) * inv1p;
          else yn = w < lo ? lo : (w > hi ? hi : w);
          const T vn = vo + rho * (yn - xb);
          y[P] = yn;
          v[P] = vn;
          if (adapt) {
            const T vh = vo + rho * (yo - sv);
            if (have) {
              T s0;
              comp_value<T>(xr, P, axis, iz, iy, ix, g, d, s0);
              const double dh = (double)sv - (double)s0;
              const double dvh = (double)vh - (double)vh0[P];
              const double dg = -((double)yn - (double)y0[P]);
              const double dv = (double)vn - (double)v0[P];
              acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
              acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
            }
            vh0[P] = vh;
            v0[P] = vn;
            y0[P] = yn;
          }
          if (check && !ident) {
            const T pc = sv < lo ? lo : (sv > hi ? hi : sv);
            const double e = (double)sv - (double)pc;
            acc[6] += e * e;
            acc[7] += (double)sv * (double)sv;
          }
        }
      }
    }
    if (adapt || check) {
      block_sum<8, kSB>(acc, lds);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[u * kUnitParts + q] = acc[q];
      }
    }
  }

  // x snapshot for adapt-rho-gamma, x history and r_evol sums
  if (adapt || d.ring) {
    T* __restrict__ xw = (T*)d.xs[call & 1];
    T* __restrict__ ring = (T*)d.ring;
    const int H = o.evol_hist;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double accx[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int P = it.begin + (int)threadIdx.x; P < end; P += kSB) {
      const T xv = x[P];
      if (adapt) xw[P] = xv;
      if (ring) {
        ring[(size_t)(k % (H + 1)) * g.N + P] = xv;
        if (check) {
          accx[0] += (double)xv * (double)xv;
#pragma unroll
          for (int jj = 1; jj < kMaxHist; ++jj) {
            if (jj > H) break;
            const double e = (double)xv - (double)ring[(size_t)((k - jj) % (H + 1)) * g.N + P];
            if (jj <= 7) acc[jj] += e * e; else accx[jj - 7] += e * e;
          }
        }
      }
    }
    if (check) {
      block_sum<8, kSB>(acc, lds);
      block_sum<8, kSB>(accx, lds);
      if (threadIdx.x == 0) {
        out[kEvolOff + 0] = accx[0];
#pragma unroll
        for (int jj = 1; jj < 8; ++jj) out[kEvolOff + jj] = acc[jj];
        out[kEvolOff + 8] = accx[1];  // evol_hist <= 8
      }
    }
  }
}

// --------------------------------------------- threshold sets: pass 1 (w)

// Pipeline 0 (every iteration): w = x-bar - v/rho for the set's components,
// stored over y (y's old value is used first for v-hat); adapt dots of the
// (dh, dvh) pair; radix histogram of the first key digit of |w|.
// Pipeline 1 (stopping-test iterations): histogram of |s| and ||s||^2.
template <typename T>
__global__ __launch_bounds__(kSB) void k_thr_w(const InstDesc* D, const Counts* cnt, const ThrItem* items, Opts o, double* parts) {
  using KT = KeyT<T>;
  __shared__ uint32_t hc[kNB];
  __shared__ double hs[kNB];
  __shared__ double lds[lds_sum<8, kSB>()];
  if ((int)blockIdx.x >= cnt->nthr) return;
  const int iti = xcd_item(blockIdx.x, cnt->nthr);
  const ThrItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const int k = (int)S[S_K];
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  if (it.src == 1 && !check) return;
  const bool have = S[S_HAVE_SNAP] != 0.0;
  const int call = adapt ? adapt_call(k, o) : 0;
  const SetDesc& s = d.sets[it.set];
  const bool l1 = s.kind == SIP_SET_L1;
  for (int b = threadIdx.x; b < kNB; b += kSB) { hc[b] = 0; hs[b] = 0.0; }
  __syncthreads();
  const Geo g(d);
  const T* x = (const T*)d.x;
  const T* xr = (const T*)d.xs[(call & 1) ^ 1];
  const int u = it.set;
  const double rho_d = S[S_RHO + u];
  const T rho = (T)rho_d, gam = (T)S[S_GAMMA + u], one_m_g = (T)(1.0 - S[S_GAMMA + u]);
  const T irho = (T)(1.0 / rho_d);
  const int sh0 = digit_shift<T>(0);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int end = it.begin + it.len;
  for (int c = 0; c < s.ncomp; ++c) {
    const int axis = s.axis[c];
    const size_t off = (size_t)c * g.N;
    T* y = (T*)s.y + off;
    const T* v = (const T*)s.v + off;
    T* vh0 = (T*)s.vh0 + off;
    for (int P = it.begin + (int)threadIdx.x; P < end; P += kSB) {
      int iz, iy, ix;
      g.coords(P, iz, iy, ix);
      T sv;
      if (!comp_value<T>(x, P, axis, iz, iy, ix, g, d, sv)) continue;
      T val;
      if (it.src == 0) {
        const T yo = y[P], vo = v[P];
        const T xb = gam * sv + one_m_g * yo;
        val = xb - vo * irho;
        y[P] = val;
        if (adapt) {
          const T vh = vo + rho * (yo - sv);
          if (have) {
            T s0;
            comp_value<T>(xr, P, axis, iz, iy, ix, g, d, s0);
            const double dh = (double)sv - (double)s0;
            const double dvh = (double)vh - (double)vh0[P];
            acc[0] += dh * dvh; acc[1] += dh * dh; acc[2] += dvh * dvh;
          }
          vh0[P] = vh;
        }
      } else {
        val = sv;
        acc[7] += (double)sv * (double)sv;
      }
      const typename KT::K key = KT::key(val);
      const int bkt = (int)(key >> sh0);
      atomicAdd(&hc[bkt], 1u);
      if (l1) atomicAdd(&hs[bkt], KT::value(key));
    }
  }
  __syncthreads();
  uint32_t* gc = s.hcnt[it.src];
  double* gs = s.hsum[it.src];
  for (int b = threadIdx.x; b < kNB; b += kSB) {
    const uint32_t cnt = hc[b];
    if (cnt) {
      atomicAdd(&gc[b], cnt);
      if (l1) atomicAdd(&gs[b], hs[b]);
    }
  }
  block_sum<8, kSB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) parts[(size_t)iti * kThrParts + q] = acc[q];
  }
}

// ---------------------------------------------- selection (one block each)

// Pick the bucket of the current digit.  l1: the largest bucket b whose lower
// edge L_b still has f(L_b) = sum_{u >= L_b} (u - L_b) >= tau (f decreases, so
// the soft threshold theta with f(theta) = tau lies in bucket b).  Cardinality:
// the largest b with at least k entries at or above L_b.  Updates the state:
// prefix gets digit b, everything in buckets above b moves to c_above/s_above.
// Returns the count of bucket b.
template <typename T>
__device__ unsigned long long select_digit(SelState& st, const uint32_t* hc, const double* hs, int nb, int dig,
                                          const SetDesc& s, bool l1, unsigned long long* lc, double* ls,
                                          int* lbest) {
  using KT = KeyT<T>;
  const int sh = digit_shift<T>(dig);
  const int per = nb / kBlock;  // nb is 1024 or 2048
  const int t = threadIdx.x;
  unsigned long long mc = 0;
  double ms = 0.0;
  for (int i = 0; i < per; ++i) { mc += hc[t * per + i]; if (l1) ms += hs[t * per + i]; }
  // totals of the threads above this one (higher buckets), in a fixed order:
  // an inclusive suffix scan inside each wave, then the wave totals
  const int lane = t & 63, wv = t >> 6;
  unsigned long long ic = mc;
  double is = ms;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long oc = __shfl_down(ic, off, 64);
    const double os = __shfl_down(is, off, 64);
    if (lane + off < 64) { ic += oc; is += os; }
  }
  unsigned long long above_c = __shfl_down(ic, 1, 64);
  double above_s = __shfl_down(is, 1, 64);
  if (lane == 63) { above_c = 0; above_s = 0.0; }
  if (lane == 0) { lc[wv] = ic; ls[wv] = is; }
  if (t == 0) *lbest = -1;
  __syncthreads();
  for (int q = kBlock / 64 - 1; q > wv; --q) { above_c += lc[q]; above_s += ls[q]; }
  __syncthreads();
  // walk own buckets from the top
  unsigned long long rc = st.c_above + above_c;
  double rs = st.s_above + above_s;
  int best = -1;
  for (int i = per - 1; i >= 0; --i) {
    const int b = t * per + i;
    const unsigned long long cb = rc + hc[b];
    const double sb = rs + (l1 ? hs[b] : 0.0);
    bool ok;
    if (l1) {
      const double L = KT::value((typename KT::K)(st.prefix | ((unsigned long long)b << sh)));
      ok = (sb - (double)cb * L) >= s.tau;
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
    double ss = st.s_above + above_s;
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

// Stage 1: totals, mode, first digit.  Clears the global histogram for the
// refine pass.  The state is worked on in LDS and written back once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sel1(const InstDesc* D, const Counts* cnt, const SelItem* items, Opts o) {
  using KT = KeyT<T>;
  __shared__ uint32_t hc[kNB];
  __shared__ double hs[kNB];
  __shared__ unsigned long long lc[kBlock];
  __shared__ double ls[kBlock];
  __shared__ int lbest;
  __shared__ double lds[lds_sum<2>()];
  __shared__ SelState st;
  if ((int)blockIdx.x >= cnt->nsel) return;
  const SelItem si = items[blockIdx.x];
  const InstDesc& d = D[si.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const int k = (int)S[S_K];
  if (si.src == 1 && !is_check_iter(k, o)) return;
  const SetDesc& s = d.sets[si.set];
  const bool l1 = s.kind == SIP_SET_L1;
  uint32_t* gc = s.hcnt[si.src];
  double* gs = s.hsum[si.src];
  double tot[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < kNB; b += kBlock) {
    hc[b] = gc[b];
    hs[b] = l1 ? gs[b] : 0.0;
    tot[0] += (double)hc[b];
    tot[1] += hs[b];
    gc[b] = 0;
    if (l1) gs[b] = 0.0;
  }
  block_sum<2>(tot, lds);
  if (threadIdx.x == 0) {
    st.prefix = 0; st.c_above = 0; st.s_above = 0.0; st.ncand = 0; st.err = 0; st.need_ties = 0;
    st.theta = 0.0; st.tkey = 0; st.tk = 0.0; st.keep_ties = 0; st.ties = 0; st.digit = 0;
    const int infb = (int)(KT::inf_key >> digit_shift<T>(0));
    unsigned long long nonfinite = 0;
    for (int b = infb; b < kNB; ++b) nonfinite += hc[b];
    if (nonfinite) st.err = SIP_ENUMERIC;
    if (l1) {
      if (!(s.tau > 0.0)) st.mode = SEL_ZERO;
      else if (tot[1] <= s.tau) st.mode = SEL_INSIDE;
      else st.mode = SEL_PROJECT;
    } else {
      st.mode = ((double)s.k >= tot[0]) ? SEL_ALL : SEL_PROJECT;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) { st.final_ = 0; st.compact_next = 0; }
  __syncthreads();
  if (st.mode == SEL_PROJECT && !st.err) {
    const unsigned long long cnt = select_digit<T>(st, hc, hs, kNB, 0, s, l1, lc, ls, &lbest);
    if (threadIdx.x == 0) {
      st.digit = 1;
      st.compact_next = cnt <= kCandCap ? 1 : 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *s.sel[si.src] = st;
}

// Whether refine pass `pass` (0 or 1) appends candidate keys: only if digits
// remain after the one it histograms, and then when the bucket it refines is
// small or on the second pass (the select kernel finishes over them).
template <typename T>
__device__ __forceinline__ bool pass_compacts(const SelState& st, int pass) {
  return st.digit + 1 < KeyT<T>::ndig && (st.compact_next || pass == 1);
}

// Refine pass over all values: histogram of digit st.digit among entries
// whose higher digits match the resolved prefix; when the bucket is small
// (or on the last pass of a long key) their keys go to the candidate list,
// appended with one atomic per block round.
template <typename T>
__global__ __launch_bounds__(kSB) void k_thr_refine(const InstDesc* D, const Counts* cnt, const ThrItem* items, Opts o, int pass) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ uint32_t hc[kNB];
  __shared__ double hs[kNB];
  __shared__ uint32_t wcnt[kSW];
  __shared__ unsigned long long bbase;
  if ((int)blockIdx.x >= cnt->nthr) return;
  const int iti = xcd_item(blockIdx.x, cnt->nthr);
  const ThrItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const int k = (int)S[S_K];
  if (it.src == 1 && !is_check_iter(k, o)) return;
  const SetDesc& s = d.sets[it.set];
  const SelState& st = *s.sel[it.src];
  if (st.mode != SEL_PROJECT || st.err || st.final_) return;
  const int dig = st.digit;
  const bool compact = pass_compacts<T>(st, pass);
  const bool l1 = s.kind == SIP_SET_L1;
  const int nb = 1 << KT::width(dig);
  for (int b = threadIdx.x; b < nb; b += kSB) { hc[b] = 0; hs[b] = 0.0; }
  __syncthreads();
  const int shp = digit_shift<T>(dig - 1), sh = digit_shift<T>(dig);
  const K want = (K)(st.prefix >> shp);
  const Geo g(d);
  const T* __restrict__ x = (const T*)d.x;
  K* __restrict__ cand = (K*)s.cand[it.src];
  unsigned long long* ncand = &s.sel[it.src]->ncand;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int end = it.begin + it.len;
  for (int c = 0; c < s.ncomp; ++c) {
    const int axis = s.axis[c];
    const T* __restrict__ y = (const T*)s.y + (size_t)c * g.N;
    for (int base = it.begin; base < end; base += kSB) {
      const int P = base + (int)threadIdx.x;
      bool hit = false;
      K key = 0;
      if (P < end) {
        int iz, iy, ix;
        g.coords(P, iz, iy, ix);
        T val = 0;
        bool valid;
        if (it.src == 0) {
          valid = comp_valid(axis, iz, iy, ix, g);
          if (valid) val = y[P];
        } else {
          valid = comp_value<T>(x, P, axis, iz, iy, ix, g, d, val);
        }
        if (valid) {
          key = KT::key(val);
          hit = (K)(key >> shp) == want;
        }
      }
      if (hit) {
        const int bkt = (int)((key >> sh) & (K)(nb - 1));
        atomicAdd(&hc[bkt], 1u);
        if (l1) atomicAdd(&hs[bkt], KT::value(key));
      }
      if (compact) {
        // block-aggregated append: wave counts, one atomic for the block
        const unsigned long long mask = __ballot(hit);
        if (lane == 0) wcnt[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
          unsigned long long tot = 0;
          for (int q = 0; q < kSW; ++q) tot += wcnt[q];
          bbase = tot ? atomicAdd(ncand, tot) : 0ull;
        }
        __syncthreads();
        if (hit) {
          unsigned long long off = bbase;
          for (int q = 0; q < wv; ++q) off += wcnt[q];
          const unsigned long long below = mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
          cand[off + __popcll(below)] = key;
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  uint32_t* gc = s.hcnt[it.src];
  double* gs = s.hsum[it.src];
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
__global__ __launch_bounds__(kBlock) void k_sel_next(const InstDesc* D, const Counts* cnt, const SelItem* items, Opts o, int pass) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ uint32_t hc[kNB];
  __shared__ double hs[kNB];
  __shared__ unsigned long long lc[kBlock];
  __shared__ double ls[kBlock];
  __shared__ int lbest;
  __shared__ SelState st;
  if ((int)blockIdx.x >= cnt->nsel) return;
  const SelItem si = items[blockIdx.x];
  const InstDesc& d = D[si.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const int k = (int)S[S_K];
  if (si.src == 1 && !is_check_iter(k, o)) return;
  const SetDesc& s = d.sets[si.set];
  if (threadIdx.x == 0) st = *s.sel[si.src];
  __syncthreads();
  if (st.mode != SEL_PROJECT || st.err || st.final_) return;
  const bool l1 = s.kind == SIP_SET_L1;
  const bool compacted = pass_compacts<T>(st, pass);
  uint32_t* gc = s.hcnt[si.src];
  double* gs = s.hsum[si.src];
  int dig = st.digit;
  int nb = 1 << KT::width(dig);
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    hc[b] = gc[b];
    hs[b] = l1 ? gs[b] : 0.0;
    gc[b] = 0;
    if (l1) gs[b] = 0.0;
  }
  __syncthreads();
  unsigned long long last = select_digit<T>(st, hc, hs, nb, dig, s, l1, lc, ls, &lbest);
  ++dig;
  if (compacted) {
    const K* cand = (const K*)s.cand[si.src];
    const unsigned long long ncand = st.ncand;
    for (; dig < KT::ndig; ++dig) {
      if (st.err) break;
      nb = 1 << KT::width(dig);
      const int shp = digit_shift<T>(dig - 1), sh = digit_shift<T>(dig);
      const K want = (K)(st.prefix >> shp);
      for (int b = threadIdx.x; b < nb; b += kBlock) { hc[b] = 0; hs[b] = 0.0; }
      __syncthreads();
      for (unsigned long long i = threadIdx.x; i < ncand; i += kBlock) {
        const K key = cand[i];
        if ((K)(key >> shp) == want) {
          const int bkt = (int)((key >> sh) & (K)(nb - 1));
          atomicAdd(&hc[bkt], 1u);
          if (l1) atomicAdd(&hs[bkt], KT::value(key));
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
  if (threadIdx.x == 0) *s.sel[si.src] = st;
}

// Cardinality ties straddling the cut: count entries equal to the k-th
// magnitude per (item, component) so the apply pass can rank them by index.
template <typename T>
__global__ __launch_bounds__(kSB) void k_card_ties(const InstDesc* D, const Counts* cnt, const ThrItem* items, Opts o,
                                                      uint32_t* tie_part) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ uint32_t tcnt[3];
  if ((int)blockIdx.x >= cnt->nthr) return;
  const int iti = xcd_item(blockIdx.x, cnt->nthr);
  const ThrItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  if (it.src != 0) return;
  const SetDesc& s = d.sets[it.set];
  if (s.kind != SIP_SET_CARD) return;
  const SelState& st = *s.sel[0];
  if (st.mode != SEL_PROJECT || st.err || !st.need_ties) return;
  if (threadIdx.x < 3) tcnt[threadIdx.x] = 0;
  __syncthreads();
  const Geo g(d);
  const K tkey = (K)st.tkey;
  const int end = it.begin + it.len;
  for (int c = 0; c < s.ncomp; ++c) {
    const T* y = (const T*)s.y + (size_t)c * g.N;
    uint32_t local = 0;
    for (int P = it.begin + (int)threadIdx.x; P < end; P += kSB) {
      int iz, iy, ix;
      g.coords(P, iz, iy, ix);
      if (!comp_valid(s.axis[c], iz, iy, ix, g)) continue;
      if (KT::key(y[P]) == tkey) ++local;
    }
    if (local) atomicAdd(&tcnt[c], local);
  }
  __syncthreads();
  if (threadIdx.x < 3) tie_part[(size_t)iti * 3 + threadIdx.x] = tcnt[threadIdx.x];
}

// Apply pass.  Pipeline 0: y = soft threshold of w (l1) or w on the kept
// support (cardinality); v = rho (y - w), which equals v + rho (y - x-bar);
// adapt dots of the (dg, dv) pair and the new y/v snapshots.  Pipeline 1:
// the feasibility distance ||s - P(s)||^2.
template <typename T>
__global__ __launch_bounds__(kSB) void k_thr_apply(const InstDesc* D, const Counts* cnt, const ThrItem* items, Opts o, double* parts,
                                                      const uint32_t* tie_part) {
  using KT = KeyT<T>;
  using K = typename KT::K;
  __shared__ double lds[lds_sum<8, kSB>()];
  __shared__ uint32_t wsum[kSW];
  __shared__ unsigned long long tie_base[3];
  if ((int)blockIdx.x >= cnt->nthr) return;
  const int iti = xcd_item(blockIdx.x, cnt->nthr);
  const ThrItem it = items[iti];
  const InstDesc& d = D[it.inst];
  const double* S = d.scal;
  if (!inst_live(S)) return;
  const int k = (int)S[S_K];
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  if (it.src == 1 && !check) return;
  const bool have = S[S_HAVE_SNAP] != 0.0;
  const SetDesc& s = d.sets[it.set];
  const SelState& st = *s.sel[it.src];
  if (st.err) return;
  const bool l1 = s.kind == SIP_SET_L1;
  const int mode = st.mode;
  const Geo g(d);
  const T* x = (const T*)d.x;
  const double rho_d = S[S_RHO + it.set];
  const T rho = (T)rho_d;
  const T theta = (T)st.theta;
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
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int end = it.begin + it.len;
  for (int c = 0; c < s.ncomp; ++c) {
    const int axis = s.axis[c];
    const size_t off = (size_t)c * g.N;
    T* y = (T*)s.y + off;
    T* v = (T*)s.v + off;
    T* y0 = (T*)s.y0 + off;
    T* v0 = (T*)s.v0 + off;
    unsigned long long run = rank_ties ? tie_base[c] : 0ull;
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
          double e2;
          const double a = fabs((double)sv);
          if (l1) {
            if (mode == SEL_PROJECT) { const double mn = a < st.theta ? a : st.theta; e2 = mn * mn; }
            else if (mode == SEL_ZERO) e2 = a * a;
            else e2 = 0.0;
          } else {
            if (mode == SEL_PROJECT) {
              const K key = KT::key(sv);
              e2 = key < tkey ? a * a : 0.0;
            } else e2 = 0.0;
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
          const double dg = -((double)yn - (double)y0[P]);
          const double dv = (double)vn - (double)v0[P];
          acc[3] += dg * dv; acc[4] += dg * dg; acc[5] += dv * dv;
        }
        y0[P] = yn;
        v0[P] = vn;
      }
    }
  }
  block_sum<8, kSB>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) parts[(size_t)iti * kThrParts + q] = acc[q];
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
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finish(const InstDesc* D, const Counts* cnt, const int32_t* insts, Opts o,
                                                   const double* proj_parts, const double* thrw_parts,
                                                   const double* thra_parts) {
  __shared__ double lds[lds_sum<8>()];
  __shared__ double dots[kMaxUnits][8];
  __shared__ double evol[16];
  if ((int)blockIdx.x >= cnt->ninst) return;
  const InstDesc& d = D[insts[blockIdx.x]];
  double* S = d.scal;
  if (S[S_STATE] != 0.0) return;
  if (S[S_ERR] != 0.0) {
    if (threadIdx.x == 0) S[S_STATE] = 3.0;
    return;
  }
  const int k = (int)S[S_K];
  const bool adapt = is_adapt_iter(k, o);
  const bool check = is_check_iter(k, o);
  const int p = d.nsets;
  int err = 0;
  if (adapt || check) {
    for (int u = 0; u <= p; ++u) {
      const bool thr = u < p && d.sets[u].thr >= 0;
      double v[8];
      if (!thr) {
        reduce_range<8>(proj_parts, d.sp_begin, d.sp_end, kProjParts, u * kUnitParts, v, lds);
      } else {
        const SetDesc& s = d.sets[u];
        double a[8], b[8];
        reduce_range<8>(thrw_parts, s.item_begin[0], s.item_end[0], kThrParts, 0, a, lds);
        reduce_range<8>(thra_parts, s.item_begin[0], s.item_end[0], kThrParts, 0, b, lds);
        for (int j = 0; j < 3; ++j) { v[j] = a[j]; v[3 + j] = b[3 + j]; }
        v[6] = v[7] = 0.0;
        if (check) {
          reduce_range<8>(thrw_parts, s.item_begin[1], s.item_end[1], kThrParts, 0, a, lds);
          reduce_range<8>(thra_parts, s.item_begin[1], s.item_end[1], kThrParts, 0, b, lds);
          v[6] = b[6];
          v[7] = a[7];
        }
      }
      if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) dots[u][j] = v[j];
      }
    }
  }
  if (threadIdx.x == 0) {
    for (int u = 0; u < p; ++u) {
      if (d.sets[u].thr < 0) continue;
      if (d.sets[u].sel[0]->err) err = d.sets[u].sel[0]->err;
      if (check && d.sets[u].sel[1]->err) err = d.sets[u].sel[1]->err;
    }
  }
  if (check && d.ring) {
    double v[8], w[8];
    reduce_range<8>(proj_parts, d.sp_begin, d.sp_end, kProjParts, kEvolOff, v, lds);
    reduce_range<8>(proj_parts, d.sp_begin, d.sp_end, kProjParts, kEvolOff + 8, w, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) { evol[j] = v[j]; evol[8 + j] = w[j]; }
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (err) { S[S_ERR] = (double)err; S[S_STATE] = 3.0; return; }
  if (d.log && k <= d.log_cap) {
    double* row = d.log + (size_t)(k - 1) * 2 * kMaxUnits;
    for (int u = 0; u <= p; ++u) { row[u] = S[S_RHO + u]; row[kMaxUnits + u] = S[S_GAMMA + u]; }
  }
  if (check) {
    bool feas = true;
    for (int u = 0; u < p; ++u) {
      double num = dots[u][6];
      const double den = dots[u][7];
      const SetDesc& s = d.sets[u];
      if (s.thr >= 0 && s.kind == SIP_SET_CARD && s.sel[1]->mode == SEL_PROJECT) {
        // the dropped entries equal to the k-th magnitude all have that magnitude
        const SelState& q = *s.sel[1];
        num += (double)(q.ties - q.keep_ties) * q.tk * q.tk;
      }
      double rf;
      if (den > 0.0) rf = sqrt(num) / sqrt(den);
      else rf = (num > 0.0) ? INFINITY : 0.0;
      S[S_RFEAS + u] = rf;
      if (!(rf < o.eps_feas)) feas = false;
    }
    double worst = 0.0;
    for (int j = 1; j <= o.evol_hist; ++j) worst = evol[j] > worst ? evol[j] : worst;
    const double xn = evol[0];
    double re;
    if (xn > 0.0) re = sqrt(worst) / sqrt(xn);
    else re = worst > 0.0 ? INFINITY : 0.0;
    S[S_REVOL] = re;
    if (re < o.eps_evol && feas) {
      S[S_STATE] = 1.0;
      S[S_ITERS] = (double)k;
      return;
    }
  }
  if (adapt) {
    if (S[S_HAVE_SNAP] != 0.0) {
      double rho[kMaxUnits], gam[kMaxUnits];
      for (int u = 0; u <= p; ++u) {
        double a = 0.0, b = 0.0;
        const bool oa = spectral(dots[u][0], dots[u][1], dots[u][2], o.eps_corr, a);
        const bool ob = spectral(dots[u][3], dots[u][4], dots[u][5], o.eps_corr, b);
        if (oa && ob) { const double gm = sqrt(a * b); rho[u] = gm; gam[u] = 1.0 + 2.0 * gm / (a + b); }
        else if (oa) { rho[u] = a; gam[u] = 1.9; }
        else if (ob) { rho[u] = b; gam[u] = 1.1; }
        else { rho[u] = S[S_RHO + u]; gam[u] = 1.5; }
        if (gam[u] > o.gamma_max) gam[u] = o.gamma_max;
      }
      const double rl = rho[p];
      for (int u = 0; u < p; ++u) {
        const double lo = rl / o.rho_ratio_max, hi = rl * o.rho_ratio_max;
        rho[u] = rho[u] < lo ? lo : (rho[u] > hi ? hi : rho[u]);
      }
      for (int u = 0; u <= p; ++u) { S[S_RHO + u] = rho[u]; S[S_GAMMA + u] = gam[u]; }
    }
    S[S_HAVE_SNAP] = 1.0;
    double c0 = S[S_RHO + p], ca[3] = {0.0, 0.0, 0.0};
    for (int u = 0; u < p; ++u) {
      const SetDesc& s = d.sets[u];
      if (s.op == SIP_OP_I) c0 += S[S_RHO + u];
      else for (int c = 0; c < s.ncomp; ++c) ca[s.axis[c]] += S[S_RHO + u];
    }
    S[S_C0] = c0;
    for (int a = 0; a < 3; ++a) S[S_CAX + a] = ca[a] * d.h2inv[a];
  }
  S[S_ITERS] = (double)k;
  S[S_K] = (double)(k + 1);
  if (k + 1 > o.max_iter) S[S_STATE] = 2.0;
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
void launch_init(hipStream_t st, const InstDesc* D, int inst, int64_t N) {
  const int64_t nb = (N + kBlock - 1) / kBlock;
  k_init<T><<<(int)(nb < 2048 ? nb : 2048), kBlock, 0, st>>>(D, inst);
}

template <typename T>
void launch_iteration(hipStream_t st, const Tables& t, const Opts& o) {
  if (t.npt > 0) {
    k_rhs<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, t.rr_part);
    for (int j = 0; j < o.cg_max; ++j) {
      k_cg_dir<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, j, t.rr_part, t.pq_part, o);
      k_cg_upd<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, j, t.pq_part, t.rr_part);
    }
    if (t.nsp) k_proj<T><<<t.nsp, kSB, 0, st>>>(t.D, t.cnt, t.sp, o, t.proj_part);
  }
  if (t.nthr > 0) {
    k_thr_w<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, t.thrw_part);
    k_sel1<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.cnt, t.sel, o);
    k_thr_refine<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, 0);
    k_sel_next<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.cnt, t.sel, o, 0);
    k_thr_refine<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, 1);
    k_sel_next<T><<<t.nsel, kBlock, 0, st>>>(t.D, t.cnt, t.sel, o, 1);
    if (t.any_card) k_card_ties<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, t.tie_part);
    k_thr_apply<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, t.thra_part, t.tie_part);
  }
  if (t.ninst > 0)
    k_finish<T><<<t.ninst, kBlock, 0, st>>>(t.D, t.cnt, t.inst, o, t.proj_part, t.thrw_part, t.thra_part);
}

// One kernel of the iteration on its own (timing); CG kernels use step 1.
template <typename T>
void launch_phase(hipStream_t st, const Tables& t, const Opts& o, int phase) {
  switch (phase) {
    case 0: if (t.npt) k_rhs<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, t.rr_part); break;
    case 1: if (t.npt) k_cg_dir<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, 1, t.rr_part, t.pq_part, o); break;
    case 2: if (t.npt) k_cg_upd<T><<<t.npt, kPB, 0, st>>>(t.D, t.cnt, t.pt, 1, t.pq_part, t.rr_part); break;
    case 3: if (t.nsp) k_proj<T><<<t.nsp, kSB, 0, st>>>(t.D, t.cnt, t.sp, o, t.proj_part); break;
    case 4: if (t.nthr) k_thr_w<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, t.thrw_part); break;
    case 5: if (t.nthr) k_thr_apply<T><<<t.nthr, kSB, 0, st>>>(t.D, t.cnt, t.thr, o, t.thra_part, t.tie_part); break;
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

}  // namespace sip
