// Level transfer kernels of multilevel PARSDMM (ML-PARSDMM listing): the
// coarse model by an anti-alias filter and subsampling, and the interpolation
// of x, y_i, v_i "as images" to the next finer grid.  They run once per level
// change, outside the iteration.
//
// Grids are in internal form (n0, n1, n2) = (z, y, x), x contiguous; a 2D
// grid has n1 = 1.  A level keeps samples 0, 2, 4, ... of each axis.
#include <hip/hip_runtime.h>

#include "sip_internal.h"

namespace sip {
namespace {

constexpr int kLvBlock = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// dst (c0 x c1 x c2) = every other sample of src (n0 x n1 x n2) after the
// binomial [1, 2, 1] / 4 filter along each axis with replicated edges.
template <typename T>
__global__ __launch_bounds__(kLvBlock) void k_restrict(const T* __restrict__ src, int n0, int n1, int n2,
                                                       T* __restrict__ dst, int c0, int c1, int c2) {
  const int64_t Nc = (int64_t)c0 * c1 * c2;
  for (int64_t q = blockIdx.x * (int64_t)kLvBlock + threadIdx.x; q < Nc; q += (int64_t)gridDim.x * kLvBlock) {
    const int jx = (int)(q % c2);
    const int64_t r = q / c2;
    const int jy = (int)(r % c1);
    const int jz = (int)(r / c1);
    double acc = 0.0;
    for (int dz = -1; dz <= 1; ++dz) {
      const int iz = clampi(2 * jz + dz, 0, n0 - 1);
      const double wz = dz == 0 ? 0.5 : 0.25;
      for (int dy = -1; dy <= 1; ++dy) {
        const int iy = clampi(2 * jy + dy, 0, n1 - 1);
        const double wy = dy == 0 ? 0.5 : 0.25;
        const int64_t row = ((int64_t)iz * n1 + iy) * n2;
        for (int dx = -1; dx <= 1; ++dx) {
          const int ix = clampi(2 * jx + dx, 0, n2 - 1);
          const double wx = dx == 0 ? 0.5 : 0.25;
          acc += wz * wy * wx * (double)src[row + ix];
        }
      }
    }
    dst[q] = (T)acc;
  }
}

// Coordinate on the coarse image of fine index i along one axis: points sit
// at i / 2; rows of a forward difference along this axis sit at
// (i + 1/2) / 2 - 1/2.  Clamped to the image.
__device__ __forceinline__ void coarse_coord(int i, bool stag, int ns, int& i0, int& i1, double& t) {
  const double off = stag ? 0.5 : 0.0;
  double c = (i + off) * 0.5 - off;
  c = c < 0.0 ? 0.0 : (c > ns - 1.0 ? ns - 1.0 : c);
  i0 = (int)c;
  i1 = i0 + 1 < ns ? i0 + 1 : ns - 1;
  t = c - i0;
}

// One image from a coarse grid to a fine one, linear along each axis.  The
// destination is walked over its full dims (f0, f1, f2) with strides
// (dsz, dsy, 1); points outside its image dims (d0, d1, d2) (the unused last
// layer of a difference component) are set to 0.  The source image has dims
// (s0, s1, s2) and strides (ssz, ssy, 1).  stag: the axis of the difference,
// -1 for a point field.
template <typename T>
__global__ __launch_bounds__(kLvBlock) void k_prolong(const T* __restrict__ src, int s0, int s1, int s2, int64_t ssz,
                                                      int64_t ssy, T* __restrict__ dst, int f0, int f1, int f2,
                                                      int d0, int d1, int d2, int64_t dsz, int64_t dsy, int stag) {
  const int64_t Nf = (int64_t)f0 * f1 * f2;
  for (int64_t q = blockIdx.x * (int64_t)kLvBlock + threadIdx.x; q < Nf; q += (int64_t)gridDim.x * kLvBlock) {
    const int ix = (int)(q % f2);
    const int64_t r = q / f2;
    const int iy = (int)(r % f1);
    const int iz = (int)(r / f1);
    T* out = dst + (int64_t)iz * dsz + (int64_t)iy * dsy + ix;
    if (iz >= d0 || iy >= d1 || ix >= d2) {
      *out = (T)0;
      continue;
    }
    int z0, z1, y0, y1, x0, x1;
    double tz, ty, tx;
    coarse_coord(iz, stag == 0, s0, z0, z1, tz);
    coarse_coord(iy, stag == 1, s1, y0, y1, ty);
    coarse_coord(ix, stag == 2, s2, x0, x1, tx);
    auto at = [&](int z, int y, int x) -> double { return (double)src[(int64_t)z * ssz + (int64_t)y * ssy + x]; };
    const double v00 = (1.0 - tx) * at(z0, y0, x0) + tx * at(z0, y0, x1);
    const double v01 = (1.0 - tx) * at(z0, y1, x0) + tx * at(z0, y1, x1);
    const double v10 = (1.0 - tx) * at(z1, y0, x0) + tx * at(z1, y0, x1);
    const double v11 = (1.0 - tx) * at(z1, y1, x0) + tx * at(z1, y1, x1);
    const double v0 = (1.0 - ty) * v00 + ty * v01;
    const double v1 = (1.0 - ty) * v10 + ty * v11;
    *out = (T)((1.0 - tz) * v0 + tz * v1);
  }
}

inline int grid_blocks(int64_t n) {
  const int64_t b = (n + kLvBlock - 1) / kLvBlock;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

template <typename T>
void launch_restrict(hipStream_t st, const T* src, const int64_t (&n)[3], T* dst, const int64_t (&c)[3]) {
  k_restrict<T><<<grid_blocks(c[0] * c[1] * c[2]), kLvBlock, 0, st>>>(src, (int)n[0], (int)n[1], (int)n[2], dst,
                                                                        (int)c[0], (int)c[1], (int)c[2]);
}

template <typename T>
void launch_prolong(hipStream_t st, const T* src, const int64_t (&s)[3], int64_t ssz, int64_t ssy, T* dst,
                    const int64_t (&f)[3], const int64_t (&d)[3], int64_t dsz, int64_t dsy, int stag) {
  k_prolong<T><<<grid_blocks(f[0] * f[1] * f[2]), kLvBlock, 0, st>>>(
      src, (int)s[0], (int)s[1], (int)s[2], ssz, ssy, dst, (int)f[0], (int)f[1], (int)f[2], (int)d[0], (int)d[1],
      (int)d[2], dsz, dsy, stag);
}

template void launch_restrict<float>(hipStream_t, const float*, const int64_t (&)[3], float*, const int64_t (&)[3]);
template void launch_restrict<double>(hipStream_t, const double*, const int64_t (&)[3], double*,
                                      const int64_t (&)[3]);
template void launch_prolong<float>(hipStream_t, const float*, const int64_t (&)[3], int64_t, int64_t, float*,
                                    const int64_t (&)[3], const int64_t (&)[3], int64_t, int64_t, int);
template void launch_prolong<double>(hipStream_t, const double*, const int64_t (&)[3], int64_t, int64_t, double*,
                                     const int64_t (&)[3], const int64_t (&)[3], int64_t, int64_t, int);

}  // namespace sip
