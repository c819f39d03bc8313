// Parallel Dykstra (Appendix A, the Parallel-DYKSTRA listing), steps 2 and 3
// on the device: the weighted average of the p projections and the update of
// the p auxiliary vectors.  The projections themselves (step 1) are
// single-set PARSDMM instances of one batch.
#include <hip/hip_runtime.h>

#include "sip_internal.h"

namespace sip {
namespace {

constexpr int kDykBlock = 256;

struct DykArgs {
  const void* y[SIP_MAX_SETS];
  void* v[SIP_MAX_SETS];
  double w[SIP_MAX_SETS];
};

// x = sum_i w_i y_i (accumulated in double, in set order); v_i = x + v_i - y_i.
template <typename T>
__global__ __launch_bounds__(kDykBlock) void k_dykstra(DykArgs a, int p, T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kDykBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDykBlock) {
    double acc = 0.0;
    for (int j = 0; j < p; ++j) acc += a.w[j] * (double)((const T*)a.y[j])[i];
    const T xv = (T)acc;
    x[i] = xv;
    for (int j = 0; j < p; ++j) {
      T* vj = (T*)a.v[j];
      vj[i] = xv + vj[i] - ((const T*)a.y[j])[i];
    }
  }
}

}  // namespace

int32_t launch_dykstra(hipStream_t st, int p, const void* const* y, void* const* v, const double* w, void* x,
                       int64_t n, bool f64) {
  DykArgs a{};
  for (int j = 0; j < p; ++j) { a.y[j] = y[j]; a.v[j] = v[j]; a.w[j] = w[j]; }
  int64_t nb = (n + kDykBlock - 1) / kDykBlock;
  const int grid = (int)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096);
  if (f64) k_dykstra<double><<<grid, kDykBlock, 0, st>>>(a, p, (double*)x, n);
  else k_dykstra<float><<<grid, kDykBlock, 0, st>>>(a, p, (float*)x, n);
  return hipGetLastError() == hipSuccess ? SIP_OK : SIP_EHIP;
}

}  // namespace sip
