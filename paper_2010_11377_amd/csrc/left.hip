// Small kernels of the left-preconditioned GMRES driver.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

// y[j] *= scale[j] (the basis columns are stored unnormalised).
__global__ void __launch_bounds__(256) k_scale_by(double *__restrict__ y,
                                                  const double *__restrict__ scale, int k) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) y[j] *= scale[j];
}

}  // namespace

namespace kern {

void scale_by(double *y, const double *scale, int k, hipStream_t st) {
  k_scale_by<<<1, 256, 0, st>>>(y, scale, k);
}

}  // namespace kern
}  // namespace irk
