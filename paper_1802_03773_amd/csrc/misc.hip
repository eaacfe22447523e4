// Small utility kernels of libqrkit.so.
#include "qrk_device.hpp"
#include "qrk_host.hpp"

namespace qrk {

// Clear or set a few ints with a kernel (not hipMemsetAsync, so the call can sit inside a
// captured HIP graph).
__global__ void k_fill_int(int* ptr, int value) {
  if (threadIdx.x < 4) ptr[threadIdx.x] = value;
}

hipError_t launch_fill_int(int* ptr, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, ptr, value);
  return hipGetLastError();
}

}  // namespace qrk
