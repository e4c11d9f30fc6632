// FP32 instantiation of the persistent grouped kernel.
#include "grouped_impl.h"

namespace dlpno {

hipError_t launch_grouped_f32(const GroupedArgs<float>& a, int workers, hipStream_t s) {
  hipLaunchKernelGGL(grouped_kernel<float>, dim3(workers), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dlpno
