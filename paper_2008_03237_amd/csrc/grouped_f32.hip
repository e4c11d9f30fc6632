// FP32 instantiation of the persistent grouped kernel.
#include "grouped_impl.h"

namespace dlpno {

hipError_t launch_grouped_f32(const GroupedArgs<float>& a, int kind, int workers, hipStream_t s) {
  if (kind == ITEM_LADDER) hipLaunchKernelGGL((grouped_kernel<float, ITEM_LADDER>), dim3(workers), dim3(256), 0, s, a);
  else if (kind == ITEM_PROJ) hipLaunchKernelGGL((grouped_kernel<float, ITEM_PROJ>), dim3(workers), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;   // the two-wave ladder launches are FP64 only
  return hipGetLastError();
}

}  // namespace dlpno
