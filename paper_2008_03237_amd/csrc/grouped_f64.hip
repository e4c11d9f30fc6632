// FP64 instantiation of the persistent grouped kernel.
#include "grouped_impl.h"

namespace dlpno {

hipError_t launch_grouped_f64(const GroupedArgs<double>& a, int kind, int workers, hipStream_t s) {
  if (kind == ITEM_LADDER) hipLaunchKernelGGL((grouped_kernel<double, ITEM_LADDER>), dim3(workers), dim3(256), 0, s, a);
  else if (kind == ITEM_LADDER2) hipLaunchKernelGGL((grouped_kernel<double, ITEM_LADDER2>), dim3(2 * workers), dim3(256), 0, s, a);
  else if (kind == ITEM_LADDER4) hipLaunchKernelGGL((grouped_coop_kernel<double>), dim3(2 * workers), dim3(256), 0, s, a);
  else if (kind == ITEM_PROJ2) hipLaunchKernelGGL((grouped_kernel<double, ITEM_PROJ2>), dim3(2 * workers), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((grouped_kernel<double, ITEM_PROJ>), dim3(workers), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace dlpno
