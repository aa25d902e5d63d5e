// Launcher of the batched FRAM kernel (batch_device.h).
#include "batch_device.h"

namespace fram {
hipError_t launch_fram_batch(Elem e, const BatchArgs& a, int grid, hipStream_t s) {
  switch (e) {
    case Elem::BF16:
      fram_batch_kernel<Elem::BF16><<<grid, kBT, 0, s>>>(a);
      break;
    case Elem::F16:
      fram_batch_kernel<Elem::F16><<<grid, kBT, 0, s>>>(a);
      break;
    case Elem::F32:
      fram_batch_kernel<Elem::F32><<<grid, kBT, 0, s>>>(a);
      break;
  }
  return hipGetLastError();
}

}  // namespace fram
