// The batched persistent kernel's variants for tetrahedra (see isb_batched_kernel.hpp).
#include "isb_batched_kernel.hpp"

namespace isb {

void* batched_kernel_3d(int precision, int mode, int block, int model, bool compact) {
  return batched_kernel_dim<3>(precision, mode, block, model, compact);
}

}  // namespace isb
