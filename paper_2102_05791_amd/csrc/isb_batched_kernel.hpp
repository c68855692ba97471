// The batched persistent kernel and the lookup of its compiled variants. The variants of each
// dimension are instantiated in a source file of their own (isb_batched_k2.hip, isb_batched_k3.hip),
// so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "isb_body.hpp"

namespace isb {

// MODE 0: step, 1: adjoint. LB is the launch bound: 1024-thread workgroups get at most 128 VGPRs,
// 768-thread ones 168 and 512-thread ones 256 (one workgroup per CU in every case). CR: the compact
// rest record (DevMesh::axis >= 0).
template <int D, typename T, int MODE, int LB, int EM = EM_NH, bool CR = false>
__global__ void __launch_bounds__(LB) k_batched(DevMesh m, DevScene sc, BatchArgs A) {
  extern __shared__ double smem[];
  batched_body<D, T, MODE, EM, CR>(m, sc, A, smem, (int)blockIdx.x);
}

// The default workgroup size of each dimension; the alternative energy models come in it only.
inline int batched_default_block(int dim) { return dim == 2 ? 768 : 512; }

// The host stub of the variant for (precision, mode, workgroup size, energy model, compact record),
// or nullptr when that variant is not compiled (an alternative model at another workgroup size).
void* batched_kernel_2d(int precision, int mode, int block, int model, bool compact);
void* batched_kernel_3d(int precision, int mode, int block, int model, bool compact);

template <typename T>
struct TypeTag {
  using type = T;
};

// Body of those lookups, instantiated for one dimension.
template <int D>
void* batched_kernel_dim(int precision, int mode, int block, int model, bool compact) {
  constexpr int DB = D == 2 ? 768 : 512;
  auto pick = [&](auto t, auto lb, auto em) -> void* {
    using T = typename decltype(t)::type;
    constexpr int LB = decltype(lb)::value;
    constexpr int EM = decltype(em)::value;
    if (mode == 0)
      return compact ? reinterpret_cast<void*>(&k_batched<D, T, 0, LB, EM, true>)
                     : reinterpret_cast<void*>(&k_batched<D, T, 0, LB, EM, false>);
    return compact ? reinterpret_cast<void*>(&k_batched<D, T, 1, LB, EM, true>)
                   : reinterpret_cast<void*>(&k_batched<D, T, 1, LB, EM, false>);
  };
  auto by_type = [&](auto lb, auto em) -> void* {
    if (precision) return pick(TypeTag<float>{}, lb, em);
    return pick(TypeTag<double>{}, lb, em);
  };
  if (model != EM_NH) {
    if (block != DB) return nullptr;
    if (model == EM_STVK) return by_type(std::integral_constant<int, DB>{}, std::integral_constant<int, EM_STVK>{});
    if (model == EM_COROT) return by_type(std::integral_constant<int, DB>{}, std::integral_constant<int, EM_COROT>{});
    return by_type(std::integral_constant<int, DB>{}, std::integral_constant<int, EM_SNH>{});
  }
  constexpr auto nh = std::integral_constant<int, EM_NH>{};
  if (block > 768) return by_type(std::integral_constant<int, 1024>{}, nh);
  if (block > 512) return by_type(std::integral_constant<int, 768>{}, nh);
  return by_type(std::integral_constant<int, 512>{}, nh);
}

}  // namespace isb
