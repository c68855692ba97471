// Runs the batched solver's body logic (isb_body.hpp) on the CPU: one workgroup of `block`
// host threads pulls every body from the work queue. Test infrastructure only.
#include <hip/hip_runtime.h>

#include <thread>

#include "isb_body.hpp"

thread_local isb_emu_dim3 threadIdx;
isb_emu_dim3 blockDim, blockIdx, gridDim;
isb_emu::Workgroup* isb_emu::g_wg = nullptr;

template <int D, typename T, int MODE>
static void run(int block, const isb::DevMesh* m, const isb::DevScene* sc, const isb::BatchArgs* A) {
  isb_emu::Workgroup wg;
  std::barrier<> all(block);
  std::vector<std::barrier<>*> waves;
  for (int w = 0; w < block / 64; ++w) waves.push_back(new std::barrier<>(64));
  wg.all = &all;
  wg.waves = waves;
  wg.buf.assign(block, 0.0);
  isb_emu::g_wg = &wg;
  blockDim.x = block;
  gridDim.x = 1;
  std::vector<double> smem(isb::kRedSlots + 2 * (size_t)A->nacc, -12345.0);
  std::vector<std::thread> th;
  for (int t = 0; t < block; ++t)
    th.emplace_back([&, t]() {
      threadIdx.x = t;
      isb::batched_body<D, T, MODE>(*m, *sc, *A, smem.data(), 0, 1);
    });
  for (auto& x : th) x.join();
  for (auto* b : waves) delete b;
}

extern "C" int emu_batched(int dim, int precision, int mode, int block, const isb::DevMesh* m,
                           const isb::DevScene* sc, const isb::BatchArgs* A) {
  if (block % 64 || block < 64 || block > 1024) return 1;
  if (dim == 2) {
    if (precision)
      mode ? run<2, float, 1>(block, m, sc, A) : run<2, float, 0>(block, m, sc, A);
    else
      mode ? run<2, double, 1>(block, m, sc, A) : run<2, double, 0>(block, m, sc, A);
  } else {
    if (precision)
      mode ? run<3, float, 1>(block, m, sc, A) : run<3, float, 0>(block, m, sc, A);
    else
      mode ? run<3, double, 1>(block, m, sc, A) : run<3, double, 0>(block, m, sc, A);
  }
  return 0;
}

extern "C" int emu_sizes(int* out) {
  out[0] = (int)sizeof(isb::DevMesh);
  out[1] = (int)sizeof(isb::DevScene);
  out[2] = (int)sizeof(isb::BatchArgs);
  out[3] = (int)sizeof(isb::DevStats);
  return 0;
}
