// Runs the batched solver's body logic (isb_body.hpp) on the CPU: one workgroup of `block`
// host threads solves every body, largest first. Built with ISB_DEBUG: the body logic's index
// checks are active (emu_debug_site). The emulated LDS starts filled with
// `lds_fill`, standing in for whatever an earlier kernel left there; the largest |value| left in
// its two accumulators afterwards is returned in *lds_left. Test infrastructure only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <thread>

#include "isb_body.hpp"

thread_local isb_emu_dim3 threadIdx;
isb_emu_dim3 blockDim, blockIdx, gridDim;
isb_emu::Workgroup* isb_emu::g_wg = nullptr;
thread_local unsigned isb_emu::wave_phase = 0;

template <int D, typename T, int MODE>
static void run(int block, const isb::DevMesh* m, const isb::DevScene* sc, const isb::BatchArgs* A, double lds_fill,
                double* lds_left) {
  isb_emu::Workgroup wg;
  std::barrier<> all(block);
  std::vector<std::barrier<>*> waves;
  for (int w = 0; w < block / 64; ++w) waves.push_back(new std::barrier<>(64));
  wg.all = &all;
  wg.waves = waves;
  wg.buf.assign(2 * block, 0.0);
  wg.ibuf.assign(2 * block, 0);
  isb_emu::g_wg = &wg;
  blockDim.x = block;
  gridDim.x = 1;
  std::vector<double> smem(isb::kRedSlots + 2 * (size_t)A->nacc, lds_fill);
  std::vector<std::thread> th;
  for (int t = 0; t < block; ++t)
    th.emplace_back([&, t]() {
      threadIdx.x = t;
      isb_emu::wave_phase = 0;
      // the compact rest record when the mesh has one (DevMesh::axis), as the library's launch does
      const bool cr = m->axis >= 0;
      switch (m->model) {
        case isb::EM_STVK:
          cr ? isb::batched_body<D, T, MODE, isb::EM_STVK, true>(*m, *sc, *A, smem.data(), 0)
             : isb::batched_body<D, T, MODE, isb::EM_STVK, false>(*m, *sc, *A, smem.data(), 0);
          break;
        case isb::EM_COROT:
          cr ? isb::batched_body<D, T, MODE, isb::EM_COROT, true>(*m, *sc, *A, smem.data(), 0)
             : isb::batched_body<D, T, MODE, isb::EM_COROT, false>(*m, *sc, *A, smem.data(), 0);
          break;
        case isb::EM_SNH:
          cr ? isb::batched_body<D, T, MODE, isb::EM_SNH, true>(*m, *sc, *A, smem.data(), 0)
             : isb::batched_body<D, T, MODE, isb::EM_SNH, false>(*m, *sc, *A, smem.data(), 0);
          break;
        default:
          cr ? isb::batched_body<D, T, MODE, isb::EM_NH, true>(*m, *sc, *A, smem.data(), 0)
             : isb::batched_body<D, T, MODE, isb::EM_NH, false>(*m, *sc, *A, smem.data(), 0);
          break;
      }
    });
  for (auto& x : th) x.join();
  for (auto* b : waves) delete b;
  double left = 0.0;
  for (size_t i = isb::kRedSlots; i < smem.size(); ++i) left = std::max(left, std::fabs(smem[i]));
  *lds_left = left;
}

extern "C" int emu_batched(int dim, int precision, int mode, int block, const isb::DevMesh* m,
                           const isb::DevScene* sc, const isb::BatchArgs* A, double lds_fill,
                           double* lds_left) {
  if (block % 64 || block < 64 || block > 1024) return 1;
  if (dim == 2) {
    if (precision)
      mode ? run<2, float, 1>(block, m, sc, A, lds_fill, lds_left) : run<2, float, 0>(block, m, sc, A, lds_fill, lds_left);
    else
      mode ? run<2, double, 1>(block, m, sc, A, lds_fill, lds_left) : run<2, double, 0>(block, m, sc, A, lds_fill, lds_left);
  } else {
    if (precision)
      mode ? run<3, float, 1>(block, m, sc, A, lds_fill, lds_left) : run<3, float, 0>(block, m, sc, A, lds_fill, lds_left);
    else
      mode ? run<3, double, 1>(block, m, sc, A, lds_fill, lds_left) : run<3, double, 0>(block, m, sc, A, lds_fill, lds_left);
  }
  return 0;
}

// the debug build's index checks (ISB_DEBUG, which this emulator is always built with): the number of
// the last check that saw an index out of range, 0 if none; reset clears it
extern "C" int emu_debug_site(int reset) {
  const int site = __atomic_load_n(&isb::g_isb_debug_site, __ATOMIC_RELAXED);
  if (reset) __atomic_store_n(&isb::g_isb_debug_site, 0, __ATOMIC_RELAXED);
  return site;
}

extern "C" int emu_sizes(int* out) {
  out[0] = (int)sizeof(isb::DevMesh);
  out[1] = (int)sizeof(isb::DevScene);
  out[2] = (int)sizeof(isb::BatchArgs);
  out[3] = (int)sizeof(isb::DevStats);
  return 0;
}

// byte offsets of BatchArgs' fields in declaration order, checked against the ctypes mirror
extern "C" int emu_batchargs_offsets(int* out) {
  int k = 0;
#define ISB_EMU_OFF(f) out[k++] = (int)offsetof(isb::BatchArgs, f)
  ISB_EMU_OFF(order); ISB_EMU_OFF(wg_off); ISB_EMU_OFF(voff); ISB_EMU_OFF(eoff); ISB_EMU_OFF(n_bodies);
  ISB_EMU_OFF(x0); ISB_EMU_OFF(v0); ISB_EMU_OFF(a); ISB_EMU_OFF(a32); ISB_EMU_OFF(x1); ISB_EMU_OFF(v1);
  ISB_EMU_OFF(xbar); ISB_EMU_OFF(vbar); ISB_EMU_OFF(w); ISB_EMU_OFF(xhat); ISB_EMU_OFF(G); ISB_EMU_OFF(Gt);
  ISB_EMU_OFF(dx); ISB_EMU_OFF(r); ISB_EMU_OFF(cv); ISB_EMU_OFF(xt); ISB_EMU_OFF(Dv); ISB_EMU_OFF(vdT);
  ISB_EMU_OFF(lconn); ISB_EMU_OFF(stats); ISB_EMU_OFF(tol); ISB_EMU_OFF(adj_tol); ISB_EMU_OFF(max_newton);
  ISB_EMU_OFF(max_cg); ISB_EMU_OFF(want_tail); ISB_EMU_OFF(nacc); ISB_EMU_OFF(Fbuf); ISB_EMU_OFF(E0);
  ISB_EMU_OFF(E1); ISB_EMU_OFF(soff); ISB_EMU_OFF(slconn); ISB_EMU_OFF(sk); ISB_EMU_OFF(sil0);
  ISB_EMU_OFF(Sbuf); ISB_EMU_OFF(n_s); ISB_EMU_OFF(adj_warm);
#undef ISB_EMU_OFF
  return k;
}
