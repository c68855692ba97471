// The library context: uploaded mesh and material, options, and every device workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/isb.h"
#include "isb_host.hpp"
#include "isb_internal.hpp"

#define ISB_HIP(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return ::isb::fail(ISB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace isb {
// A named roctx range over a scope: the solver's phases (step, Newton solve, line search, CG
// solve, adjoint, VJP, batched launches) appear in a rocprofv3 marker trace; without a tool
// attached a range costs two library calls.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace isb

struct isb_ctx {
  int device = 0;
  int precision = ISB_FP64;

  // mesh
  int dim = 0, n_bodies = 0, n_v = 0, n_e = 0;
  std::vector<int64_t> voff, eoff;
  bool have_mesh = false, have_material = false;
  std::vector<void*> mesh_allocs, work_allocs;  // freed on re-upload / destroy
  int32_t* conn = nullptr;
  double *X = nullptr, *Dinv = nullptr, *W = nullptr, *gf = nullptr, *wmu = nullptr, *wlam = nullptr,
         *wkf = nullptr, *mass = nullptr, *rho = nullptr;
  float *Dinv32 = nullptr, *gf32 = nullptr, *wmu32 = nullptr, *wlam32 = nullptr, *wkf32 = nullptr,
        *W32 = nullptr;
  uint8_t* pinned = nullptr;
  // the material is uniform with the fibre along axis `uni_axis` (-1: not); see DevMesh::axis
  int uni_axis = -1;
  double uni_mu = 0.0, uni_lam = 0.0, uni_kf = 0.0;

  // element colouring: elements of body b and colour k are clist[col_off[b*(nc+1)+k] .. +1)
  int n_colours = 0;
  std::vector<int32_t> col_off;
  int32_t* clist = nullptr;

  // element patches of the LDS-staged scatter; body b owns patches [body_patch_off[b], body_patch_off[b+1])
  int n_patches = 0;
  std::vector<int32_t> body_patch_off;
  isb::PatchPlan plan{};

  // the resident CG solver's plan (isb::build_resident_patches): body b's patches
  // [res_patch_off[b], res_patch_off[b+1]) of rplan, largest vertex list res_max_nv[b]; res_ok[b]
  // when the body takes the resident solver; res_cu: the compute units the plan was cut for.
  // rplan regroups each patch's elements (eperm) for the kernel that holds them in registers;
  // rplan_fixed keeps the elements' order (its loads stay coalesced) and only renumbers vertices.
  std::vector<int32_t> res_patch_off, res_max_nv;
  std::vector<uint8_t> res_ok;
  isb::PatchPlan rplan{}, rplan_fixed{};
  int res_cu = 0;
  isb::GridBar* gbar = nullptr;  // the resident solver's barrier (device)

  // vertex-pair springs (isb_spring_upload); body b owns springs [soff[b], soff[b+1]); colour k of
  // body b is sclist[scol_off[b*(nsc+1)+k] .. +1) as for the elements
  int n_s = 0, n_scolours = 0;
  std::vector<int64_t> soff;
  std::vector<int32_t> scol_off;
  std::vector<void*> spring_allocs;  // freed on spring or mesh re-upload / destroy
  int32_t* sconn = nullptr;          // [2][n_s]
  double *sk = nullptr, *sil0 = nullptr;
  int32_t* sclist = nullptr;

  isb_scene scene{};

  // options
  int solver = 0, scatter = 2, graph_safe = 0, block = 0 /* 0: 768 in 2D, 512 in 3D */, cg_check = 4;
  int model = 0;  // ISB_ENERGY_*
  int forward = 0, lbfgs_m = 8, lbfgs_max_iters = 20000;  // ISB_OPT_FORWARD and the L-BFGS settings
  int cg_graph = 0;                    // ISB_OPT_CG_GRAPH
  int fp64_fallback = 1;               // ISB_OPT_FP64_FALLBACK
  int adj_warm = 0;                    // ISB_OPT_ADJ_WARM_START
  int compact_rest = 1;                // ISB_OPT_COMPACT_REST
  int patch_block = 0;                 // ISB_OPT_PATCH_BLOCK (0: kPatchBlock)
  int cg_single = 1;                   // ISB_OPT_CG_SINGLE_REDUCTION
  int cg_resident = 1;                 // ISB_OPT_CG_RESIDENT
  int64_t barrier_limit_us = 4000000;  // ISB_OPT_CG_BARRIER_LIMIT_US
  hipStream_t cap_stream = nullptr;    // internal stream the CG chunk is captured on

  // plain-solver workspaces, [n_v*dim] unless noted
  double *w_x = nullptr, *w_xt = nullptr, *w_xhat = nullptr, *w_cv = nullptr /*[n_v]*/, *w_G = nullptr,
         *w_Gt = nullptr, *w_xs = nullptr, *w_r = nullptr, *w_p = nullptr, *w_Hp = nullptr, *w_Dinvp = nullptr,
         *w_vdiag = nullptr, *w_diag = nullptr;
  double *w_u = nullptr, *w_s = nullptr;  // single-reduction CG: u = D^-1 r and s = H p
  double* hv_part = nullptr;        // [min(n_patches, kMaxPatchGrid)] curvature partials of the patch Hv
  float* w_a32 = nullptr;           // [n_e]
  double *w_lbS = nullptr, *w_lbY = nullptr;  // [lbfgs_m][n_v*dim] L-BFGS pairs (allocated on first use)
  int lbfgs_alloc_m = 0;
  std::vector<void*> lbfgs_allocs;           // the two arrays above; freed when lbfgs_m changes
  double* partials = nullptr;       // reduction partials
  double* dscal = nullptr;          // small device results (finalize outputs)
  double* ebuf = nullptr;           // [3*n_bodies] per-body energy comps
  isb::CgScal* scal = nullptr;      // device CG scalars
  double* hscal = nullptr;          // pinned host mirror of dscal
  isb::CgScal* hcg = nullptr;       // pinned host mirror of scal
  isb::CgScal* hcg_ring = nullptr;  // [2] pinned copies of scal taken after alternate CG batches
  hipEvent_t cg_ev[2] = {nullptr, nullptr};  // completion of the copy into hcg_ring[k]

  // batched-solver state (owned by the batched solver); batched64: the FP64 state of the mixed
  // solver's fallback, prepared on first use
  void* batched = nullptr;
  void* batched64 = nullptr;

  ~isb_ctx();
  void free_list(std::vector<void*>& v);
};

namespace isb {

DevMesh devmesh(const isb_ctx* c);
DevScene devscene(const isb_ctx* c);
DevSprings devsprings(const isb_ctx* c);

// batched persistent solver (isb_batched.hip)
isb_status batched_prepare(isb_ctx* c);
void batched_release(isb_ctx* c);
isb_status batched_step(isb_ctx* c, hipStream_t s, const double* x0, const double* v0, const double* a, double* x1,
                        double* v1, isb_stats* stats);
isb_status batched_adjoint(isb_ctx* c, hipStream_t s, const double* x1, const double* x0, const double* a,
                           const double* x1_bar, const double* v1_bar, double* w, isb_stats* stats);
int64_t batched_lds_bytes(const isb_ctx* c);

}  // namespace isb
