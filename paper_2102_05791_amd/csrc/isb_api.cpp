// C-ABI implementation: context lifetime, upload, and the plain host-driven Newton-PCG solver.
//
// The plain solver handles one body at a time with grid-wide kernels. Per Newton iteration
// (Sec. 3 and 5: x1 is the minimiser of the step objective; the paper leaves the minimiser free):
//   gradient -> |G| (host read) -> Jacobi diagonal -> PCG on H dx = -G with device-resident
//   scalars (host polls the stop flag every cg_check iterations) -> Armijo backtracking on
//   element-wise energy differences (host read per trial) -> x += alpha dx.
// The adjoint (Eq. 9) is one PCG solve with the same Hessian-vector kernel at x1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "isb_ctx.hpp"

using namespace isb;

static constexpr double kArmijoC1 = 1e-4;
static constexpr int kMaxBacktracks = 30;
static constexpr double kEps = 2.220446049250313e-16;
// Below the FP64 resolution of g the line search accepts a step only if it at least halves
// |grad g| or brings it under the stopping threshold; a smaller decrease is rounding noise, and the
// solve stops there as stagnated.
static constexpr double kFloorDecrease = 0.5;

void isb_ctx::free_list(std::vector<void*>& v) {
  for (void* p : v) (void)hipFree(p);
  v.clear();
}

isb_ctx::~isb_ctx() {
  (void)hipSetDevice(device);
  batched_release(this);
  free_list(work_allocs);
  free_list(lbfgs_allocs);
  free_list(spring_allocs);
  free_list(mesh_allocs);
  if (hscal) (void)hipHostFree(hscal);
  if (hcg) (void)hipHostFree(hcg);
  if (hcg_ring) (void)hipHostFree(hcg_ring);
  for (hipEvent_t& e : cg_ev)
    if (e) (void)hipEventDestroy(e);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

namespace isb {

DevMesh devmesh(const isb_ctx* c) {
  DevMesh m;
  m.dim = c->dim;
  m.n_v = c->n_v;
  m.n_e = c->n_e;
  m.conn = c->conn;
  m.Dinv = c->Dinv;
  m.gf = c->gf;
  m.W = c->W;
  m.wmu = c->wmu;
  m.wlam = c->wlam;
  m.wkf = c->wkf;
  m.Dinv32 = c->Dinv32;
  m.gf32 = c->gf32;
  m.wmu32 = c->wmu32;
  m.wlam32 = c->wlam32;
  m.wkf32 = c->wkf32;
  m.mass = c->mass;
  m.pinned = c->pinned;
  m.model = c->model;
  m.axis = c->compact_rest ? c->uni_axis : -1;
  m.mu_u = c->uni_mu;
  m.lam_u = c->uni_lam;
  m.kf_u = c->uni_kf;
  m.W32 = c->W32;
  return m;
}

DevSprings devsprings(const isb_ctx* c) { return DevSprings{c->n_s, c->sconn, c->sk, c->sil0}; }

DevScene devscene(const isb_ctx* c) {
  DevScene s;
  s.be = c->scene.integrator == ISB_BACKWARD_EULER;
  s.h = c->scene.h;
  s.s_pot = s.be ? c->scene.h * c->scene.h : 1.0;
  s.grav = c->scene.gravity;
  s.kc = c->scene.k_contact;
  s.kfr = c->scene.k_friction;
  s.eps = c->scene.eps_friction;
  s.ih2 = 1.0 / (s.h * s.h);
  return s;
}

}  // namespace isb

template <typename T>
static isb_status dalloc(std::vector<void*>& list, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  ISB_HIP(hipMalloc(&q, count * sizeof(T)));
  list.push_back(q);
  *p = static_cast<T*>(q);
  return ISB_OK;
}

#define ISB_TRY(expr)                 \
  do {                                \
    isb_status st_ = (expr);          \
    if (st_ != ISB_OK) return st_;    \
  } while (0)

static isb_status check_ctx(isb_ctx* c, bool need_material) {
  if (!c) return fail(ISB_E_ARG, "NULL context");
  if (!c->have_mesh) return fail(ISB_E_STATE, "no mesh uploaded");
  if (need_material && !c->have_material) return fail(ISB_E_STATE, "no material uploaded");
  ISB_HIP(hipSetDevice(c->device));
  return ISB_OK;
}

static isb_status check_scene(const isb_scene* s) {
  if (!s) return fail(ISB_E_ARG, "NULL scene");
  if (s->integrator != ISB_QUASISTATIC && s->integrator != ISB_BACKWARD_EULER)
    return fail(ISB_E_ARG, "unknown integrator");
  if (!(s->h > 0.0)) return fail(ISB_E_ARG, "h must be > 0");
  if (s->max_newton < 0 || s->max_cg < 1) return fail(ISB_E_ARG, "iteration caps must be >= 0 / >= 1");
  if (!(s->tol_rel >= 0.0) || !(s->adj_tol_rel >= 0.0)) return fail(ISB_E_ARG, "tolerances must be >= 0");
  if (!std::isfinite(s->gravity) || !std::isfinite(s->k_contact) || !std::isfinite(s->k_friction) ||
      !std::isfinite(s->eps_friction))
    return fail(ISB_E_ARG, "non-finite scene constant");
  return ISB_OK;
}

// read n doubles of dscal into hscal (synchronises the stream)
static isb_status read_scal(isb_ctx* c, hipStream_t s, int n) {
  ISB_HIP(hipMemcpyAsync(c->hscal, c->dscal, n * sizeof(double), hipMemcpyDeviceToHost, s));
  ISB_HIP(hipStreamSynchronize(s));
  return ISB_OK;
}

static isb_status read_cg(isb_ctx* c, hipStream_t s) {
  ISB_HIP(hipMemcpyAsync(c->hcg, c->scal, sizeof(CgScal), hipMemcpyDeviceToHost, s));
  ISB_HIP(hipStreamSynchronize(s));
  return ISB_OK;
}

// run fn(ERange, atomic) over the elements of body b (all bodies when b < 0)
template <class Fn>
static void elem_ranges(const isb_ctx* c, int b, Fn fn) {
  const int b0 = b < 0 ? 0 : b, b1 = b < 0 ? c->n_bodies : b + 1;
  if (c->scatter != 1) {
    fn(ERange{(int)c->eoff[b0], (int)c->eoff[b1], nullptr}, true);
    return;
  }
  const int nc1 = c->n_colours + 1;
  for (int bb = b0; bb < b1; ++bb)
    for (int k = 0; k < c->n_colours; ++k) {
      const int s = c->col_off[bb * nc1 + k], e = c->col_off[bb * nc1 + k + 1];
      if (e > s) fn(ERange{s, e, c->clist}, false);
    }
}

// Bodies below this many elements keep the per-corner atomic scatter in patch mode: a launch over
// them is latency bound and patches of a small body cannot fill the GPU.
static constexpr int64_t kPatchMinElems = 16384;

// spring scatter of op (PATCH_GRAD / PATCH_HV / PATCH_DIAG) over body b (all bodies when b < 0):
// one pass per colour in colour mode (bitwise reproducible), FP64 global atomics otherwise
static void spring_scatter(isb_ctx* c, int b, int op, const double* x, const double* a, const double* p,
                           double* out, const int* done, hipStream_t s) {
  if (c->n_s == 0) return;
  const DevSprings sp = devsprings(c);
  const DevScene sc = devscene(c);
  const double* as = a + c->n_e;
  const int b0 = b < 0 ? 0 : b, b1 = b < 0 ? c->n_bodies : b + 1;
  if (c->scatter != 1) {
    launch_spring_op(c->dim, sp, sc, ERange{(int)c->soff[b0], (int)c->soff[b1], nullptr}, true, op, x, as, p, out,
                     done, s);
    return;
  }
  const int nc1 = c->n_scolours + 1;
  for (int bb = b0; bb < b1; ++bb)
    for (int k = 0; k < c->n_scolours; ++k) {
      const int s0 = c->scol_off[bb * nc1 + k], s1 = c->scol_off[bb * nc1 + k + 1];
      if (s1 > s0) launch_spring_op(c->dim, sp, sc, ERange{s0, s1, c->sclist}, false, op, x, as, p, out, done, s);
    }
}

// element scatter of op (PATCH_GRAD / PATCH_HV / PATCH_DIAG) over body b (all bodies when b < 0),
// in the context's scatter mode: FP64 global atomics, colour passes, or LDS-staged patches. Only
// the Hessian-vector product takes the context's precision; gradient and diagonal are FP64.
// a32: the FP32 copy of the actuation that mixed Hessian-vector products read (nullptr: they read a)
static void elem_scatter(isb_ctx* c, int b, int op, const double* x, const double* a, const double* p, double* out,
                         const int* done, hipStream_t s, const float* a32 = nullptr) {
  const DevMesh m = devmesh(c);
  const DevScene sc = devscene(c);
  const int64_t ne_scope = b < 0 ? c->n_e : c->eoff[b + 1] - c->eoff[b];
  if (c->scatter == 2 && ne_scope >= kPatchMinElems) {
    const int p0 = b < 0 ? 0 : c->body_patch_off[b];
    const int p1 = b < 0 ? c->n_patches : c->body_patch_off[b + 1];
    PatchPlan plan = c->plan;
    plan.block = c->patch_block;
    launch_elem_patch(m, sc, plan, p0, p1, op, op == PATCH_HV ? c->precision : 0, x, a, a32, p, out, done, s);
  } else {
    elem_ranges(c, b, [&](ERange r, bool atomic) {
      if (op == PATCH_GRAD)
        launch_elem_grad(m, sc, r, atomic, x, a, out, s);
      else if (op == PATCH_HV)
        launch_elem_hv(m, sc, r, atomic, c->precision, x, a, a32, p, out, done, s);
      else
        launch_elem_diag(m, sc, r, atomic, x, a, out, s);
    });
  }
  spring_scatter(c, b, op, x, a, p, out, done, s);
}

struct BodyRange {
  int v0, v1, e0, e1, n, off;
};

static BodyRange body_range(const isb_ctx* c, int b) {
  BodyRange r;
  if (b < 0) {
    r.v0 = 0;
    r.v1 = c->n_v;
    r.e0 = 0;
    r.e1 = c->n_e;
  } else {
    r.v0 = (int)c->voff[b];
    r.v1 = (int)c->voff[b + 1];
    r.e0 = (int)c->eoff[b];
    r.e1 = (int)c->eoff[b + 1];
  }
  r.n = (r.v1 - r.v0) * c->dim;
  r.off = r.v0 * c->dim;
  return r;
}

// ---------------------------------------------------------------------------------------------
// building blocks of the plain solver (body b, or all bodies with b < 0)
// ---------------------------------------------------------------------------------------------
static void eval_grad(isb_ctx* c, int b, const double* x, const double* x0, const double* a, double* G,
                      hipStream_t s) {
  const DevMesh m = devmesh(c);
  const DevScene sc = devscene(c);
  const BodyRange br = body_range(c, b);
  launch_vertex_grad(m, sc, br.v0, br.v1, x, x0, c->w_xhat, c->w_cv, G, s);
  elem_scatter(c, b, PATCH_GRAD, x, a, nullptr, G, nullptr, s);
  launch_mask(m, br.v0, br.v1, G, s);
}

// |v|_2 over body b's DOFs into dscal[slot]
static void enqueue_norm2(isb_ctx* c, int b, const double* v, int slot, hipStream_t s) {
  const BodyRange br = body_range(c, b);
  int nb = 0;
  launch_dot(br.n, v + br.off, v + br.off, c->partials, s, &nb);
  launch_finalize(c->partials, nb, 1, c->dscal + slot, s);
}

static void eval_precond(isb_ctx* c, int b, const double* x, const double* a, hipStream_t s) {
  const DevMesh m = devmesh(c);
  const DevScene sc = devscene(c);
  const BodyRange br = body_range(c, b);
  launch_vertex_hdiag(m, sc, br.v0, br.v1, x, c->w_cv, c->w_vdiag, s);
  launch_copy(br.n, c->w_vdiag + br.off, c->w_diag + br.off, s);
  elem_scatter(c, b, PATCH_DIAG, x, a, nullptr, c->w_diag, nullptr, s);
  launch_finish_diag(m, br.v0, br.v1, c->w_diag, c->w_Dinvp, s);
}

// energy change along dx at step alpha: dscal[0..3) = (sum dE, sum |E(x)|, E(x + alpha dx));
// dx == nullptr gives the energy at x in dscal[2]
static void enqueue_energy(isb_ctx* c, int b, const double* x, const double* dx, double alpha, const double* x0,
                           const double* a, double* out, hipStream_t s) {
  const DevMesh m = devmesh(c);
  const DevScene sc = devscene(c);
  const BodyRange br = body_range(c, b);
  int nbe = 0, nbs = 0, nbv = 0;
  launch_elem_energy(m, sc, ERange{br.e0, br.e1, nullptr}, x, dx, alpha, a, c->partials, 0, s, &nbe);
  if (c->n_s > 0) {
    const int b0 = b < 0 ? 0 : b, b1 = b < 0 ? c->n_bodies : b + 1;
    launch_spring_energy(c->dim, devsprings(c), sc, ERange{(int)c->soff[b0], (int)c->soff[b1], nullptr}, x, dx,
                         alpha, a + c->n_e, c->partials, nbe, s, &nbs);
  }
  launch_vertex_energy(m, sc, br.v0, br.v1, x, dx, alpha, x0, c->w_xhat, c->w_cv, c->partials, nbe + nbs, s, &nbv);
  launch_finalize(c->partials, nbe + nbs + nbv, 3, out, s);
}

// The single-reduction CG runs where the Hessian-vector product is one patch launch that can also
// return its curvature partials: LDS-staged patches, no springs (their curvature would need a pass
// of its own).
static bool single_reduction_cg(const isb_ctx* c, int b) {
  const int64_t ne = b < 0 ? c->n_e : c->eoff[b + 1] - c->eoff[b];
  return c->cg_single && c->scatter == 2 && ne >= kPatchMinElems && c->n_s == 0;
}

// one CG iteration over body b (every kernel returns at once when the device flag says the solve is
// done). Classic PCG: the Hessian-vector product, then three vector kernels (p.Hp; x, r, r.z; the
// next p). Single-reduction PCG: the Hessian-vector product with its curvature partials (w += H u),
// then one vector kernel.
static void cg_iteration(isb_ctx* c, int b, const double* x, const double* a, hipStream_t s) {
  const BodyRange br = body_range(c, b);
  const int o = br.off;
  if (single_reduction_cg(c, b)) {
    const int p0 = b < 0 ? 0 : c->body_patch_off[b];
    const int p1 = b < 0 ? c->n_patches : c->body_patch_off[b + 1];
    PatchPlan plan = c->plan;
    plan.block = c->patch_block;
    const int nhv = launch_elem_patch(devmesh(c), devscene(c), plan, p0, p1, PATCH_HV, c->precision, x, a, c->w_a32,
                                      c->w_u, c->w_Hp, &c->scal->done, s, c->hv_part);
    launch_cgcg_vec(br.n, c->hv_part, nhv, c->partials, c->w_Dinvp + o, c->w_vdiag + o, c->w_r + o, c->w_u + o,
                    c->w_Hp + o, c->w_p + o, c->w_s + o, c->w_xs + o, c->scal, s);
    return;
  }
  elem_scatter(c, b, PATCH_HV, x, a, c->w_p, c->w_Hp, &c->scal->done, s, c->w_a32);
  launch_cg_dot(br.n, c->w_p + o, c->w_Hp + o, c->partials, c->scal, s);
  launch_cg_update(br.n, c->w_p + o, c->w_Hp + o, c->w_Dinvp + o, c->w_r + o, c->w_xs + o, c->partials, c->scal, s);
  launch_cg_p(br.n, c->w_r + o, c->w_Dinvp + o, c->w_vdiag + o, c->w_p + o, c->w_Hp + o, c->partials, c->scal, s);
}

// Iterations per captured chunk of the graph mode: a chunk is replayed until the device flag says
// the solve is done; the iterations of the last chunk past that point return at once.
static constexpr int kCgChunk = 8;

// The resident form of the single-reduction CG on body b (one cooperative launch for the whole
// solve) where the body has a resident plan that fits the device; *ran = false when it does not run.
static isb_status resident_cg(isb_ctx* c, int b, const double* x, const double* a, const double* rhs, double sign,
                              double tol, int max_cg, hipStream_t s, bool* ran) {
  *ran = false;
  if (!c->cg_resident || b < 0 || (size_t)b >= c->res_ok.size() || !c->res_ok[b]) return ISB_OK;
  const TraceRange trace("isb: CG solve, resident");
  PatchPlan P = resident_caches_elements(c->precision, c->model) ? c->rplan : c->rplan_fixed;
  P.max_nv = c->res_max_nv[b];
  const int p0 = c->res_patch_off[b], np = c->res_patch_off[b + 1] - p0;
  // W0..W2 are the workspaces the launch-per-iteration form uses for H u, u and s
  const hipError_t e = launch_cg_resident(devmesh(c), devscene(c), P, p0, np, c->res_cu, c->precision, x, a,
                                          c->w_a32, rhs, sign, c->w_Dinvp, c->w_vdiag, c->w_xs, c->w_Hp, c->w_u,
                                          c->w_s, c->partials, c->gbar, c->scal, tol * tol, max_cg,
                                          c->barrier_limit_us, s);
  if (e == hipErrorCooperativeLaunchTooLarge) {
    c->res_ok[b] = 0;  // its workgroups cannot all be resident here: the launch-per-iteration form
    return ISB_OK;
  }
  if (e != hipSuccess) return fail(ISB_E_HIP, std::string("resident CG launch: ") + hipGetErrorString(e));
  ISB_TRY(read_cg(c, s));
  if (c->hcg->fault) return fail(ISB_E_HIP, "resident CG: a grid barrier timed out");
  *ran = true;
  return ISB_OK;
}

// PCG on H(x) xs = sign * rhs over body b, one launch per kernel, leaving the outcome in c->hcg.
// Graph mode (ISB_OPT_CG_GRAPH): a chunk of kCgChunk iterations is captured once per solve on an
// internal stream and replayed on `s`, one launch and one host read per chunk instead of the
// iteration's launches and a read every cg_check iterations.
static isb_status launched_cg(isb_ctx* c, int b, const double* x, const double* a, const double* rhs, double sign,
                              double tol, int max_cg, hipStream_t s, bool single) {
  const TraceRange trace("isb: CG solve, launch per kernel");
  const BodyRange br = body_range(c, b);
  const int o = br.off;
  if (single)
    launch_cgcg_start(br.n, rhs + o, sign, c->w_Dinvp + o, c->w_vdiag + o, c->w_r + o, c->w_u + o, c->w_Hp + o,
                      c->w_p + o, c->w_s + o, c->w_xs + o, c->partials, c->scal, tol * tol, max_cg, s);
  else
    launch_cg_start(br.n, rhs + o, sign, c->w_Dinvp + o, c->w_vdiag + o, c->w_r + o, c->w_p + o, c->w_xs + o,
                    c->w_Hp + o, c->partials, c->scal, tol * tol, max_cg, s);
  if (c->cg_graph && max_cg > kCgChunk) {
    if (!c->cap_stream) ISB_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ISB_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kCgChunk; ++k) cg_iteration(c, b, x, a, c->cap_stream);
    const hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
    if (ce != hipSuccess) return fail(ISB_E_HIP, std::string("CG graph capture: ") + hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(ISB_E_HIP, std::string("CG graph instantiation: ") + hipGetErrorString(ie));
    isb_status st = ISB_OK;
    for (int done_its = 0; done_its < max_cg; done_its += kCgChunk) {
      const hipError_t le = hipGraphLaunch(exec, s);
      if (le != hipSuccess) {
        st = fail(ISB_E_HIP, std::string("CG graph launch: ") + hipGetErrorString(le));
        break;
      }
      if ((st = read_cg(c, s)) != ISB_OK || c->hcg->done) break;
    }
    (void)hipGraphExecDestroy(exec);
    if (st != ISB_OK) return st;
  } else {
    // Batches of cg_check iterations with one batch of look-ahead: each batch ends with an
    // asynchronous copy of the CG scalars to pinned host memory and an event; the host waits for the
    // previous batch's event while the current batch is already queued, so the GPU does not drain at
    // every check. Iterations enqueued after convergence return at once (the device flag).
    const int check = std::max(1, c->cg_check);
    int k = 0, enq = 0;
    bool pending = false;
    while (enq < max_cg) {
      const int n = std::min(check, max_cg - enq);
      for (int j = 0; j < n; ++j) cg_iteration(c, b, x, a, s);
      enq += n;
      ISB_HIP(hipMemcpyAsync(c->hcg_ring + (k & 1), c->scal, sizeof(CgScal), hipMemcpyDeviceToHost, s));
      ISB_HIP(hipEventRecord(c->cg_ev[k & 1], s));
      if (pending) {
        ISB_HIP(hipEventSynchronize(c->cg_ev[(k - 1) & 1]));
        if (c->hcg_ring[(k - 1) & 1].done) break;
      }
      pending = true;
      ++k;
    }
  }
  if (single) launch_cgcg_final(br.n, c->partials, c->scal, s);
  return read_cg(c, s);
}

// PCG on H(x) xs = sign * rhs over body b; returns iterations, sets negcurv and the final r.r.
static isb_status run_cg(isb_ctx* c, int b, const double* x, const double* a, const double* rhs, double sign,
                         double tol, int max_cg, hipStream_t s, int* iters, bool* negcurv, double* rr) {
  const bool single = single_reduction_cg(c, b);
  bool resident = false;
  if (single) ISB_TRY(resident_cg(c, b, x, a, rhs, sign, tol, max_cg, s, &resident));
  if (!resident) ISB_TRY(launched_cg(c, b, x, a, rhs, sign, tol, max_cg, s, single));
  *iters = c->hcg->iters;
  *negcurv = c->hcg->negcurv != 0;
  *rr = c->hcg->rr;
  if (single && *negcurv) {
    // The single-reduction form obtains p^T H p from a recurrence, delta - beta gamma / alpha_prev,
    // which cancels when beta^2 p_prev^T H p_prev approaches delta (long, slowly converging solves):
    // a non-positive value there may be rounding. Solve again in the classic form, which forms
    // p^T H p from a fresh product and decides the curvature itself.
    const int keep = c->cg_single;
    int it2 = 0;
    c->cg_single = 0;
    const isb_status st = run_cg(c, b, x, a, rhs, sign, tol, max_cg, s, &it2, negcurv, rr);
    c->cg_single = keep;
    ISB_TRY(st);
    *iters += it2;
  }
  return ISB_OK;
}

// one Newton-PCG solve of body b; x is the iterate (workspace), G its gradient
// Armijo backtracking along dx from the iterate *px (gradient *pG, norm *res, g^T dx = gTd < 0) on
// sum_e [g_e(x + alpha dx) - g_e(x)]. Below the FP64 resolution of g the gradient decides instead:
// Newton takes the step if |grad g| at least halves or falls to res_stop (the stopping threshold)
// and otherwise stops (shorter steps of a quadratically convergent method cannot do better at the
// floor); a first-order method takes it if |grad g| falls to res_stop or the slope along dx has not
// turned past half its initial size, grad g(x + alpha dx) . dx <= |gTd| / 2 (on a quadratic that
// holds up to 1.5 times the exact line minimiser, where g still decreases), and otherwise halves
// alpha. On acceptance *px, *pG and *res hold the new iterate (the buffers may swap with *pxt, *pGt)
// and *alpha_out the step taken.
static isb_status line_search(isb_ctx* c, int b, hipStream_t s, const double* x0, const double* a, const double* dx,
                              double gTd, double res_stop, bool first_order, double** px, double** pxt, double** pG,
                              double** pGt, double* res, isb_stats* st, bool* accepted_out, double* alpha_out) {
  const TraceRange trace("isb: line search");
  const BodyRange br = body_range(c, b);
  double *x = *px, *xt = *pxt, *G = *pG, *Gt = *pGt;
  double alpha = 1.0;
  bool accepted = false, via_grad = false;
  for (int ls = 0; ls <= kMaxBacktracks; ++ls) {
    enqueue_energy(c, b, x, dx, alpha, x0, a, c->dscal, s);
    ISB_TRY(read_scal(c, s, 3));
    const double dg = c->hscal[0], gabs = c->hscal[1];
    if (!std::isfinite(dg)) {
      // overflow or an invalid trial point: backtrack
    } else if (std::fabs(dg) > 1e3 * kEps * gabs) {
      accepted = dg <= kArmijoC1 * alpha * gTd;
    } else {
      // below the resolution of g the Armijo test only sees rounding
      launch_copy(br.n, x + br.off, xt + br.off, s);
      launch_axpy(br.n, xt + br.off, alpha, dx + br.off, s);
      eval_grad(c, b, xt, x0, a, Gt, s);
      enqueue_norm2(c, b, Gt, 0, s);
      ISB_TRY(read_scal(c, s, 1));
      const double rt = std::sqrt(c->hscal[0]);
      bool take;
      if (first_order) {
        int nb = 0;
        launch_dot(br.n, Gt + br.off, dx + br.off, c->partials, s, &nb);
        launch_finalize(c->partials, nb, 1, c->dscal, s);
        ISB_TRY(read_scal(c, s, 1));
        take = rt <= res_stop || c->hscal[0] <= 0.5 * std::fabs(gTd);
      } else {
        take = rt <= kFloorDecrease * *res || rt <= res_stop;
        if (!take) break;  // shorter steps cannot do better at the rounding floor
      }
      if (take) {
        accepted = via_grad = true;
        std::swap(x, xt);
        std::swap(G, Gt);
        *res = rt;
      }
    }
    if (accepted) break;
    alpha *= 0.5;
    st->ls_backtracks += 1;
  }
  if (accepted && !via_grad) {
    launch_axpy(br.n, x + br.off, alpha, dx + br.off, s);
    eval_grad(c, b, x, x0, a, G, s);
    enqueue_norm2(c, b, G, 0, s);
    ISB_TRY(read_scal(c, s, 1));
    *res = std::sqrt(c->hscal[0]);
  }
  *px = x;
  *pxt = xt;
  *pG = G;
  *pGt = Gt;
  *accepted_out = accepted;
  *alpha_out = alpha;
  return ISB_OK;
}

static isb_status plain_newton(isb_ctx* c, int b, hipStream_t s, const double* x0, const double* a, double** px,
                               double** pxt, double** pG, double** pGt, isb_stats* st) {
  const TraceRange trace("isb: Newton solve");
  const BodyRange br = body_range(c, b);
  const isb_scene& sc = c->scene;
  double *x = *px, *xt = *pxt, *G = *pG, *Gt = *pGt;
  eval_grad(c, b, x, x0, a, G, s);
  enqueue_norm2(c, b, G, 0, s);
  ISB_TRY(read_scal(c, s, 1));
  const double res0 = std::sqrt(c->hscal[0]);
  double res = res0;
  double eta = 0.5, res_prev = res0;  // forcing term and the gradient norm it was set from
  // a body large enough for the resident CG plan (whichever CG form runs, so that the Newton path
  // does not depend on it)
  const bool large = b >= 0 && (size_t)b < c->res_ok.size() && c->res_ok[b];
  st->res0 = res0;
  isb_status status = ISB_OK;
  if (!std::isfinite(res0)) {
    st->flags |= ISB_FLAG_NONFINITE;
    status = fail(ISB_E_NONFINITE, "non-finite gradient at the initial guess");
  }
  while (status == ISB_OK) {
    if (res <= sc.tol_rel * res0 || res == 0.0) {
      st->flags |= ISB_FLAG_CONVERGED;
      break;
    }
    if (st->newton_iters >= sc.max_newton) {
      status = fail(ISB_E_NOT_CONVERGED, "Newton iteration cap reached");
      break;
    }
    eval_precond(c, b, x, a, s);
    // the CG tolerance eta |g| never goes below half the Newton stopping threshold, which a more
    // accurate last step could not improve on
    // inexact Newton forcing: on a small body each Newton iteration costs as much as several CG
    // iterations (launches and host round trips), and Eisenstat and Walker's second choice (eta
    // following the square of the last step's reduction of the gradient, with its safeguard)
    // saves Newton iterations; on a large body CG iterations dominate, and the square-root rule,
    // which spends fewer of them, is the faster
    if (large) {
      eta = std::min(0.5, std::sqrt(res / res0));
    } else if (st->newton_iters > 0) {
      const double q = res / res_prev;
      double e = 0.9 * q * q;
      if (0.9 * eta * eta > 0.1) e = std::max(e, 0.9 * eta * eta);
      eta = std::min(0.5, e);
    }
    res_prev = res;
    const double cg_tol = std::max(eta * res, 0.5 * sc.tol_rel * res0);
    int cg_it = 0;
    bool neg = false;
    double rr = 0.0;
    ISB_TRY(run_cg(c, b, x, a, G, -1.0, cg_tol, sc.max_cg, s, &cg_it, &neg, &rr));
    st->cg_iters += cg_it;
    st->negcurv_exits += neg ? 1 : 0;
    double* dx = c->w_xs;
    int nb = 0;
    launch_dot(br.n, G + br.off, dx + br.off, c->partials, s, &nb);
    launch_finalize(c->partials, nb, 1, c->dscal, s);
    ISB_TRY(read_scal(c, s, 1));
    double gTd = c->hscal[0];
    if (!(gTd < 0.0)) {
      // not a descent direction (CG stopped before any progress): preconditioned steepest descent
      launch_neg_precond(br.n, c->w_Dinvp + br.off, G + br.off, dx + br.off, s);
      launch_dot(br.n, G + br.off, dx + br.off, c->partials, s, &nb);
      launch_finalize(c->partials, nb, 1, c->dscal, s);
      ISB_TRY(read_scal(c, s, 1));
      gTd = c->hscal[0];
      if (!(gTd < 0.0)) {
        st->flags |= ISB_FLAG_STAGNATED;
        break;
      }
    }
    bool accepted = false;
    double alpha = 0.0;
    ISB_TRY(line_search(c, b, s, x0, a, dx, gTd, sc.tol_rel * res0, false, &x, &xt, &G, &Gt, &res, st, &accepted,
                        &alpha));
    if (!accepted) {
      st->flags |= ISB_FLAG_STAGNATED;
      break;
    }
    st->newton_iters += 1;
    if (!std::isfinite(res)) {
      st->flags |= ISB_FLAG_NONFINITE;
      status = fail(ISB_E_NONFINITE, "non-finite gradient");
    }
  }
  st->res_final = res;
  if (res <= sc.tol_rel * res0) st->flags |= ISB_FLAG_CONVERGED;
  *px = x;
  *pxt = xt;
  *pG = G;
  *pGt = Gt;
  return status;
}

// dot product of two vectors over body b's DOFs, read back to the host
static isb_status body_dot(isb_ctx* c, int b, const double* u, const double* v, hipStream_t s, double* out) {
  const BodyRange br = body_range(c, b);
  int nb = 0;
  launch_dot(br.n, u + br.off, v + br.off, c->partials, s, &nb);
  launch_finalize(c->partials, nb, 1, c->dscal, s);
  ISB_TRY(read_scal(c, s, 1));
  *out = c->hscal[0];
  return ISB_OK;
}

// The first-order forward solver (ISB_FORWARD_LBFGS): limited-memory BFGS on the step objective,
// which uses gradients only (Nocedal & Wright, Alg. 7.4 and 7.5, two-loop recursion with the
// scaling s^T y / y^T y of the newest pair), the same Armijo line search and stopping rule as
// Newton, and steepest descent of unit length as the first direction and whenever the recursion
// does not give a descent direction. Pairs with s^T y <= 1e-12 |s| |y| are not stored. Iterations
// are reported as newton_iters.
static isb_status plain_lbfgs(isb_ctx* c, int b, hipStream_t s, const double* x0, const double* a, double** px,
                              double** pxt, double** pG, double** pGt, isb_stats* st) {
  const TraceRange trace("isb: L-BFGS solve");
  const BodyRange br = body_range(c, b);
  const isb_scene& sc = c->scene;
  const int m = c->lbfgs_m, n = br.n, o = br.off;
  const size_t nd = (size_t)c->n_v * c->dim;
  double *x = *px, *xt = *pxt, *G = *pG, *Gt = *pGt;
  double* q = c->w_p;      // the recursion's vector, then the direction's negative
  double* Gold = c->w_r;   // gradient at the previous iterate
  double* dx = c->w_xs;    // search direction
  std::vector<double> rho(m), al(m);
  std::vector<int> slot;   // history, oldest first; entries index the S and Y planes
  int next = 0;
  eval_grad(c, b, x, x0, a, G, s);
  enqueue_norm2(c, b, G, 0, s);
  ISB_TRY(read_scal(c, s, 1));
  const double res0 = std::sqrt(c->hscal[0]);
  double res = res0;
  st->res0 = res0;
  isb_status status = ISB_OK;
  if (!std::isfinite(res0)) {
    st->flags |= ISB_FLAG_NONFINITE;
    status = fail(ISB_E_NONFINITE, "non-finite gradient at the initial guess");
  }
  while (status == ISB_OK) {
    if (res <= sc.tol_rel * res0 || res == 0.0) {
      st->flags |= ISB_FLAG_CONVERGED;
      break;
    }
    if (st->newton_iters >= c->lbfgs_max_iters) {
      status = fail(ISB_E_NOT_CONVERGED, "L-BFGS iteration cap reached");
      break;
    }
    double gTd = 0.0;
    if (!slot.empty()) {
      // two-loop recursion: q = H_k G
      launch_copy(n, G + o, q + o, s);
      for (int k = (int)slot.size() - 1; k >= 0; --k) {
        const int j = slot[k];
        double sq = 0.0;
        ISB_TRY(body_dot(c, b, c->w_lbS + (size_t)j * nd, q, s, &sq));
        al[j] = rho[j] * sq;
        launch_axpy(n, q + o, -al[j], c->w_lbY + (size_t)j * nd + o, s);
      }
      const int jn = slot.back();
      double yy = 0.0;
      ISB_TRY(body_dot(c, b, c->w_lbY + (size_t)jn * nd, c->w_lbY + (size_t)jn * nd, s, &yy));
      const double gamma = 1.0 / (rho[jn] * yy);
      launch_axpy(n, q + o, gamma - 1.0, q + o, s);
      for (int k = 0; k < (int)slot.size(); ++k) {
        const int j = slot[k];
        double yq = 0.0;
        ISB_TRY(body_dot(c, b, c->w_lbY + (size_t)j * nd, q, s, &yq));
        launch_axpy(n, q + o, al[j] - rho[j] * yq, c->w_lbS + (size_t)j * nd + o, s);
      }
      launch_copy(n, q + o, dx + o, s);
      launch_axpy(n, dx + o, -2.0, dx + o, s);  // dx = -q
      ISB_TRY(body_dot(c, b, G, dx, s, &gTd));
    }
    if (!(gTd < 0.0)) {
      // steepest descent of unit length; the history restarts
      slot.clear();
      launch_copy(n, G + o, dx + o, s);
      launch_axpy(n, dx + o, -1.0 - 1.0 / res, dx + o, s);  // dx = -G / |G|
      gTd = -res;
    }
    launch_copy(n, G + o, Gold + o, s);
    bool accepted = false;
    double alpha = 0.0;
    ISB_TRY(line_search(c, b, s, x0, a, dx, gTd, sc.tol_rel * res0, true, &x, &xt, &G, &Gt, &res, st, &accepted,
                        &alpha));
    if (!accepted) {
      st->flags |= ISB_FLAG_STAGNATED;
      break;
    }
    st->newton_iters += 1;
    if (!std::isfinite(res)) {
      st->flags |= ISB_FLAG_NONFINITE;
      status = fail(ISB_E_NONFINITE, "non-finite gradient");
      break;
    }
    // the new pair s = alpha dx, y = G - G_old, written over the oldest pair when the history is full
    const int j = next;
    for (size_t k = 0; k < slot.size(); ++k)
      if (slot[k] == j) {
        slot.erase(slot.begin() + k);
        break;
      }
    double* Sj = c->w_lbS + (size_t)j * nd;
    double* Yj = c->w_lbY + (size_t)j * nd;
    launch_copy(n, dx + o, Sj + o, s);
    launch_axpy(n, Sj + o, alpha - 1.0, Sj + o, s);
    launch_copy(n, G + o, Yj + o, s);
    launch_axpy(n, Yj + o, -1.0, Gold + o, s);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    ISB_TRY(body_dot(c, b, Sj, Yj, s, &sy));
    ISB_TRY(body_dot(c, b, Sj, Sj, s, &ss));
    ISB_TRY(body_dot(c, b, Yj, Yj, s, &yy));
    if (sy > 1e-12 * std::sqrt(ss * yy)) {
      slot.push_back(j);
      rho[j] = 1.0 / sy;
      next = (j + 1) % m;
    }
  }
  st->res_final = res;
  if (res <= sc.tol_rel * res0) st->flags |= ISB_FLAG_CONVERGED;
  *px = x;
  *pxt = xt;
  *pG = G;
  *pGt = Gt;
  return status;
}

static isb_status fill_stats_tail(isb_ctx* c, int b, hipStream_t s, const double* x, const double* x0,
                                  const double* a, isb_stats* st) {
  const BodyRange br = body_range(c, b);
  const DevMesh m = devmesh(c);
  enqueue_energy(c, b, x, nullptr, 0.0, x0, a, c->dscal, s);
  int nb = 0;
  launch_elem_minmax_J(m, ERange{br.e0, br.e1, nullptr}, x, c->partials + 6 * kMaxRedBlocks, s, &nb);
  launch_finalize_minmax(c->partials + 6 * kMaxRedBlocks, nb, c->dscal + 3, s);
  ISB_TRY(read_scal(c, s, 5));
  st->energy = c->hscal[2];
  st->min_J = c->hscal[3];
  st->max_J = c->hscal[4];
  return ISB_OK;
}

// check a > 0 and finite over the elements' and springs' actions (one reduction, host read)
static isb_status check_actuation(isb_ctx* c, hipStream_t s, const double* a) {
  launch_min_count(c->n_e + c->n_s, a, c->partials, c->dscal, s);
  ISB_TRY(read_scal(c, s, 2));
  if (c->hscal[1] != 0.0) return fail(ISB_E_NONFINITE, "non-finite actuation");
  if (!(c->hscal[0] > 0.0)) return fail(ISB_E_ARG, "actuation a must be > 0");
  return ISB_OK;
}

static isb_status plain_step(isb_ctx* c, hipStream_t s, const double* x0, const double* v0, const double* a,
                             double* x1, double* v1, isb_stats* per_body) {
  const TraceRange trace("isb: step, plain");
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  if (c->precision == ISB_MIXED) launch_to_f32(c->n_e, a, c->w_a32, s);
  if (c->forward == ISB_FORWARD_LBFGS && c->lbfgs_alloc_m != c->lbfgs_m) {
    // the first-order solver's history: lbfgs_m pairs (s, y) of full DOF vectors
    c->free_list(c->lbfgs_allocs);
    c->lbfgs_alloc_m = 0;
    const size_t nd = (size_t)c->n_v * c->dim * (size_t)c->lbfgs_m;
    ISB_TRY(dalloc(c->lbfgs_allocs, &c->w_lbS, nd));
    ISB_TRY(dalloc(c->lbfgs_allocs, &c->w_lbY, nd));
    ISB_HIP(hipMemset(c->w_lbS, 0, nd * sizeof(double)));
    ISB_HIP(hipMemset(c->w_lbY, 0, nd * sizeof(double)));
    c->lbfgs_alloc_m = c->lbfgs_m;
  }
  isb_status worst = ISB_OK;
  for (int b = 0; b < c->n_bodies; ++b) {
    const BodyRange br = body_range(c, b);
    isb_stats st;
    std::memset(&st, 0, sizeof(st));
    double *x = c->w_x, *xt = c->w_xt, *G = c->w_G, *Gt = c->w_Gt;
    launch_setup(m, dsc, br.v0, br.v1, x0, dsc.be ? v0 : nullptr, x, c->w_xhat, c->w_cv, s);
    isb_status r = c->forward == ISB_FORWARD_LBFGS ? plain_lbfgs(c, b, s, x0, a, &x, &xt, &G, &Gt, &st)
                                                   : plain_newton(c, b, s, x0, a, &x, &xt, &G, &Gt, &st);
    if (r == ISB_E_HIP) return r;
    launch_copy(br.n, x + br.off, x1 + br.off, s);
    if (dsc.be && v1) launch_velocity(br.n, x1 + br.off, x0 + br.off, 1.0 / dsc.h, v1 + br.off, s);
    if (per_body) {
      ISB_TRY(fill_stats_tail(c, b, s, x, x0, a, &st));
      per_body[b] = st;
    }
    if (r != ISB_OK && worst == ISB_OK) worst = r;
  }
  if (worst != ISB_OK) return worst;
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

static isb_status plain_adjoint(isb_ctx* c, hipStream_t s, const double* x1, const double* x0, const double* a,
                                const double* x1_bar, const double* v1_bar, double* w, isb_stats* per_body) {
  const TraceRange trace("isb: adjoint, plain");
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  if (c->precision == ISB_MIXED) launch_to_f32(c->n_e, a, c->w_a32, s);
  isb_status worst = ISB_OK;
  for (int b = 0; b < c->n_bodies; ++b) {
    const BodyRange br = body_range(c, b);
    launch_setup(m, dsc, br.v0, br.v1, x0, nullptr, c->w_x, c->w_xhat, c->w_cv, s);
    launch_adjoint_rhs(m, dsc, br.v0, br.v1, x1_bar, dsc.be ? v1_bar : nullptr, c->w_G, s);
    enqueue_norm2(c, b, c->w_G, 0, s);
    ISB_TRY(read_scal(c, s, 1));
    const double bnorm = std::sqrt(c->hscal[0]);
    int iters = 0;
    bool neg = false;
    double rr = 0.0;
    if (!std::isfinite(bnorm)) return fail(ISB_E_NONFINITE, "non-finite adjoint right-hand side");
    if (bnorm == 0.0) {
      launch_fill(br.n, 0.0, w + br.off, s);
    } else {
      eval_precond(c, b, x1, a, s);
      if (c->adj_warm) {
        // start from the caller's w: CG solves H d = b - H w for the correction d, whose residual is
        // that of H (w + d) = b, so the tolerance stays relative to |b|
        launch_mask(m, br.v0, br.v1, w, s);
        launch_copy(br.n, w + br.off, c->w_p + br.off, s);
        launch_mul(br.n, c->w_vdiag + br.off, c->w_p + br.off, c->w_Hp + br.off, s);
        elem_scatter(c, b, PATCH_HV, x1, a, c->w_p, c->w_Hp, nullptr, s, c->w_a32);
        launch_mask(m, br.v0, br.v1, c->w_Hp, s);
        launch_axpy(br.n, c->w_G + br.off, -1.0, c->w_Hp + br.off, s);
      }
      ISB_TRY(run_cg(c, b, x1, a, c->w_G, 1.0, c->scene.adj_tol_rel * bnorm, c->scene.max_cg, s, &iters, &neg, &rr));
      if (!neg && c->precision == ISB_MIXED && single_reduction_cg(c, b)) {
        // The single-reduction CG carries H p in a recurrence (s = w + beta s), in which the FP32
        // operator's rounding accumulates: its recursive residual can fall below the tolerance before
        // the true one does. Check the true residual G - H xs once and, if it is too large, solve for
        // the correction from there (the adjoint is the solve whose accuracy the gradient inherits).
        double* xs0 = c->w_Gt;
        double* rt = c->w_xt;
        launch_copy(br.n, c->w_xs + br.off, xs0 + br.off, s);
        launch_mul(br.n, c->w_vdiag + br.off, xs0 + br.off, c->w_Hp + br.off, s);
        elem_scatter(c, b, PATCH_HV, x1, a, xs0, c->w_Hp, nullptr, s, c->w_a32);
        launch_mask(m, br.v0, br.v1, c->w_Hp, s);
        launch_copy(br.n, c->w_G + br.off, rt + br.off, s);
        launch_axpy(br.n, rt + br.off, -1.0, c->w_Hp + br.off, s);
        enqueue_norm2(c, b, rt, 0, s);
        ISB_TRY(read_scal(c, s, 1));
        const double true_res = std::sqrt(c->hscal[0]);
        if (true_res > c->scene.adj_tol_rel * bnorm) {
          int it2 = 0;
          ISB_TRY(run_cg(c, b, x1, a, rt, 1.0, c->scene.adj_tol_rel * bnorm, c->scene.max_cg, s, &it2, &neg, &rr));
          iters += it2;
          launch_axpy(br.n, c->w_xs + br.off, 1.0, xs0 + br.off, s);
        } else {
          rr = true_res * true_res;
        }
      }
      if (c->adj_warm)
        launch_axpy(br.n, w + br.off, 1.0, c->w_xs + br.off, s);
      else
        launch_copy(br.n, c->w_xs + br.off, w + br.off, s);
    }
    const double rel = bnorm > 0.0 ? std::sqrt(rr) / bnorm : 0.0;
    const bool ok = rel <= c->scene.adj_tol_rel && !neg;
    if (per_body) {
      per_body[b].adj_cg_iters = iters;
      per_body[b].adj_res_final = rel;
      if (ok)
        per_body[b].flags |= ISB_FLAG_ADJ_CONVERGED;
      else
        per_body[b].flags &= ~ISB_FLAG_ADJ_CONVERGED;
    }
    if (neg && worst == ISB_OK) worst = fail(ISB_E_NOT_CONVERGED, "adjoint CG met non-positive curvature");
    if (!ok && !neg && worst == ISB_OK) worst = fail(ISB_E_NOT_CONVERGED, "adjoint CG iteration cap reached");
  }
  ISB_HIP(hipGetLastError());
  return worst;
}

// ---------------------------------------------------------------------------------------------
// workspace allocation
// ---------------------------------------------------------------------------------------------
static isb_status alloc_workspaces(isb_ctx* c) {
  c->free_list(c->work_allocs);
  c->free_list(c->lbfgs_allocs);
  c->w_lbS = c->w_lbY = nullptr;
  c->lbfgs_alloc_m = 0;
  const size_t nd = (size_t)c->n_v * c->dim;
  auto& L = c->work_allocs;
  for (double** p : {&c->w_x, &c->w_xt, &c->w_xhat, &c->w_G, &c->w_Gt, &c->w_xs, &c->w_r, &c->w_p, &c->w_Hp,
                     &c->w_Dinvp, &c->w_vdiag, &c->w_diag, &c->w_u, &c->w_s})
    ISB_TRY(dalloc(L, p, nd));
  ISB_TRY(dalloc(L, &c->hv_part, (size_t)std::max(1, std::min(c->n_patches, kMaxPatchGrid))));
  ISB_TRY(dalloc(L, &c->w_cv, (size_t)c->n_v));
  ISB_TRY(dalloc(L, &c->w_a32, (size_t)c->n_e));
  ISB_TRY(dalloc(L, &c->partials, (size_t)12 * kMaxRedBlocks));
  ISB_TRY(dalloc(L, &c->dscal, (size_t)64));
  ISB_TRY(dalloc(L, &c->ebuf, (size_t)3 * c->n_bodies));
  ISB_TRY(dalloc(L, &c->scal, (size_t)1));
  ISB_TRY(dalloc(L, &c->gbar, (size_t)1));
  // zero the vectors once so that the Hessian-vector kernel never reads uninitialised memory
  for (double* p : {c->w_x, c->w_xt, c->w_xhat, c->w_G, c->w_Gt, c->w_xs, c->w_r, c->w_p, c->w_Hp, c->w_Dinvp,
                    c->w_vdiag, c->w_diag, c->w_u, c->w_s})
    ISB_HIP(hipMemset(p, 0, nd * sizeof(double)));
  ISB_HIP(hipMemset(c->scal, 0, sizeof(CgScal)));
  return ISB_OK;
}

// ---------------------------------------------------------------------------------------------
// the Hessian-vector product of isb_hessvec and isb_hessvec_noalloc
// ---------------------------------------------------------------------------------------------
// Device memory the product stages besides its inputs and output: the friction factor cv [n_v],
// the vertex-term diagonal vdiag [n_v*dim], the masked operand pm [n_v*dim] and, in mixed
// precision, the FP32 actuation a32 [n_e]. Every entry is written before it is read.
struct HvScratch {
  double *cv, *vdiag, *pm;
  float* a32;
};

// hp = P H(x) P p: vertex terms from the friction factor of x0, then the elements (and springs)
static void enqueue_hessvec(isb_ctx* c, hipStream_t s, const double* x, const double* x0, const double* a,
                            const double* p, double* hp, const HvScratch& w) {
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  const int n = c->n_v * c->dim;
  if (c->precision == ISB_MIXED) launch_to_f32(c->n_e, a, w.a32, s);
  launch_setup(m, dsc, 0, c->n_v, x0, nullptr, nullptr, nullptr, w.cv, s);
  launch_vertex_hdiag(m, dsc, 0, c->n_v, x, w.cv, w.vdiag, s);
  launch_copy(n, p, w.pm, s);
  launch_mask(m, 0, c->n_v, w.pm, s);
  launch_mul(n, w.vdiag, w.pm, hp, s);
  elem_scatter(c, -1, PATCH_HV, x, a, w.pm, hp, nullptr, s, w.a32);
  launch_mask(m, 0, c->n_v, hp, s);
}

// Scratch of isb_hessvec_noalloc: a fixed array in device memory, one copy per GPU for the life of
// the process, shared by every call on that GPU (calls that overlap on one GPU race on it). Host
// code must not pass the array's name to a kernel: its device address is resolved per device with
// hipGetSymbolAddress (scratch_resolve, called by isb_create with the device current) and only that
// address is used.
static constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];
static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxScratchDevices] = {};

static isb_status scratch_resolve(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return fail(ISB_E_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return ISB_OK;
  void* ptr = nullptr;
  ISB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(ISB_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_dev[device] = ptr;
  return ISB_OK;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_dev[device];
}

// word offsets of HvScratch inside the scratch array, each segment 256-byte aligned
struct NoallocLayout {
  size_t cv, vdiag, pm, a32, words;
};

static NoallocLayout noalloc_layout(const isb_ctx* c) {
  auto up = [](size_t w) { return (w + 31) / 32 * 32; };
  const size_t nv = (size_t)c->n_v, nd = nv * (size_t)c->dim;
  NoallocLayout L;
  L.cv = 0;
  L.vdiag = L.cv + up(nv);
  L.pm = L.vdiag + up(nd);
  L.a32 = L.pm + up(nd);
  L.words = L.a32 + (c->precision == ISB_MIXED ? up(((size_t)c->n_e + 1) / 2) : 0);
  return L;
}

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
extern "C" {

isb_status isb_create(int device, int precision, isb_ctx** out) {
  clear_error();
  if (!out) return fail(ISB_E_ARG, "NULL out pointer");
  *out = nullptr;
  if (precision != ISB_FP64 && precision != ISB_MIXED) return fail(ISB_E_ARG, "unknown precision");
  int n = 0;
  ISB_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(ISB_E_ARG, "device index out of range");
  ISB_HIP(hipSetDevice(device));
  ISB_TRY(scratch_resolve(device));
  isb_ctx* c = new isb_ctx();
  c->device = device;
  c->precision = precision;
  if (hipHostMalloc((void**)&c->hscal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->hcg, sizeof(CgScal), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->hcg_ring, 2 * sizeof(CgScal), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->cg_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->cg_ev[1], hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(ISB_E_HIP, "pinned host allocation or event creation failed");
  }
  *out = c;
  return ISB_OK;
}

isb_status isb_destroy(isb_ctx* ctx) {
  clear_error();
  if (!ctx) return ISB_OK;
  delete ctx;
  return ISB_OK;
}

// The resident CG plan (after the patch plan, on the context's device): one patch per compute
// unit for every body of at least kPatchMinElems elements whose patches fit the LDS a workgroup may
// hold; bodies far too large for that are not cut at all. Nothing is uploaded when no body qualifies.
static isb_status build_resident_plan(isb_ctx* c, const int32_t* T, const int64_t* body_e_off) {
  const int dim = c->dim, nb = c->n_bodies;
  c->res_ok.assign(nb, 0);
  c->res_patch_off.assign(nb + 1, 0);
  c->res_max_nv.assign(nb, 0);
  c->rplan = c->rplan_fixed = PatchPlan{};
  int n_cu = 0, max_lds = 0;
  ISB_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  ISB_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  // the partials of one solve (two banks of four per workgroup) live in the reduction workspace
  if (n_cu < 1 || 8 * n_cu > 12 * kMaxRedBlocks) return ISB_OK;
  const int max_verts = std::min(65535, max_lds / resident_vertex_bytes(dim));
  bool any = false;
  for (int b = 0; b < nb; ++b) {
    const int64_t ne_b = body_e_off[b + 1] - body_e_off[b];
    // a simplex mesh has at most about six elements per vertex: larger bodies cannot fit
    any |= ne_b >= kPatchMinElems && ne_b <= (int64_t)n_cu * 8 * max_verts;
  }
  if (!any) return ISB_OK;
  Patches rp, rp0;
  std::vector<uint8_t> eligible;
  std::vector<int32_t> bpo0;
  ISB_TRY(build_resident_patches(dim, c->n_v, nb, c->voff.data(), body_e_off, T, n_cu, max_verts, true, &rp,
                                 &c->res_patch_off, &eligible));
  int n_ok = 0;
  for (int b = 0; b < nb; ++b) {
    c->res_ok[b] = eligible[b] && body_e_off[b + 1] - body_e_off[b] >= kPatchMinElems;
    for (int k = c->res_patch_off[b]; k < c->res_patch_off[b + 1]; ++k)
      c->res_max_nv[b] = std::max(c->res_max_nv[b], rp.voff[k + 1] - rp.voff[k]);
    n_ok += c->res_ok[b];
  }
  if (n_ok == 0) return ISB_OK;
  // the same patches with the elements left in place (their vertex sets and owners are the same)
  std::vector<uint8_t> eligible0;
  ISB_TRY(build_resident_patches(dim, c->n_v, nb, c->voff.data(), body_e_off, T, n_cu, max_verts, false, &rp0,
                                 &bpo0, &eligible0));
  if (bpo0 != c->res_patch_off || rp0.eoff != rp.eoff || rp0.voff != rp.voff || rp0.nshared != rp.nshared)
    return fail(ISB_E_STATE, "resident plan: the two patch orders disagree");
  auto& L = c->mesh_allocs;
  int32_t *r_eoff, *r_voff, *r_verts, *r_eperm, *r_verts0, *r_nsh;
  uint16_t *r_lconn, *r_lconn0;
  ISB_TRY(dalloc(L, &r_nsh, rp.nshared.size()));
  ISB_HIP(hipMemcpy(r_nsh, rp.nshared.data(), rp.nshared.size() * 4, hipMemcpyHostToDevice));
  ISB_TRY(dalloc(L, &r_eperm, rp.eperm.size()));
  ISB_HIP(hipMemcpy(r_eperm, rp.eperm.data(), rp.eperm.size() * 4, hipMemcpyHostToDevice));
  ISB_TRY(dalloc(L, &r_verts0, rp0.verts.size()));
  ISB_HIP(hipMemcpy(r_verts0, rp0.verts.data(), rp0.verts.size() * 4, hipMemcpyHostToDevice));
  ISB_TRY(dalloc(L, &r_lconn0, rp0.lconn.size()));
  ISB_HIP(hipMemcpy(r_lconn0, rp0.lconn.data(), rp0.lconn.size() * 2, hipMemcpyHostToDevice));
  ISB_TRY(dalloc(L, &r_eoff, rp.eoff.size()));
  ISB_TRY(dalloc(L, &r_voff, rp.voff.size()));
  ISB_TRY(dalloc(L, &r_verts, rp.verts.size()));
  ISB_TRY(dalloc(L, &r_lconn, rp.lconn.size()));
  ISB_HIP(hipMemcpy(r_eoff, rp.eoff.data(), rp.eoff.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(r_voff, rp.voff.data(), rp.voff.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(r_verts, rp.verts.data(), rp.verts.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(r_lconn, rp.lconn.data(), rp.lconn.size() * 2, hipMemcpyHostToDevice));
  c->rplan = PatchPlan{r_eoff, r_voff, r_verts, r_lconn, rp.max_nv, 0, r_eperm, r_nsh};
  c->rplan_fixed = PatchPlan{r_eoff, r_voff, r_verts0, r_lconn0, rp0.max_nv, 0, nullptr, r_nsh};
  c->res_cu = n_cu;
  return ISB_OK;
}

isb_status isb_mesh_upload(isb_ctx* c, int dim, int32_t n_bodies, const int64_t* body_v_off,
                           const int64_t* body_e_off, const double* X_rest, const int32_t* T,
                           const uint8_t* dof_pinned) {
  clear_error();
  if (!c) return fail(ISB_E_ARG, "NULL context");
  if (!body_v_off || !body_e_off || !X_rest || !T || !dof_pinned || n_bodies <= 0)
    return fail(ISB_E_ARG, "NULL mesh argument");
  const int64_t n_v = body_v_off[n_bodies], n_e = body_e_off[n_bodies];
  ISB_TRY(validate_mesh(dim, n_v, X_rest, n_e, T, n_bodies, body_v_off, body_e_off));
  ISB_HIP(hipSetDevice(c->device));
  batched_release(c);
  c->free_list(c->work_allocs);
  c->free_list(c->lbfgs_allocs);
  c->w_lbS = c->w_lbY = nullptr;
  c->lbfgs_alloc_m = 0;
  c->free_list(c->mesh_allocs);
  c->have_mesh = c->have_material = false;
  c->dim = dim;
  c->uni_axis = -1;
  c->W32 = nullptr;
  c->n_bodies = n_bodies;
  c->n_v = (int)n_v;
  c->n_e = (int)n_e;
  c->voff.assign(body_v_off, body_v_off + n_bodies + 1);
  c->eoff.assign(body_e_off, body_e_off + n_bodies + 1);
  c->free_list(c->spring_allocs);
  c->n_s = c->n_scolours = 0;
  c->soff.assign(n_bodies + 1, 0);
  c->scol_off.clear();
  c->sconn = nullptr;
  c->sk = c->sil0 = nullptr;
  c->sclist = nullptr;

  // colouring, then per-(body, colour) element lists
  std::vector<int32_t> colour((size_t)n_e);
  int32_t nc = 0;
  ISB_TRY(colour_elements(dim, n_v, n_e, T, colour.data(), &nc));
  c->n_colours = nc;
  const int nc1 = nc + 1;
  c->col_off.assign((size_t)n_bodies * nc1, 0);
  std::vector<int32_t> clist((size_t)n_e);
  {
    int32_t pos = 0;
    for (int b = 0; b < n_bodies; ++b) {
      std::vector<int32_t> count(nc, 0);
      for (int64_t e = body_e_off[b]; e < body_e_off[b + 1]; ++e) count[colour[e]]++;
      std::vector<int32_t> start(nc, 0);
      for (int k = 0; k < nc; ++k) {
        c->col_off[b * nc1 + k] = pos;
        start[k] = pos;
        pos += count[k];
      }
      c->col_off[b * nc1 + nc] = pos;
      for (int64_t e = body_e_off[b]; e < body_e_off[b + 1]; ++e) clist[start[colour[e]]++] = (int32_t)e;
    }
  }

  // element patches for the LDS-staged scatter, sized to the patch workgroup's LDS budget
  Patches pt;
  {
    ISB_TRY(build_patches(dim, n_v, n_bodies, body_e_off, T, kPatchMaxElems, patch_max_verts(dim), &pt));
    c->n_patches = (int)pt.eoff.size() - 1;
    c->body_patch_off.assign(n_bodies + 1, 0);
    int k = 0;
    for (int b = 0; b <= n_bodies; ++b) {
      while (k < c->n_patches && pt.eoff[k] < body_e_off[b]) ++k;
      c->body_patch_off[b] = k;
    }
  }

  // SoA connectivity
  std::vector<int32_t> connh((size_t)(dim + 1) * n_e);
  for (int64_t e = 0; e < n_e; ++e)
    for (int k = 0; k <= dim; ++k) connh[(size_t)k * n_e + e] = T[e * (dim + 1) + k];

  auto& L = c->mesh_allocs;
  const size_t ne = (size_t)n_e, nd = (size_t)n_v * dim;
  ISB_TRY(dalloc(L, &c->conn, (size_t)(dim + 1) * ne));
  ISB_TRY(dalloc(L, &c->X, nd));
  ISB_TRY(dalloc(L, &c->Dinv, (size_t)dim * dim * ne));
  ISB_TRY(dalloc(L, &c->W, ne));
  ISB_TRY(dalloc(L, &c->gf, (size_t)dim * ne));
  ISB_TRY(dalloc(L, &c->wmu, ne));
  ISB_TRY(dalloc(L, &c->wlam, ne));
  ISB_TRY(dalloc(L, &c->wkf, ne));
  ISB_TRY(dalloc(L, &c->rho, ne));
  ISB_TRY(dalloc(L, &c->mass, (size_t)n_v));
  ISB_TRY(dalloc(L, &c->pinned, nd));
  ISB_TRY(dalloc(L, &c->clist, ne));
  int32_t *p_eoff, *p_voff, *p_verts;
  uint16_t* p_lconn;
  ISB_TRY(dalloc(L, &p_eoff, pt.eoff.size()));
  ISB_TRY(dalloc(L, &p_voff, pt.voff.size()));
  ISB_TRY(dalloc(L, &p_verts, pt.verts.size()));
  ISB_TRY(dalloc(L, &p_lconn, pt.lconn.size()));
  ISB_HIP(hipMemcpy(p_eoff, pt.eoff.data(), pt.eoff.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(p_voff, pt.voff.data(), pt.voff.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(p_verts, pt.verts.data(), pt.verts.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(p_lconn, pt.lconn.data(), pt.lconn.size() * 2, hipMemcpyHostToDevice));
  c->plan = PatchPlan{p_eoff, p_voff, p_verts, p_lconn, pt.max_nv};
  ISB_TRY(build_resident_plan(c, T, body_e_off));
  if (c->precision == ISB_MIXED) {
    ISB_TRY(dalloc(L, &c->W32, ne));
    ISB_TRY(dalloc(L, &c->Dinv32, (size_t)dim * dim * ne));
    ISB_TRY(dalloc(L, &c->gf32, (size_t)dim * ne));
    ISB_TRY(dalloc(L, &c->wmu32, ne));
    ISB_TRY(dalloc(L, &c->wlam32, ne));
    ISB_TRY(dalloc(L, &c->wkf32, ne));
  }
  ISB_HIP(hipMemcpy(c->conn, connh.data(), connh.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(c->X, X_rest, nd * sizeof(double), hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(c->pinned, dof_pinned, nd, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(c->clist, clist.data(), ne * sizeof(int32_t), hipMemcpyHostToDevice));
  launch_precompute_geom(dim, (int)n_e, c->X, c->conn, c->Dinv, c->W, nullptr);
  if (c->W32) launch_to_f32((int)n_e, c->W, c->W32, nullptr);
  ISB_HIP(hipGetLastError());
  ISB_HIP(hipDeviceSynchronize());
  ISB_TRY(alloc_workspaces(c));
  c->have_mesh = true;
  return ISB_OK;
}

isb_status isb_material_upload(isb_ctx* c, const double* mu, const double* lam, const double* k_fibre,
                               const double* fibre_dir, const double* density, const isb_scene* scene) {
  clear_error();
  ISB_TRY(check_ctx(c, false));
  if (!mu || !lam || !k_fibre || !fibre_dir || !density) return fail(ISB_E_ARG, "NULL material array");
  ISB_TRY(check_scene(scene));
  const size_t ne = (size_t)c->n_e;
  for (size_t e = 0; e < ne; ++e) {
    if (!std::isfinite(mu[e]) || !std::isfinite(lam[e]) || !std::isfinite(k_fibre[e]) || !(density[e] > 0.0) ||
        !std::isfinite(density[e]))
      return fail(ISB_E_ARG, "material entry " + std::to_string(e) + " invalid (density must be > 0)");
    double n2 = 0.0;
    for (int c2 = 0; c2 < c->dim; ++c2) n2 += fibre_dir[e * c->dim + c2] * fibre_dir[e * c->dim + c2];
    if (!(std::fabs(n2 - 1.0) < 1e-6)) return fail(ISB_E_ARG, "fibre_dir must be unit vectors");
  }
  std::vector<void*> tmp;
  double *dmu, *dlam, *dkf, *dfd;
  ISB_TRY(dalloc(tmp, &dmu, ne));
  ISB_TRY(dalloc(tmp, &dlam, ne));
  ISB_TRY(dalloc(tmp, &dkf, ne));
  ISB_TRY(dalloc(tmp, &dfd, ne * c->dim));
  isb_status st = ISB_OK;
  auto copy_all = [&]() -> isb_status {
    ISB_HIP(hipMemcpy(dmu, mu, ne * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(dlam, lam, ne * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(dkf, k_fibre, ne * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(dfd, fibre_dir, ne * c->dim * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(c->rho, density, ne * 8, hipMemcpyHostToDevice));
    launch_precompute_material(c->dim, c->n_e, c->Dinv, c->W, dfd, dmu, dlam, dkf, c->gf, c->wmu, c->wlam, c->wkf,
                               c->Dinv32, c->gf32, c->wmu32, c->wlam32, c->wkf32, nullptr);
    // lumped mass, one colour at a time so that the sum order is fixed
    ISB_HIP(hipMemset(c->mass, 0, (size_t)c->n_v * 8));
    const int nc1 = c->n_colours + 1;
    for (int b = 0; b < c->n_bodies; ++b)
      for (int k = 0; k < c->n_colours; ++k) {
        ERange r{c->col_off[b * nc1 + k], c->col_off[b * nc1 + k + 1], c->clist};
        launch_mass_colour(c->dim, r, c->conn, c->n_e, c->W, c->rho, c->mass, nullptr);
      }
    ISB_HIP(hipGetLastError());
    ISB_HIP(hipDeviceSynchronize());
    return ISB_OK;
  };
  st = copy_all();
  c->free_list(tmp);
  if (st != ISB_OK) return st;
  // compact rest record: one (mu, lam, k_f) for every element and every fibre along one coordinate axis
  c->uni_axis = -1;
  if (ne > 0) {
    int axis = -1;
    for (int k = 0; k < c->dim; ++k)
      if (fibre_dir[k] == 1.0) axis = k;
    bool uniform = axis >= 0;
    for (size_t e = 0; e < ne && uniform; ++e) {
      uniform = mu[e] == mu[0] && lam[e] == lam[0] && k_fibre[e] == k_fibre[0];
      for (int k = 0; k < c->dim && uniform; ++k) uniform = fibre_dir[e * c->dim + k] == (k == axis ? 1.0 : 0.0);
    }
    if (uniform) {
      c->uni_axis = axis;
      c->uni_mu = mu[0];
      c->uni_lam = lam[0];
      c->uni_kf = k_fibre[0];
    }
  }
  c->scene = *scene;
  c->have_material = true;
  batched_release(c);
  return ISB_OK;
}

isb_status isb_set_scene(isb_ctx* c, const isb_scene* scene) {
  clear_error();
  if (!c) return fail(ISB_E_ARG, "NULL context");
  ISB_TRY(check_scene(scene));
  c->scene = *scene;
  return ISB_OK;
}

isb_status isb_set_option(isb_ctx* c, int key, int64_t value) {
  clear_error();
  if (!c) return fail(ISB_E_ARG, "NULL context");
  switch (key) {
    case ISB_OPT_SOLVER:
      if (value != 0 && value != 1) return fail(ISB_E_ARG, "solver must be 0 or 1");
      c->solver = (int)value;
      return ISB_OK;
    case ISB_OPT_SCATTER:
      if (value < 0 || value > 2) return fail(ISB_E_ARG, "scatter must be 0, 1 or 2");
      c->scatter = (int)value;
      return ISB_OK;
    case ISB_OPT_GRAPH_SAFE:
      c->graph_safe = value != 0;
      return ISB_OK;
    case ISB_OPT_BLOCK:
      if (value != 0 && value != 256 && value != 512 && value != 768 && value != 1024)
        return fail(ISB_E_ARG, "block must be 0 (automatic), 256, 512, 768 or 1024");
      c->block = (int)value;
      return ISB_OK;
    case ISB_OPT_CG_CHECK:
      if (value < 1 || value > 1000) return fail(ISB_E_ARG, "cg_check must be in [1, 1000]");
      c->cg_check = (int)value;
      return ISB_OK;
    case ISB_OPT_ENERGY:
      if (value < ISB_ENERGY_NEOHOOKEAN || value > ISB_ENERGY_STABLE_NEOHOOKEAN)
        return fail(ISB_E_ARG, "energy must be one of ISB_ENERGY_*");
      c->model = (int)value;
      return ISB_OK;
    case ISB_OPT_CG_GRAPH:
      c->cg_graph = value != 0;
      return ISB_OK;
    case ISB_OPT_FP64_FALLBACK:
      if (value < 0 || value > 2) return fail(ISB_E_ARG, "fp64 fallback must be 0, 1 or 2");
      c->fp64_fallback = (int)value;
      return ISB_OK;
    case ISB_OPT_ADJ_WARM_START:
      if (value != 0 && value != 1) return fail(ISB_E_ARG, "adjoint warm start must be 0 or 1");
      c->adj_warm = (int)value;
      return ISB_OK;
    case ISB_OPT_CG_SINGLE_REDUCTION:
      if (value != 0 && value != 1) return fail(ISB_E_ARG, "single-reduction CG must be 0 or 1");
      c->cg_single = (int)value;
      return ISB_OK;
    case ISB_OPT_CG_RESIDENT:
      if (value != 0 && value != 1) return fail(ISB_E_ARG, "resident CG must be 0 or 1");
      c->cg_resident = (int)value;
      return ISB_OK;
    case ISB_OPT_CG_BARRIER_LIMIT_US:
      if (value < 1 || value > 60000000) return fail(ISB_E_ARG, "barrier limit must be in [1, 6e7] us");
      c->barrier_limit_us = value;
      return ISB_OK;
    case ISB_OPT_PATCH_BLOCK:
      if (value != 0 && value != 256 && value != 512 && value != 1024)
        return fail(ISB_E_ARG, "patch block must be 0 (default), 256, 512 or 1024");
      c->patch_block = (int)value;
      return ISB_OK;
    case ISB_OPT_COMPACT_REST:
      if (value != 0 && value != 1) return fail(ISB_E_ARG, "compact rest record must be 0 or 1");
      c->compact_rest = (int)value;
      batched_release(c);
      return ISB_OK;
    case ISB_OPT_FORWARD:
      if (value != ISB_FORWARD_NEWTON && value != ISB_FORWARD_LBFGS)
        return fail(ISB_E_ARG, "forward must be ISB_FORWARD_NEWTON or ISB_FORWARD_LBFGS");
      c->forward = (int)value;
      return ISB_OK;
    case ISB_OPT_LBFGS_MEMORY:
      if (value < 1 || value > 64) return fail(ISB_E_ARG, "lbfgs memory must be in [1, 64]");
      c->lbfgs_m = (int)value;
      return ISB_OK;
    case ISB_OPT_LBFGS_MAX_ITERS:
      if (value < 1 || value > 10000000) return fail(ISB_E_ARG, "lbfgs iteration cap must be in [1, 1e7]");
      c->lbfgs_max_iters = (int)value;
      return ISB_OK;
    default:
      return fail(ISB_E_ARG, "unknown or read-only option key " + std::to_string(key));
  }
}

isb_status isb_get_option(isb_ctx* c, int key, int64_t* value) {
  clear_error();
  if (!c || !value) return fail(ISB_E_ARG, "NULL argument");
  switch (key) {
    case ISB_OPT_SOLVER: *value = c->solver; return ISB_OK;
    case ISB_OPT_SCATTER: *value = c->scatter; return ISB_OK;
    case ISB_OPT_GRAPH_SAFE: *value = c->graph_safe; return ISB_OK;
    case ISB_OPT_BLOCK: *value = c->block > 0 ? c->block : (c->dim == 3 ? 512 : 768); return ISB_OK;
    case ISB_OPT_CG_CHECK: *value = c->cg_check; return ISB_OK;
    case ISB_OPT_PRECISION: *value = c->precision; return ISB_OK;
    case ISB_OPT_ENERGY: *value = c->model; return ISB_OK;
    case ISB_OPT_FORWARD: *value = c->forward; return ISB_OK;
    case ISB_OPT_CG_GRAPH: *value = c->cg_graph; return ISB_OK;
    case ISB_OPT_FP64_FALLBACK: *value = c->fp64_fallback; return ISB_OK;
    case ISB_OPT_ADJ_WARM_START: *value = c->adj_warm; return ISB_OK;
    case ISB_OPT_COMPACT_REST: *value = c->compact_rest; return ISB_OK;
    case ISB_OPT_PATCH_BLOCK: *value = c->patch_block; return ISB_OK;
    case ISB_OPT_CG_SINGLE_REDUCTION: *value = c->cg_single; return ISB_OK;
    case ISB_OPT_CG_RESIDENT: *value = c->cg_resident; return ISB_OK;
    case ISB_OPT_CG_BARRIER_LIMIT_US: *value = c->barrier_limit_us; return ISB_OK;
    case ISB_INFO_RESIDENT: {
      int64_t n = 0;
      for (uint8_t ok : c->res_ok) n += ok;
      *value = n;
      return ISB_OK;
    }
    case ISB_INFO_COMPACT_AXIS: *value = c->have_material && c->compact_rest ? c->uni_axis : -1; return ISB_OK;
    case ISB_OPT_LBFGS_MEMORY: *value = c->lbfgs_m; return ISB_OK;
    case ISB_OPT_LBFGS_MAX_ITERS: *value = c->lbfgs_max_iters; return ISB_OK;
    case ISB_INFO_N_VERTICES: *value = c->n_v; return ISB_OK;
    case ISB_INFO_N_ELEMENTS: *value = c->n_e; return ISB_OK;
    case ISB_INFO_N_BODIES: *value = c->n_bodies; return ISB_OK;
    case ISB_INFO_DIM: *value = c->dim; return ISB_OK;
    case ISB_INFO_N_COLOURS: *value = c->n_colours; return ISB_OK;
    case ISB_INFO_LDS_BYTES: *value = c->have_mesh ? batched_lds_bytes(c) : 0; return ISB_OK;
    default: return fail(ISB_E_ARG, "unknown option key " + std::to_string(key));
  }
}

isb_status isb_get_mass(isb_ctx* c, isb_stream stream, double* mass_out) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!mass_out) return fail(ISB_E_ARG, "NULL output");
  ISB_HIP(hipMemcpyAsync(mass_out, c->mass, (size_t)c->n_v * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return ISB_OK;
}

isb_status isb_step(isb_ctx* c, isb_stream stream, const double* x0, const double* v0, const double* a, double* x1,
                    double* v1, isb_stats* per_body) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  const bool be = c->scene.integrator == ISB_BACKWARD_EULER;
  if (!x0 || !a || !x1 || (be && !v0)) return fail(ISB_E_ARG, "NULL state argument");
  hipStream_t s = (hipStream_t)stream;
  if (per_body) std::memset(per_body, 0, sizeof(isb_stats) * c->n_bodies);
  if (c->solver == 1) {
    if (c->forward != ISB_FORWARD_NEWTON)
      return fail(ISB_E_ARG, "the batched solver runs Newton-PCG only (ISB_OPT_FORWARD)");
    const TraceRange trace("isb: step, batched");
    return batched_step(c, s, x0, be ? v0 : nullptr, a, x1, be ? v1 : nullptr, per_body);
  }
  ISB_TRY(check_actuation(c, s, a));
  return plain_step(c, s, x0, v0, a, x1, v1, per_body);
}

isb_status isb_solve_adjoint(isb_ctx* c, isb_stream stream, const double* x1, const double* x0, const double* a,
                             const double* x1_bar, const double* v1_bar, double* w, isb_stats* per_body) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x1 || !x0 || !a || !x1_bar || !w) return fail(ISB_E_ARG, "NULL adjoint argument");
  hipStream_t s = (hipStream_t)stream;
  if (c->solver == 1) {
    const TraceRange trace("isb: adjoint, batched");
    return batched_adjoint(c, s, x1, x0, a, x1_bar, v1_bar, w, per_body);
  }
  ISB_TRY(check_actuation(c, s, a));
  return plain_adjoint(c, s, x1, x0, a, x1_bar, v1_bar, w, per_body);
}

isb_status isb_vjp_params(isb_ctx* c, isb_stream stream, const double* w, const double* x1, const double* x0,
                          const double* a, const double* v1_bar, double* a_bar, double* x0_bar, double* v0_bar,
                          double* mu_bar, double* lam_bar, double* kf_bar) {
  const TraceRange trace("isb: VJP");
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!w || !x1 || !x0 || !a) return fail(ISB_E_ARG, "NULL vjp argument");
  hipStream_t s = (hipStream_t)stream;
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  if (a_bar || mu_bar || lam_bar || kf_bar)
    launch_elem_vjp(m, dsc, ERange{0, c->n_e, nullptr}, w, x1, a, a_bar, mu_bar, lam_bar, kf_bar, s);
  if (a_bar && c->n_s > 0)
    launch_spring_vjp(c->dim, devsprings(c), dsc, ERange{0, c->n_s, nullptr}, w, x1, a + c->n_e, a_bar + c->n_e,
                      nullptr, s);
  launch_vertex_vjp(m, dsc, 0, c->n_v, w, x1, x0, dsc.be ? v1_bar : nullptr, x0_bar, v0_bar, s);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_vjp_spring_stiffness(isb_ctx* c, isb_stream stream, const double* w, const double* x1,
                                    const double* a, double* k_bar) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!w || !x1 || !a || !k_bar) return fail(ISB_E_ARG, "NULL vjp argument");
  launch_spring_vjp(c->dim, devsprings(c), devscene(c), ERange{0, c->n_s, nullptr}, w, x1, a + c->n_e, nullptr, k_bar,
                    (hipStream_t)stream);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_spring_upload(isb_ctx* c, int64_t n_s, const int64_t* body_s_off, const int32_t* pairs,
                             const double* k) {
  clear_error();
  if (!c) return fail(ISB_E_ARG, "NULL context");
  if (!c->have_mesh) return fail(ISB_E_STATE, "isb_spring_upload needs the mesh first");
  if (n_s < 0 || n_s > INT32_MAX / 2) return fail(ISB_E_ARG, "spring count out of range");
  if (n_s > 0 && (!pairs || !k)) return fail(ISB_E_ARG, "NULL spring array");
  const int nb = c->n_bodies;
  std::vector<int64_t> soff(nb + 1, 0);
  if (body_s_off) {
    soff.assign(body_s_off, body_s_off + nb + 1);
  } else if (nb == 1) {
    soff[1] = n_s;
  } else {
    return fail(ISB_E_ARG, "body_s_off is required with several bodies");
  }
  if (soff[0] != 0 || soff[nb] != n_s) return fail(ISB_E_ARG, "body_s_off must run from 0 to n_s");
  for (int b = 0; b < nb; ++b)
    if (soff[b + 1] < soff[b]) return fail(ISB_E_ARG, "body_s_off must be non-decreasing");
  // rest lengths from the uploaded rest positions
  const int D = c->dim;
  std::vector<double> X((size_t)c->n_v * D);
  ISB_HIP(hipSetDevice(c->device));
  ISB_HIP(hipMemcpy(X.data(), c->X, X.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<int32_t> connh((size_t)2 * n_s);
  std::vector<double> il0((size_t)n_s);
  for (int b = 0; b < nb; ++b)
    for (int64_t s = soff[b]; s < soff[b + 1]; ++s) {
      const int32_t i = pairs[2 * s], j = pairs[2 * s + 1];
      if (i < c->voff[b] || i >= c->voff[b + 1] || j < c->voff[b] || j >= c->voff[b + 1])
        return fail(ISB_E_MESH, "spring " + std::to_string(s) + " joins vertices outside its body");
      if (i == j) return fail(ISB_E_MESH, "spring " + std::to_string(s) + " joins a vertex to itself");
      if (!std::isfinite(k[s]) || k[s] < 0.0)
        return fail(ISB_E_ARG, "spring " + std::to_string(s) + " needs a finite stiffness >= 0");
      double l2 = 0.0;
      for (int r = 0; r < D; ++r) {
        const double d = X[(size_t)j * D + r] - X[(size_t)i * D + r];
        l2 += d * d;
      }
      if (!(l2 > 0.0)) return fail(ISB_E_MESH, "spring " + std::to_string(s) + " has zero rest length");
      il0[s] = 1.0 / std::sqrt(l2);
      connh[s] = i;
      connh[(size_t)n_s + s] = j;
    }
  // colouring (pairs are elements of two vertices), then per-(body, colour) lists
  std::vector<int32_t> colour((size_t)n_s);
  int32_t nc = 0;
  if (n_s > 0) ISB_TRY(colour_elements(1, c->n_v, n_s, pairs, colour.data(), &nc));
  const int nc1 = nc + 1;
  std::vector<int32_t> scol_off((size_t)nb * nc1, 0), sclist((size_t)n_s);
  {
    int32_t pos = 0;
    for (int b = 0; b < nb; ++b) {
      std::vector<int32_t> start(nc, 0), count(nc, 0);
      for (int64_t s = soff[b]; s < soff[b + 1]; ++s) count[colour[s]]++;
      for (int q = 0; q < nc; ++q) {
        scol_off[b * nc1 + q] = pos;
        start[q] = pos;
        pos += count[q];
      }
      scol_off[b * nc1 + nc] = pos;
      for (int64_t s = soff[b]; s < soff[b + 1]; ++s) sclist[start[colour[s]]++] = (int32_t)s;
    }
  }
  batched_release(c);
  c->free_list(c->spring_allocs);
  c->sconn = nullptr;
  c->sk = c->sil0 = nullptr;
  c->sclist = nullptr;
  c->n_s = 0;
  if (n_s > 0) {
    auto& L = c->spring_allocs;
    ISB_TRY(dalloc(L, &c->sconn, (size_t)2 * n_s));
    ISB_TRY(dalloc(L, &c->sk, (size_t)n_s));
    ISB_TRY(dalloc(L, &c->sil0, (size_t)n_s));
    ISB_TRY(dalloc(L, &c->sclist, (size_t)n_s));
    ISB_HIP(hipMemcpy(c->sconn, connh.data(), connh.size() * 4, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(c->sk, k, (size_t)n_s * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(c->sil0, il0.data(), (size_t)n_s * 8, hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(c->sclist, sclist.data(), (size_t)n_s * 4, hipMemcpyHostToDevice));
  }
  c->n_s = (int)n_s;
  c->n_scolours = nc;
  c->soff = soff;
  c->scol_off = scol_off;
  return ISB_OK;
}

isb_status isb_autotune(isb_ctx* c, isb_stream stream, const double* x0, const double* v0, const double* a,
                        int64_t* chosen_out) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  const bool be = c->scene.integrator == ISB_BACKWARD_EULER;
  if (!x0 || !a || (be && !v0)) return fail(ISB_E_ARG, "NULL state argument");
  hipStream_t s = (hipStream_t)stream;
  // candidates: the batched solver's workgroup size (the alternative energies have one size only),
  // the plain solver's scatter (atomic or LDS-staged patches; the colour mode is for reproducibility)
  const bool batched = c->solver == 1;
  std::vector<int> cand;
  if (batched)
    cand = c->model == ISB_ENERGY_NEOHOOKEAN ? std::vector<int>{512, 768, 1024} : std::vector<int>{0};
  else
    cand = {0, 2};
  const int keep_block = c->block, keep_scatter = c->scatter;
  const size_t nd = (size_t)c->n_v * c->dim;
  double *x1 = nullptr, *v1 = nullptr;
  ISB_HIP(hipMalloc(&x1, nd * sizeof(double)));
  if (hipMalloc(&v1, nd * sizeof(double)) != hipSuccess) {
    (void)hipFree(x1);
    return fail(ISB_E_HIP, "isb_autotune: out of device memory");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int best = -1;
  float best_ms = 0.0f;
  isb_status st = ISB_OK;
  for (int v : cand) {
    if (batched)
      c->block = v;
    else
      c->scatter = v;
    float ms = 0.0f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {  // the first run prepares state and warms the caches
      (void)hipEventRecord(e0, s);
      const isb_status r = isb_step(c, stream, x0, v0, a, x1, be ? v1 : nullptr, nullptr);
      (void)hipEventRecord(e1, s);
      if (r != ISB_OK && r != ISB_E_NOT_CONVERGED) {
        ok = false;  // this configuration cannot run on the context (e.g. too little LDS)
        break;
      }
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(ISB_E_HIP, "isb_autotune: event timing failed");
        ok = false;
      }
    }
    if (st != ISB_OK) break;
    if (ok && (best < 0 || ms < best_ms)) {
      best = v;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x1);
  (void)hipFree(v1);
  c->block = keep_block;
  c->scatter = keep_scatter;
  if (st != ISB_OK) return st;
  if (best < 0) return fail(ISB_E_ARG, "isb_autotune: no candidate configuration ran");
  if (batched)
    c->block = best;
  else
    c->scatter = best;
  clear_error();
  if (chosen_out) {
    chosen_out[0] = batched ? ISB_OPT_BLOCK : ISB_OPT_SCATTER;
    chosen_out[1] = best;
  }
  return ISB_OK;
}

isb_status isb_energy(isb_ctx* c, isb_stream stream, const double* x, const double* x0, const double* v0,
                      const double* a, double* energy) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  const DevScene dsc = devscene(c);
  if (!x || !x0 || !a || !energy || (dsc.be && !v0)) return fail(ISB_E_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const DevMesh m = devmesh(c);
  launch_setup(m, dsc, 0, c->n_v, x0, dsc.be ? v0 : nullptr, c->w_xt, c->w_xhat, c->w_cv, s);
  for (int b = 0; b < c->n_bodies; ++b) enqueue_energy(c, b, x, nullptr, 0.0, x0, a, c->ebuf + 3 * b, s);
  ISB_HIP(hipMemcpy2DAsync(energy, sizeof(double), c->ebuf + 2, 3 * sizeof(double), sizeof(double), c->n_bodies,
                           hipMemcpyDeviceToDevice, s));
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_gradient(isb_ctx* c, isb_stream stream, const double* x, const double* x0, const double* v0,
                        const double* a, double* g) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  const DevScene dsc = devscene(c);
  if (!x || !x0 || !a || !g || (dsc.be && !v0)) return fail(ISB_E_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  launch_setup(devmesh(c), dsc, 0, c->n_v, x0, dsc.be ? v0 : nullptr, c->w_xt, c->w_xhat, c->w_cv, s);
  eval_grad(c, -1, x, x0, a, g, s);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_hessvec(isb_ctx* c, isb_stream stream, const double* x, const double* x0, const double* a,
                       const double* p, double* hp) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x || !x0 || !a || !p || !hp) return fail(ISB_E_ARG, "NULL argument");
  enqueue_hessvec(c, (hipStream_t)stream, x, x0, a, p, hp, HvScratch{c->w_cv, c->w_vdiag, c->w_p, c->w_a32});
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_hessvec_noalloc(isb_ctx* c, isb_stream stream, const double* x, const double* x0, const double* a,
                               const double* p, double* hp) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x || !x0 || !a || !p || !hp) return fail(ISB_E_ARG, "NULL argument");
  double* base = static_cast<double*>(scratch_ptr(c->device));
  if (!base) return fail(ISB_E_STATE, "isb_hessvec_noalloc: scratch of this device not resolved");
  const NoallocLayout L = noalloc_layout(c);
  if (L.words * sizeof(double) > kNoallocScratchBytes)
    return fail(ISB_E_ARG, "isb_hessvec_noalloc: the mesh needs " + std::to_string(L.words * sizeof(double)) +
                               " B of scratch, the maximum is " + std::to_string(kNoallocScratchBytes) + " B");
  const HvScratch w{base + L.cv, base + L.vdiag, base + L.pm,
                    c->precision == ISB_MIXED ? reinterpret_cast<float*>(base + L.a32) : nullptr};
  enqueue_hessvec(c, (hipStream_t)stream, x, x0, a, p, hp, w);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_hessvec_elements(isb_ctx* c, isb_stream stream, const double* x, const double* a,
                                const double* p, double* hp) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x || !a || !p || !hp) return fail(ISB_E_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  // one pass: the element kernels read the FP64 actuation directly (no FP32 copy)
  elem_scatter(c, -1, PATCH_HV, x, a, p, hp, nullptr, s);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_gradient_elements(isb_ctx* c, isb_stream stream, const double* x, const double* a, double* g) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x || !a || !g) return fail(ISB_E_ARG, "NULL argument");
  elem_scatter(c, -1, PATCH_GRAD, x, a, nullptr, g, nullptr, (hipStream_t)stream);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_hessdiag(isb_ctx* c, isb_stream stream, const double* x, const double* x0, const double* a,
                        double* diag) {
  clear_error();
  ISB_TRY(check_ctx(c, true));
  if (!x || !x0 || !a || !diag) return fail(ISB_E_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const DevMesh m = devmesh(c);
  const DevScene dsc = devscene(c);
  launch_setup(m, dsc, 0, c->n_v, x0, nullptr, c->w_xt, c->w_xhat, c->w_cv, s);
  launch_vertex_hdiag(m, dsc, 0, c->n_v, x, c->w_cv, diag, s);
  elem_scatter(c, -1, PATCH_DIAG, x, a, nullptr, diag, nullptr, s);
  launch_set_pinned(m, 0, c->n_v, 1.0, diag, s);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

isb_status isb_stream_copy(isb_stream stream, const double* src, double* dst, int64_t n) {
  clear_error();
  if (n < 0 || (n > 0 && (!src || !dst))) return fail(ISB_E_ARG, "isb_stream_copy: bad argument");
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(ISB_E_ARG, "isb_stream_copy: buffers must be 16-byte aligned");
  if (n > 0 && src < dst + n && dst < src + n) return fail(ISB_E_ARG, "isb_stream_copy: buffers overlap");
  launch_stream_copy(n, src, dst, (hipStream_t)stream);
  ISB_HIP(hipGetLastError());
  return ISB_OK;
}

}  // extern "C"
