// Batched persistent solver: many bodies of uneven size in one launch per phase (the
// body-level logic is in isb_body.hpp). Mixed precision: the Hessian-vector product and the
// diagonal evaluate elements in FP32 from FP32 rest data; gradients, energies, CG vectors, dot
// products, norms and the state are FP64. No host synchronisation happens inside a launch, so
// the launches are graph-capturable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <utility>
#include <vector>

#include "isb_batched_kernel.hpp"
#include "isb_ctx.hpp"

namespace isb {

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
struct BatchedState {
  std::vector<void*> allocs;
  int32_t *order = nullptr, *wg_off = nullptr, *voff = nullptr, *eoff = nullptr;
  DevStats* stats = nullptr;
  DevStats* hstats = nullptr;  // pinned host mirror
  void* Fbuf = nullptr;        // per-element Hessian-vector state in the element precision
  double *E0 = nullptr, *E1 = nullptr;  // per-element energies (iterate, trial)
  float* Dv = nullptr;                  // FP32 Jacobi preconditioner
  void* vdT = nullptr;                  // vertex-term diagonal, element precision
  uint16_t* lconn = nullptr;            // body-local connectivity
  int32_t* soff = nullptr;              // springs per body
  uint16_t* slconn = nullptr;           // body-local spring ends
  void* Sbuf = nullptr;                 // per-spring block K in the element precision
  int32_t *fb_order = nullptr, *fb_wgoff = nullptr;  // schedule of a fallback launch (FP64 state only)
  int nacc = 0, grid = 0, block = 0, precision = -1, dim = 0, model = 0;
  bool compact = false;  // the compact rest record (the kernel variant the launches take)
  size_t lds = 0;
};

static int default_block(int dim) { return batched_default_block(dim); }

// nullptr: no kernel of this configuration (an alternative energy model at another block size)
static void* pick_kernel(int dim, int precision, int mode, int block, int model, bool compact) {
  const int prec = precision == ISB_MIXED ? 1 : 0;
  return dim == 2 ? batched_kernel_2d(prec, mode, block, model, compact)
                  : batched_kernel_3d(prec, mode, block, model, compact);
}

// LDS of one workgroup: reduction slots, the FP64 accumulator and the FP64 CG direction, sized for
// the body with the most DOFs
int64_t batched_lds_bytes(const isb_ctx* c) {
  int64_t mx = 0;
  for (int b = 0; b < c->n_bodies; ++b) mx = std::max<int64_t>(mx, (c->voff[b + 1] - c->voff[b]) * c->dim);
  return (int64_t)(kRedSlots + 2 * mx) * (int64_t)sizeof(double);
}

static int64_t batched_max_dof(const isb_ctx* c) {
  int64_t mx = 0;
  for (int b = 0; b < c->n_bodies; ++b) mx = std::max<int64_t>(mx, (c->voff[b + 1] - c->voff[b]) * c->dim);
  return mx;
}

static void release_state(void** slot) {
  auto* st = static_cast<BatchedState*>(*slot);
  if (!st) return;
  for (void* p : st->allocs) (void)hipFree(p);
  if (st->hstats) (void)hipHostFree(st->hstats);
  delete st;
  *slot = nullptr;
}

void batched_release(isb_ctx* c) {
  release_state(&c->batched);
  release_state(&c->batched64);
}

// Cost of a body in element-equivalents for the static schedule: a fixed part per body (the
// vector passes, reductions and barriers of every CG iteration, which do not shrink with the
// body) plus its elements.
static constexpr double kBodyFixedCost = 1152.0;

// Longest-processing-time schedule: bodies in decreasing cost go, one at a time, to the
// workgroup with the least load so far (ties to the lowest index). Workgroup g solves
// order[wg_off[g] .. wg_off[g+1]) in that order. eoff: cumulative work items (elements and
// springs) per body.
static void lpt_schedule(const std::vector<int32_t>& eoff, int nb, int G, std::vector<int32_t>& order,
                         std::vector<int32_t>& wg_off) {
  std::vector<int32_t> byc(nb);
  std::iota(byc.begin(), byc.end(), 0);
  std::stable_sort(byc.begin(), byc.end(),
                   [&](int a, int b) { return (eoff[a + 1] - eoff[a]) > (eoff[b + 1] - eoff[b]); });
  using Load = std::pair<double, int>;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int g = 0; g < G; ++g) heap.push({0.0, g});
  std::vector<std::vector<int32_t>> lists(G);
  for (int b : byc) {
    Load l = heap.top();
    heap.pop();
    lists[l.second].push_back(b);
    heap.push({l.first + kBodyFixedCost + (double)(eoff[b + 1] - eoff[b]), l.second});
  }
  order.clear();
  wg_off.assign(1, 0);
  for (int g = 0; g < G; ++g) {
    order.insert(order.end(), lists[g].begin(), lists[g].end());
    wg_off.push_back((int32_t)order.size());
  }
}

// the batched state of one precision in *slot (the context's, or the FP64 fallback's)
static isb_status prepare_state(isb_ctx* c, void** slot, int precision) {
  auto* st = static_cast<BatchedState*>(*slot);
  const int want_block = c->block > 0 ? c->block : default_block(c->dim);
  const bool compact = devmesh(c).axis >= 0;
  if (st && st->block == want_block && st->precision == precision && st->dim == c->dim && st->model == c->model &&
      st->compact == compact)
    return ISB_OK;
  if (!pick_kernel(c->dim, precision, 0, want_block, c->model, compact))
    return fail(ISB_E_ARG, "batched solver: the alternative energy models run with the default workgroup size only");
  release_state(slot);
  st = new BatchedState();
  *slot = st;
  const int nb = c->n_bodies;
  st->lds = (size_t)batched_lds_bytes(c);
  st->nacc = (int)batched_max_dof(c);
  st->block = want_block;
  st->precision = precision;
  st->dim = c->dim;
  st->model = c->model;
  st->compact = compact;
  int max_lds = 0, n_cu = 0;
  ISB_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  ISB_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  if ((int64_t)st->lds > (int64_t)max_lds)
    return fail(ISB_E_ARG, "batched solver: the largest body needs " + std::to_string(st->lds) +
                               " B of LDS, the device allows " + std::to_string(max_lds) + " B per workgroup");
  int occ = 0;
  for (int mode = 0; mode < 2; ++mode) {
    void* k = pick_kernel(c->dim, precision, mode, st->block, c->model, compact);
    ISB_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)st->lds));
    int o = 0;
    ISB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, st->block, st->lds));
    occ = mode == 0 ? o : std::min(occ, o);
  }
  if (occ < 1) return fail(ISB_E_ARG, "batched solver: kernel does not fit one workgroup per CU");
  st->grid = std::min(nb, occ * n_cu);

  std::vector<int32_t> order, wg_off, voff(nb + 1), eoff(nb + 1);
  for (int b = 0; b <= nb; ++b) {
    voff[b] = (int32_t)c->voff[b];
    eoff[b] = (int32_t)c->eoff[b];
  }
  {
    std::vector<int32_t> work(nb + 1);
    for (int b = 0; b <= nb; ++b) work[b] = eoff[b] + (int32_t)c->soff[b];
    lpt_schedule(work, nb, st->grid, order, wg_off);
  }
  auto alloc = [&](void** p, size_t bytes) -> isb_status {
    ISB_HIP(hipMalloc(p, bytes));
    st->allocs.push_back(*p);
    return ISB_OK;
  };
  isb_status r;
  if ((r = alloc((void**)&st->order, nb * 4)) != ISB_OK) return r;
  if ((r = alloc((void**)&st->wg_off, (st->grid + 1) * 4)) != ISB_OK) return r;
  if ((r = alloc((void**)&st->voff, (nb + 1) * 4)) != ISB_OK) return r;
  if ((r = alloc((void**)&st->eoff, (nb + 1) * 4)) != ISB_OK) return r;
  if ((r = alloc((void**)&st->stats, nb * sizeof(DevStats))) != ISB_OK) return r;
  if ((r = alloc((void**)&st->fb_order, nb * 4)) != ISB_OK) return r;
  if ((r = alloc((void**)&st->fb_wgoff, (st->grid + 1) * 4)) != ISB_OK) return r;
  const size_t fwords = (size_t)hv_state_words(c->dim) * (size_t)c->n_e;
  if ((r = alloc(&st->Fbuf, fwords * (precision == ISB_MIXED ? 4 : 8))) != ISB_OK) return r;
  const size_t nterms = (size_t)c->n_e + (size_t)c->n_s;
  if ((r = alloc((void**)&st->E0, nterms * sizeof(double))) != ISB_OK) return r;
  if ((r = alloc((void**)&st->E1, nterms * sizeof(double))) != ISB_OK) return r;
  if (c->n_s > 0) {
    const size_t ns = (size_t)c->n_s;
    if ((r = alloc(&st->Sbuf, (size_t)spring_state_words(c->dim) * ns * (precision == ISB_MIXED ? 4 : 8))) != ISB_OK)
      return r;
    if ((r = alloc((void**)&st->soff, (nb + 1) * 4)) != ISB_OK) return r;
    if ((r = alloc((void**)&st->slconn, 2 * ns * sizeof(uint16_t))) != ISB_OK) return r;
    std::vector<int32_t> sconn(2 * ns), soff(nb + 1);
    ISB_HIP(hipMemcpy(sconn.data(), c->sconn, 2 * ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<uint16_t> loc(2 * ns);
    for (int b = 0; b < nb; ++b) {
      soff[b] = (int32_t)c->soff[b];
      for (int k = 0; k < 2; ++k)
        for (int64_t q = c->soff[b]; q < c->soff[b + 1]; ++q)
          loc[(size_t)k * ns + q] = (uint16_t)(sconn[(size_t)k * ns + q] - voff[b]);
    }
    soff[nb] = (int32_t)c->soff[nb];
    ISB_HIP(hipMemcpy(st->slconn, loc.data(), 2 * ns * sizeof(uint16_t), hipMemcpyHostToDevice));
    ISB_HIP(hipMemcpy(st->soff, soff.data(), (nb + 1) * 4, hipMemcpyHostToDevice));
  }
  const size_t ndof = (size_t)c->n_v * c->dim;
  if ((r = alloc((void**)&st->Dv, ndof * sizeof(float))) != ISB_OK) return r;
  if ((r = alloc(&st->vdT, ndof * (precision == ISB_MIXED ? 4 : 8))) != ISB_OK) return r;
  // 16-bit body-local connectivity: every body passed the LDS check, so it has fewer than 65536
  // vertices (2 x 8 bytes of LDS per DOF)
  {
    const size_t nk = (size_t)(c->dim + 1) * (size_t)c->n_e;
    std::vector<int32_t> conn(nk);
    ISB_HIP(hipMemcpy(conn.data(), c->conn, nk * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<uint16_t> loc(nk);
    for (int b = 0; b < nb; ++b) {
      if (voff[b + 1] - voff[b] > 65536) return fail(ISB_E_ARG, "batched solver: body with more than 65536 vertices");
      for (int k = 0; k <= c->dim; ++k)
        for (int64_t e = eoff[b]; e < eoff[b + 1]; ++e)
          loc[(size_t)k * c->n_e + e] = (uint16_t)(conn[(size_t)k * c->n_e + e] - voff[b]);
    }
    if ((r = alloc((void**)&st->lconn, nk * sizeof(uint16_t))) != ISB_OK) return r;
    ISB_HIP(hipMemcpy(st->lconn, loc.data(), nk * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  ISB_HIP(hipHostMalloc((void**)&st->hstats, nb * sizeof(DevStats), hipHostMallocDefault));
  ISB_HIP(hipMemcpy(st->order, order.data(), nb * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(st->wg_off, wg_off.data(), (st->grid + 1) * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(st->voff, voff.data(), (nb + 1) * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(st->eoff, eoff.data(), (nb + 1) * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemset(st->stats, 0, nb * sizeof(DevStats)));
  return ISB_OK;
}

isb_status batched_prepare(isb_ctx* c) { return prepare_state(c, &c->batched, c->precision); }

static BatchArgs make_args(isb_ctx* c, BatchedState* st) {
  BatchArgs A;
  std::memset(&A, 0, sizeof(A));
  A.order = st->order;
  A.wg_off = st->wg_off;
  A.voff = st->voff;
  A.eoff = st->eoff;
  A.n_bodies = c->n_bodies;
  A.a32 = c->w_a32;
  A.xhat = c->w_xhat;
  A.G = c->w_G;
  A.Gt = c->w_Gt;
  A.xt = c->w_xt;
  A.dx = c->w_xs;
  A.r = c->w_r;
  A.Dv = st->Dv;
  A.vdT = st->vdT;
  A.lconn = st->lconn;
  A.cv = c->w_cv;
  A.stats = st->stats;
  A.tol = c->scene.tol_rel;
  A.adj_tol = c->scene.adj_tol_rel;
  A.max_newton = c->scene.max_newton;
  A.max_cg = c->scene.max_cg;
  A.adj_warm = c->adj_warm;
  A.nacc = st->nacc;
  A.Fbuf = st->Fbuf;
  A.E0 = st->E0;
  A.E1 = st->E1;
  A.n_s = c->n_s;
  A.soff = st->soff;
  A.slconn = st->slconn;
  A.sk = c->sk;
  A.sil0 = c->sil0;
  A.Sbuf = st->Sbuf;
  return A;
}

static isb_status launch(isb_ctx* c, BatchedState* st, hipStream_t s, int mode, const BatchArgs& A, int grid = 0) {
  void* k = pick_kernel(c->dim, st->precision, mode, st->block, c->model, st->compact);
  const DevMesh m = devmesh(c);
  const DevScene sc = devscene(c);
  void* args[] = {(void*)&m, (void*)&sc, (void*)&A};
  ISB_HIP(hipLaunchKernel(k, dim3(grid > 0 ? grid : st->grid), dim3(st->block), args, st->lds, s));
  return ISB_OK;
}

// Mixed-precision recovery: the bodies whose solve did not converge are solved again from the same
// inputs by the FP64 kernel (its own batched state), in one launch over just those bodies, which
// overwrites their outputs; their stats come from that solve and carry ISB_FLAG_FP64_FALLBACK.
static isb_status fp64_fallback(isb_ctx* c, BatchedState* st, hipStream_t s, int mode, const BatchArgs& A0,
                                const std::vector<int32_t>& bodies) {
  isb_status r = prepare_state(c, &c->batched64, ISB_FP64);
  if (r != ISB_OK) return r;
  auto* fb = static_cast<BatchedState*>(c->batched64);
  const int n = (int)bodies.size(), grid = std::min(n, fb->grid);
  std::vector<int32_t> order, wg_off(1, 0);
  for (int g = 0; g < grid; ++g) {
    for (int k = g; k < n; k += grid) order.push_back(bodies[k]);
    wg_off.push_back((int32_t)order.size());
  }
  ISB_HIP(hipMemcpy(fb->fb_order, order.data(), order.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(fb->fb_wgoff, wg_off.data(), wg_off.size() * 4, hipMemcpyHostToDevice));
  ISB_HIP(hipMemcpy(fb->stats, st->hstats, c->n_bodies * sizeof(DevStats), hipMemcpyHostToDevice));
  BatchArgs A = make_args(c, fb);
  A.order = fb->fb_order;
  A.wg_off = fb->fb_wgoff;
  A.x0 = A0.x0;
  A.v0 = A0.v0;
  A.a = A0.a;
  A.x1 = A0.x1;
  A.v1 = A0.v1;
  A.xbar = A0.xbar;
  A.vbar = A0.vbar;
  A.w = A0.w;
  A.want_tail = A0.want_tail;
  if ((r = launch(c, fb, s, mode, A, grid)) != ISB_OK) return r;
  ISB_HIP(hipGetLastError());
  ISB_HIP(hipMemcpyAsync(fb->hstats, fb->stats, c->n_bodies * sizeof(DevStats), hipMemcpyDeviceToHost, s));
  ISB_HIP(hipStreamSynchronize(s));
  for (int32_t b : bodies) {
    st->hstats[b] = fb->hstats[b];
    st->hstats[b].flags |= ISB_FLAG_FP64_FALLBACK;
  }
  // the context's stats keep the merged record (a later call merges its own phase into it)
  ISB_HIP(hipMemcpy(st->stats, st->hstats, c->n_bodies * sizeof(DevStats), hipMemcpyHostToDevice));
  return ISB_OK;
}

static bool body_failed(const DevStats& d, int mode) {
  if (d.flags & ISB_FLAG_INVALID_ACTION) return false;  // an input error: a re-solve cannot help
  if (d.flags & ISB_FLAG_NONFINITE) return true;
  return mode == 0 ? !(d.flags & ISB_FLAG_CONVERGED) : !(d.flags & ISB_FLAG_ADJ_CONVERGED);
}

static isb_status collect(isb_ctx* c, BatchedState* st, hipStream_t s, isb_stats* per_body, int mode,
                          const BatchArgs& A) {
  if (c->graph_safe && !per_body) return ISB_OK;
  ISB_HIP(hipMemcpyAsync(st->hstats, st->stats, c->n_bodies * sizeof(DevStats), hipMemcpyDeviceToHost, s));
  ISB_HIP(hipStreamSynchronize(s));
  if (c->precision == ISB_MIXED && c->fp64_fallback) {
    std::vector<int32_t> failed;
    for (int b = 0; b < c->n_bodies; ++b)
      if (c->fp64_fallback == 2 || body_failed(st->hstats[b], mode)) failed.push_back(b);
    if (!failed.empty()) {
      const isb_status r = fp64_fallback(c, st, s, mode, A, failed);
      if (r != ISB_OK) return r;
    }
  }
  if (per_body) std::memcpy(per_body, st->hstats, c->n_bodies * sizeof(DevStats));
  for (int b = 0; b < c->n_bodies; ++b) {
    const DevStats& d = st->hstats[b];
    if (d.flags & ISB_FLAG_NONFINITE)
      return fail(ISB_E_NONFINITE, "body " + std::to_string(b) + ": non-finite value in the solve");
    if (d.flags & ISB_FLAG_INVALID_ACTION)
      return fail(ISB_E_ARG, "body " + std::to_string(b) + ": actuation a must be > 0");
    if (mode == 0 && !(d.flags & (ISB_FLAG_CONVERGED | ISB_FLAG_STAGNATED)))
      return fail(ISB_E_NOT_CONVERGED, "body " + std::to_string(b) + ": Newton iteration cap reached");
    if (mode == 1 && !(d.flags & ISB_FLAG_ADJ_CONVERGED))
      return fail(ISB_E_NOT_CONVERGED, "body " + std::to_string(b) + ": adjoint CG did not converge");
  }
  return ISB_OK;
}

isb_status batched_step(isb_ctx* c, hipStream_t s, const double* x0, const double* v0, const double* a, double* x1,
                        double* v1, isb_stats* per_body) {
  isb_status r = batched_prepare(c);
  if (r != ISB_OK) return r;
  auto* st = static_cast<BatchedState*>(c->batched);
  if (c->precision == ISB_MIXED) launch_to_f32(c->n_e, a, c->w_a32, s);
  BatchArgs A = make_args(c, st);
  A.x0 = x0;
  A.v0 = v0;
  A.a = a;
  A.x1 = x1;
  A.v1 = v1;
  A.want_tail = per_body != nullptr;
  if ((r = launch(c, st, s, 0, A)) != ISB_OK) return r;
  ISB_HIP(hipGetLastError());
  return collect(c, st, s, per_body, 0, A);
}

isb_status batched_adjoint(isb_ctx* c, hipStream_t s, const double* x1, const double* x0, const double* a,
                           const double* x1_bar, const double* v1_bar, double* w, isb_stats* per_body) {
  isb_status r = batched_prepare(c);
  if (r != ISB_OK) return r;
  auto* st = static_cast<BatchedState*>(c->batched);
  if (c->precision == ISB_MIXED) launch_to_f32(c->n_e, a, c->w_a32, s);
  BatchArgs A = make_args(c, st);
  A.x0 = x0;
  A.a = a;
  A.x1 = const_cast<double*>(x1);
  A.xbar = x1_bar;
  A.vbar = v1_bar;
  A.w = w;
  if ((r = launch(c, st, s, 1, A)) != ISB_OK) return r;
  ISB_HIP(hipGetLastError());
  return collect(c, st, s, per_body, 1, A);
}

}  // namespace isb
