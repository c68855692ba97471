// Grid-wide kernels of the vertex-pair springs (Eq. 2 between two vertices; isb_spring.hpp) for
// the plain solver and the single-pass entry points: one spring per thread over a spring range,
// FP64 arithmetic in both precisions, results scattered with FP64 global atomics or, over one
// colour of the spring colouring (no two springs of a colour share a vertex), with plain
// read-modify-writes. The action of spring s is as[s] (the caller offsets the action vector past
// the elements' entries).
#include <hip/hip_runtime.h>

#include "isb_device.hpp"
#include "isb_internal.hpp"
#include "isb_spring.hpp"

namespace isb {

namespace {

int spring_grid(int n) {
  int b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return b > 65535 ? 65535 : b;
}

template <int D>
__device__ __forceinline__ void spring_load(const DevSprings& sp, int s, const double* __restrict__ x, int& i, int& j,
                                            double d[D]) {
  i = sp.conn[s];
  j = sp.conn[(size_t)sp.n_s + s];
#pragma unroll
  for (int r = 0; r < D; ++r) d[r] = x[(size_t)j * D + r] - x[(size_t)i * D + r];
}

template <int D, bool ATOMIC>
__device__ __forceinline__ void spring_scatter(double* out, int i, int j, const double y[D], double scale, bool both_plus) {
#pragma unroll
  for (int r = 0; r < D; ++r) {
    scatter_add<ATOMIC>(out, (size_t)j * D + r, scale * y[r]);
    scatter_add<ATOMIC>(out, (size_t)i * D + r, both_plus ? scale * y[r] : -scale * y[r]);
  }
}

// op: PATCH_GRAD (gradient), PATCH_HV (K (p_j - p_i) at j, its negative at i), PATCH_DIAG
template <int D, bool ATOMIC, int OP>
__global__ void __launch_bounds__(kBlock) k_spring_op(DevSprings sp, DevScene sc, ERange rg,
                                                      const double* __restrict__ x, const double* __restrict__ as,
                                                      const double* __restrict__ p, double* out, const int* done) {
  if (OP == PATCH_HV && done && *done) return;
  for (int k = rg.begin + blockIdx.x * blockDim.x + threadIdx.x; k < rg.end; k += gridDim.x * blockDim.x) {
    const int s = elem_id(rg, k);
    int i, j;
    double d[D];
    spring_load<D>(sp, s, x, i, j, d);
    SpringTerms<D> S;
    spring_terms<D>(d, sp.k[s], sp.il0[s], as[s], S);
    double y[D];
    if constexpr (OP == PATCH_GRAD) {
#pragma unroll
      for (int r = 0; r < D; ++r) y[r] = S.f * S.n[r];
      spring_scatter<D, ATOMIC>(out, i, j, y, sc.s_pot, false);
    } else if constexpr (OP == PATCH_HV) {
      double u[D];
#pragma unroll
      for (int r = 0; r < D; ++r) u[r] = p[(size_t)j * D + r] - p[(size_t)i * D + r];
      spring_apply<D>(S, u, y);
      spring_scatter<D, ATOMIC>(out, i, j, y, sc.s_pot, false);
    } else {
      spring_diag<D>(S, y);
      spring_scatter<D, ATOMIC>(out, i, j, y, sc.s_pot, true);
    }
  }
}

// comps per block: (sum s_pot [E_s(x + alpha dx) - E_s(x)], sum s_pot |E_s(x)|, sum s_pot E_s(x + alpha dx))
template <int D>
__global__ void __launch_bounds__(kBlock) k_spring_energy(DevSprings sp, DevScene sc, ERange rg,
                                                          const double* __restrict__ x, const double* __restrict__ dx,
                                                          double alpha, const double* __restrict__ as,
                                                          double* partials) {
  __shared__ double sh[kBlock / 64];
  double sd = 0.0, sa = 0.0, st = 0.0;
  for (int k = rg.begin + blockIdx.x * blockDim.x + threadIdx.x; k < rg.end; k += gridDim.x * blockDim.x) {
    const int s = elem_id(rg, k);
    int i, j;
    double d[D];
    spring_load<D>(sp, s, x, i, j, d);
    const double ks = sp.k[s], il0 = sp.il0[s], a = as[s];
    SpringTerms<D> S;
    spring_terms<D>(d, ks, il0, a, S);
    const double ea = sc.s_pot * spring_energy<D>(S, ks);
    double eb = ea;
    if (dx) {
#pragma unroll
      for (int r = 0; r < D; ++r)
        d[r] = (x[(size_t)j * D + r] + alpha * dx[(size_t)j * D + r]) - (x[(size_t)i * D + r] + alpha * dx[(size_t)i * D + r]);
      spring_terms<D>(d, ks, il0, a, S);
      eb = sc.s_pot * spring_energy<D>(S, ks);
    }
    sd += eb - ea;
    sa += fabs(ea);
    st += eb;
  }
  sd = block_sum(sd, sh);
  sa = block_sum(sa, sh);
  st = block_sum(st, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = sd;
    partials[blockIdx.x * 3 + 1] = sa;
    partials[blockIdx.x * 3 + 2] = st;
  }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_spring_vjp(DevSprings sp, DevScene sc, ERange rg,
                                                       const double* __restrict__ w, const double* __restrict__ x1,
                                                       const double* __restrict__ as, double* a_bar, double* k_bar) {
  for (int k = rg.begin + blockIdx.x * blockDim.x + threadIdx.x; k < rg.end; k += gridDim.x * blockDim.x) {
    const int s = elem_id(rg, k);
    int i, j;
    double d[D], dw[D];
    spring_load<D>(sp, s, x1, i, j, d);
#pragma unroll
    for (int r = 0; r < D; ++r) dw[r] = w[(size_t)j * D + r] - w[(size_t)i * D + r];
    const double ks = sp.k[s], a = as[s];
    SpringTerms<D> S;
    spring_terms<D>(d, ks, sp.il0[s], a, S);
    double ab, kb;
    spring_vjp<D>(S, ks, a, dw, ab, kb);
    if (a_bar) a_bar[s] = sc.s_pot * ab;
    if (k_bar) k_bar[s] = sc.s_pot * kb;
  }
}

template <int D, bool ATOMIC>
void spring_op_d(const DevSprings& sp, const DevScene& sc, ERange r, int op, const double* x, const double* as,
                 const double* p, double* out, const int* done, hipStream_t s) {
  const int g = spring_grid(r.end - r.begin);
  if (op == PATCH_GRAD)
    k_spring_op<D, ATOMIC, PATCH_GRAD><<<g, kBlock, 0, s>>>(sp, sc, r, x, as, p, out, done);
  else if (op == PATCH_HV)
    k_spring_op<D, ATOMIC, PATCH_HV><<<g, kBlock, 0, s>>>(sp, sc, r, x, as, p, out, done);
  else
    k_spring_op<D, ATOMIC, PATCH_DIAG><<<g, kBlock, 0, s>>>(sp, sc, r, x, as, p, out, done);
}

}  // namespace

void launch_spring_op(int dim, const DevSprings& sp, const DevScene& sc, ERange r, bool atomic, int op,
                      const double* x, const double* as, const double* p, double* out, const int* done,
                      hipStream_t s) {
  if (r.end <= r.begin) return;
  if (dim == 2)
    atomic ? spring_op_d<2, true>(sp, sc, r, op, x, as, p, out, done, s)
           : spring_op_d<2, false>(sp, sc, r, op, x, as, p, out, done, s);
  else
    atomic ? spring_op_d<3, true>(sp, sc, r, op, x, as, p, out, done, s)
           : spring_op_d<3, false>(sp, sc, r, op, x, as, p, out, done, s);
}

void launch_spring_energy(int dim, const DevSprings& sp, const DevScene& sc, ERange r, const double* x,
                          const double* dx, double alpha, const double* as, double* partials, int part_off,
                          hipStream_t s, int* nblocks_out) {
  if (r.end <= r.begin) {
    *nblocks_out = 0;
    return;
  }
  const int nb = red_blocks(r.end - r.begin);
  if (dim == 2)
    k_spring_energy<2><<<nb, kBlock, 0, s>>>(sp, sc, r, x, dx, alpha, as, partials + 3 * part_off);
  else
    k_spring_energy<3><<<nb, kBlock, 0, s>>>(sp, sc, r, x, dx, alpha, as, partials + 3 * part_off);
  *nblocks_out = nb;
}

void launch_spring_vjp(int dim, const DevSprings& sp, const DevScene& sc, ERange r, const double* w,
                       const double* x1, const double* as, double* a_bar, double* k_bar, hipStream_t s) {
  if (r.end <= r.begin || (!a_bar && !k_bar)) return;
  const int g = spring_grid(r.end - r.begin);
  if (dim == 2)
    k_spring_vjp<2><<<g, kBlock, 0, s>>>(sp, sc, r, w, x1, as, a_bar, k_bar);
  else
    k_spring_vjp<3><<<g, kBlock, 0, s>>>(sp, sc, r, w, x1, as, a_bar, k_bar);
}

}  // namespace isb
