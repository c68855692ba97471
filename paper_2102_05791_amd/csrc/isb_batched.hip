// Batched persistent solver: one workgroup per body, the whole Newton-PCG step and the adjoint
// solve inside one launch (written after the plain path).
#include <hip/hip_runtime.h>

#include "isb_ctx.hpp"

namespace isb {

isb_status batched_prepare(isb_ctx* c) {
  (void)c;
  return fail(ISB_E_ARG, "batched solver not available");
}
void batched_release(isb_ctx* c) { (void)c; }
isb_status batched_step(isb_ctx* c, hipStream_t s, const double* x0, const double* v0, const double* a, double* x1,
                        double* v1, isb_stats* stats) {
  (void)c; (void)s; (void)x0; (void)v0; (void)a; (void)x1; (void)v1; (void)stats;
  return fail(ISB_E_ARG, "batched solver not available");
}
isb_status batched_adjoint(isb_ctx* c, hipStream_t s, const double* x1, const double* x0, const double* a,
                           const double* x1_bar, const double* v1_bar, double* w, isb_stats* stats) {
  (void)c; (void)s; (void)x1; (void)x0; (void)a; (void)x1_bar; (void)v1_bar; (void)w; (void)stats;
  return fail(ISB_E_ARG, "batched solver not available");
}
int64_t batched_lds_bytes(const isb_ctx* c) { (void)c; return 0; }

}  // namespace isb
