// Internal device data layout and kernel launchers of libisb (not part of the C ABI).
//
// HBM layout (all SoA, indexed by element or vertex id in the caller's order):
//   conn  [D+1][n_e] int32      vertex ids of each simplex (global ids)
//   Dinv  [D*D][n_e] f64        Dm^-1, entry (j, c) at plane j*D + c
//   gf    [D][n_e]   f64        Dm^-1 d (fibre direction pulled back, so F d = Ds gf)
//   W, wmu, wlam, wkf [n_e] f64 rest volume and W mu, W lam, W k_f
//   *32 copies of Dinv, gf, wmu, wlam, wkf in f32 (mixed precision only)
//   mass  [n_v] f64, pinned [n_v*D] u8
// Vertex vectors (positions, gradients, CG vectors) are [n_v][D] f64, the boundary layout:
// one vertex is one contiguous 16 B (2D) / 24 B (3D) record, which is what a simplex gathers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isb {

constexpr int kBlock = 256;        // threads per block of the grid-wide kernels
constexpr int kMaxRedBlocks = 512; // cap on blocks of any kernel that writes reduction partials

struct DevMesh {
  int dim;
  int n_v, n_e;
  const int32_t* conn;
  const double *Dinv, *gf, *W, *wmu, *wlam, *wkf;
  const float *Dinv32, *gf32, *wmu32, *wlam32, *wkf32;
  const double* mass;
  const uint8_t* pinned;
  int model;  // isotropic energy model (EM_* of isb_elem.hpp, ISB_ENERGY_* of the C ABI)
  // Compact rest record: when every element has the same (mu, lam, k_f) and its fibre along the
  // coordinate axis `axis`, kernels with a compact variant read only Dm^-1 and W per element (W32 in
  // FP32 element math) and form W mu, W lam, W k_f from the scalars below and Dm^-1 d as column
  // `axis` of Dm^-1. axis < 0: the general per-element record.
  int axis;
  double mu_u, lam_u, kf_u;
  const float* W32;
};

// Vertex-pair springs, SoA over the caller's spring order:
//   conn [2][n_s] int32 end vertices i, j (global ids), k [n_s] stiffness, il0 [n_s] 1 / rest length
struct DevSprings {
  int n_s;
  const int32_t* conn;
  const double *k, *il0;
};

struct DevScene {
  int be;          // 1 = backward Euler, 0 = quasistatic
  double h;        // time step
  double s_pot;    // h^2 (backward Euler) or 1 (quasistatic): scale of the potential energy
  double grav;     // gravity along -y
  double kc;       // contact stiffness
  double kfr;      // friction stiffness
  double eps;      // friction contact tolerance
  double ih2;      // 1 / h^2
};

// Element index range: element k of [begin, end) is list[k] when list != nullptr, else k.
struct ERange {
  int begin, end;
  const int32_t* list;
};

// Element patches of the LDS-staged scatter (see Patches in isb_host.hpp), on the device.
struct PatchPlan {
  const int32_t* eoff;    // [n_patch+1] element range of each patch
  const int32_t* voff;    // [n_patch+1] range of each patch's vertex list
  const int32_t* verts;   // distinct vertices of each patch (sorted, but in the resident plan)
  const uint16_t* lconn;  // [(D+1)][n_e] corner index into the patch's vertex list
  int max_nv;             // largest vertex list
  int block;              // threads per patch workgroup: 256, 512 or 1024 (0: the default)
  const int32_t* eperm;   // [n_e] element of each slot of a patch's range (null: the slot itself)
  // [n_patch] the first nshared[k] vertices of patch k are held by other patches too, the rest by
  // it alone (null: no such split)
  const int32_t* nshared;
};

constexpr int kPatchBlock = 512;        // threads per patch workgroup (FP32 element math; FP64 takes half)

enum PatchOp { PATCH_GRAD = 0, PATCH_HV = 1, PATCH_DIAG = 2 };

// Device-resident CG scalars of the plain solver (one solve at a time). The iteration index lives
// here too, so that a captured chunk of iterations can be replayed: k_cg_update reads the completed
// count and publishes it in it_cur, k_cg_p reads it_cur and advances the count (each kernel only
// reads what the previous one wrote).
struct CgScal {
  double rz[2];    // r.z of the current iterate, double-buffered by iteration parity
  double rr;       // r.r
  double pHp;
  double rr0;      // r.r at the start
  double tol2;     // stop when r.r <= tol2
  int done;        // converged, stopped by curvature, or at the iteration cap
  int negcurv;     // non-positive curvature met
  int iters;       // completed iterations
  int it_cur;      // the iteration in progress
  int max_it;      // iteration cap
  int fault;       // resident solver: a grid barrier waited past its limit and the launch gave up
  double alpha_prev, gamma_prev;  // single-reduction CG: alpha and r.u of the previous iteration
};

constexpr int kMaxPatchGrid = 65535;  // workgroups of one patch launch (grid-stride beyond)

// Resident CG solver: threads per workgroup (one workgroup per CU), and LDS per patch vertex: nine
// FP64 vectors of D components (x, u, r, p, s, the preconditioner, the vertex diagonal, the
// accumulator, the solution) and the vertex id
constexpr int kResidentBlockF32 = 512;
constexpr int kResidentBlockF64 = 512;
constexpr int resident_vertex_bytes(int dim) { return 9 * dim * (int)sizeof(double) + 4; }

// the resident solver's grid barrier (zeroed before each launch): arrival counters per group of
// workgroups (workgroup b in group b % kBarGroups, the XCD it is dispatched to), the arrivals of
// the groups' last workgroups, the number of the last completed barrier and the abort flag, each on
// a 128-byte line of its own
constexpr int kBarGroups = 8;
struct GridBar {
  unsigned group[kBarGroups][32];
  unsigned top;
  unsigned pad0[31];
  unsigned flag;
  unsigned pad1[31];
  unsigned abort;
  unsigned pad2[31];
};

// ---- precompute ----
void launch_precompute_geom(int D, int n_e, const double* X, const int32_t* conn, double* Dinv, double* W,
                            hipStream_t s);
void launch_precompute_material(int D, int n_e, const double* Dinv, const double* W, const double* fdir,
                                const double* mu, const double* lam, const double* kf, double* gf, double* wmu,
                                double* wlam, double* wkf, float* Dinv32, float* gf32, float* wmu32, float* wlam32,
                                float* wkf32, hipStream_t s);
void launch_mass_colour(int D, ERange r, const int32_t* conn, int n_e, const double* W, const double* rho,
                        double* mass, hipStream_t s);

// ---- vertex kernels (range of vertices [v0, v1)) ----
void launch_setup(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x0, const double* v0p,
                  double* x, double* xhat, double* cv, hipStream_t s);
void launch_vertex_grad(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* x0,
                        const double* xhat, const double* cv, double* G, hipStream_t s);
void launch_vertex_hdiag(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* cv,
                         double* vdiag, hipStream_t s);
void launch_mask(const DevMesh& m, int v0, int v1, double* vec, hipStream_t s);
void launch_finish_diag(const DevMesh& m, int v0, int v1, const double* diag, double* Dinvp, hipStream_t s);
void launch_vertex_energy(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x, const double* dx,
                          double alpha, const double* x0, const double* xhat, const double* cv, double* partials,
                          int part_off, hipStream_t s, int* nblocks_out);
void launch_velocity(int n, const double* x1, const double* x0, double inv_h, double* v1, hipStream_t s);
void launch_vertex_vjp(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* w, const double* x1,
                       const double* x0, const double* v1_bar, double* x0_bar, double* v0_bar, hipStream_t s);
void launch_adjoint_rhs(const DevMesh& m, const DevScene& sc, int v0, int v1, const double* x1_bar,
                        const double* v1_bar, double* b, hipStream_t s);

// ---- element kernels ----
// precision: 0 = f64 element math, 1 = f32 element math (Hessian-vector product and diagonal)
void launch_elem_grad(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                      double* G, hipStream_t s);
void launch_elem_hv(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, int precision, const double* x,
                    const double* a, const float* a32, const double* p, double* Hp, const int* done, hipStream_t s);
void launch_elem_diag(const DevMesh& m, const DevScene& sc, ERange r, bool atomic, const double* x, const double* a,
                      double* diag, hipStream_t s);
void launch_elem_energy(const DevMesh& m, const DevScene& sc, ERange r, const double* x, const double* dx,
                        double alpha, const double* a, double* partials, int part_off, hipStream_t s,
                        int* nblocks_out);
void launch_elem_vjp(const DevMesh& m, const DevScene& sc, ERange r, const double* w, const double* x1,
                     const double* a, double* a_bar, double* mu_bar, double* lam_bar, double* kf_bar, hipStream_t s);
void launch_elem_minmax_J(const DevMesh& m, ERange r, const double* x, double* partials, hipStream_t s,
                          int* nblocks_out);
void launch_to_f32(int n, const double* src, float* dst, hipStream_t s);
// LDS-staged scatter over patches [p0, p1): op = PatchOp; p is the Hessian-vector operand (HV only);
// out receives one global atomic add per distinct vertex DOF of each patch. curv (HV only, may be
// null): per-workgroup partials of p^T H_elem p (s_pot-scaled). Returns the number of workgroups.
int launch_elem_patch(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int p0, int p1, int op,
                      int precision, const double* x, const double* a, const float* a32, const double* p,
                      double* out, const int* done, hipStream_t s, double* curv = nullptr);

// single-reduction PCG over the patch Hessian-vector kernel (partials: 6 x kMaxRedBlocks values)
void launch_cgcg_start(int n, const double* b, double sign, const double* Dinvp, const double* vdiag, double* r,
                       double* u, double* w, double* p, double* sv, double* xs, double* partials, CgScal* scal,
                       double tol2, int max_it, hipStream_t s);
void launch_cgcg_vec(int n, const double* hvpart, int nhv, double* partials, const double* Dinvp,
                     const double* vdiag, double* r, double* u, double* w, double* p, double* sv, double* xs,
                     CgScal* scal, hipStream_t s);
void launch_cgcg_final(int n, const double* partials, CgScal* scal, hipStream_t s);

// ---- resident single-reduction PCG (isb_resident.hip): body patches [p0, p0 + np) of the resident
// plan P (P.max_nv: the largest of them), one cooperative workgroup each, solve H(x) xs = sign * rhs
// to r.r <= tol2 in one launch and leave the outcome in *scal (fault = 1: a barrier waited longer
// than barrier_limit_us and every workgroup left the launch).
// Vectors are the global [n_v][D] arrays; W0..W2 are [n_v][D] scratch, part 8 * np values.
// Returns hipErrorCooperativeLaunchTooLarge, launching nothing, when np workgroups cannot all be
// resident. ----
// whether the resident kernel for this precision (1: mixed) and energy model keeps its elements'
// state in registers (and so takes the plan whose element slots are regrouped)
bool resident_caches_elements(int precision, int model);
hipError_t launch_cg_resident(const DevMesh& m, const DevScene& sc, const PatchPlan& P, int p0, int np, int n_cu,
                              int precision, const double* x, const double* a, const float* a32, const double* rhs,
                              double sign, const double* Dinvp, const double* vdiag, double* xs, double* W0,
                              double* W1, double* W2, double* part, GridBar* bar, CgScal* scal, double tol2,
                              int max_it, int64_t barrier_limit_us, hipStream_t s);

// ---- spring kernels (isb_springs.hip): spring range r (ids through r.list when given); as = the
// springs' actions (the action vector past the elements' entries); op = PatchOp; FP64 throughout ----
void launch_spring_op(int dim, const DevSprings& sp, const DevScene& sc, ERange r, bool atomic, int op,
                      const double* x, const double* as, const double* p, double* out, const int* done,
                      hipStream_t s);
void launch_spring_energy(int dim, const DevSprings& sp, const DevScene& sc, ERange r, const double* x,
                          const double* dx, double alpha, const double* as, double* partials, int part_off,
                          hipStream_t s, int* nblocks_out);
void launch_spring_vjp(int dim, const DevSprings& sp, const DevScene& sc, ERange r, const double* w,
                       const double* x1, const double* as, double* a_bar, double* k_bar, hipStream_t s);

// ---- reductions and CG vector kernels (vectors of length n, pointers already offset) ----
// partial sums of ncomp products per block; finalize into out[0..ncomp)
void launch_dot(int n, const double* a, const double* b, double* partials, hipStream_t s, int* nblocks_out);
void launch_finalize(const double* partials, int nblocks, int ncomp, double* out, hipStream_t s);
void launch_finalize_minmax(const double* partials, int nblocks, double* out, hipStream_t s);
void launch_axpy(int n, double* x, double alpha, const double* dx, hipStream_t s);
void launch_copy(int n, const double* src, double* dst, hipStream_t s);
void launch_stream_copy(int64_t n, const double* src, double* dst, hipStream_t s);

// CG on H xs = sign * b (b is masked to the free DOFs, where D^-1 != 0)
void launch_cg_start(int n, const double* b, double sign, const double* Dinvp, const double* vdiag, double* r,
                     double* p, double* xs, double* Hp, double* partials, CgScal* scal, double tol2, int max_it,
                     hipStream_t s);
void launch_cg_dot(int n, const double* p, const double* Hp, double* partials, const CgScal* scal, hipStream_t s);
void launch_cg_update(int n, const double* p, const double* Hp, const double* Dinvp, double* r, double* xs,
                      double* partials, CgScal* scal, hipStream_t s);
void launch_cg_p(int n, const double* r, const double* Dinvp, const double* vdiag, double* p, double* Hp,
                 const double* partials, CgScal* scal, hipStream_t s);
int red_blocks(int n);
void launch_fill(int n, double value, double* out, hipStream_t s);
void launch_mul(int n, const double* a, const double* b, double* out, hipStream_t s);
void launch_neg_precond(int n, const double* Dinvp, const double* g, double* out, hipStream_t s);
void launch_set_pinned(const DevMesh& m, int v0, int v1, double value, double* vec, hipStream_t s);
void launch_min_count(int n, const double* a, double* partials, double* out, hipStream_t s);

}  // namespace isb
