/*
 * isb.h - C ABI of the implicit soft-body step and its adjoint (libisb.so, gfx950).
 *
 * One call of isb_step advances every body of an uploaded mesh by one implicit
 * step posed as energy minimisation:
 *   quasistatic      x1 = argmin_x E(x, a)                                 (Sec. 3, Eq. 1)
 *   backward Euler   x1 = argmin_x 1/2 |x - (x0 + h v0)|_M^2 + h^2 E(x, a)  (Sec. 5, Eq. 13-14)
 *                    v1 = (x1 - x0) / h
 * E is, per element, the neo-Hookean density of Eq. 3 (log J replaced by its
 * quadratic expansion about J = 1, as Sec. 3 prescribes for inverted elements)
 * plus the contractile fibre term of Eq. 2 taken along a per-element material
 * direction d (l / l0 = |F d|), scaled by the rest volume W; and, per vertex,
 * gravity m g y, ground contact k_c ReLU(-y)^2 (Eq. 15) and friction
 * k_fr ((x_t - x0_t)/h)^2 ReLU(-y0 + eps) on the tangential axes (Eq. 16-17);
 * and, per vertex-pair spring (optional, isb_spring_upload), Eq. 2 with l the
 * distance between the spring's two vertices (Fig. 2's energies of d = x_j - x_i).
 * The minimiser is found by Newton's method with a preconditioned conjugate
 * gradient inner solve over matrix-free Hessian-vector products (Sec. 4.1,
 * Eq. 10); the backward pass is the adjoint of Eq. 9: one CG solve with the
 * symmetric Hessian H(x1), followed by per-element vector-Jacobian products.
 *
 * Conventions shared by every call
 *   - Vertex arrays are [n_v][dim] row-major FP64 (the n x d layout of Sec. 4.1);
 *     element arrays are [n_e] or [n_e][dim]; y (axis 1) is "up"; dim is 2
 *     (triangles) or 3 (tetrahedra).
 *   - The action vector a (and its cotangent a_bar) has n_e + n_s entries: one per
 *     element's fibre, then one per spring (n_s = 0 without springs).
 *   - Pointers named "host" are CPU memory, copied before the call returns.
 *     Every other array argument is device memory on the context's GPU, owned
 *     by the caller; the library never keeps a caller pointer past the call.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). All device
 *     work of a call is enqueued on it. A call that returns statistics to host
 *     memory synchronises the stream; with stats == NULL and the graph-safe
 *     option set, isb_step / isb_solve_adjoint / isb_vjp_params enqueue work
 *     only (no host synchronisation, no allocation) and may be captured.
 *   - Pinned (Dirichlet) DOFs keep their x0 value; the adjoint, x0_bar and
 *     v0_bar are 0 on them (pins are boundary data, not differentiable state).
 *   - Every call returns an isb_status; on failure isb_last_error() describes it.
 *     The library owns the context and every workspace; isb_destroy frees them.
 */
#ifndef ISB_H
#define ISB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isb_ctx isb_ctx;   /* opaque, library-owned */
typedef void* isb_stream;         /* a hipStream_t */

typedef enum {
  ISB_OK = 0,
  ISB_E_ARG = 1,            /* bad argument: NULL pointer, size, a <= 0, unknown key */
  ISB_E_MESH = 2,           /* invalid mesh: index out of body range, non-positive rest volume */
  ISB_E_HIP = 3,            /* HIP runtime error */
  ISB_E_NOT_CONVERGED = 4,  /* Newton or CG hit its iteration cap; outputs hold the last iterate */
  ISB_E_NONFINITE = 5,      /* NaN or Inf in an energy, residual or input */
  ISB_E_STATE = 6           /* call order: e.g. step before mesh and material upload */
} isb_status;

typedef enum { ISB_FP64 = 0, ISB_MIXED = 1 } isb_precision;
typedef enum { ISB_QUASISTATIC = 0, ISB_BACKWARD_EULER = 1 } isb_integrator;

/* Isotropic element energy (ISB_OPT_ENERGY). Each density is a function of F = Ds Dm^-1, linear in
 * the Lame pair (mu, lam) of isb_material_upload, zero with zero stress at rest, and its Hessian at
 * rest is the linear-elastic stiffness of that Lame pair; the fibre term of Eq. 2 is added in all.
 *   NEOHOOKEAN         Eq. 3 with log J replaced by (J-1) - (J-1)^2/2 (Sec. 3)
 *   STVK               St. Venant-Kirchhoff, E = (F^T F - I)/2: mu E:E + lam/2 tr(E)^2
 *   COROTATED          mu |F - R|^2 + lam/2 tr(R^T F - I)^2, R the rotation closest to F
 *                      (argmax of tr(R^T F) over rotations, so det R = 1 also for inverted F)
 *   STABLE_NEOHOOKEAN  mu/2 (I1 - dim) - mu (J - 1) + (lam + mu)/2 (J - 1)^2: the stable neo-Hookean
 *                      form without its log barrier, Lame pair reparametrised to rest stress zero
 * Sec. 3 names these models as alternatives to Eq. 3. */
typedef enum {
  ISB_ENERGY_NEOHOOKEAN = 0,
  ISB_ENERGY_STVK = 1,
  ISB_ENERGY_COROTATED = 2,
  ISB_ENERGY_STABLE_NEOHOOKEAN = 3
} isb_energy_model;

/* Forward minimiser of the step objective (ISB_OPT_FORWARD). The adjoint of Eq. 9 does not depend
 * on it (Sec. 4: the rule differentiates the minimiser, not the iterations that found it).
 *   NEWTON  inexact Newton with Jacobi-preconditioned CG over matrix-free Hessian-vector products
 *   LBFGS   the paper's kind of forward pass: a descent method with line search that uses first
 *           derivatives only (Sec. 6), here limited-memory BFGS (two-loop recursion, scaling
 *           s^T y / y^T y); same Armijo line search and stopping rule as NEWTON; plain solver only */
typedef enum { ISB_FORWARD_NEWTON = 0, ISB_FORWARD_LBFGS = 1 } isb_forward;

/* Option keys for isb_set_option / isb_get_option. */
typedef enum {
  ISB_OPT_SOLVER = 0,       /* 0 = plain: host-driven Newton-PCG, one body at a time, grid-wide kernels;
                               1 = batched: one persistent launch, one workgroup per body (default 0) */
  ISB_OPT_SCATTER = 1,      /* plain solver scatter: 0 = FP64 global atomics per element corner,
                               1 = graph colouring (deterministic, bitwise reproducible),
                               2 = LDS-staged element patches (default): one workgroup per patch of
                               consecutive elements accumulates in LDS and adds each distinct vertex DOF
                               to global memory once */
  ISB_OPT_GRAPH_SAFE = 2,   /* 1 = no host synchronisation inside step/adjoint/vjp (batched solver only) */
  ISB_OPT_BLOCK = 3,        /* batched solver workgroup size: 256, 512, 768 or 1024; 0 (default) = 768 for
                               triangles, 512 for tetrahedra */
  ISB_OPT_CG_CHECK = 4,     /* plain solver: CG iterations are enqueued in batches of k (default 4); the host reads the
                             * convergence flag of each batch while the next one is already queued, so up to 2k
                             * iterations past convergence are enqueued and return at once */
  ISB_OPT_PRECISION = 5,    /* isb_precision; equals the value given to isb_create */
  ISB_OPT_ENERGY = 6,       /* isotropic element energy, one of isb_energy_model (default neo-Hookean); the
                             * batched solver runs the alternatives with the default workgroup size only */
  ISB_OPT_FORWARD = 7,      /* forward minimiser of the plain solver, one of isb_forward (default Newton-PCG);
                             * the batched solver takes ISB_FORWARD_NEWTON only (ISB_E_ARG otherwise) */
  ISB_OPT_LBFGS_MEMORY = 8, /* pairs kept by ISB_FORWARD_LBFGS, 1..64 (default 8) */
  ISB_OPT_LBFGS_MAX_ITERS = 9, /* iteration cap of ISB_FORWARD_LBFGS (default 20000; max_newton caps Newton) */
  ISB_OPT_FP64_FALLBACK = 11, /* batched solver in ISB_MIXED: 1 (default) = a body whose step or adjoint did not
                             * converge is solved again from the same inputs in FP64 (its stats then carry
                             * ISB_FLAG_FP64_FALLBACK); needs the host check, so not in graph-safe mode without
                             * stats; 0 = off; 2 = re-solve every body in FP64 (exercises the fallback path) */
  ISB_OPT_ADJ_WARM_START = 12, /* 1 = isb_solve_adjoint reads w on entry as the starting point of its CG
                             * (pinned DOFs ignored; e.g. the adjoint of the step after, in a backward pass
                             * through time, whose solution is close) and solves H d = b - H w for the
                             * correction, to the same tolerance on the residual of H w = b; 0 (default) =
                             * w is output only and CG starts from zero. An FP64 re-solve (ISB_OPT_FP64_FALLBACK)
                             * starts from the first attempt's w */
  ISB_OPT_COMPACT_REST = 13, /* 1 (default) = when every element has the same (mu, lam, k_f) and every fibre
                             * direction is the same coordinate axis, the kernels that have a compact variant
                             * (the LDS-staged patch kernels, the batched solver) read per element only Dm^-1
                             * and W, and take the material from three scalars and the fibre from a column of
                             * Dm^-1 (the same FP64 values; ISB_INFO_COMPACT_AXIS tells whether it applies);
                             * 0 = always the general per-element record */
  ISB_OPT_PATCH_BLOCK = 14, /* threads per workgroup of the LDS-staged patch kernels: 256, 512 or 1024; 0 = the
                             * default (512 for FP32 element math, 256 for FP64); the alternative energy models
                             * run with the default only */
  ISB_OPT_CG_SINGLE_REDUCTION = 15, /* plain solver: 1 (default) = where the Hessian-vector product is one
                             * LDS-staged patch launch (bodies of >= 16,384 elements in ISB_OPT_SCATTER 2, no
                             * springs), CG runs in the single-reduction form of Chronopoulos and Gear: the
                             * product also returns its share of u^T H u and one vector kernel forms every
                             * scalar from one reduction, two launches per iteration instead of four;
                             * 0 = the classic form everywhere. Same iterates in exact arithmetic */
  ISB_OPT_CG_RESIDENT = 16, /* plain solver: 1 (default) = where the single-reduction CG runs and the body's
                             * resident patches (one workgroup per compute unit, the patch's CG vectors in
                             * LDS; ISB_INFO_RESIDENT tells whether a body has them) can all be resident at
                             * once, the whole CG solve is one cooperative launch with one grid barrier per
                             * iteration; 0 = one Hessian-vector launch and one vector launch per iteration.
                             * The same single-reduction iteration either way. A barrier that waits longer
                             * than ISB_OPT_CG_BARRIER_LIMIT_US (workgroups that are not all resident) ends
                             * the launch, and the call returns ISB_E_HIP */
  ISB_OPT_CG_BARRIER_LIMIT_US = 17, /* resident CG: the longest wait at one grid barrier, in microseconds,
                             * 1 .. 60,000,000 (default 4,000,000); a barrier that waits longer ends the
                             * launch and the call returns ISB_E_HIP. A small value forces that path, for
                             * tests of the error handling; every workgroup still leaves the launch */
  ISB_OPT_CG_GRAPH = 10     /* plain solver: 1 = run CG as a graph of 8 iterations, captured once per solve and
                             * replayed until converged (one launch and one host read per 8 iterations);
                             * 0 (default) = one launch per kernel and a read every ISB_OPT_CG_CHECK iterations.
                             * Same kernels in the same order either way */
} isb_option;

/* Read-only context facts for isb_get_option. */
#define ISB_INFO_N_VERTICES 100
#define ISB_INFO_N_ELEMENTS 101
#define ISB_INFO_N_BODIES 102
#define ISB_INFO_DIM 103
#define ISB_INFO_N_COLOURS 104    /* colours of the element colouring (max over bodies) */
#define ISB_INFO_LDS_BYTES 105    /* LDS bytes per workgroup of the batched solver for the largest body */
#define ISB_INFO_COMPACT_AXIS 106 /* the fibre axis of the compact rest record in use, -1 when not in use */
#define ISB_INFO_RESIDENT 107     /* bodies that have a resident CG plan (ISB_OPT_CG_RESIDENT) */

/* Per-body solver statistics (host memory). */
typedef struct {
  int32_t newton_iters;     /* Newton iterations taken */
  int32_t cg_iters;         /* CG iterations summed over the Newton iterations */
  int32_t adj_cg_iters;     /* CG iterations of the last adjoint solve */
  int32_t ls_backtracks;    /* line-search halvings */
  int32_t negcurv_exits;    /* CG solves cut short by non-positive curvature */
  int32_t flags;            /* bit 0 converged, bit 1 stagnated (rounding floor), bit 2 non-finite,
                               bit 3 adjoint converged */
  double res0;              /* |grad g(x_init)|_2 over free DOFs */
  double res_final;         /* |grad g(x1)|_2 over free DOFs */
  double adj_res_final;     /* |H w - xbar|_2 / |xbar|_2 (CG recursive residual) of the last adjoint */
  double energy;            /* g(x1) */
  double min_J, max_J;      /* extreme element volume ratios det F at x1 */
} isb_stats;

#define ISB_FLAG_CONVERGED 1
#define ISB_FLAG_STAGNATED 2
#define ISB_FLAG_NONFINITE 4
#define ISB_FLAG_ADJ_CONVERGED 8
#define ISB_FLAG_FP64_FALLBACK 16 /* the mixed solve did not converge; these stats are the FP64 re-solve's */
#define ISB_FLAG_INVALID_ACTION 32 /* batched solver: an action of the body was <= 0 or non-finite (non-finite
                                    * also sets ISB_FLAG_NONFINITE); the body was not solved: x1 = x_init,
                                    * v1 = (x1 - x0) / h, or w = 0 for the adjoint */

/* Scene constants (one set for every body of the context). */
typedef struct {
  int32_t integrator;       /* isb_integrator */
  int32_t max_newton;       /* Newton iteration cap (e.g. 50) */
  int32_t max_cg;           /* CG iteration cap per solve (e.g. 1000) */
  int32_t pad_;
  double h;                 /* time step (backward Euler; also the friction velocity scale) */
  double gravity;           /* g >= 0, acting along -y */
  double k_contact;         /* ground penalty stiffness k_c (Eq. 15), ground at y = 0 */
  double k_friction;        /* friction stiffness k_fr (Eq. 17) */
  double eps_friction;      /* friction contact tolerance eps (Eq. 17) */
  double tol_rel;           /* Newton stop: |grad g| <= tol_rel |grad g(x_init)| */
  double adj_tol_rel;       /* adjoint CG stop: |H w - xbar| <= adj_tol_rel |xbar| */
} isb_scene;

/* ---- lifetime ---------------------------------------------------------------------------- */

/* Create a context on HIP device `device` computing in `precision`: the holder of one simulated
 * system, whose state transition s1 = sim(s0, a0) (Sec. 5, Eq. 12) isb_step evaluates (ISB_FP64: every element
 * kernel in FP64; ISB_MIXED: Hessian-vector products in FP32 element arithmetic, while
 * gradients, energies, the preconditioner diagonal, CG vectors, dot products, norms and the
 * state stay FP64). The boundary is FP64 in both modes. */
isb_status isb_create(int device, int precision, isb_ctx** out);
isb_status isb_destroy(isb_ctx* ctx);
/* Thread-local description of the last failure on this thread; valid until the next isb_ call. */
const char* isb_last_error(void);
/* Library version string. */
const char* isb_version(void);

/* ---- host-only helpers (no GPU needed) ---------------------------------------------------- */

/* Check a mesh: dim in {2,3}; offsets monotone with body_v_off[0] = body_e_off[0] = 0 and
 * body_v_off[n_bodies] = n_v, body_e_off[n_bodies] = n_e; each element's vertices distinct and
 * inside its body's vertex range; every rest volume det(Dm)/dim! > 0 (Sec. 3: F = Ds Dm^-1).
 * X host [n_v][dim], T host [n_e][dim+1] int32 (global vertex ids). Returns ISB_OK or ISB_E_MESH. */
isb_status isb_validate_mesh(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T,
                             int32_t n_bodies, const int64_t* body_v_off, const int64_t* body_e_off);

/* Greedy element colouring: no two elements of one colour share a vertex. colour_out host [n_e]
 * receives each element's colour; *n_colours_out the number of colours used. Deterministic. */
isb_status isb_colour_elements(int dim, int64_t n_v, int64_t n_e, const int32_t* T,
                               int32_t* colour_out, int32_t* n_colours_out);

/* A locality order of the elements: perm_out host [n_e] receives, for each new position, the
 * element that goes there, sorting each body's elements (body_e_off host [n_bodies+1], or NULL for
 * one body) by the Morton key of their rest centroids (X host [n_v][dim]). The LDS-staged patch
 * scatter takes consecutive elements, so a mesh whose elements come in such an order loads and
 * flushes each vertex in fewer patches; a caller applies the permutation to T and to every
 * per-element array once, before isb_mesh_upload. Deterministic; ISB_E_MESH for an out-of-range
 * vertex, ISB_E_ARG otherwise. */
isb_status isb_locality_order(int dim, int64_t n_v, const double* X, int64_t n_e, const int32_t* T,
                              int32_t n_bodies, const int64_t* body_e_off, int64_t* perm_out);

/* An order of the elements for the patch scatter's wavefronts, applied after a locality order:
 * perm_out host [n_e] receives, for each new position, the element that goes there. It only
 * permutes elements inside each patch of the plan isb_mesh_upload builds for this T (n_v
 * vertices, T host [n_e][dim+1] int32, body_e_off host [n_bodies+1] or NULL for one body): the
 * patches, their vertex sets and the plan's boundaries are unchanged. Inside a patch, each group of
 * 64 consecutive elements from the patch's first (one wavefront of the patch kernels) receives
 * elements with distinct vertices in each corner slot where a greedy placement finds them, so that
 * the lanes of one LDS atomic add address distinct vertices; then elements move between the groups
 * of 32 (the lanes the LDS serves together in an FP64 access) so that each group's vertices in a
 * corner slot spread over the LDS bank classes (the plan's local id mod 32 in 3D, mod 16 in 2D),
 * where a short local search lowers the largest class counts. A caller applies the permutation to T
 * and to every per-element array once, before isb_mesh_upload; results change only by the
 * rounding of the summation order. Deterministic; ISB_E_MESH for an out-of-range vertex,
 * ISB_E_ARG otherwise. */
isb_status isb_wave_order(int dim, int64_t n_v, int64_t n_e, const int32_t* T, int32_t n_bodies,
                          const int64_t* body_e_off, int64_t* perm_out);

/* ---- upload ------------------------------------------------------------------------------- */

/* Copy a mesh of n_bodies independent bodies to the device and precompute Dm^-1 and W per element:
 * F = Ds Dm^-1 is linear in the vertex positions (Sec. 3, beside Eq. 3) and W = det(Dm) / dim! is the
 * rest volume that scales each element's energy; the positions are the n x dim tensor of Sec. 4.1.
 * body_v_off / body_e_off host [n_bodies+1]; X_rest host [n_v][dim]; T host [n_e][dim+1]
 * (positively oriented); dof_pinned host [n_v][dim], 1 = Dirichlet. Validates first (ISB_E_MESH).
 * Replaces any previous mesh (the material must then be uploaded again). */
isb_status isb_mesh_upload(isb_ctx* ctx, int dim, int32_t n_bodies, const int64_t* body_v_off,
                           const int64_t* body_e_off, const double* X_rest, const int32_t* T,
                           const uint8_t* dof_pinned);

/* Per-element material, all host [n_e] except fibre_dir host [n_e][dim] (unit material-space
 * direction d of the fibre, Eq. 2) and the scene. mu, lam: Lame pair of Eq. 3; k_fibre: k of
 * Eq. 2 per unit rest volume; density: rho, giving the lumped mass m_v = sum rho W / (dim+1)
 * (the M of Eq. 14). Requires a mesh. */
isb_status isb_material_upload(isb_ctx* ctx, const double* mu, const double* lam, const double* k_fibre,
                               const double* fibre_dir, const double* density, const isb_scene* scene);

/* Vertex-pair springs of Eq. 2: spring s joins vertices i = pairs[2s] and j = pairs[2s+1] (global
 * ids, both inside the body that owns s, i != j) with energy k[s]/2 (l / (a l0) - 1)^2, l = |x_j - x_i|,
 * rest length l0 = |X_j - X_i| from the uploaded rest positions (must be > 0) and its own action
 * a[n_e + s]. body_s_off host [n_bodies+1] (springs of body b are [body_s_off[b], body_s_off[b+1]);
 * may be NULL for one body); pairs host [n_s][2] int32; k host [n_s], finite and >= 0 (no volume
 * weight). Spring arithmetic is FP64, except that the batched solver in ISB_MIXED applies the
 * FP64-formed spring block to the CG direction in FP32, as it does the element blocks. n_s = 0
 * removes the springs. Requires a
 * mesh; a new mesh upload removes them. ISB_E_MESH for a bad pair or rest length, ISB_E_ARG otherwise. */
isb_status isb_spring_upload(isb_ctx* ctx, int64_t n_s, const int64_t* body_s_off, const int32_t* pairs,
                             const double* k);

/* Replace the scene constants (tolerances, stiffnesses, h) without re-uploading the material. */
isb_status isb_set_scene(isb_ctx* ctx, const isb_scene* scene);

isb_status isb_set_option(isb_ctx* ctx, int key, int64_t value);
isb_status isb_get_option(isb_ctx* ctx, int key, int64_t* value);

/* Lumped vertex masses, device out [n_v] (FP64). */
isb_status isb_get_mass(isb_ctx* ctx, isb_stream stream, double* mass_out);

/* Pick the fastest launch configuration for this context on the caller's inputs: each candidate
 * runs two steps from (x0, v0, a) (the first prepares and warms up; the second is timed with HIP
 * events on `stream`) and the fastest is kept as the context's option. Candidates: the batched
 * solver's workgroup size (ISB_OPT_BLOCK 512, 768, 1024; the alternative energies have one size),
 * the plain solver's scatter (ISB_OPT_SCATTER 0 atomic or 2 patches). chosen_out host [2] or NULL
 * receives (option key, value). Allocates two temporary state buffers; synchronises the stream.
 * Candidates that cannot run on the context are skipped; ISB_E_ARG if none ran. */
isb_status isb_autotune(isb_ctx* ctx, isb_stream stream, const double* x0, const double* v0,
                        const double* a, int64_t* chosen_out);

/* ---- the step and its adjoint ------------------------------------------------------------- */

/* One implicit step (Eq. 1 or Eq. 14) of every body. x0, v0: device [n_v][dim] (v0 ignored and
 * may be NULL in quasistatic mode); a: device [n_e + n_s], actuation of Eq. 2 (1 = relaxed, < 1
 * contracts; must be > 0); x1, v1: device out [n_v][dim] (v1 may be NULL; it is not written in
 * quasistatic mode). per_body: host [n_bodies] stats or NULL. Returns ISB_E_NOT_CONVERGED if
 * any body hit max_newton (x1, v1 then hold the last iterate), ISB_E_NONFINITE on NaN/Inf, ISB_E_ARG
 * if an action is <= 0. The batched solver checks the actions on the device, per body
 * (ISB_FLAG_INVALID_ACTION), and reports them with the other per-body failures when the call reads its
 * stats back; a graph-safe call without stats reports no per-body failure. */
isb_status isb_step(isb_ctx* ctx, isb_stream stream, const double* x0, const double* v0,
                    const double* a, double* x1, double* v1, isb_stats* per_body);

/* Adjoint solve of Eq. 9: w = H(x1)^-1 (x1_bar + v1_bar / h) over the free DOFs (the v1_bar term
 * only in backward Euler; v1_bar may be NULL), w = 0 on pinned DOFs. H is the unprojected
 * Hessian of the step objective at x1, symmetric and positive definite at a minimiser (Sec. 4),
 * so CG needs no transpose. x1, x0: device [n_v][dim]; a: device [n_e + n_s]; w: device out (also
 * the starting point on entry with ISB_OPT_ADJ_WARM_START). */
isb_status isb_solve_adjoint(isb_ctx* ctx, isb_stream stream, const double* x1, const double* x0,
                             const double* a, const double* x1_bar, const double* v1_bar, double* w,
                             isb_stats* per_body);

/* Vector-Jacobian products given the adjoint w: theta_bar = -w^T dG/dtheta with G = grad_x g
 * (Eq. 9 and the remark after Eq. 10), evaluated at x1. Outputs (device, any may be NULL):
 *   a_bar [n_e + n_s]                      actuation cotangents (elements, then springs)
 *   mu_bar, lam_bar, kf_bar [n_e]          per-element material cotangents
 *   x0_bar, v0_bar [n_v][dim]              previous-state cotangents, including the explicit
 *                                          v1 = (x1 - x0)/h path (-v1_bar / h) in backward Euler */
isb_status isb_vjp_params(isb_ctx* ctx, isb_stream stream, const double* w, const double* x1,
                          const double* x0, const double* a, const double* v1_bar, double* a_bar,
                          double* x0_bar, double* v0_bar, double* mu_bar, double* lam_bar,
                          double* kf_bar);

/* Spring stiffness cotangents k_bar = -w^T dG/dk (Eq. 9) at x1, device out [n_s]; a: device
 * [n_e + n_s]. Nothing to do without springs. */
isb_status isb_vjp_spring_stiffness(isb_ctx* ctx, isb_stream stream, const double* w, const double* x1,
                                    const double* a, double* k_bar);

/* ---- single evaluations of the step objective (the kernels of the solver, exposed) --------- */

/* g(x) per body, device out energy [n_bodies]; v0 may be NULL in quasistatic mode. */
isb_status isb_energy(isb_ctx* ctx, isb_stream stream, const double* x, const double* x0,
                      const double* v0, const double* a, double* energy);
/* grad_x g(x), device out g [n_v][dim], 0 on pinned DOFs. */
isb_status isb_gradient(isb_ctx* ctx, isb_stream stream, const double* x, const double* x0,
                        const double* v0, const double* a, double* g);
/* Hessian-vector product hp = P H(x) P p with P the projection onto free DOFs (Eq. 10);
 * FP32 element arithmetic in ISB_MIXED. device [n_v][dim] in/out. */
isb_status isb_hessvec(isb_ctx* ctx, isb_stream stream, const double* x, const double* x0,
                       const double* a, const double* p, double* hp);
/* isb_hessvec for callers that cannot allocate device memory during the call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments, result and errors as
 * isb_hessvec, from the same kernels; no allocation and no library routine that allocates. The
 * product's staging (friction factor, vertex-term diagonal, masked operand, FP32 actuation in
 * ISB_MIXED: 8 (n_v (1 + 2 dim)) + 4 n_e bytes, each part rounded up to 256 B) lives in a fixed
 * 32 MiB array of device memory that every GPU the library runs on holds until the process ends;
 * a mesh that needs more returns ISB_E_ARG. Every call on one GPU shares that array, so calls that
 * overlap on one GPU (several streams or host threads) race; serialise them. Nothing in the array
 * needs to start at zero: each call writes every entry it reads. */
isb_status isb_hessvec_noalloc(isb_ctx* ctx, isb_stream stream, const double* x, const double* x0,
                               const double* a, const double* p, double* hp);
/* Element part of the Hessian-vector product only, added into hp: hp += sum_e W_e dP(F_e; dF_e(p)) Dm^-T
 * scattered to the element's vertices, plus the springs' K (p_j - p_i) (Eq. 10 without the vertex
 * terms and without the projection onto free DOFs), scaled by h^2 in backward Euler. This is the hot kernel of the CG iteration on
 * its own, for callers that add their own vertex terms and for timing. device [n_v][dim] in/in-out. */
isb_status isb_hessvec_elements(isb_ctx* ctx, isb_stream stream, const double* x, const double* a,
                                const double* p, double* hp);
/* Element part of the gradient only, added into g: g += sum_e W_e P(F_e) Dm^-T scattered to the
 * element's vertices (Eq. 4-5), plus the springs' forces (no vertex terms, no projection onto free
 * DOFs), scaled by h^2 in backward Euler; FP64 in both precisions. The gradient kernel on its own,
 * for callers that add their own vertex terms and for timing. device [n_v][dim] in/in-out. */
isb_status isb_gradient_elements(isb_ctx* ctx, isb_stream stream, const double* x, const double* a, double* g);
/* Diagonal of H(x) over free DOFs (1 on pinned DOFs), FP64 in both precisions, device out [n_v][dim]. */
isb_status isb_hessdiag(isb_ctx* ctx, isb_stream stream, const double* x, const double* x0,
                        const double* a, double* diag);

/* ---- bandwidth probe ------------------------------------------------------------------------ */

/* dst[i] = src[i] for i < n by a plain streaming copy kernel (one 16-byte load and store per
 * thread), enqueued on `stream` on the current device: timed around a large n,
 * it gives the HBM ceiling the element and solver kernels are compared with. Device buffers of n
 * doubles owned by the caller, 16-byte aligned, not overlapping; n >= 0 (n == 0 does nothing).
 * Returns ISB_E_ARG for NULL or misaligned pointers or negative n. Needs no context. */
isb_status isb_stream_copy(isb_stream stream, const double* src, double* dst, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* ISB_H */
