/*
 * kfbi.h -- C ABI of libkfbi, an MI355X (gfx950) implementation of one evaluation of the
 * kernel-free boundary integral (KFBI) operator for 3D Stokes and Navier (linear elasticity)
 * Dirichlet problems on irregular domains, after Zhao, Dong and Ying, "Kernel free boundary
 * integral method for 3D Stokes and Navier equations on irregular domains".
 *
 * Plain C: no C++ or torch types cross this boundary.  Every call returns a kfbi_status;
 * on error the outputs are unspecified and kfbi_last_error() returns a message.  Nothing
 * aborts or throws.
 *
 * Memory: the caller owns every buffer passed in.  Arguments named *_dev are device
 * pointers (HIP device memory of the current device, float64, C-contiguous); *_host are
 * host pointers.  The library owns only what its context holds (geometry, sparse maps and
 * device workspaces), allocated in kfbi_create and released by kfbi_destroy.
 *
 * Ordering: work is issued on cfg.stream (a hipStream_t; NULL = a stream that kfbi_create
 * creates and kfbi_destroy destroys) and every call returns after its work has completed (the
 * CG and GMRES loops read scalars back to the host).  One context per thread/stream; contexts
 * are independent.
 *
 * Grid layout of exported fields (numpy C order [i][j][k] <-> (x, y, z), box [lo,hi]^3,
 * h = (hi-lo)/N): u1 has shape (N+1, N, N) with u1[i][j][k] the x-velocity at
 * (lo + i h, lo + (j+1/2) h, lo + (k+1/2) h) (i = 0 and N are box faces, zero); u2, u3 are
 * analogous; p has shape (N, N, N) at cell centres.  Packed u = u1 | u2 | u3.
 */
#ifndef KFBI_H
#define KFBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kfbi_ctx kfbi_ctx; /* opaque */

typedef enum {
  KFBI_OK = 0,
  KFBI_EINVAL = -1,  /* bad argument, non-finite input, unsupported size */
  KFBI_ENOMEM = -2,  /* host or device allocation failed */
  KFBI_EGEOM = -3,   /* geometry not resolved by the grid (too few fit neighbours, an
                        interpolation stencil or a crossed arm touching the box boundary) */
  KFBI_ENOCONV = -4, /* CG, refinement or GMRES did not reach its tolerance in maxit */
  KFBI_EDEVICE = -5  /* a HIP runtime call failed */
} kfbi_status;

/* Problem (Sec. 2 of the paper): Stokes  -mu lap u + grad p = f, div u = 0;
 * Navier  -mu lap u - (lambda+mu) grad div u = f, written in generalised Stokes form with
 * p = -(lambda+mu) div u and div u + p/(lambda+mu) = 0 (Remark 3.1). */
typedef enum { KFBI_STOKES = 0, KFBI_NAVIER = 1 } kfbi_pde;

/* Arithmetic of the MAC solve.  FP64: everything in float64.  MIXED_FP32: transforms and
 * inner Schur CG in float32 inside float64 residual refinement of the full MAC system;
 * corrections, jumps, interpolation, residuals and all dot products stay float64. */
typedef enum { KFBI_FP64 = 0, KFBI_MIXED_FP32 = 1 } kfbi_precision;

typedef enum { KFBI_SPHERE = 0, KFBI_ELLIPSOID = 1, KFBI_STAR = 2, KFBI_TORUS = 3 } kfbi_shape_kind;

/* How the trace K phi = 1/2 phi - M phi is read off the grid solution (Prop. 4.2 / 4.4,
 * Sec. 4.4).  AVERAGE (the default): 1/2 phi plus the mean of the interior and exterior
 * limits (-M phi = (u+ + u-)/2), both interpolated from the same ten grid nodes with the jump
 * function whose value part is the least-squares fitted value at the control point;
 * equivalently u+ + (1/2 - alpha)(phi - S phi) with alpha the exterior weight fraction of the
 * stencil and S phi the fitted value.  INTERIOR: the interior limit u+ alone, with the
 * density itself as the value part of the jump function.  The forms agree to the fit's
 * O(h^3) error on smooth densities; on grid-scale oscillations AVERAGE acts like 1/2 (as the
 * second-kind equation does) while INTERIOR acts like alpha in [0, 1], so GMRES needs a
 * mesh-dependent and several times larger number of iterations with INTERIOR. */
typedef enum { KFBI_TRACE_AVERAGE = 0, KFBI_TRACE_INTERIOR = 1 } kfbi_trace;

/* Omega = {psi <= 0}.  param: sphere R | ellipsoid semi-axes a,b,c (body axes rotated by
 * rot_z_deg about z) | star r0, eps, k, l with r = r0 + eps sin(k theta) cos(l phi),
 * theta = arccos(z/|x|), phi = atan2(y,x) | torus tube radius a, centre-line radius c. */
typedef struct {
  kfbi_shape_kind kind;
  double center[3];
  double param[6];
  double rot_z_deg;
} kfbi_shape;

typedef struct {
  int32_t N;          /* cells per axis; power of two, 16 <= N <= 512 */
  double lo, hi;      /* box [lo,hi]^3 */
  kfbi_pde pde;
  double mu, lambda;  /* lambda ignored for Stokes */
  kfbi_shape shape;
  kfbi_precision precision;
  double cg_rtol;     /* relative tolerance of the MAC solve (Schur CG residual for FP64,
                         full-system refinement residual for MIXED_FP32); <= 0: 1e-12 */
  int32_t cg_maxit;   /* <= 0: 2000 */
  double inner_rtol;  /* MIXED_FP32: tolerance of each float32 inner solve; <= 0: 1e-5 */
  double gmres_rtol;  /* <= 0: 1e-8 */
  int32_t gmres_maxit;/* <= 0: 200 */
  void* stream;       /* hipStream_t; NULL = a stream owned by the context */
  kfbi_trace trace;   /* trace form of K (eval, adjoint and the GMRES operator) */
} kfbi_config;

typedef struct {
  int32_t cg_iters;        /* total Schur CG iterations of the call */
  int32_t refine_rounds;   /* MIXED_FP32 refinement rounds of the last MAC solve */
  int32_t gmres_iters;
  double final_rel_residual;
  double ms_total;         /* device time of the call's evaluations (HIP events on the stream) */
  double ms_stage[6];      /* of which: [0] surface fit + jumps (and their transposes),
                              [1] corrections, [2] MAC right-hand side, [3] Schur CG iterations
                              and mixed refinement passes, [4] velocity back-substitution,
                              [5] interpolation (and probes) */
  double model_bytes;      /* algorithmic HBM bytes of the call's kernels: one read or write of
                              every field value or map entry touched, gathers counted per
                              element (model_bytes / ms_total = the call's effective bandwidth) */
} kfbi_info;

/* Host callback for body forces: fill out[i][3] with f at xyz[i][3], i < m. */
typedef void (*kfbi_vec_fn)(const double* xyz, int64_t m, double* out, void* user);

/* Builds the geometry and every sparse map (Algorithm 1 step 1): node classification,
 * crossings of the surface with the nine grid-line families, control points, local frames,
 * least-squares surface-fit weights, jump maps, correction arms and interpolation weights,
 * and uploads them.  *out receives a new context (NULL on error). */
kfbi_status kfbi_create(const kfbi_config* cfg, kfbi_ctx** out);
void kfbi_destroy(kfbi_ctx* ctx);
const char* kfbi_last_error(const kfbi_ctx* ctx);
/* Message of the last kfbi_create failure in this thread (kfbi_create has no context). */
const char* kfbi_create_error(void);

/* Number n of control points; the density and K phi are n x 3. */
kfbi_status kfbi_num_points(const kfbi_ctx* ctx, int64_t* n);
/* Control points and outward unit normals, host arrays [n][3] (normal may be NULL). */
kfbi_status kfbi_get_points(const kfbi_ctx* ctx, double* xyz_host, double* normal_host);
/* Number of crossings (surface points where jumps are evaluated) and of irregular MAC nodes
 * (grid equations that receive a correction term). */
kfbi_status kfbi_sizes(const kfbi_ctx* ctx, int64_t* n_crossings, int64_t* n_irregular);

/* K phi = 1/2 phi - M phi (Prop. 4.2 / 4.4) at the control points, read off the double-layer
 * interface problem  -mu lap u + grad p = 0, div u + c p = 0 off the surface, [[u]] = phi,
 * [[sigma n]] = 0, u = 0 on the box (Sec. 4.4 interpolation), in the context's trace form:
 * AVERAGE (default) 1/2 phi + (u+ + u-)/2, INTERIOR the interior limit u+.  phi_dev, out_dev:
 * [n][3] float64 device arrays (may not alias).  info may be NULL.  A non-finite phi gives
 * EINVAL. */
kfbi_status kfbi_eval(kfbi_ctx* ctx, const double* phi_dev, double* out_dev, kfbi_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): kfbi_eval with every per-call work buffer
 * (MAC solver fields, right-hand side, grid solution, surface-stage values, partial sums)
 * carved from a static device array of KFBI_NOALLOC_MAX_BYTES that each device holds until
 * the process ends, instead of the context's own workspaces; it calls no allocator.  Same
 * arguments, result and errors as kfbi_eval, and EINVAL when the context's evaluation needs
 * more scratch than the limit (64 MiB: N <= 64 in either precision).  All calls on one device
 * share that device's array: calls that overlap in time on one device (several host threads or
 * streams) race and must be serialised by the caller. */
#define KFBI_NOALLOC_MAX_BYTES (64ull << 20)
kfbi_status kfbi_eval_noalloc(kfbi_ctx* ctx, const double* phi_dev, double* out_dev, kfbi_info* info);

/* K phi for several densities in one call (Sec. 3: the second-kind equation is linear, so the
 * densities of several boundary data, finite-difference directions or Krylov blocks can be
 * evaluated together): out[r] = K phi[r] for r < nrhs (1 <= nrhs <= KFBI_BATCH_MAX),
 * phi_dev and out_dev [nrhs][n][3] float64 device arrays.  The right-hand sides run in lockstep:
 * every kernel serves all of them (the surface fit weights and jump maps are read once per
 * group of four), their Schur CG and refinement scalars come back to the host in one copy per
 * iteration, and each right-hand side stops by the same rule as its own kfbi_eval, so the
 * results equal those of nrhs calls to rounding.  The context keeps nrhs work arenas (each the
 * size of one evaluation's work buffers) for later batches; ENOMEM if they cannot be
 * allocated.  info: CG iterations summed over the right-hand sides, the largest refinement
 * count, the call's device time and model bytes. */
#define KFBI_BATCH_MAX 64
kfbi_status kfbi_eval_batch(kfbi_ctx* ctx, int32_t nrhs, const double* phi_dev, double* out_dev, kfbi_info* info);

/* Transpose of kfbi_eval (in the context's trace form): out = K^T w (same shapes). */
kfbi_status kfbi_eval_adjoint(kfbi_ctx* ctx, const double* w_dev, double* out_dev, kfbi_info* info);

/* Dirichlet BVP (Sec. 3, Algorithm 1 step 3): u = g at the control points, body force f
 * (f == NULL: zero).  Volume trace b, GMRES (zero initial guess, unrestarted) on
 * K phi = g - b to gmres_rtol, then the unified interface solve.  g_dev, phi_dev: [n][3]
 * device; u_dev (packed u1|u2|u3 in the exported layout) and p_dev ([N][N][N]) are optional
 * (NULL = not returned). */
kfbi_status kfbi_solve_bvp(kfbi_ctx* ctx, const double* g_dev, kfbi_vec_fn f, void* f_user,
                           double* phi_dev, double* u_dev, double* p_dev, kfbi_info* info);

/* Grid velocity of the unified interface solve for density phi (and the body force of the
 * last kfbi_solve_bvp with f != NULL if use_force != 0), exported layout. */
kfbi_status kfbi_interface_solve(kfbi_ctx* ctx, const double* phi_dev, int32_t use_force,
                                 double* u_dev, double* p_dev, kfbi_info* info);

/* Probes for losses on interior values (the differentiation layer; not in the paper): m
 * points, host array [m][3]; each velocity component is interpolated trilinearly from its
 * face grid, so the 8 nodes of every probe's cell must be interior nodes (EINVAL otherwise).
 * Replaces earlier probes. */
kfbi_status kfbi_set_probes(kfbi_ctx* ctx, const double* xyz_host, int64_t m);
/* Velocity at the probes ([m][3] device) of the unified interface solve with density phi
 * (and the stored body force of the last kfbi_solve_bvp if use_force != 0). */
kfbi_status kfbi_probe(kfbi_ctx* ctx, const double* phi_dev, int32_t use_force, double* vals_dev,
                       kfbi_info* info);
/* Transpose of phi -> probe values (the affine body-force part drops out): phi_bar [n][3]. */
kfbi_status kfbi_probe_adjoint(kfbi_ctx* ctx, const double* vals_bar_dev, double* phi_bar_dev,
                               kfbi_info* info);
/* y = K^{-T} rhs by unrestarted GMRES with kfbi_eval_adjoint as the operator (zero initial
 * guess, gmres_rtol, gmres_maxit): the adjoint of the second-kind equation of Sec. 3, used for
 * gradients with respect to the Dirichlet data. */
kfbi_status kfbi_solve_adjoint(kfbi_ctx* ctx, const double* rhs_dev, double* y_dev, kfbi_info* info);
/* Reverse mode of the probe values of the Dirichlet BVP (Sec. 3: phi = K^{-1}(g - b), the
 * representation u = G f - M phi read at the probes): for the cotangent vals_bar [m][3] of
 * the probe values, phi_bar = P^T vals_bar (P: density -> probe values of the unified
 * interface solve) and g_bar = K^{-T} phi_bar (GMRES on the transposed operator, as
 * kfbi_solve_adjoint).  Either output may be NULL (not both); [n][3] device arrays. */
kfbi_status kfbi_solve_bvp_adjoint(kfbi_ctx* ctx, const double* vals_bar_dev, double* g_bar_dev,
                                   double* phi_bar_dev, kfbi_info* info);

/* Kernels of the MAC solver that the measurement helpers can time: the single transform
 * pass (kind 0 DCT-II, 1 DST-II, 2 DCT-III, 3 DST-III, 4 DST-I, along one axis) and the
 * fused kernels of one Schur-complement CG iteration. */
enum {
  KFBI_K_XMID = 5, /* x: forward transform, spectral weight, inverse, three components */
  KFBI_K_ZFWD = 6, /* x += alpha d, r -= alpha (q - mean q), d = r + beta d, DST-II_z d and DCT-II_z d */
  KFBI_K_ZINV = 7, /* q = DST-III_z A + DCT-III_z B + c d, partial dot products */
  KFBI_K_YFWD = 8, /* DST-II_y A and DCT-II_y A */
  KFBI_K_YINV = 9,  /* DST-III_y A1 + DCT-III_y B2 */
  KFBI_K_GEMM_X = 10 /* DCT-II along x as a split-bfloat16 matrix product on the matrix cores
                        (MIXED_FP32 contexts, N = 128, 256, 512; a measured alternative to the
                        radix pass, not used by the evaluation) */
};

/* Measurement helper: launches one kernel of the context's MAC solver (kind: a transform
 * kind 0..4 along axis 0..2, or a KFBI_K_* fused kernel; precision of the context's inner
 * solver) reps times back to back on the context stream between two HIP events, on the
 * solver's own work fields (contents are overwritten).  Returns the mean duration of one
 * launch and the algorithmic HBM bytes of one launch (one read or write per N^3 field
 * touched: 2 fields for a transform pass, 6 XMID, 9 ZFWD, 4 ZINV, 3 YFWD, 3 YINV). */
kfbi_status kfbi_time_pass(kfbi_ctx* ctx, int32_t kind, int32_t axis, int32_t reps, double* avg_ms,
                           double* bytes_per_launch);

/* Transform helper (for checking the transform engine): out = the one-dimensional pass `kind`
 * (0 DCT-II, 1 DST-II, 2 DCT-III, 3 DST-III, all orthonormal, length N; 4 DST-I on indices
 * 1..N-1 of the axis, index 0 being the box face: out 0 there; or KFBI_K_GEMM_X, the DCT-II
 * along x on the matrix cores) of in along axis (0 x, 1 y, 2 z) for an N^3 field, layout
 * [x][y][z], computed in the context's inner precision (float32 for MIXED_FP32): in_dev and
 * out_dev are float64 device arrays of N^3 values (may alias). */
kfbi_status kfbi_apply_pass(kfbi_ctx* ctx, int32_t kind, int32_t axis, const double* in_dev, double* out_dev);

/* Measurement helper: live timing of one kernel (kind as above; for transform passes axis
 * 0..2 or -1 for every axis) inside the evaluations.  Calling it returns the launches and summed duration recorded since the
 * previous call (HIP events around every matching launch on the context stream) and the
 * algorithmic bytes of one launch, then resets the counters and enables (enable != 0) or
 * disables the timing. */
kfbi_status kfbi_profile_pass(kfbi_ctx* ctx, int32_t kind, int32_t axis, int32_t enable, int64_t* launches,
                              double* total_ms, double* bytes_per_launch);

/* Host-only setup (no device is touched): the same geometry and maps as kfbi_create, for
 * inspection and testing on machines without a GPU. */
typedef struct kfbi_plan kfbi_plan;
kfbi_status kfbi_plan_create(const kfbi_config* cfg, kfbi_plan** out);
void kfbi_plan_destroy(kfbi_plan* plan);
/* Copies the named host array into out (if non-NULL) and returns its element count, or -1
 * for an unknown name.  Names: xyz normal t1 t2 kappa (float64, per crossing), fam line1
 * line2 (int32), cp_target (int64), nb_ptr (int64) nb_idx (int32) fitw (float64, 6 per
 * neighbour entry), jmap (5x18 per crossing) jfmap (5x3) emap (3x18 per control point, then
 * 3x3), stab_a (1/2 - exterior weight fraction, 3 per control point), sv_ptr (int64) sv_idx
 * (int32) sv_w (fitted-value weights of the control points, CSR over control points), irr_node irr_ptr (int64) arm_t (int32) arm_o (int8) arm_a (3 per arm), itp_idx
 * (int64) itp_w (10 per control point and component), side0 side1 side2 sidep (uint8 N^3,
 * face index 0..N-1 along the face normal). */
int64_t kfbi_plan_get(const kfbi_plan* plan, const char* name, void* out);

#ifdef __cplusplus
}
#endif
#endif /* KFBI_H */
