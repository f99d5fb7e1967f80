/*
 * cans_poisson.h -- C ABI of the MI355X (gfx950) direct Poisson solver.
 *
 * The library solves the second-order finite-difference Poisson equation on a
 * staggered Cartesian grid, eq. (poi) of Costa et al., "GPU acceleration of
 * CaNS" (arXiv 2001.05234), Section 2, by eigenfunction expansion
 * (eq. (poi_reduced)): a real-to-real transform along x, then along y, chosen
 * by the boundary conditions of each axis (real DFT for periodic, DCT-II for
 * Neumann-Neumann, DST-II for Dirichlet-Dirichlet, DCT-IV / DST-IV for the
 * mixed pairs), one tridiagonal solve along z per (kx, ky) pair by Gauss
 * elimination without pivoting, then the inverse transforms.  x and y are
 * uniform; z may be stretched (the remark after eq. (poi_reduced)), in which
 * case the z operator is taken in conservative form
 *     [(p_{k+1}-p_k)/dzc_k - (p_k-p_{k-1})/dzc_{k-1}] / dzf_k,
 *     dzc_k = (dzf_k + dzf_{k+1})/2, mirror ghost cell at a wall.
 * Boundary conditions are homogeneous and located on the cell faces
 * (staggered): periodic p_0 = p_n; Neumann p_0 = p_1; Dirichlet p_0 = -p_1.
 * A field may instead live on the cell faces of an axis themselves (a
 * velocity component along its own direction, as in the implicit diffusion
 * steps of eq. (up_id_2)): CANS_BC_DIRICHLET_FACE and CANS_BC_NEUMANN_FACE
 * below, which take the DST-I, DCT-I and type-III transforms (the rest of
 * the transform types Section 3 lists for the CPU solver).
 *
 * Layout of every field: double, x fastest, element (i,j,k) at
 * i + nx*(j + ny*k), i.e. a C array [nz][ny][nx].
 *
 * All functions return CANS_OK (0) or a negative cans_status.  Nothing throws
 * across this interface.  Device pointers are HIP device memory of the
 * device that was current when the plan was created.
 */
#ifndef CANS_POISSON_H
#define CANS_POISSON_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary condition of one face */
enum cans_bc {
    CANS_BC_PERIODIC = 0,
    CANS_BC_NEUMANN = 1,
    CANS_BC_DIRICHLET = 2,
    /* z only, on both z faces: Dirichlet for a field located on the z faces
       instead of the cell centres, zero on the two wall faces -- the
       wall-normal velocity of the implicit diffusion steps, eq. (up_id_2).
       The nz unknowns of a column are the interior faces of a grid of nz+1
       cells, and dz then holds those nz+1 cell widths.  Row k of the z
       operator is
         [(w_{k+1}-w_k)/dz_{k+1} - (w_k-w_{k-1})/dz_k] / ((dz_k + dz_{k+1})/2)
       with w_{-1} = w_nz = 0.  Never singular; element (i,j,k) of rhs and p
       is the value on face k (between cells k and k+1). */
    CANS_BC_DIRICHLET_FACE = 3,
    /* A field located on the faces of x or y (codes 3 and 4, both ends of the
       axis one of them): code 3 is Dirichlet on the boundary face (the field
       is zero there and the face is no unknown), code 4 Neumann on the
       boundary face (the face is an unknown and the field is mirrored about
       it, w_{-1} = w_1).  With C cells of width dx along x the nx unknowns
       are the C-1 interior faces for (3,3) (DST-I), all C+1 faces for (4,4)
       (DCT-I), and the C faces other than the Dirichlet one for (3,4) (a
       DST-III) and (4,3) (a DCT-III); element i is the i-th of those faces
       from x-.  The operator is (w_{i-1} - 2 w_i + w_{i+1})/dx^2.  Along z
       only (3,3).  A problem that a (4,4) pair would make singular (shift 0,
       every other axis periodic or Neumann) is unsupported; so are the
       dense transform, the projection step and the time-step bound on such
       an axis. */
    CANS_BC_NEUMANN_FACE = 4
};

enum cans_status {
    CANS_OK = 0,
    CANS_ERR_INVALID_ARG = -1,  /* bad size, spacing, pointer or boundary pair */
    CANS_ERR_UNSUPPORTED = -2,  /* valid problem the library does not handle
                                   (an x/y transform line that is odd, > 4096 or not
                                   {2,3,5}-smooth -- see cans_poisson_plan --,
                                   periodic z that is stretched or shorter
                                   than 3 cells, a transform form the options
                                   do not allow, shift > 0) */
    CANS_ERR_ALLOC = -3,        /* device or host allocation failed */
    CANS_ERR_HIP = -4,          /* HIP runtime or launch error */
    CANS_ERR_ALIAS = -5,        /* rhs == p where the mode forbids it */
    CANS_ERR_TOO_LARGE = -6     /* the problem's workspace exceeds the fixed
                                   scratch of cans_poisson_solve_noalloc */
};

/* arithmetic of the transforms (the z elimination is always FP64) */
enum cans_precision {
    CANS_PREC_FP64 = 0,         /* everything FP64 */
    CANS_PREC_FP32_REFINE = 1   /* FP32 transforms, FP64 z elimination, FP64
                                   residual and iterative refinement */
};

/* how the transform along an axis is evaluated */
enum cans_xform_mode {
    CANS_XFORM_AUTO = 0,
    CANS_XFORM_FFT = 1,         /* LDS radix FFT with fused pre/post twiddles */
    CANS_XFORM_DENSE = 2        /* dense matrix product on the matrix cores,
                                   split-bf16 operands, FP32 accumulation
                                   (FP32_REFINE only; x axis only; nx = 128,
                                   256, 384 or 512) */
};

typedef struct cans_opts {
    int precision;      /* enum cans_precision, default FP64 */
    int xform_x;        /* enum cans_xform_mode for x, default AUTO */
    int xform_y;        /* enum cans_xform_mode for y, default AUTO */
    double tol;         /* FP32_REFINE: stop when the relative residual
                           ||Pi f - L p||_2 / ||Pi f||_2 <= tol; default 1e-10 */
    int max_iter;       /* FP32_REFINE: most refinement steps enqueued per
                           solve (0..16); default 4.  The solve is enqueued
                           without a host synchronisation, so all max_iter
                           steps are launched; those after convergence return
                           at once but still cost their six launches (about
                           12 us per step on MI355X, which is what separates
                           max_iter 1 and 4 on a 32^3 grid: 0.108 vs 0.144
                           ms).  Small problems that converge in one step
                           gain from max_iter 1 or 2. */
    int autotune;       /* 1: at plan time, time candidate transform tiles
                           (lines per tile, radix-8 or radix-4 first) for
                           every transform kernel the plan uses on the
                           current device and keep the fastest; with
                           xform_x AUTO on a single-problem FP32_REFINE plan
                           whose x axis the dense form takes, also time whole
                           refined solves with either x form and keep the
                           faster (batched plans keep the FFT form, which
                           joins the batch's grouped launches)
                           (allocates temporary fields and synchronises);
                           0: built-in choice (FFT).  Default 0. */
    int graph;          /* 1: cans_poisson_solve records the solve's kernel
                           sequence into a HIP graph on its first call with a
                           given (rhs, p) pair and replays it on later calls
                           with the same pair (one launch per solve instead of
                           some 5 to 35); a new pair records again.  The
                           recording allocates graph resources on the first
                           call.  0: kernels are launched one by one.  Batched
                           plans always use a graph.  Default 0. */
    double shift;       /* s <= 0: solve the Helmholtz form (L_h + s) p = f of
                           implicit diffusion (eq. (up_id_2): s = -2/(gamma_k
                           nu dt)) for a cell-centred quantity: the same
                           expansion, every column's diagonal moved by s; no
                           singular case when s < 0.  s > 0 (indefinite) is
                           unsupported.  Default 0: eq. (poi). */
} cans_opts;

#define CANS_HISTORY 17

typedef struct cans_info {
    int iterations;         /* refinement corrections applied (0 for FP64) */
    int converged;          /* 1 if the residual test passed (always 1 for FP64) */
    double residual;        /* last relative residual measured (FP32_REFINE);
                               -1 when not measured (FP64) */
    double history[CANS_HISTORY]; /* relative residual before each correction
                                     and after the last; unused entries -1 */
    double removed_mean;    /* singular problems (every axis periodic or
                               Neumann-Neumann): dzf-weighted mean of the rhs
                               removed to make it compatible; else 0 */
    double residual_inf;    /* max-norm form of the last residual check,
                               max|Pi f - L_h p| / max|Pi f| (FP32_REFINE);
                               -1 when not measured (FP64) */
} cans_info;

typedef struct cans_plan_s *cans_plan_t;

/* Fill *opts with the defaults listed above. */
void cans_default_opts(cans_opts *opts);

/*
 * Build a plan for an nx x ny x nz grid (Section 2, eqs. (poi) and
 * (poi_reduced)).
 *   bc[6]  = {x-, x+, y-, y+, z-, z+}, enum cans_bc; periodic must be paired
 *            with periodic on the same axis.
 *   dx, dy = uniform spacings (> 0).
 *   dz     = host array of nz cell widths dzf (> 0), copied into the plan; a
 *            periodic z must be uniform.  With CANS_BC_DIRICHLET_FACE on z:
 *            the nz+1 widths of the cells around the face-located unknowns.
 *   nx, ny: the line the transform sees -- the line itself, or for a
 *            face-located (3,3) / (4,4) pair its odd / even extension of
 *            2(n+1) / 2(n-1) reals -- has an even length of at most 4096
 *            whose half is a product of 2, 3 and 5 (so n even for the
 *            cell-centred pairs and the face pairs (3,4), (4,3));
 *   nz >= 1 (>= 3 if periodic).
 * The plan owns its tables and device workspace (allocated on the current
 * device).  One solve may be in flight per plan at a time.
 */
int cans_poisson_plan(cans_plan_t *out, int nx, int ny, int nz, const int bc[6],
                      double dx, double dy, const double *dz);

/* As cans_poisson_plan, with options (NULL = defaults). */
int cans_poisson_plan_ex(cans_plan_t *out, int nx, int ny, int nz, const int bc[6],
                         double dx, double dy, const double *dz, const cans_opts *opts);

/*
 * Enqueue one solve of L_h p = rhs, eq. (poi) of Section 2, by the
 * eigenfunction expansion that follows it (eq. (poi_reduced)): forward
 * transform along x, then y; one tridiagonal solve along z per (kx, ky) pair
 * by Gauss elimination; inverse transforms along y, then x.  FP32_REFINE plans
 * run the transforms in FP32 and correct p by iterative refinement on the FP64
 * residual of eq. (poi) until opts.tol (the z elimination stays FP64).
 * Enqueued on `stream`; the call returns without host synchronisation.  rhs and p are device arrays of nx*ny*nz doubles owned by
 * the caller, alive until the stream work completes.  FP64 mode allows
 * rhs == p (in place); FP32_REFINE re-reads rhs and returns CANS_ERR_ALIAS
 * for rhs == p.  For a singular problem the rhs is projected on the range
 * (its dzf-weighted mean removed) and p is returned with zero dzf-weighted
 * mean.  Errors here are enqueue-time errors only; convergence is reported by
 * cans_poisson_get_info.
 */
int cans_poisson_solve(cans_plan_t plan, const double *rhs, double *p, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as cans_poisson_solve, with the same arguments, results and rules,
 * but every per-solve device buffer it writes (the FP32 spectral field of
 * FP32_REFINE plans, block partial sums, the info record, the convergence
 * flag, the z-solve tile counters, and the plain elimination's multipliers
 * where nz needs them) carved from one fixed array compiled into the library,
 * CANS_NOALLOC_SCRATCH_BYTES bytes per device, held until the process ends.
 * The call allocates nothing: no hipMalloc, no graph (opts.graph is ignored,
 * kernels are launched directly).  Plans with more than one problem give
 * CANS_ERR_INVALID_ARG, a problem whose buffers exceed the array gives
 * CANS_ERR_TOO_LARGE (FP32_REFINE: about 4 bytes per grid point, so up to
 * roughly 20 million points; FP64 plans need a few hundred bytes unless nz >
 * 512 or z is periodic with nz > 128, which need 16-24 bytes per point), and a
 * current device other than the plan's gives CANS_ERR_INVALID_ARG.  The info
 * record is copied into the plan's at the end, so cans_poisson_get_info
 * reports this solve after a stream sync.  Every call on one device shares
 * that device's array: calls that overlap on one device (other streams or
 * threads, before the previous one completed) race and give wrong results.
 */
#define CANS_NOALLOC_SCRATCH_BYTES (80u << 20)
int cans_poisson_solve_noalloc(cans_plan_t plan, const double *rhs, double *p, hipStream_t stream);

/*
 * Enqueue one projection (pressure-correction) step, the equations that
 * follow eq. (up): Phi solves L_h Phi = D u / gdt, then u -= gdt G Phi and
 * p += Phi, with gdt = gamma_k dt > 0 of the Runge-Kutta substep.
 *   u, v, w = staggered velocity (device, nx*ny*nz doubles each, x fastest):
 *             element (i,j,k) of u lies on the +x face of cell (i,j,k), of v
 *             on its +y face, of w on its +z face.  Updated in place.
 *   p       = pressure (device, nx*ny*nz doubles), incremented by Phi.
 * D u = (u - u_below)/dx + (v - v_below)/dy + (w - w_below)/dzf_k and G Phi =
 * (Phi_next - Phi)/dx, /dy, /dzc_k.  Every axis must be periodic (the face
 * below the first cell is the last face) or bounded by walls (Neumann pairs:
 * zero normal velocity below the first cell; the last face is the wall, its
 * value is used as given and left unchanged).  Phi has zero dzf-weighted
 * mean; the weighted mean removed from D u / gdt is reported by
 * cans_poisson_get_info.  The plan must be a single FP64 plan without shift
 * and every pair periodic or Neumann, else CANS_ERR_UNSUPPORTED; u, v, w, p
 * must be distinct arrays (CANS_ERR_ALIAS).  The first call allocates the
 * plan's Phi field (nx*ny*nz doubles) on the current device, so that call is
 * not capturable in a HIP graph.  It shares the plan's Phi field and info
 * record, so, as for solves, one call may be in flight per plan.  Enqueued
 * on `stream`; no host synchronisation.
 */
int cans_poisson_project(cans_plan_t plan, double *u, double *v, double *w, double *p, double gdt,
                         hipStream_t stream);

/*
 * cans_poisson_project with the two other pieces of a Runge-Kutta substep
 * that sit on the same fields (Section 2, "Numerical method"):
 *   alpha  = gamma_k nu dt / 2 >= 0: the pressure update of implicit
 *            diffusion, p += Phi - alpha L_h Phi (the last equation after
 *            eq. (poi_ns_id)); alpha = 0 gives the explicit-diffusion update
 *            p += Phi of cans_poisson_project.  L_h is the operator of
 *            eq. (poi) with the pressure's ghost rules.
 *   dt_max = NULL, or a device pointer to one double that receives the
 *            time-step bound of eq. (dt) on the corrected velocity:
 *            sqrt(3) / (largest advective rate), and with nu > 0 at most
 *            1.65 dl^2 / nu, dl = min(dx, dy, min dzf).  The advective rate is
 *            taken as the Listing of Section 3 takes it: at the +x, +y and +z
 *            face of every cell, the face-normal component plus the
 *            magnitudes of the four-point means of the other two, each over
 *            its spacing (dx, dy, dzf_k; the centre distance dzc_k at z faces,
 *            the wall cell's width on a wall face).  Beyond the last cell of a
 *            walled axis the tangential components are the no-slip mirror
 *            (negated); the normal component below the first cell is zero.  A
 *            velocity at rest with nu = 0 gives +inf.
 *   nu     >= 0: the viscosity of the viscous bound (0 omits it, as with
 *            implicit diffusion).
 * Layout, boundary rules, ownership, the one-call-in-flight rule and errors
 * are those of cans_poisson_project; a negative or non-finite alpha or nu is
 * CANS_ERR_INVALID_ARG and dt_max equal to one of the fields CANS_ERR_ALIAS.
 * The first projection call of a plan (either form) allocates Phi and a
 * table of 2048 block maxima.
 */
int cans_poisson_project_ex(cans_plan_t plan, double *u, double *v, double *w, double *p, double gdt,
                            double alpha, double nu, double *dt_max, hipStream_t stream);

/* Copy the last solve's cans_info to *out.  Synchronises with the device, so
 * it is meant to be called after the solve's stream has been synchronised. */
int cans_poisson_get_info(cans_plan_t plan, cans_info *out);

/* Release the plan and its device memory.  NULL is ignored. */
void cans_poisson_destroy(cans_plan_t plan);

/* Static text for a status code. */
const char *cans_status_string(int code);

/* Bytes of device workspace the plan holds. */
size_t cans_poisson_workspace_bytes(cans_plan_t plan);

/*
 * The form a single-problem plan evaluates the transform of an axis in
 * (axis 0 = x, 1 = y): CANS_XFORM_FFT or CANS_XFORM_DENSE, as the options
 * fixed it or, for CANS_XFORM_AUTO with autotune = 1 on a refinement plan
 * whose x axis the dense form takes, as the plan-time timing of whole
 * refined solves chose it (the transforms F^x, F^y of eq. (poi_reduced)
 * evaluated as FFTs or as dense matrix products); CANS_ERR_INVALID_ARG for
 * a bad handle, axis or a batched plan.
 */
int cans_poisson_xform_mode(cans_plan_t plan, int axis);

/*
 * Run one stage of a plan on device arrays of nx*ny*nz doubles (test and
 * timing hook).  FP64 plans (`in` and `out` may be equal):
 *   1 forward x transform      T_x along x
 *   2 forward y transform      T_y along y
 *   3 z solve on spectral data  (columns of eq. (poi_reduced)), rhs scaled by
 *                               1/(s_x s_y)
 *   4 inverse y transform      B_y along y
 *   5 inverse x transform      B_x along x
 * T is the unnormalised transform: real DFT (rows 1, (-1)^i, cos, -sin of
 * each wavenumber), DCT-II, DST-II, DCT-IV, DST-IV for P, NN, DD, ND, DN;
 * B satisfies B T = s I with s = n for P, NN, DD and s = n/2 for ND, DN.  Stages 1..5 composed equal one FP64 solve.
 * FP32_REFINE plans run single kernels on the plan's internal FP32 field:
 *   0 clear the refinement state (needed before 6 after a finished solve),
 *   1 in -> field (forward x), 2 / 4 forward / inverse y, 3 z solve,
 *   5 field -> out (inverse x), 6 residual of p = out for rhs = in fused with
 *   the forward x transform, 7 out += inverse x of the field, 8 residual
 *   norms of p = out for rhs = in (6 and 8 need state 0 first).
 */
int cans_poisson_debug_stage(cans_plan_t plan, int stage, const double *in, double *out,
                             hipStream_t stream);

/* ----------------------------------------------------------------------- */
/* Batched solves: many independent problems of different sizes and
 * boundary conditions enqueued as one unit. */
typedef struct cans_desc {
    int nx, ny, nz;
    int bc[6];
    double dx, dy;
    const double *dz;   /* host, nz cell widths (nz+1 for a face-located z) */
} cans_desc;

/* Build one plan holding `count` independent problems, each the eq. (poi)
 * problem of Section 2 with its own sizes, boundary pairs and spacings
 * (descs[i], validated as for cans_poisson_plan; dz is copied).  Every
 * problem gets the tables and workspace a single plan would; opts apply to
 * all of them.  On error nothing is allocated and *out is NULL. */
int cans_poisson_plan_batched(cans_plan_t *out, int count, const cans_desc *descs,
                              const cans_opts *opts);

/* Solve every problem of a batched plan, each by the expansion of
 * eq. (poi_reduced) (Section 2) as cans_poisson_solve does: rhs[i], p[i] are
 * device arrays of nx_i*ny_i*nz_i doubles of problem i.  The whole batch is one graph launch on `stream` (no host
 * synchronisation): the first call, and any call with different array
 * addresses, captures the kernels of all problems into a HIP graph whose
 * independent branches run problems concurrently; later calls replay it.
 * Same ownership and aliasing rules as cans_poisson_solve. */
int cans_poisson_solve_batched(cans_plan_t plan, const double *const *rhs, double *const *p,
                               hipStream_t stream);

/* Info of problem `index` of a batched plan (after a stream sync). */
int cans_poisson_get_info_batched(cans_plan_t plan, int index, cans_info *out);

#ifdef __cplusplus
}
#endif
#endif /* CANS_POISSON_H */
