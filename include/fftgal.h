/*
 * fftgal -- guaranteed bounds on the homogenized conductivity of a periodic
 * medium by the Fourier-Galerkin method with exact integration (the "Ga"
 * scheme of J. Vondrejc, arXiv:1412.2033), on one AMD MI355X (gfx950).
 *
 * Problem (Sec. 1.1, eq. intro_HP; Def. homog_problem): for a Y-periodic,
 * symmetric, uniformly elliptic A(x) on the unit cell Y = (-1/2, 1/2)^d,
 * d in {2, 3}, find A_H.  The Ga scheme (Def. Ga, eq. Ga) minimises the exact
 * energy over trigonometric fields of odd order N (eq. N_odd): the primal
 * minimum over E_N gives A_{H,N}, the dual minimum of the A^{-1} energy over
 * J_N gives B_{H,N}, and Prop. struct_bounds gives
 *
 *      B_{H,N}^{-1}  <=  A_H  <=  A_{H,N}        (Loewner order),
 *
 * guaranteed because the energies are evaluated exactly by the double-grid
 * quadrature of Lemma integ_eval_VM on M >= 2N-1 points per axis.  Each
 * minimiser is found by conjugate gradients (Remark CG) on the linear systems
 * of Cor. Ga_linsys (eq. Ga_linsys_orig), whose matrix-vector product is
 * Algorithm 2 (material multiply, FFT, projection, inverse FFT).
 *
 * Conventions.  Axis 1 is the slowest in every array; frequencies and grid
 * points follow eqs. index_set and grid_points; the M-grid point with index j
 * is x = j/M (mod 1).  M is the smallest odd 3,5,7-smooth integer >= 2N-1
 * (Lemma integ_eval_VM allows any M >= 2N-1; the bounds do not depend on it).
 *
 * Memory.  The library never allocates device memory: the caller passes one
 * device workspace of fftgal_workspace_bytes() bytes and a HIP stream (as a
 * void*; NULL is the default stream) to fftgal_plan().  All device work of a
 * plan is ordered on that stream.  Host arrays passed in are copied before the
 * call returns.  The plan object itself is host memory owned by the library
 * and released by fftgal_destroy().  One plan must not be used from two
 * threads at once; distinct plans are independent (no global mutable state).
 *
 * Errors.  Every entry point returns an fftgal_status code and never aborts;
 * fftgal_last_error() gives a message for the last failing call on a plan
 * (or for a failing fftgal_plan() when called with NULL).
 */
#ifndef FFTGAL_H
#define FFTGAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fftgal_status {
    FFTGAL_OK = 0,
    FFTGAL_EINVAL = -1,     /* invalid argument (message says which)            */
    FFTGAL_ENOMEM = -2,     /* workspace smaller than fftgal_workspace_bytes()   */
    FFTGAL_EDEVICE = -3,    /* a HIP call failed                                */
    FFTGAL_ENOTCONV = -4,   /* CG stopped at maxit, or (FP32_ITER) stalled by
                               rounding; the field kept is still admissible, so
                               fftgal_bounds() still returns guaranteed bounds */
    FFTGAL_ESTATE = -5,     /* call out of order (e.g. bounds before solves)     */
    FFTGAL_EBREAKDOWN = -6  /* CG breakdown: (p, Kp) <= 0 or not finite (a
                               non-SPD or non-finite material)                   */
};

enum fftgal_precision {
    FFTGAL_FP64 = 0,      /* every step in FP64                                  */
    FFTGAL_FP32_ITER = 1  /* CG iterations (FFTs, projection, material multiply,
                             vector updates) in FP32 with inner products
                             accumulated in FP64; the final re-projection and the
                             bound quadrature in FP64                            */
};

/* Layout flag of the reduced Ga (or-ed into `precision` of
 * fftgal_workspace_bytes_reduced and fftgal_plan_reduced): one set of transform
 * intermediates, the 2^d shifts of every operator pass run one after another
 * (smallest workspace).  Without it every shift has intermediates and a
 * projected vector of its own and the shifts of a pass share one launch
 * (faster, larger workspace).  EINVAL with the other plan kinds. */
#define FFTGAL_REDUCED_LEAN 0x100

/* Flag or-ed into `precision` of fftgal_workspace_bytes* and fftgal_plan /
 * fftgal_plan_static: the plan stores the material as d (d + 1) / 2 fields per
 * side (the entries of the symmetric A_M and B_M of eq. MBA_GA) instead of one
 * scalar field with constant matrices.  Materials without that scalar form
 * need it: matrix voxel images (image_tensor) and inclusion sets whose phases
 * differ and are not all isotropic (eq. inclcomp with one SPD A_i per
 * inclusion).  Ga plans only (EINVAL with GaNi and reduced plans); the
 * workspace grows by (d (d + 1) / 2 - 1) material fields per side. */
#define FFTGAL_TENSOR 0x200

/* Flag or-ed into `precision` of fftgal_workspace_bytes* and fftgal_plan /
 * fftgal_plan_gani: the plan keeps 2d copies of the per-solve buffers (transform
 * intermediates, CG vectors, partial sums), so that all its d primal and d dual
 * solves can run at once -- as members of a batch, or through
 * fftgal_solve_all.  Without it a plan runs one solve at a time.  The
 * workspace grows by 2d - 1 copies of that region plus the internal batch of
 * fftgal_solve_all.  EINVAL with reduced plans. */
#define FFTGAL_CONCURRENT 0x400

/* Flag or-ed into `precision` of fftgal_workspace_bytes* and the plan
 * constructors.  By default the CG iterations of 2D Ga plans whose double
 * grid is 81 x 81 (N = 41, or smaller N with FFTGAL_FAST_GRID; FP32-iteration
 * form also 81 or 125 on either axis) run entirely inside one work-group per
 * solve: the CG vectors
 * in registers, the operator of Algorithm 2 on the M_1 x M_2 grid in LDS, the
 * update and the stopping test in the same kernel, many iterations per launch
 * (timing class FFTGAL_K_SOLO).  Solves of such plans in a batch run that way
 * too, side by side on a stream of the batch's own.  The flag keeps these
 * plans on the per-pass kernels instead (one launch per pass and iteration).
 * Both forms compute the same iterations; their results agree to rounding.
 * It changes no workspace size. */
#define FFTGAL_SEPARATE_PASSES 0x800

/* Flag or-ed into `precision` of fftgal_workspace_bytes* and fftgal_plan /
 * fftgal_plan_static.  By default a Ga plan takes per axis the smallest
 * 3,5,7-smooth double grid M >= 2N - 1.  With the flag it takes instead the
 * smallest length with specialised kernels (81, 125, 225, 245, 729 or 2025
 * points) at least 2N - 1 on each axis whose default length is at least 9,
 * when the grid then holds at most four times the points of the default grid
 * or at most 2^21 points (else the default grid).  The double-grid
 * quadrature is exact for every M >= 2N - 1 (Lemma integ_eval_VM, eq. MBA_GA),
 * so the bounds are those of the default grid up to rounding.  The specialised
 * transforms run several times faster per point than the generic ones, and the
 * workspace grows with the grid.  fftgal_grid_size reports the grid taken.
 * EINVAL with GaNi and reduced plans, whose grids the scheme fixes. */
#define FFTGAL_FAST_GRID 0x1000

enum fftgal_material_kind {
    FFTGAL_INCLUSIONS = 0, /* eq. inclcomp: matrix phase plus inclusions          */
    FFTGAL_VOXELS = 1      /* eq. gridcomp: piecewise-constant voxel image        */
};

enum fftgal_shape {
    FFTGAL_RECT = 0, /* box |x_a - c_a| < h_a / 2 (eq. def_cube)                 */
    FFTGAL_CIRC = 1  /* disc |x - c| < r, d = 2 only (eq. char_func_Four)         */
};

/*
 * Material description (host memory; copied by fftgal_set_material).
 *
 * FFTGAL_INCLUSIONS (eq. inclcomp, eq. inclcomp_formula): A0 is the matrix
 *   phase (d x d, row-major, SPD).  Inclusion i has shape[i], centre
 *   center[i*d .. i*d+d-1] in the cell, size[i*d ..] = side lengths h
 *   (0 < h_a <= 1) for RECT or size[i*d] = radius r (0 < r <= 1/2) for CIRC,
 *   and ABSOLUTE conductivity A_in[i*d*d ..] (SPD; not the increment
 *   A_i = A_in - A0 of eq. inclcomp, because the dual needs A_in^{-1}).
 *   Inclusions must not overlap (periodic minimum image); the dual material
 *   is then A^{-1} = A0^{-1} + sum_i f_i [A_in^{-1} - A0^{-1}].  Any plan
 *   takes all A_in equal (two-phase, any SPD matrices) or A0 and every A_in
 *   isotropic (multiples of I); a plan made with FFTGAL_TENSOR takes any SPD
 *   A0 and A_in (one per inclusion).
 * FFTGAL_VOXELS (eq. gridcomp with psi = rect_{1/P}, Lemma grid_compos,
 *   Remark eval_with_FFT): image holds P[0]*...*P[d-1] positive scalar
 *   conductivities, row-major, voxel p centred at x = p/P; the dual uses
 *   1/image.  With image_tensor non-zero (plans made with FFTGAL_TENSOR) it
 *   holds instead one symmetric positive definite d x d matrix C^p per voxel
 *   (P[0]*...*P[d-1]*d*d doubles, voxel-major, each matrix row-major), and
 *   the dual uses the voxel-wise inverse (C^p)^{-1}.  Each P[a] must be odd
 *   (lengths that are not 3,5,7-smooth are transformed by Bluestein's chirp
 *   convolution, through the generic kernels).  If image_device is non-zero, image is a device
 *   pointer that is read (stream-ordered, on the plan's stream) during
 *   fftgal_set_material only and validated on the device; otherwise it is
 *   host memory (a matrix image is then copied in chunks through the plan's
 *   scratch).  Voxels that are not positive (scalars) or not finite,
 *   symmetric and positive definite (matrices) give EINVAL.
 */
typedef struct fftgal_material {
    int32_t kind;
    double A0[9];
    int32_t n_incl;
    const int32_t *shape;
    const double *center;
    const double *size;
    const double *A_in;
    int32_t P[3];
    const double *image;
    int32_t image_device;
    /* optional second image of the same resolution and residency for the dual
     * side (NULL: the same image): the primal solves use `image`, the dual
     * solves its voxel-wise inverse 1 / image_dual -- upper and lower
     * approximations of A for Lemma bounds_bounds */
    const double *image_dual;
    /* non-zero: image (and image_dual) hold a d x d matrix per voxel */
    int32_t image_tensor;
} fftgal_material;

/* Outcome of one CG solve (Remark CG). */
typedef struct fftgal_info {
    int32_t iters;      /* CG iterations taken                                  */
    int32_t converged;  /* 1 if the stopping test was met within maxit          */
    double rel_res;     /* ||r_k|| / ||b|| at exit (0 if b = 0)                  */
    double res0;        /* ||b|| (= ||r_0|| from e_0 = 0), (.,.)_{R^{d x M}}    */
    int32_t stagnated;  /* FP32_ITER only: 1 if the iteration stopped because
                           FP32 rounding stalled it (see fftgal_solve_primal)   */
    int32_t iterate;    /* the CG iteration whose field the plan keeps           */
} fftgal_info;

/*
 * Bytes of device workspace a plan of dimension d (2 or 3), orders N[0..d-1]
 * (odd, >= 1) and precision needs; 0 if the arguments are invalid.  Used for
 * admission by HBM footprint.  If voxel images with resolution P other than
 * the plan's M will be set, pass the largest P through fftgal_workspace_bytes_p.
 */
size_t fftgal_workspace_bytes(int d, const int32_t *N, int precision);
size_t fftgal_workspace_bytes_p(int d, const int32_t *N, int precision, const int32_t *P);

/*
 * Create a plan on `dev_workspace` (device pointer, 256-byte aligned, at least
 * fftgal_workspace_bytes() bytes; owned by the caller and used until
 * fftgal_destroy) and `hip_stream` (hipStream_t or NULL).  Writes FFT twiddle
 * tables into the workspace (stream-ordered).  Returns EINVAL for d not in
 * {2,3}, even or non-positive N, unknown precision, or a misaligned workspace;
 * ENOMEM if bytes is too small.
 */
int fftgal_plan(struct fftgal_plan **out, int d, const int32_t *N, int precision,
                void *dev_workspace, size_t bytes, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * allocation): fftgal_plan on a workspace the library owns, a static device
 * array of fftgal_static_workspace_bytes() = 64 MiB that each GPU the library
 * runs on holds until the process ends (it fits 2D plans up to N = 365 and 3D
 * plans up to N = 41 in either precision).  Allocates no device memory.  The
 * plan works like one from fftgal_plan on the current device and `hip_stream`.
 * All calls on one GPU share that GPU's array, so only one plan at a time may
 * hold it: a second fftgal_plan_static on the same device while the first is
 * alive returns ESTATE (the array is not cleared between plans; a plan
 * initialises what it reads, as with a caller's workspace).  fftgal_destroy
 * waits for the plan's stream and releases the array.  ENOMEM if the plan
 * needs more than the array holds; EINVAL as fftgal_plan.
 */
int fftgal_plan_static(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *hip_stream);
size_t fftgal_static_workspace_bytes(void);

/*
 * Build the double-grid material fields A_M and B_M (eq. MBA_GA; Lemma
 * integ_eval_VM) on the device from closed-form Fourier coefficients
 * (Remark anal_Fourier) or from the voxel image (Lemma grid_compos), for both
 * the primal (A) and the dual (A^{-1}) problem.  Invalidates earlier solves.
 * EINVAL on any violation listed above.
 */
int fftgal_set_material(struct fftgal_plan *plan, const fftgal_material *m);

/*
 * Solve the primal cell problem G A_M e = -G A_M E (eq. Ga_linsys_orig) by CG
 * from e_0 = 0 -- or from the initial iterate placed by fftgal_warm_start --
 * for E = e_alpha (alpha in 0..d-1) or for all d unit fields (alpha = -1).
 * Stops when ||r_k|| <= rtol ||b|| with b = -G A_M E (= r_0 from e_0 = 0), or when ||r_k|| <=
 * 1e-14 ||A_M E|| (FP64) / 1e-7 ||A_M E|| (FP32_ITER) -- a right-hand side at
 * rounding level of the load is treated as zero -- or at maxit.  `info` (may be
 * NULL; an array of d entries when alpha = -1) receives the outcome.  Returns
 * OK, ENOTCONV, EBREAKDOWN, ESTATE (no material) or EINVAL.
 *
 * Every CG iterate is admissible, so the energy of each is a guaranteed bound
 * (Sec. 6.4).  With FP32_ITER, once FP32 rounding dominates (tolerances near
 * or below the FP32 attainable accuracy, high contrast) the iterates drift and
 * their exact energies rise again.  FP32_ITER solves therefore measure the
 * exact energy of the iterate every 64 iterations (one more operator
 * application) and keep a copy of the lowest one; they stop when that energy
 * rises by more than 1e-5 of itself, when it stops falling while the residual
 * has made no new minimum for 64 iterations, or when (p, K p) <= 0 after the
 * first step.  The kept field is then restored and the call returns ENOTCONV
 * with info.stagnated = 1 and info.iterate = the iteration of that field.  A
 * solve that reaches maxit keeps the better of its last iterate and the copy.
 */
int fftgal_solve_primal(struct fftgal_plan *plan, int alpha, double rtol, int maxit,
                        fftgal_info *info);

/* The dual problem G^J B_M j = -G^J B_M J with J = e_alpha, as above. */
int fftgal_solve_dual(struct fftgal_plan *plan, int alpha, double rtol, int maxit,
                      fftgal_info *info);

/*
 * All d primal and all d dual solves (Cor. Ga_linsys, Remark CG; the solves
 * are independent), with the arguments and stopping tests of
 * fftgal_solve_primal; `info` (may be NULL) receives 2d entries, primal
 * alpha = 0..d-1 then dual.  A plan made with FFTGAL_CONCURRENT runs the 2d
 * solves at once: every launch of an iteration covers all unfinished ones (a
 * small grid fills the GPU that one solve leaves idle), each with its own
 * reductions, so every result equals bitwise that of its solve alone.  Other
 * plans run them one after another.  Returns the first non-OK outcome
 * (ENOTCONV, EBREAKDOWN) after all solves ran, or ESTATE / EINVAL / EDEVICE.
 */
int fftgal_solve_all(struct fftgal_plan *plan, double rtol, int maxit, fftgal_info *info);

/*
 * Guaranteed bounds from the d primal and d dual fields (Prop. struct_bounds):
 * upper = A_{H,N} and lower = B_{H,N}^{-1}, each d x d row-major on the host,
 * and gap = tr(upper - lower)/2 (eq. error).  The energy Gram matrices
 * (A_M (E_a + e_a), E_b + e_b)_{R^{d x M}} are evaluated in FP64 on the device
 * from fields that lie in E_N (J_N) by construction, then symmetrised; B is
 * inverted on the host.  Any pointer may be NULL.  ESTATE unless all 2d
 * solves exist.
 */
int fftgal_bounds(struct fftgal_plan *plan, double *upper, double *lower, double *gap);

/*
 * Coarse-to-fine warm start (Sec. 6.4: a solution on a coarse grid used as
 * the initial approximation on a fine grid, through the prolongation
 * I_N o I_M^{-1}).  For every solve (primal/dual, alpha) that `coarse` has
 * finished, the fine plan's next solve of the same (kind, alpha) starts from
 * the coarse field: the coefficients of the frequencies of Z_{N_coarse} are
 * copied and all others are zero, so the trigonometric polynomial -- and its
 * exact energy -- is the same on both grids (along an axis where the fine
 * grid is smaller the field is truncated, which is still admissible).  The
 * plans must have the same d and may differ in N, grid and precision; the
 * fine plan must have its material set (setting a material clears pending
 * warm starts).  The coarse plan's stream is synchronised if it differs.
 * Returns OK, ESTATE (no material / nothing solved / a plan in a batch) or
 * EINVAL.
 */
int fftgal_warm_start(struct fftgal_plan *fine, struct fftgal_plan *coarse);

/*
 * Energies of the CG iterates of the last solve of (kind 0 primal / 1 dual,
 * alpha) on the plan (Sec. 6.4: bounds during the iterations).  energy[k] =
 * (A_M (E + e_k), E + e_k) for the primal (B_M, J for the dual), k = 0 ..
 * iters: energy[0] is the exact energy of the initial iterate (the Voigt entry
 * <A>_{alpha alpha} from e_0 = 0); later entries follow the CG recurrence
 * energy_k = energy_{k-1} - alpha_k (r_{k-1}, r_{k-1}), which holds in exact
 * arithmetic and here accumulates rounding (and, in FP32_ITER, the FP32
 * iterates' error): a monitor, not a guaranteed bound -- fftgal_bounds
 * evaluates the guaranteed ones.  Primal entries decrease towards
 * A_{H,N}[alpha, alpha]; the reciprocal of a dual entry increases towards a
 * lower bound on A_H[alpha, alpha].  Writes min(cap, iters + 1) values and
 * *n = iters + 1.  ESTATE unless the solve was run with maxit <= 20000.
 */
int fftgal_history(struct fftgal_plan *plan, int kind, int alpha, double *energy, int cap, int *n);

/*
 * Stop on the bound as well as on the residual (Sec. 6.4: the energy of every
 * CG iterate is a guaranteed bound, and it decreases monotonically).  With
 * btol > 0 the plan's later solves also stop once the estimated remaining
 * decrease of the bound entry -- the last decrease d_k times q / (1 - q), q =
 * d_k / d_{k-1} -- is below btol times the entry (after at least two steps).
 * The bounds fftgal_bounds returns stay guaranteed; btol states how far they
 * are estimated to be from the converged Ga bounds.  0 (the default)
 * disables the test.  EINVAL for a negative or non-finite btol.
 */
int fftgal_set_bound_tol(struct fftgal_plan *plan, double btol);

/*
 * GaNi plans (Def. GaNi, Algorithm 1): the material is sampled at the grid
 * points x = k / N of the grid of the approximation order N (a point on an
 * inclusion boundary counts as outside; a voxel p covers [p/P - 1/(2P),
 * p/P + 1/(2P))), and the transforms run on that grid: every N_a must be odd;
 * a length that is not 3,5,7-smooth is transformed by Bluestein's chirp
 * convolution of the smooth length L >= 2 N_a - 1 (generic kernels).  The solve and bounds calls then return the GaNi
 * minimisers and A~_{H,N} (upper) and B~_{H,N}^{-1} (lower) -- equal for odd
 * N (Remark duality_gani) and NOT guaranteed bounds; fftgal_bounds_of turns
 * the minimisers into guaranteed ones.  Workspace, arguments and errors as
 * for fftgal_plan / fftgal_workspace_bytes_p (P may be NULL).
 */
size_t fftgal_workspace_bytes_gani(int d, const int32_t *N, int precision, const int32_t *P);
int fftgal_plan_gani(struct fftgal_plan **out, int d, const int32_t *N, int precision,
                     void *dev_workspace, size_t bytes, void *hip_stream);

/*
 * A-posteriori guaranteed bounds (eq. GaNi_apost; Prop. struct_bounds): the
 * exact energies, on this plan's double grid, of the fields of all 2d solves
 * of `src` (e.g. a GaNi plan of the same N), carried over as in
 * fftgal_warm_start.  `plan` must be a Ga plan with its material set; its
 * solution storage is overwritten and its solves are marked done.  Outputs as
 * fftgal_bounds.  ESTATE unless `src` has all 2d solves.
 */
int fftgal_bounds_of(struct fftgal_plan *plan, struct fftgal_plan *src, double *upper, double *lower,
                     double *gap);

/*
 * Reduced Ga plan (Lemma reduce_grid, eq. Ga_linsys_R, Algorithm 3): the same
 * guaranteed bounds as fftgal_plan, with every transform of size N on the grid
 * of the approximation order itself.  The double grid of 2N points per axis is
 * split into its 2^d interleaved N-grids (k = 2r - s, s in {0,1}^d); the
 * material is the double-grid series (eq. MBA_GA) evaluated on each of them
 * (the series on Z_{2N-1} folded onto Z_N with the phase of s, then one
 * inverse DFT of size N), and every operator application runs the transform
 * passes once per shift with the phases S(s), S*(s) of the lemma, summing the
 * projected results.  Every N_a must be odd; 81, 125, 225, 245, 729 and 2025
 * run the specialised kernels, other 3,5,7-smooth lengths the generic ones,
 * and the other lengths (the primes 41, 113, 1013 among them) Bluestein's chirp
 * convolution of the smooth length L >= 2 N_a - 1 in the generic kernels.  Solves, bounds, history and
 * the bound tolerance work as for fftgal_plan; warm starts, a-posteriori
 * bounds and batches are not available (EINVAL).  The workspace holds 2^d
 * material fields of |N| values and transform intermediates of the N-grid:
 * fftgal_workspace_bytes_reduced (P as in fftgal_workspace_bytes_p).  With the
 * default layout and specialised transform lengths the shifts of each operator
 * pass run in one launch, each on intermediates and a projected vector of its
 * own, summed by the CG update in shift order; with FFTGAL_REDUCED_LEAN in
 * `precision` (both calls) one set of intermediates serves the shifts in turn.
 */
size_t fftgal_workspace_bytes_reduced(int d, const int32_t *N, int precision, const int32_t *P);
int fftgal_plan_reduced(struct fftgal_plan **out, int d, const int32_t *N, int precision, void *dev_workspace,
                        size_t bytes, void *hip_stream);

/*
 * Upper and lower voxel approximations of an inclusion composite (Remark
 * adjusting_A, for Lemma bounds_bounds): on the P-grid of voxels (voxel p
 * centred at p/P with sides 1/P), `upper` receives the largest and `lower` the
 * smallest eigenvalue of the phases that meet the voxel with positive measure
 * (the matrix counts unless one inclusion contains the whole voxel), so that
 * lower I <= A(x) <= upper I almost everywhere.  `upper` and `lower` are
 * device buffers of P^d doubles (row-major, P[0] slowest) written on the
 * plan's stream; the plan supplies d, the stream and scratch for the tables
 * (it must not be in a batch; its state is otherwise untouched).  Passing them
 * as `image` and `image_dual` of a voxel material yields guaranteed
 * upper-upper and lower-lower bounds.  EINVAL for a material that is not an
 * inclusion description or fails validation; ENOMEM if the tables do not fit.
 */
int fftgal_envelope_images(struct fftgal_plan *plan, const fftgal_material *m, const int32_t *P, double *upper,
                           double *lower);

/* Release the plan (host memory only; the workspace stays the caller's). */
int fftgal_destroy(struct fftgal_plan *plan);

/* Message for the last error on `plan` (or of the last failed fftgal_plan()
 * call on this thread when plan is NULL).  Never NULL. */
const char *fftgal_last_error(const struct fftgal_plan *plan);

/* The grid size M the plan uses along axis a (0 if invalid). */
int fftgal_grid_size(const struct fftgal_plan *plan, int axis);

/*
 * Kernel timing (tracing).  While enabled, every kernel launch of the plan is
 * timed by a pair of HIP events tagged with one of the classes below: the
 * specialised kernels and the CG kernels are dispatched so that the dispatch
 * itself records the events at the kernel's start and end; other launches are
 * bracketed by two event records on the plan's stream.  fftgal_read_timing()
 * waits for the stream, writes the summed milliseconds and the launch counts
 * per class (arrays of FFTGAL_K_COUNT entries; either may be NULL) since the
 * previous read, and resets them.
 */
enum fftgal_kernel_class {
    FFTGAL_K_EXPAND = 0,      /* CG state -> d components, inverse DFT along axis 1 */
    FFTGAL_K_PENCIL_INV = 1,  /* inverse DFT along axis 2 (d = 3)                   */
    FFTGAL_K_ROW = 2,         /* C2R along axis d, material multiply, R2C           */
    FFTGAL_K_PENCIL_FWD = 3,  /* forward DFT along axis 2 (d = 3)                   */
    FFTGAL_K_PROJECT = 4,     /* forward DFT along axis 1, projection, (p, Kp)      */
    FFTGAL_K_CG_UPDATE = 5,   /* alpha, x += alpha p, r -= alpha q, (r, r)          */
    FFTGAL_K_CG_SCALAR = 6,   /* beta / stopping test, initial state, clears        */
    FFTGAL_K_RHS = 7,         /* right-hand side -G A_M E                           */
    FFTGAL_K_BOUNDS = 8,      /* FP64 fields and energy Gram quadrature             */
    FFTGAL_K_SETUP = 9,       /* material fields A_M, B_M                           */
    FFTGAL_K_CHECKPOINT = 10, /* FP32 best-iterate checkpoints (exact energies)     */
    FFTGAL_K_SOLO = 11,       /* whole CG iterations of small 2D solves, one
                                 work-group per solve (see FFTGAL_SEPARATE_PASSES) */
    FFTGAL_K_COUNT = 12
};
int fftgal_set_timing(struct fftgal_plan *plan, int enable);
/* As fftgal_set_timing, for the classes whose bit (1 << class) is set only
 * (0 disables timing). */
int fftgal_set_timing_classes(struct fftgal_plan *plan, uint32_t mask);
int fftgal_read_timing(struct fftgal_plan *plan, double *ms, int32_t *count);

/*
 * Batched CG (continuous batching of solves across plans; not in the paper).
 *
 * A batch advances many solves at once: every launch of one CG iteration
 * (each transform pass, the alpha/update/check kernels) covers all member
 * solves that share a grid size, precision and dimension, with per-solve
 * argument tables in the batch workspace.  Members join with
 * fftgal_batch_add (which computes the right-hand side at once) and leave when
 * their stopping test is met, so new solves can join while others run.  Each
 * solve's reductions use only its own work-groups in a fixed order, so its
 * result is bitwise identical whether it runs alone, through
 * fftgal_solve_primal/dual, or in any mix.
 *
 * Every plan added must use the batch's stream.  A plan can have one solve in
 * batches at a time, or 2d (each of its solves once) when made with
 * FFTGAL_CONCURRENT (its CG vectors and transform buffers are per solve slot).
 * The workspace is caller-owned device memory of
 * fftgal_batch_workspace_bytes(capacity) bytes.
 */
size_t fftgal_batch_workspace_bytes(int capacity);
int fftgal_batch_create(struct fftgal_batch **out, int capacity, void *dev_workspace, size_t bytes,
                        void *hip_stream);
/* Start solve (kind 0 = primal, 1 = dual; alpha in 0..d-1) of `plan`; writes
 * an identifier to *solve_id.  ESTATE if the plan has no material, if this
 * solve of the plan is already in a batch or if all its solve slots are in
 * use; ENOMEM if the batch is full. */
int fftgal_batch_add(struct fftgal_batch *b, struct fftgal_plan *plan, int kind, int alpha, double rtol,
                     int maxit, int *solve_id);
/* Enqueue `iterations` batched CG iterations, wait, and retire finished
 * solves; *n_active receives the number still running. */
int fftgal_batch_step(struct fftgal_batch *b, int iterations, int *n_active);
/* Pop one retired solve: returns 1 and fills *solve_id, *info and *status (the
 * code fftgal_solve_* would have returned), or 0 if none is waiting. */
int fftgal_batch_poll(struct fftgal_batch *b, int *solve_id, fftgal_info *info, int *status);
int fftgal_batch_destroy(struct fftgal_batch *b);
const char *fftgal_batch_last_error(const struct fftgal_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* FFTGAL_H */
