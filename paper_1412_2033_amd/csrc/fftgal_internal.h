// Internal declarations shared by the host library (fftgal.cpp) and the HIP
// kernels (fftgal_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fftgal {

constexpr int kThreads = 256;   // work-group size of every kernel
constexpr int kMaxStages = 16;  // radix-3/5/7 stages per FFT length

// Mixed-radix factorisation of one FFT length and where its twiddles live.
// Stage s has radix radix[s] and twiddles w(q, k) = exp(-2 pi i q k / (p r)),
// q = 1..r-1, k = 0..p-1 (p = product of the earlier radices), stored at
// twoff[s] + (q - 1) * p + k in the plan's twiddle tables.
// A length n that is not 3,5,7-smooth is transformed by Bluestein's chirp
// convolution: with c_m = exp(sg i pi m^2 / n), sum_j x_j exp(sg 2 pi i j k / n)
// = c_k sum_j (x_j c_j) conj(c_{k-j}), a circular convolution of length L >= 2n - 1
// (3,5,7-smooth) done with two transforms of length L; the stages then describe
// L, and the tables hold the chirp exp(i pi m^2 / n) (m < n) at choff and
// H = DFT_L^-(conj chirp, placed at m mod L for |m| < n) / L at hoff.
struct FftDesc {
    int n;
    int nst;
    int radix[kMaxStages];
    int twoff[kMaxStages];
    int L;      // transform buffer length in LDS: n, or the Bluestein length
    int blue;   // 1: Bluestein transform of length n through length L
    int choff;
    int hoff;
};

// Grid sizes with compile-time specialised kernels, and their radix
// schedules (composite radices are done in registers).  The host builds the
// twiddle tables of these lengths with the same schedule.  Schedules read the
// same forwards and backwards where the length allows: then the last stage of
// an inverse transform leaves each thread holding exactly the points that the
// first stage of a forward transform consumes.
struct FastSched {
    int n;
    int nst;
    int r[4];
};
constexpr FastSched kFastSched[] = {
    {81, 2, {9, 9, 0, 0}},      {125, 2, {25, 5, 0, 0}},  {225, 2, {15, 15, 0, 0}},
    {245, 3, {7, 5, 7, 0}},     {729, 3, {9, 9, 9, 0}},   {2025, 3, {15, 9, 15, 0}},
};
constexpr int kNumFast = sizeof(kFastSched) / sizeof(kFastSched[0]);
constexpr int fast_index(int n) {
    for (int i = 0; i < kNumFast; ++i)
        if (kFastSched[i].n == n) return i;
    return -1;
}

// Device-resident state of one CG solve (Remark CG), advanced by the scalar
// kernels; every kernel of an iteration returns at once when `done` is set.
struct CgStatus {
    double rr;       // (r_k, r_k)
    double rr0;      // (r_0, r_0)
    double pq;       // (p_k, K p_k)
    double alpha;    // rr / pq
    double beta;     // rr_{k+1} / rr_k (0 before the first step)
    double tol2;     // rtol^2
    double floor2;   // (floor * ||A_M E||)^2
    double load2;    // ||A_M E||^2
    double energy;   // energy of the current iterate (CG recurrence)
    double dprev;    // energy decrease of the previous step
    double btol;     // bound tolerance (0: residual test only)
    // best-iterate guard of the FP32-iteration form: exact energies of the
    // iterate at checkpoints, the lowest one kept in a copy of the field
    double eAE;      // (A_M E, E): the energy of e = 0
    double ebest;    // lowest checkpoint energy (the initial iterate's at start)
    double rrmin;    // smallest (r_k, r_k) so far
    int32_t rrmin_it;  // iteration of rrmin
    int32_t best_it;   // iteration of the kept copy
    int32_t stagnated; // stopped because FP32 rounding stalled the iteration
    int32_t ck_copy;   // set by a checkpoint: copy the iterate into the best copy
    int32_t ck_restore;  // set by a checkpoint: restore the iterate from the best copy
    int32_t iter;
    int32_t maxit;
    int32_t done;
    int32_t converged;
    int32_t breakdown;
    int32_t pad;
};

enum Prologue { PRO_PLAIN = 0, PRO_EXPAND = 1 };
enum Epilogue { EPI_PLAIN = 0, EPI_PROJECT = 1, EPI_WINDOW = 2 };
enum RowMode { ROW_OPER = 0, ROW_RHS = 1, ROW_GRAM = 2, ROW_C2R = 3, ROW_R2C = 4 };
enum SolveKind { KIND_E = 0, KIND_J = 1 };

// A batched 1D DFT along one strided axis ("pencils"), with optional
// prologue/epilogue.  Element (component c, outer o, position l, batch b) of
// an operand lives at base + c*cs + o*os + l*ls + b (complex units).  Stored
// position l of a length-L operand holds frequency wrap_L(l) (or grid point l
// when L equals the transform length n), placed in the transform at
// wrap_L(l) mod n.
struct PencilArgs {
    const void *in;
    void *out;
    long in_cs, out_cs, in_os, out_os, in_ls, out_ls;
    int L_in, L_out;
    int nb;       // batch extent (contiguous)
    int B;        // pencils per work-group
    int ncomp;    // transformed components (per solution)
    int cb;       // generic kernel: components transformed together (1 .. ncomp)
    int twl;      // generic kernel: table entries staged in LDS (0: read from the table)
    int sgn;      // +1: inverse DFT (omega^{+mk}); -1: forward
    double scale; // applied to every output value
    FftDesc f;
    const void *tw;
    int pro, epi;
    int fast;     // set by configure_pencil: specialised kernel for this length
    // frequency decoding for EXPAND / PROJECT / WINDOW
    int d, kind, nc, Nmid, Nh;
    // EXPAND: state vectors (component stride st_cs, solution stride st_ss)
    const void *st_r;
    void *st_p;
    const void *st_x;
    long st_cs, st_ss;
    int nsol;
    int update_p;
    const CgStatus *status;
    // PROJECT
    void *st_q;
    const void *st_dot;
    double *partial;
    // WINDOW: sinc window of a P-voxel image, times 1/|P|
    int Pw[3];
    double winscale;
    // reduced Ga (Lemma reduce_grid): EXPAND multiplies frequency k by
    // exp(-i pi sum_a shift_a k_a / Nfull_a) (S(s)), PROJECT by its conjugate
    // (S*(s)) and, with accumulate, adds to the vector already in out
    int shift[3];
    int Nfull[3];
    int accumulate;
};

// Batched real transforms along the last (contiguous, half-spectrum) axis,
// two rows packed per complex transform, with the material multiply fused.
struct RowArgs {
    void *data;       // complex rows: comp stride cs, row stride Nh_row
    long cs;
    int nrows;
    int Nh_row;
    int n;
    FftDesc f;
    const void *tw;
    int ncomp;
    int d;
    int mode;
    int RP;           // row pairs per work-group
    int fast;         // set by configure_row (1 specialised, 2 specialised isotropic, 3 isotropic
                      // with all loads of a work-group staged in LDS)
    int iso;          // A0 and D are multiples of the identity
    const void *g;    // material field g (M^d, precision of the kernel)
    double A0[9];     // A(x) = A0 + g(x) D
    double D[9];
    // nfield > 1: A(x) is the symmetric matrix whose entries 11, 12, [13,] 22,
    // [23,] 33 are the fields g + f * gstride (f = 0 .. nfield - 1); A0 and D
    // are unused
    int nfield;
    long gstride;
    // ROW_GRAM, generic kernel: 1 packs two components of one row per complex
    // transform (RP rows per work-group) instead of two rows of one component
    // (RP row pairs), halving the transform buffers for long rows
    int gpack;
    // generic kernel: the components' rows form one batch of transforms (LDS
    // for two buffers of every component) instead of one batch per component
    int zbatch;
    double E[3];      // load for ROW_RHS
    void *real_out;   // ROW_C2R output rows (length n)
    const void *real_in;  // ROW_R2C input rows (length n)
    long real_stride;
    int imgmap;       // ROW_R2C: voxel value mapping (see map_voxel)
    double vmax;
    double scale;
    double *partial;  // RHS: |A_M E|^2 sums; GRAM: d*d sums per work-group
    double *partial2; // RHS: sums of (A_M E).E per work-group (may be null)
    const CgStatus *status;
};

// Per-problem arguments of the multi-problem CG kernels.
struct UpdArgs {
    void *x;
    void *r;
    const void *p;
    const void *q;
    long n_per_comp;
    long cs;
    int nc;
    int Nh;
    int nblocks;  // work-groups of this problem (fixes the reduction order)
    CgStatus *st;
    double *partial;
    const double *pq_part;  // partials of (p, K p) from the projection pass, or nullptr
    int npq;
    // K p as the sum of nq vectors q, q + q_ss, ... (the shifts of the reduced
    // Ga, added in that order); nq = 1 otherwise
    int nq;
    long q_ss;
};

// One 2D CG solve run entirely by one work-group (launch_solo): the CG
// vectors x, r, p (nc = 1 component of N0 x Nh coefficients, half spectrum),
// the status, the material A(x) = A0 + g(x) D (nfield = 1) or the fields g +
// f gstride holding the entries 11, 12, 22 of A(x) (nfield = 3) on the M0 x M1
// grid, the stage twiddles of both axes (entries tw0, tw1 of tw), the basis
// kind and the scale 1 / (M0 M1) of the forward transforms.
struct SoloArgs {
    void *x, *r, *p;
    CgStatus *st;
    CgStatus *mirror;  // copy of the status at the end of a launch, or nullptr
    double *hist;      // (rr, alpha) per iteration, or nullptr
    int hist_cap;
    const void *g;
    long gstride;
    int nfield;
    double A0[4], D[4];
    const void *tw;
    int tw0, tw1;
    int M0, M1, N0, Nh;
    int kind;
    double scale;
};

struct CgItem {
    CgStatus *st;
    const double *rr_part;
    int nrr;
    double *hist;      // (rr, alpha) per iteration, or nullptr
    int hist_cap;      // entries available in hist
    CgStatus *mirror;  // copy of the status after each check, or nullptr
};

struct InclDev {
    int shape;
    double c[3];
    double h[3];
    double w;  // weight of this inclusion's indicator
};

// ---- launchers (fftgal_kernels.hip) ----
// GaNi material at the grid points x = k / M (centred): w0 + sum_i w_i chi_i(x)
// for inclusions (periodic minimum image; boundary points outside), and the
// mapped value of the voxel containing x for images (voxel p covers
// [p/P - 1/(2P), p/P + 1/(2P))).  Output layout [x1][x2][x3], FP64.
hipError_t launch_sample_incl(double *g, int d, const int *M, const InclDev *inc, int n, double w0, hipStream_t s);
hipError_t launch_sample_voxel(double *g, const double *img, int d, const int *P, const int *M, int map, double vmax,
                               hipStream_t s);
// Upper / lower voxel images of an inclusion composite (Remark adjusting_A):
// per voxel (centre p/P, sides 1/P) the largest / smallest eigenvalue of the
// phases meeting it with positive measure; ext = (hi, lo) of the matrix, then
// of each inclusion phase.
hipError_t launch_envelope(double *upper, double *lower, int d, const int *P, const InclDev *inc, int n,
                           const double *ext, hipStream_t s);
size_t pencil_lds_bytes(const PencilArgs &a, bool fp64);
size_t row_lds_bytes(const RowArgs &a, bool fp64);
// Choose pencils per work-group / row pairs per work-group (and whether the
// specialised kernel runs) for a launch; sets a.B / r.RP.
void configure_pencil(PencilArgs &a, bool fp64);
void configure_row(RowArgs &r, bool fp64);
// LDS of a generic-kernel work-group (its transform buffers): at most 80 KB,
// two work-groups per CU
constexpr size_t kGenericLds = 80 * 1024;
// Generic pencil kernel: the most components per transform batch (a.cb) whose
// buffers fit kGenericLds at the batch a.B, then a.twl > 0 when the
// transform's table fits beside them too.
void fit_pencil_components(PencilArgs &a, bool fp64);
// Generic row kernel: a.zbatch = 1 when the batched buffers fit kGenericLds at a.RP.
void fit_row_batch(RowArgs &r, bool fp64);
hipError_t launch_pencil(const PencilArgs &a, int nouter, bool fp64, hipStream_t s);
hipError_t launch_row(const RowArgs &a, bool fp64, hipStream_t s);
int row_grid(const RowArgs &a);
int pencil_grid_x(const PencilArgs &a);

// Best-iterate checkpoint of an FP32 solve (between iterations, after the
// operator was applied to the iterate x with partials of (x, K x) in
// part_xkx): partials of (b, x) per update work-group, then the exact energy
// (A_M E, E) - 2 (b, x) + (x, K x) compared with the best one: a lower energy
// is copied into xbest; a clear rise, or no gain while the residual has not
// reached a new minimum for `window` iterations, stops the solve and restores
// x from xbest.  final = 1 (after the last iteration of a solve that did not
// converge) only restores x when the kept copy is better.  Every kernel does
// nothing when the solve is done, except in the final checkpoint.
hipError_t launch_cg_checkpoint(const UpdArgs &u, const void *b, void *xbest, const double *part_xkx, int n_xkx,
                                double *part_bx, int window, int final, bool fp64, hipStream_t s);
hipError_t launch_copy_vec(void *dst, const void *src, size_t bytes, hipStream_t s);
// Matrix voxel images (n voxels of d x d, row-major per voxel): per work-group
// counts of voxels that are not finite, symmetric and positive definite into
// part (one entry per work-group of the launch, nparts returned in *nparts).
hipError_t launch_tensor_check(const double *img, long n, int d, double *part, int *nparts, hipStream_t s);
// out[i] = entry (a, b) of voxel i's matrix, or of its inverse (invert = 1).
hipError_t launch_tensor_component(const double *img, long n, int d, int a, int b, int invert, double *out,
                                   hipStream_t s);
hipError_t launch_cg_init(CgStatus *st, const double *rr_part, int n_rr, const double *load_part, int n_load,
                          const double *work_part, double inv_mtot, double tol, double floor_rel, int maxit,
                          double btol, double *hist, hipStream_t s);
// Multi-problem launches: `args` and `woff` are device arrays; problem i
// owns work-groups [woff[i], woff[i + 1]) of a grid of `total` work-groups.
// Optional pair of events that a dispatch records itself at its start and at
// its end (hipExtLaunchKernel): the kernel's own duration, with no marker
// packets between launches.  Both null: an ordinary launch.
struct LaunchEv {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
hipError_t launch_pencil_multi(const PencilArgs &proto, const PencilArgs *args, const int *woff, int np,
                               int total, bool fp64, hipStream_t s, LaunchEv ev = LaunchEv{});
hipError_t launch_row_multi(const RowArgs &proto, const RowArgs *args, const int *woff, int np, int total,
                            bool fp64, hipStream_t s, LaunchEv ev = LaunchEv{});
hipError_t launch_cg_check_multi(const CgItem *items, int np, hipStream_t s, LaunchEv ev = LaunchEv{});
// Whether a 2D Ga grid M0 x M1 has the single-work-group solver (both lengths
// specialised, the complex grid within the LDS of one work-group).
bool solo_fits(int M0, int M1, bool fp64);
// `niter` CG iterations (fewer once a solve is done) of each of the np solves
// in `args` (device array; all of one grid and precision), one work-group each.
hipError_t launch_solo(const SoloArgs &proto, const SoloArgs *args, int np, int niter, bool fp64, hipStream_t s,
                       LaunchEv ev = LaunchEv{});
hipError_t launch_cg_update_multi(const UpdArgs *ua, const int *woff, int np, int total, bool fp64,
                                  hipStream_t s, LaunchEv ev = LaunchEv{});
int pencil_grid(const PencilArgs &a, int nouter);  // work-groups of one problem
int update_blocks(long n);                         // work-groups of one CG update
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// Warm start: r <- r - q (r holds b on entry), partials of (r, r), (b, x0),
// (r, x0) into part_rr / part_bx / part_rx (one per work-group, update grid).
hipError_t launch_warm_residual(const UpdArgs &u, double *part_rr, double *part_bx, double *part_rx, bool fp64,
                                hipStream_t s);
// Status of a warm-started solve: rr = sum part_rr, reference rr0 = scal[0]
// ((b, b)), load2 = scal[1], energy at the initial iterate
// scal[2] / mtot - sum part_bx - sum part_rx (history slot 1).
hipError_t launch_cg_init_warm(CgStatus *st, const double *part_rr, const double *part_bx, const double *part_rx,
                               int nparts, const double *scal, double mtot, double tol, double floor_rel, int maxit,
                               double btol, double *hist, hipStream_t s);
// Copy the coefficient arrays of a coarse solve into a fine one: entries of
// frequencies inside the coarse grid are copied, all others set to zero.
hipError_t launch_prolong(const void *src, bool src64, void *dst, bool dst64, int d, int nc, const int *Nf,
                          const int *Nc, hipStream_t s);
hipError_t launch_convert_f2d(double *dst, const float *src, size_t n, hipStream_t s);
hipError_t launch_convert_d2f(float *dst, const double *src, size_t n, hipStream_t s);
hipError_t launch_sum_partials(double *out, const double *part, int nparts, int nvals,
                               hipStream_t s);
hipError_t launch_image_stats(const double *img, long n, double *part, double *out, hipStream_t s);
// Reduced Ga material (Lemma reduce_grid): fold a Fourier half-grid on
// Z_{2N-1} (layout [L0][L1][Lh], wrapped) onto Z_N (layout [N0][N1][Nh]) with
// the phase of the shift s: b(j) = sum_{k = j mod N} c(k) exp(-i pi s.k / N).
hipError_t launch_fold_series(void *out, const void *coef, int d, const int *N, const int *L, int Lh,
                              const int *shift, hipStream_t s);
hipError_t launch_incl_coeff(void *out, int d, int L1, int L2, int Lh, const InclDev *incl, int n_incl,
                             double w0, hipStream_t s);

}  // namespace fftgal
