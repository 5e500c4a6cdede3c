/*
 * lalm.h -- C ABI of the MI355X (gfx950) OS-LALM library for penalized
 * weighted least-squares X-ray CT reconstruction.
 *
 * The calls follow the problem statement of Nien & Fessler, arXiv 1402.4381,
 * Sec. IV (eq. "ct_recon"):
 *
 *     x^ = argmin_{x >= 0} 1/2 ||y - A x||_W^2 + R(x),
 *
 * solved with the ordered-subsets linearized augmented Lagrangian method
 * (Sec. III-A, eq. "os_lalm_iterates") and its deterministic downward
 * continuation of rho (Sec. III-B, eq. "rho_l_formula_qp").
 *
 * Conventions shared by every call
 *   - Device pointers are plain HIP device addresses (for instance from a
 *     torch tensor's data_ptr()); the caller owns every image and sinogram
 *     buffer.  The plan owns its geometry tables and workspace, allocated once
 *     by lalm_plan_geometry; no other call allocates device memory.
 *   - Images are float32 [z][y][x], x fastest.  Voxel centres are
 *     X_i = (i - (nx-1)/2) dx (same for y, z): the image centre is the
 *     isocentre.
 *   - A plan holds a batch of B images of the same geometry (B = 1 for a
 *     single reconstruction).  Every image argument then holds B images one
 *     after the other ([batch][z][y][x]), every sinogram argument B
 *     sinograms ([batch][sinogram]), every subset argument B subset arrays
 *     ([batch][rays of the subset]); each kernel launch covers all B, and the
 *     B reconstructions are independent (each has its own data, weights,
 *     D_L and continuation state).
 *   - Sinograms are float32 and subset-major: views are grouped by subset
 *     (subset m holds the views v with v mod M == m, in increasing order);
 *     lalm_plan_info returns the view of every slot and the ray offset of
 *     every subset.  Within a view the layout is [row][bin], bin fastest.
 *   - All calls are asynchronous on the given stream unless stated; a plan is
 *     not thread-safe and must be used by one stream at a time.
 *   - Errors: no call throws; each returns a lalm_status, and
 *     lalm_last_error() returns a thread-local text describing the last
 *     failure.  Arguments are validated before any work is queued.
 */
#ifndef LALM_H
#define LALM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hipStream_t;

#if defined(__GNUC__)
#define LALM_API __attribute__((visibility("default")))
#else
#define LALM_API
#endif

typedef int32_t lalm_status;
#define LALM_OK 0
#define LALM_E_INVALID (-1)   /* bad argument, geometry or size */
#define LALM_E_HIP (-2)       /* a HIP runtime call or kernel launch failed */
#define LALM_E_NOMEM (-3)     /* device allocation failed (plan creation) */
#define LALM_E_NONFINITE (-4) /* a non-finite restart indicator was met */
#define LALM_E_STATE (-5)     /* state inconsistent with plan or options */

/* Thread-local text of the last failure ("" if none). */
LALM_API const char *lalm_last_error(void);

/* Library version string. */
LALM_API const char *lalm_version(void);

#define LALM_FAN2D 0
#define LALM_CONE_AXIAL 1
#define LALM_CONE_HELICAL 2

/*
 * Scanner and image geometry.  Lengths in mm, angles in radians.  The paper
 * names no projector or scanner model; the reading implemented is a
 * third-generation scanner with an arc (equiangular, cylindrical) detector:
 *   view angle  beta_v = start_angle + 2 pi v / n_views_per_turn,
 *   source      S_v = (dso cos beta_v, dso sin beta_v, z_s(v)),
 *   channel     gamma_b = (b - (n_bins-1)/2 - channel_offset) ds / dsd,
 *               in-plane ray direction at angle beta_v + pi + gamma_b,
 *   row         v_r = (r - (n_rows-1)/2) dt at distance dsd from the source,
 *   helical     z_s(v) = (v - (n_views-1)/2) feed / n_views_per_turn with
 *               feed = pitch n_rows dt dso / dsd (0 for axial and 2D).
 */
typedef struct {
    int32_t kind;                  /* LALM_FAN2D, LALM_CONE_AXIAL, LALM_CONE_HELICAL */
    int32_t nx, ny, nz;            /* nz = 1 for LALM_FAN2D */
    double dx, dy, dz;
    int32_t n_views, n_views_per_turn; /* equal for axial and 2D */
    int32_t n_bins, n_rows;        /* n_rows = 1 for LALM_FAN2D */
    double ds, dt;                 /* channel arc length and row height at the detector */
    double dso, dsd;               /* source-isocentre, source-detector distances */
    double start_angle, pitch;     /* pitch only for LALM_CONE_HELICAL */
    double channel_offset;         /* in bins */
    int32_t detector;              /* 0 = arc; no other detector is implemented */
} lalm_geometry;

typedef struct lalm_plan lalm_plan;

/*
 * Plan a geometry with M = n_subsets ordered subsets (Sec. IV-A: subsets
 * visited in bit-reversal order; Sec. IV-B: views spread uniformly over each
 * subset) for batch images reconstructed together (the problem statement of
 * Sec. IV, once per image).  Builds the per-view and per-ray tables in FP64
 * on the host, stores them as FP32 on the current device, and allocates the
 * workspace, per image of the batch (two padded image copies, one image of
 * regularizer gradient, two partial images, one inner-iteration image, one
 * subset residual, reduction buffers, device scalars; 2D also a second
 * pair of padded copies and four x-candidate images; 2D and full-turn axial
 * cone beam the filtered sinogram of the FBP).
 * Errors: LALM_E_INVALID for non-positive sizes, dsd <= dso, a source inside
 * the image's circumscribed cylinder, n_subsets outside [1, n_views], batch
 * outside [1, 65535 / nz], an unsupported detector, more than 256 detector
 * rows or 2^20 channels, or (cone beam) a subset sinogram of 4 GiB or more;
 * LALM_E_NOMEM when allocation fails.
 */
LALM_API lalm_status lalm_plan_geometry(const lalm_geometry *geom, int32_t n_subsets, int32_t batch,
                                        lalm_plan **out);

/*
 * Plan facts (the ordered subsets of Sec. IV-A, visited in bit-reversal
 * order, with their views spread over the scan as Sec. IV-B asks; the
 * Joseph sample count of every subset is the unit of the projector's work),
 * written to host arrays the caller provides (any may be NULL):
 *   image_elems      nx*ny*nz;  sino_elems  n_views*n_rows*n_bins;
 *   subset_ray_offset [M+1] first ray (element) of each subset in the
 *                    subset-major sinogram, and the total at [M];
 *   order            [M] subset visiting order (bit reversal);
 *   view_of_slot     [n_views] natural view index of each sinogram slot;
 *   subset_samples   [M] Joseph samples per subset (ray/slice pairs with at
 *                    least one tap inside the volume), for byte accounting.
 */
LALM_API lalm_status lalm_plan_info(const lalm_plan *plan, int64_t *image_elems, int64_t *sino_elems,
                           int64_t *subset_ray_offset, int32_t *order, int32_t *view_of_slot,
                           int64_t *subset_samples);

/* Release the plan and its device memory (synchronizes the device). */
LALM_API lalm_status lalm_plan_destroy(lalm_plan *plan);

/*
 * Forward projection of subset m (system matrix A of Sec. IV): for every ray
 * of the subset, out = w .* (A_m x - y).  y_sub NULL means y = 0 and w_sub
 * NULL means w = 1, so (NULL, NULL) gives A_m x.  x is an image; out_sub,
 * y_sub, w_sub hold the subset's rays (subset_ray_offset[m+1] -
 * subset_ray_offset[m] elements, layout [view][row][bin]).
 * Projector: ray-driven Joseph interpolation, one ray per detector-cell
 * centre, sampled at every slice of the in-plane dominant axis, linear (2D)
 * or bilinear (3D) interpolation, zero outside the volume; weight per sample
 * = ray length per slice.  With a batch, x holds B images and out_sub,
 * y_sub, w_sub B subset arrays.
 */
LALM_API lalm_status lalm_project_subset(lalm_plan *plan, int32_t m, const float *x, float *out_sub,
                                const float *y_sub, const float *w_sub, hipStream_t stream);

/*
 * Back-projection of subset m: the transpose A_m' of the subset system
 * matrix, the operator of the subset gradient M grad l_m(x) =
 * M A_m' W_m (A_m x - y_m) that every OS-LALM step evaluates (Sec. III-A,
 * eq. "os_lalm_iterates", with the substitution of eq. "ct_substitution").
 * Exact transpose of lalm_project_subset's weights (matched adjoint,
 * deterministic gather, no atomics): x_out = scale * A_m' r
 * (accumulate = 0) or x_out += scale * A_m' r (accumulate = 1).  r_sub
 * holds the subset's rays ([view][row][bin], as lalm_project_subset's
 * output), x_out is an image; both are caller-owned device arrays (B subset
 * arrays and B images with a batch).
 * Errors: LALM_E_INVALID for a null pointer or m outside [0, M).
 */
LALM_API lalm_status lalm_backproject_subset(lalm_plan *plan, int32_t m, const float *r_sub, float *x_out,
                                    float scale, int32_t accumulate, hipStream_t stream);

/*
 * SQS denominator (Sec. IV-A): denom = A' (w .* (A 1)) over all subsets,
 * the diagonal majorizer L_diag = diag{A'WA1}.  w_full is the whole
 * subset-major weight sinogram (B of them with a batch; denom then holds
 * the B denominators).
 */
LALM_API lalm_status lalm_sqs_denom(lalm_plan *plan, const float *w_full, float *denom, hipStream_t stream);

/* Initial image by filtered back-projection (the paper's experiments start
 * from an FBP image; figure captions), over one full turn, FP32, into x_out
 * (device image [z][y][x]) from the line integrals y_full (device,
 * subset-major like lalm_iterate's y; rays with zero counts carry y = 0).
 * The paper gives no formula; these are the textbook reconstructions for
 * the arc (equiangular, cylindrical) detector:
 *   2D fan beam   cosine weighting D cos(gamma), the fan-beam Ram-Lak
 *                 kernel along the channels, 1/L^2-weighted back-projection
 *                 with linear interpolation in channel;
 *   axial cone    FDK (Feldkamp, Davis & Kress): the weight also carries the
 *                 row's cone angle dsd / sqrt(dsd^2 + v_r^2), each detector
 *                 row is filtered on its own, and a voxel at height z reads
 *                 the row height z dsd / L (L: in-plane distance from the
 *                 source), bilinear in (channel, row), weight 1/L^2.
 * The helical cone beam has no such one-pass reconstruction (its rays cover
 * each slice from a different set of angles) and is rejected.
 * With a batch, y_full holds B sinograms and x_out receives B images.
 * Errors: LALM_E_INVALID for helical plans, scans that are not one full
 * turn, or more than 4096 channels. */
LALM_API lalm_status lalm_fbp(lalm_plan *plan, const float *y_full, float *x_out, hipStream_t stream);

/* The PWLS problem of Sec. IV: data, weights, SQS denominator, and the
 * hyperbola edge-preserving regularizer
 *   R(x) = beta sum_{pairs j~k} kappa_jk psi(x_j - x_k),
 *   psi(t) = delta^2 (sqrt(1 + (t/delta)^2) - 1),
 * over the 8- (2D) or 26- (3D) neighbourhood with kappa = 1/|offset| in index
 * units; pairs leaving the grid are dropped.  nonneg = 1 imposes x >= 0
 * (the box constraint Omega). */
typedef struct {
    const float *y, *w, *denom; /* full subset-major sinograms; denom image (B of each with a batch) */
    double beta, delta;         /* the same for every image of a batch */
    int32_t nonneg;
} lalm_problem;

/* Caller-owned iteration state.  x: image; g: split gradient; grad: the
 * latest scaled subset gradient M grad l_m.  step counts subset steps done;
 * l and rho are the continuation counter and the rho of the next step.  When
 * step == 0, lalm_iterate initializes grad = g = M grad l_{order[0]}(x),
 * l = 0 and rho = 1 (continuation) or rho_fixed.  The struct is updated on
 * return, so a state saved after a call resumes bit-exactly.
 * Barzilai-Borwein history (used only with lalm_options.bb = 1, else may be
 * null / ignored): x_prev, grad_prev are device images holding x and grad at
 * the start of the current iteration (written by the library at every
 * iteration start), alpha the current scale of D_L (set to 1 at step 0).
 * With a batch the images hold B images each, every image has its own
 * continuation state, and l_b, rho_b, alpha_b are HOST arrays of B entries
 * (read on resume, written on return; required when B > 1, may be null
 * when B = 1); l, rho and alpha then mirror image 0 and step counts the
 * steps the batch has taken (all images step together). */
typedef struct {
    float *x, *g, *grad;
    int64_t step;
    int64_t l;
    double rho;
    float *x_prev, *grad_prev;
    double alpha;
    int64_t *l_b;
    double *rho_b, *alpha_b;
} lalm_state;

/* continuation: 1 = downward continuation with adaptive restart (Sec. III-B),
 * 0 = fixed rho = rho_fixed.  rho_min: lower bound of rho_l (1e-3 in the
 * paper).  n_inner: FISTA iterations (Beck & Teboulle) on the inner
 * constrained-denoising problem of each step, from the warm start x (Sec.
 * IV-A), 1 .. LALM_MAX_INNER; 1 is one projected, diagonally majorized
 * gradient step (the paper's default), n > 1 costs n - 1 more image passes
 * with a regularizer gradient each.  forced_restart: optional DEVICE array of
 * forced_len bytes indexed by global step ([batch][forced_len] with a
 * batch); when step < forced_len its value replaces the restart test
 * (replay of a restart sequence).
 * bb = 1: Barzilai-Borwein acceleration (supplement, eq.
 * scale_factor_alpha_k): the majorizer D_L is replaced by alpha_k D_L with
 * alpha_k = min(1, <s, y> / <s, D_L s>) (FP64), s and y the differences of
 * the image and of the scaled gradient M grad l_{order[0]} between the
 * starts of iterations k and k - 1 (every M steps); alpha_k >= bb_alpha_min,
 * and 1 when <s, y> <= 0.  Needs state.x_prev and state.grad_prev. */
#define LALM_MAX_INNER 16

typedef struct {
    int32_t continuation;
    double rho_fixed, rho_min;
    int32_t n_inner;
    const uint8_t *forced_restart;
    int64_t forced_len;
    int32_t bb;
    double bb_alpha_min;
} lalm_options;

/* Optional per-step record, DEVICE arrays indexed by global step (entries at
 * step >= capacity are not written; [batch][capacity] with a batch): rho
 * used by the step, the restart indicator xi (FP64) and whether the step
 * restarted the continuation. */
typedef struct {
    double *rho, *xi;
    uint8_t *restart;
    int64_t capacity;
} lalm_stats;

/*
 * Run n_steps OS-LALM subset steps (an iteration is M steps).  Step j:
 *   s = rho grad + (1 - rho) g,
 *   x <- max(0, x - (s + grad R(x)) / (rho denom + D_R))
 *        (one projected gradient step on the inner constrained denoising
 *        problem, n = 1; D_R = 2 beta sum kappa, the SQS curvature of R;
 *        n_inner > 1 continues with FISTA iterations, see lalm_options),
 *   grad+ = M A_m' W_m (A_m x - y_m) with m = order[(j+1) mod M],
 *   g <- (rho grad+ + g) / (rho + 1),
 *   xi = <g_old - grad+, grad+ - grad_old> in FP64; with continuation,
 *   l <- 0 if xi > 0 else l + 1, and the next step uses rho_l.
 * Synchronizes the stream once at the end to return the continuation state.
 * Errors: LALM_E_INVALID for null pointers (also l_b, rho_b, alpha_b with a
 * batch) or n_inner outside [1, LALM_MAX_INNER]; LALM_E_STATE for a
 * negative step or an inconsistent continuation state; LALM_E_NONFINITE
 * when xi of an image became non-finite (that image keeps the last image
 * computed from finite gradients and skips its later steps; the other
 * images of a batch run on).
 */
LALM_API lalm_status lalm_iterate(lalm_plan *plan, const lalm_problem *prob, lalm_state *state,
                         int64_t n_steps, const lalm_options *opt, const lalm_stats *stats,
                         hipStream_t stream);

/* FP64 monitors (reduced in a fixed order: deterministic). */
/* out_dev[0..2] = Psi(x), 1/2 ||y - A x||_W^2, R(x)   (Sec. IV, eq. "ct_recon");
 * with a batch out_dev[3 b .. 3 b + 2] for image b. */
LALM_API lalm_status lalm_cost_f64(lalm_plan *plan, const lalm_problem *prob, const float *x,
                          double *out_dev, hipStream_t stream);
/* out_dev[0] = sum_i a_i b_i over n elements (for the adjoint test). */
LALM_API lalm_status lalm_dot_f64(lalm_plan *plan, const float *a, const float *b, int64_t n,
                         double *out_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the same
 * out_dev[0] = sum_i a_i b_i as lalm_dot_f64, with the same kernels and
 * bits, without a plan.  Its scratch, 1024 FP64 block partials (8 KiB), is
 * a file-scope device array of the library, one per GPU, held until the
 * process ends; the call allocates nothing.  Calls that overlap on one GPU
 * (concurrent streams, threads) share that array and race: serialize them.
 * Errors: LALM_E_INVALID for null pointers, n < 0 or n > 2^40; LALM_E_HIP
 * when the scratch address or a launch fails. */
LALM_API lalm_status lalm_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *out_dev,
                                          hipStream_t stream);
/* out_dev[0] = RMS of (a - b) over voxels whose centre lies within radius_mm
 * of the rotation axis, all slices (Sec. V: RMS difference in the ROI);
 * with a batch out_dev[b] for image b. */
LALM_API lalm_status lalm_roi_rmsd_f64(lalm_plan *plan, const float *a, const float *b, double radius_mm,
                              double *out_dev, hipStream_t stream);

/*
 * Kernel timing (measurement aid, not part of the method).  While profiling
 * is on, every kernel lalm_iterate launches carries start / stop HIP events
 * on its own dispatch (on the caller's stream), and their elapsed times are
 * summed per kernel class.  lalm_profile_read returns, per class, the total
 * milliseconds and the number of subset steps that ran the class since
 * lalm_profile_begin: [0] x-update (2D within a call: the step kernel that
 * sums the partial back-projections and makes the next x candidates; also
 * the inner FISTA iterations), [1] forward projection (with the
 * continuation decision where it takes it), [2] back-projection (2D within
 * a call: the line kernel; otherwise with its epilogue and, in 3D, the
 * continuation decision).  ms and counts are host arrays of 3.
 */
LALM_API lalm_status lalm_profile_begin(lalm_plan *plan);
LALM_API lalm_status lalm_profile_read(lalm_plan *plan, double *ms, int64_t *counts);
LALM_API lalm_status lalm_profile_end(lalm_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* LALM_H */
