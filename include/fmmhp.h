/*
 * fmmhp.h -- fast multipole evaluation of the 2-D half-plane Laplace potential
 * with a Robin (impedance) boundary condition, on AMD gfx950 (MI355X).
 *
 * Computes, for N charged points r_j = (x_j, y_j) with y_j > 0 and charges q_j,
 *
 *     phi_i = sum_j q_j G(r_i, r_j),      i = 1..N            (Section 2.2, eq. (potential1))
 *
 * where G is the Green's function of Section 2.1, eq. (ddGreensfunimp):
 *
 *     G(r, r') = -(1/2pi) ln|r - r'| + (1/2pi) ln|r - r'_im| + G_Z(r, r'),
 *     r'_im = (x', -y'),  G_Z = I_0(x - x', y + y') + I_0(x' - x, y + y')   (eq. (reactdecomposition)),
 *     I_n(x, y) = 1/(2 pi n!) int_0^inf exp(-lam y + i lam x) lam^n / (lam - Z_eps) dlam   (eq. (generalintegral)),
 *
 * with impedance Z_eps = lambda_re + i lambda_im (lambda_re > 0, lambda_im >= 0; lambda_im = 0 is the
 * lossless case, understood by limiting absorption, eq. (dzGreensfunimplossless)).  The free-space
 * log term skips j with r_j == r_i (eq. (1.2)); the image and reaction terms keep every j.  phi is
 * complex even for real charges and real impedance.
 *
 * The potential is split as Algorithm 2 of the paper does (free-space, image and reaction parts) and
 * evaluated with an adaptive quadtree over the points and their images (Algorithm 1), the paper's
 * reaction-field expansions and translation operators (S2M, M2M, M2L, L2L, S2L: eqs. (MEcoefficients),
 * (metome), (truncatedM2Lcoef), (truncatedL2L), (LEcoefficients)), the textbook log-kernel
 * expansions, and direct summation between neighbouring leaves.
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] are device pointers on the current HIP device; [host] are host
 *     pointers.  The caller owns every buffer it passes.  Arrays are dense, float64, SoA.
 *   - Work is issued on `stream` (0 = the null stream) and is asynchronous with respect to the host
 *     unless stated otherwise; outputs are valid once the stream reaches that point.
 *   - Every call returns a status and never throws.  On failure, fmmhp_last_error_message() (per
 *     host thread) describes the cause.  Kernel faults surface as FMMHP_EHIP on a later call.
 *   - A plan is bound to the device that was current at creation and must be used from that device.
 *     Calls that share a plan must not overlap in time (the plan owns one workspace).
 */
#ifndef FMMHP_H
#define FMMHP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmmhp_plan_s *fmmhp_plan_t;

typedef enum {
    FMMHP_OK = 0,
    FMMHP_EINVAL = 1,       /* null pointer, size or option out of range, non-finite input */
    FMMHP_EDOMAIN = 2,      /* outside the problem's domain: a point with y <= 0, Re Z <= 0,
                               Im Z < 0, or image arrays that are not exactly (x, -y) */
    FMMHP_ENOMEM = 3,       /* device or host allocation failed */
    FMMHP_EHIP = 4,         /* a HIP runtime call failed */
    FMMHP_ESTATE = 5,       /* plan handle is NULL or already destroyed */
    FMMHP_EUNSUPPORTED = 6  /* valid request this build does not handle (see message) */
} fmmhp_status;

#define FMMHP_MAX_P 40

typedef struct {
    int p;          /* truncation order: expansion coefficients n = 0..p (the paper's p,
                       eq. (truncatedME)).  1 <= p <= FMMHP_MAX_P.  The kernels are compiled for
                       p in {5, 10, ..., 40}; other values are rounded UP to the next of these and
                       fmmhp_plan_info reports the order actually used. */
    int leaf_size;  /* a box with more than leaf_size points is split (>= 1) */
    int max_level;  /* deepest tree level, 1..30 (1..27 for a forest); 0 selects the maximum */
    unsigned flags; /* 0, or a combination of FMMHP_FLAG_GRAPH, FMMHP_FLAG_M2L_FP32,
                       FMMHP_FLAG_SERIAL, one of FMMHP_FLAG_M2L_VECTOR, FMMHP_FLAG_M2L_MFMA and
                       one of FMMHP_FLAG_DIRICHLET, FMMHP_FLAG_NEUMANN */
    /* Launch shape of the near field (the U-list sums), which runs beside the far-field kernels on
     * a bounded grid.  Neither changes what is computed beyond rounding; fmmhp_tune picks both by
     * timing.  0 selects the default for the plan's p. */
    int near_walk;   /* 0: default; 1: source points loaded one step ahead of their use (hides
                        memory latency, more instructions per pair); 2: plain walk; 3: symmetric
                        leaf pairs (potential evaluations: each pair of leaves once, its column
                        sums gathered by a second kernel; other passes use walk 1); 4: symmetric
                        leaf pairs with the pairs blocked in registers (each lane holds up to 8
                        targets; column sums reduced over a few lanes; potential evaluations,
                        other passes use walk 1) */
    int near_groups; /* 0: default; 1..16: near-field workgroups per compute unit (potential passes;
                        gradient and double-layer passes take at least 8) */
} fmmhp_opts;

/* fmmhp_eval records its launches into a HIP graph on the first call with a given (n_vec, q, phi,
 * stream) and replays the graph on later calls with the same four; another combination records a
 * new graph.  The stream must not be the null stream (graph capture needs a created stream; the
 * null stream runs eagerly).  Phase timing is unavailable while recording. */
#define FMMHP_FLAG_GRAPH 1u

/* The M2L of upper (free-space) sources runs on the FP32 matrix cores (MFMA), with operands scaled
 * into FP32 range and each offset slot's FP32 sums folded into FP64 (addition 3).  Everything else
 * stays FP64.  Expect a relative error of ~1e-7 on top of the truncation error: for tolerances of
 * 1e-6, not 1e-10. */
#define FMMHP_FLAG_M2L_FP32 2u

/* The half-plane Green's functions of eq. (ddd1.2) instead of the Robin one:
 *   Dirichlet  G = -(1/2pi) ln|r - r'| + (1/2pi) ln|r - r'_im|   (G = 0 on y = 0; the Z -> infinity limit)
 *   Neumann    G = -(1/2pi) ln|r - r'| - (1/2pi) ln|r - r'_im|   (d_y G = 0 on y = 0)
 * The same tree and expansions without the reaction part (no reaction M2L, near-field reaction
 * sums or surface term); the impedance arguments are ignored (not checked), the potential is real
 * (its imaginary part is zero) and fmmhp_backward reports a zero impedance gradient.  At most one of
 * the two may be set. */
#define FMMHP_FLAG_DIRICHLET 4u
#define FMMHP_FLAG_NEUMANN 8u
/* Every kernel of an evaluation on the caller's stream, one after another, instead of the near field
 * and the deep-level M2L on streams of their own beside the rest: a profiling aid (each kernel's
 * duration is then its own, not shared with concurrent kernels); slower. */
#define FMMHP_FLAG_SERIAL 16u
/* Form of the FP64 M2L of upper sources (eq. (truncatedM2Lcoef) and the log-kernel M2L): the vector
 * ALUs (one lane per target box, operators in scalar registers; the default) or the FP64 matrix cores
 * (v_mfma_f64_16x16x4f64, complex numbers as 2 x 2 real blocks); at most one of the two flags.  The
 * same sums in another order (agreement to rounding).  Ignored with FMMHP_FLAG_M2L_FP32. */
#define FMMHP_FLAG_M2L_VECTOR 32u
#define FMMHP_FLAG_M2L_MFMA 64u

typedef struct {
    int64_t n;              /* number of points */
    int p;                  /* truncation order in use */
    int leaf_size, max_level;
    int depth;              /* deepest level present */
    int64_t nbox;           /* upper-half boxes (each has an implicit mirror image box) */
    int64_t nleaf;
    int64_t list_len[4];    /* total entries of the U, V, W, X lists */
    double x_lo, S, scale;  /* root square [x_lo, x_lo + S] x [-S/2, S/2]; cells = 2^30 / S */
    double lambda_re, lambda_im;
    int real_impedance;     /* 1 if lambda_im == 0 (one local expansion + rank-one surface term) */
    int64_t device_bytes;   /* device memory held by the plan */
    int64_t p2p_pairs[2];   /* near-field (target, source) pairs per charge vector: upper sources,
                               image sources (the U list expanded to points) */
    int64_t m2l_pairs[2];   /* M2L (target box, source box) pairs: upper, image (the V list) */
    int32_t n_inst;         /* instances (1 for fmmhp_plan_create) */
    int32_t near_walk;      /* near-field launch shape in use (see fmmhp_opts) */
    int32_t near_groups;
    int64_t n_sources;      /* sources (n unless the plan has separate targets: then n - n_sources
                               targets follow the sources in the tree's point set) */
} fmmhp_plan_stats;

/* Phases of fmmhp_eval whose device time fmmhp_plan_phase_times reports. */
enum {
    FMMHP_PHASE_P2M = 0,    /* charge gather and leaf multipoles (S2M) */
    FMMHP_PHASE_M2M = 1,    /* upward pass, one launch per level */
    FMMHP_PHASE_M2L = 2,    /* multipole-to-local over all levels, one launch */
    FMMHP_PHASE_P2L = 3,    /* X list */
    FMMHP_PHASE_L2L = 4,    /* downward pass, one launch per level */
    FMMHP_PHASE_SURF = 5,   /* surface term sum (real impedance) */
    FMMHP_PHASE_LEAF = 6,   /* L2P, W list and output (after the near field has joined) */
    FMMHP_PHASE_NEAR = 7,   /* near field (U list), on the plan's side stream, concurrent with 1-5 */
    FMMHP_NUM_PHASES = 8
};

/* Build a plan: the adaptive quadtree over the points and their images, interaction lists and
 * translation tables (Algorithm 1, its image, tree and table steps; tables from eq.
 * (integralrecursion)).
 *
 *   n              number of points (sources = targets), 1 <= n < 2^31
 *   x, y           [device] point coordinates, y > 0, finite
 *   img_x, img_y   [device] the image sources r_j^im = (x_j, -y_j) (Section 2.2), or both NULL.  When
 *                  given they must equal (x, -y) bitwise, else FMMHP_EDOMAIN: the tree is built
 *                  over the points and their exact mirror images.
 *   lambda_re/im   impedance Z_eps; lambda_re > 0, lambda_im >= 0
 *   opts           [host] options (see fmmhp_opts); NULL selects p = 20, leaf_size = 40
 *   stream         stream for the build; this call synchronises it (tree sizes are read back)
 *   plan_out       [host] receives the plan handle, owned by the caller until fmmhp_plan_destroy
 *
 * The plan keeps its own sorted copy of the coordinates: x, y may be freed after the call returns.
 */
fmmhp_status fmmhp_plan_create(int64_t n, const double *x, const double *y, const double *img_x,
                               const double *img_y, double lambda_re, double lambda_im,
                               const fmmhp_opts *opts, hipStream_t stream,
                               fmmhp_plan_t *plan_out);

/* Build a plan with separate target points: the potential of the sources is wanted at the targets
 * (the paper's Example 2 evaluates the field of charged circles on a grid that reaches y = 0).
 *
 *   n_src, xs, ys  [device] source coordinates, y > 0, finite; n_src >= 1
 *   n_tgt, xt, yt  [device] target coordinates, y >= 0, finite; n_tgt >= 1, n_src + n_tgt < 2^31
 *   lambda_re/im, opts, stream, plan_out   as for fmmhp_plan_create
 *
 * The tree is built over the sources and the targets together (the targets take part as points
 * without charge).  fmmhp_eval / fmmhp_eval_complex on this plan take q [n_vec][n_src] and return
 * phi [n_vec][n_tgt][2].  A target that coincides with a source skips that source's free-space term
 * (as coincident points do in fmmhp_plan_create); a target on y = 0 is the limit of the potential
 * from y > 0.  fmmhp_backward returns FMMHP_EUNSUPPORTED for this plan.  xs, ys, xt, yt may be freed
 * after the call returns. */
fmmhp_status fmmhp_plan_create_targets(int64_t n_src, const double *xs, const double *ys, int64_t n_tgt,
                                       const double *xt, const double *yt, double lambda_re, double lambda_im,
                                       const fmmhp_opts *opts, hipStream_t stream, fmmhp_plan_t *plan_out);

/* Build a batched plan: n_inst independent problems ("instances") in one forest, each with its own
 * points, root square and impedance; every evaluation runs all instances in the same launches
 * (Algorithm 1 per instance).
 *
 *   n_inst    number of instances, 1 <= n_inst <= 512
 *   offsets   [host] [n_inst + 1] point ranges: instance k owns points offsets[k] .. offsets[k+1]-1;
 *             offsets[0] = 0, strictly increasing (no empty instance), total < 2^31
 *   x, y      [device] coordinates of all points, instance after instance (y > 0)
 *   lambda    [host] [n_inst][2] impedance (re, im) of each instance, re > 0, im >= 0
 *   opts      [host] as for fmmhp_plan_create; with n_inst > 1 the cells have 27 bits per axis, so
 *             max_level <= 27
 *
 * n_inst = 1 gives the same plan as fmmhp_plan_create.  Errors as for fmmhp_plan_create, plus
 * FMMHP_EINVAL for bad offsets or n_inst.  Sources and targets coincide within each instance;
 * instances do not interact.
 */
fmmhp_status fmmhp_batch_plan_create(int n_inst, const int64_t *offsets, const double *x,
                                     const double *y, const double *lambda,
                                     const fmmhp_opts *opts, hipStream_t stream,
                                     fmmhp_plan_t *plan_out);

/* Evaluate phi = A q for n_vec real charge vectors (Algorithm 2), over every instance of the plan.
 *
 *   n_vec   number of charge vectors, >= 1
 *   q       [device] charges, [n_vec][n] row-major, real, in the caller's point order (n = all
 *           points of all instances)
 *   phi     [device] output, [n_vec][n][2] (re, im) interleaved, caller's point order
 *
 * Vectors are evaluated eight at a time where possible: the near field computes each pair's kernel
 * once for the eight, the far-field kernels take the vector as a grid dimension.  The first call
 * with n_vec >= 8 grows the plan's workspace for eight vectors.  Complex charges: see
 * fmmhp_eval_complex.  No host synchronisation.
 */
fmmhp_status fmmhp_eval(fmmhp_plan_t plan, int n_vec, const double *q, double *phi,
                        hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): fmmhp_eval with each pass's per-vector workspace (multipoles,
 * locals, sorted charges, near-field and surface sums) taken from a static device array of the
 * library, FMMHP_NOALLOC_SCRATCH_BYTES (128 MiB) per device, instead of the plan's memory.  Calls no
 * hipMalloc, hipFree or allocating routine; launches eagerly on stream (the plan's graph flag is
 * not used).  Same arguments, layout, ordering and results as fmmhp_eval, for plans whose points are
 * the targets (fmmhp_plan_create, fmmhp_batch_plan_create).
 *
 * Eight vectors share a pass when their workspace fits the array, else vectors run one at a time;
 * the workspace of one vector is 16 (p + 1)(1 + nloc) bytes per box plus 24 bytes per point (nloc =
 * 1 for a real impedance, 2 for a complex one, p rounded up to a multiple of 5).  The plan's device
 * must be the current device.  The first call on a device looks up the array's address there
 * (hipGetSymbolAddress); each device holds the array until the process ends.  Every call on a device
 * shares that device's array and leaves its contents behind; evaluations overwrite all of the
 * workspace they read, so nothing needs clearing, but calls that overlap on one device (different
 * streams or host threads) race and give wrong results.
 *
 * Errors: FMMHP_EINVAL for the arguments fmmhp_eval rejects, or when one vector's workspace exceeds
 * the array; FMMHP_EUNSUPPORTED for plans with separate targets; FMMHP_ESTATE when phase timing is on
 * (fmmhp_plan_set_timing) or the plan's device is not current; FMMHP_EHIP when the address lookup
 * fails.
 */
#define FMMHP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
fmmhp_status fmmhp_eval_noalloc(fmmhp_plan_t plan, int n_vec, const double *q, double *phi,
                                hipStream_t stream);

/* Evaluate phi = A q for n_vec complex charge vectors: the operator is linear over the reals in the
 * charges, so phi[q] = phi[Re q] + i phi[Im q], computed as two real passes and combined on the
 * device (eqs. (potential1), (1.2), (reactioncomp1) with complex q_j).
 *
 *   q     [device] charges, [n_vec][n][2] (re, im) interleaved, caller's point order
 *   phi   [device] output, [n_vec][n][2], caller's point order
 *
 * The first call allocates 48 bytes per point of workspace, owned by the plan.  No host
 * synchronisation.  Errors as for fmmhp_eval.
 */
fmmhp_status fmmhp_eval_complex(fmmhp_plan_t plan, int n_vec, const double *q, double *phi,
                                hipStream_t stream);

/* The field of one real charge vector: the potential and its gradient at the targets (every point,
 * or the separate targets of fmmhp_plan_create_targets), for field and boundary-integral uses of the
 * potential (the paper's introduction and conclusion).  The gradient comes from the same expansions
 * differentiated in the target: the far field H' of the local expansions, d_x log|r - r'| = (x -
 * x') / |r - r'|^2 and alike in the near field, and d_x I_0 = i I_1, d_y I_0 = -I_1 for the reaction
 * term (eq. (integralrecursion), n = 1).
 *
 *   q              [device] [n_src] real charges (n_src = n for fmmhp_plan_create plans)
 *   phi            [device] [n_tgt][2] complex potential
 *   grad_x, grad_y [device] [n_tgt][2] complex d phi / d x and d phi / d y at the targets
 *
 * A target that coincides with a source skips that source's free-space term in both.  Asynchronous
 * on stream. */
/* The double-layer potential of dipole sources at the targets (every point, or the separate
 * targets of fmmhp_plan_create_targets), the other layer potential of the boundary-integral uses of
 * the Green's function in the paper's introduction:
 *
 *   phi_i = sum_j mu_j n_j . grad_{r_j} G(r_i, r_j)
 *
 * with G the plan's Green's function (Robin, eq. (ddGreensfunimp); Dirichlet or Neumann,
 * eq. (ddd1.2)).  The free-space term is skipped where r_i == r_j, as for the potential.  The same
 * tree and translations serve: the multipoles, the point-to-local terms, the near field and the
 * surface sums take the derivative of each source's term along its normal.
 *
 *   n_vec        number of density vectors (>= 1), evaluated one after another
 *   mu           [device] densities, [n_vec][n_src] real (mu_complex = 0) or [n_vec][n_src][2]
 *                (re, im) interleaved (mu_complex = 1; phi[mu] = phi[Re mu] + i phi[Im mu])
 *   nx, ny       [device] [n_src] source normals (the result is linear in them: a non-unit vector
 *                scales its dipole), caller's point order
 *   phi          [device] output, [n_vec][n_tgt][2]
 *
 * The first call allocates 16 bytes per point for the sorted normals (and, for complex densities or
 * a plan with separate targets, the workspaces of fmmhp_eval_complex and fmmhp_eval).  Asynchronous
 * on stream; not captured in a graph.  FMMHP_EINVAL for a NULL pointer, n_vec < 1 or mu_complex
 * outside {0, 1}.
 */
fmmhp_status fmmhp_eval_double_layer(fmmhp_plan_t plan, int n_vec, const double *mu, int mu_complex,
                                     const double *nx, const double *ny, double *phi, hipStream_t stream);

fmmhp_status fmmhp_eval_field(fmmhp_plan_t plan, const double *q, double *phi, double *grad_x, double *grad_y,
                              hipStream_t stream);

/* The normal derivative of the potential of one real charge vector at the targets, for the
 * second-kind boundary-integral uses of the paper's introduction:
 *
 *   dphi_i = n_i . grad phi(r_i) = n_x d_x phi + n_y d_y phi,
 *
 * from the field of fmmhp_eval_field (same expansions, same coincidence rule).
 *
 *   q        [device] [n_src] real charges
 *   nx, ny   [device] [n_tgt] target normals (the result is linear in them)
 *   dphi     [device] output, [n_tgt][2] complex
 *
 * The first call allocates 48 bytes per target of workspace (plus that of fmmhp_eval_field).
 * Asynchronous on stream.  FMMHP_EINVAL for a NULL pointer. */
fmmhp_status fmmhp_eval_normal_derivative(fmmhp_plan_t plan, const double *q, const double *nx, const double *ny,
                                          double *dphi, hipStream_t stream);

/* Adjoint of fmmhp_eval for one real charge vector: gradients of a real loss l of phi with respect
 * to the charges, the point positions and the impedance (the reverse-mode step of phi = A q; the
 * paper's Green's function, eqs. (1.2) and (reactdecomposition), differentiated).
 *
 *   q          [device] charges [n], real, caller's point order (those of the forward call)
 *   grad_phi   [device] incoming gradient [n][2]: g_i = dl/dRe phi_i + i dl/dIm phi_i
 *   grad_q     [device] output [n]: dl/dq_j = Re sum_i conj(g_i) G(r_i, r_j), or NULL
 *   grad_x, grad_y  [device] outputs [n]: dl/dx_k, dl/dy_k, or NULL.  A point moves as a target
 *              and as a source; both are included, so are its own image and reaction terms.
 *   grad_lambda [host] output [n_inst][2]: (dl/dRe Z_k, dl/dIm Z_k) per instance, or NULL.  When
 *              given, the call synchronises the stream.
 *
 * The potential's gradient fields come from the same expansions as phi (derivatives of the local
 * expansions, the multipole series and the near-field kernels), so their accuracy follows p like
 * phi's.  dl/dZ uses the scale homogeneity of the Green's function, G_Z(s r, s r') = G_{sZ}(r, r')
 * up to the log of s for skipped coincident pairs.  Cost: three evaluations (one gradient pass for
 * q, two potential-and-gradient passes for Re and Im of conj(g)); two potential passes when only
 * grad_q is asked for.  The first call allocates the adjoint workspace (about 150 bytes per
 * point), owned by the plan.  Calls on one plan must be ordered (one stream, or synchronised).
 * Errors: FMMHP_EINVAL for a NULL q or grad_phi; with all outputs NULL the call does nothing.
 */
fmmhp_status fmmhp_backward(fmmhp_plan_t plan, const double *q, const double *grad_phi,
                            double *grad_q, double *grad_x, double *grad_y,
                            double *grad_lambda, hipStream_t stream);

/* fmmhp_backward with the impedance gradient left on the device, for training loops that must not
 * synchronise the host: identical gradients, and grad_lambda is a [device] output [n_inst][2]
 * (dl/dRe Z_k, dl/dIm Z_k), written by a kernel on stream; the call never synchronises.  (The
 * reduction of eq. (reactdecomposition)'s homogeneity sums runs on the device either way; only
 * the place the result lands differs.)  Errors as for fmmhp_backward. */
fmmhp_status fmmhp_backward_device(fmmhp_plan_t plan, const double *q, const double *grad_phi, double *grad_q,
                                   double *grad_x, double *grad_y, double *grad_lambda, hipStream_t stream);

/* Plan statistics (sizes, root square, order in use).  stats: [host]. */
fmmhp_status fmmhp_plan_info(fmmhp_plan_t plan, fmmhp_plan_stats *stats);

/* Copy the tree and interaction lists to host arrays, for bit-exact comparison with a reference
 * build.  Box arrays have stats.nbox entries, perm has n, list offsets nbox + 1, list entries
 * stats.list_len[k].  Boxes are numbered by (level, Morton prefix); list entries are
 * 2 * box + image (image = 1 refers to the mirror image of that box below y = 0), ascending.
 * Any pointer may be NULL to skip that array.  Synchronises the plan's stream.
 *
 *   level, bx, by   box level (1..30) and full-tree integer coordinates (by >= 2^(level-1))
 *   first, count    range of the box's points in sorted order
 *   parent          parent box, -1 at level 1;  leaf: 1 if the box is a leaf
 *   child_first, nchild   children are the nchild boxes starting at child_first (-1 if none)
 *   perm            sorted position -> input index
 *   {u,v,w,x}_off, _ent   CSR lists U (near field), V (M2L), W (M2P), X (P2L)
 */
fmmhp_status fmmhp_plan_export_tree(fmmhp_plan_t plan, int32_t *level, int32_t *bx, int32_t *by,
                                    int32_t *first, int32_t *count, int32_t *parent,
                                    int32_t *leaf, int32_t *child_first, int32_t *nchild,
                                    int64_t *perm, int64_t *u_off, int32_t *u_ent,
                                    int64_t *v_off, int32_t *v_ent, int64_t *w_off,
                                    int32_t *w_ent, int64_t *x_off, int32_t *x_ent);

/* Per-phase device timing of fmmhp_eval (profiling aid).  enable = 1 clears the totals and starts
 * recording HIP events around every phase of every subsequent eval on that eval's stream;
 * enable = 0 stops recording.  Recording adds one event per phase boundary. */
fmmhp_status fmmhp_plan_set_timing(fmmhp_plan_t plan, int enable);

/* Totals since timing was enabled: ms[k] = summed device milliseconds of phase k
 * (k < FMMHP_NUM_PHASES), n_evals = number of charge vectors evaluated.  Waits for the recorded
 * events.  ms: [host] FMMHP_NUM_PHASES doubles; n_evals: [host], may be NULL. */
fmmhp_status fmmhp_plan_phase_times(fmmhp_plan_t plan, double *ms, int64_t *n_evals);

/* Totals since timing was enabled of the upper-source M2L kernel alone (profiling aid): ms = summed
 * device milliseconds of its launches, each bracketed by HIP events on the stream it runs on (it
 * runs as up to two launches per charge-vector pass: the deepest levels on a second stream, the
 * coarse levels on the eval stream, concurrently with the near field), n_launches = their number.
 * With FMMHP_FLAG_M2L_FP32 each bracket covers the FP32 source-row conversion and the matrix-core
 * M2L of those levels.  Waits for the recorded events.  ms: [host] one double; n_launches: [host], may be NULL. */
fmmhp_status fmmhp_plan_m2l_kernel_times(fmmhp_plan_t plan, double *ms, int64_t *n_launches);

/* Release the plan and its device memory.  Synchronises the device.  plan may be NULL (no-op). */
fmmhp_status fmmhp_plan_destroy(fmmhp_plan_t plan);

/* Direct O(n_tgt * n_src) evaluation of phi_i = sum_j q_j G(r_i, r_j) on the GPU, with the same
 * kernel arithmetic as the FMM's near field (eqs. (1.2), (reactioncomp1)).  Targets may differ from
 * sources; the free-space term skips pairs with identical coordinates.
 *   src_x, src_y, q  [device] [n_src] (q: [n_vec][n_src]);  tgt_x, tgt_y [device] [n_tgt]
 *   phi              [device] [n_vec][n_tgt][2]
 */
fmmhp_status fmmhp_direct_eval(int64_t n_src, const double *src_x, const double *src_y,
                               int n_vec, const double *q, int64_t n_tgt, const double *tgt_x,
                               const double *tgt_y, double lambda_re, double lambda_im,
                               double *phi, hipStream_t stream);

/* The reaction integrals I_0 .. I_nmax of eq. (generalintegral) at m points (x_k, y_k), y_k > 0,
 * computed on the GPU from the closed form of I_0 (exponential integral) and the upward recursion
 * of eq. (integralrecursion).
 *   x, y  [device] [m];  out [device] [m][nmax + 1][2];  0 <= nmax <= 2 * FMMHP_MAX_P
 */
fmmhp_status fmmhp_reaction_integrals(int64_t m, const double *x, const double *y, int nmax,
                                      double lambda_re, double lambda_im, double *out,
                                      hipStream_t stream);

/* Autotuner: choose the truncation order p and the leaf size for a point set, an impedance and an
 * accuracy target (p from tolerance, leaf size from measured eval time).
 *
 * The error of a candidate is measured, not modelled: the FMM potential is compared with the
 * GPU direct sum (fmmhp_direct_eval) at `sample` fixed targets (indices floor(k n / sample)),
 * for the given charges.  For each candidate leaf size the smallest p in {5, 10, ..., 40} whose
 * relative l2 error is at most tol is kept, and the (p, leaf) pair with the fastest
 * fmmhp_eval time (n_vec vectors) wins; an eval time is the median over three rounds of the mean
 * of five back-to-back evaluations (the steady state of a loop of evaluations).
 *
 *   n, x, y, lambda_re, lambda_im   as for fmmhp_plan_create ([device] x, y)
 *   q            [device] [n] charges used for the trial evaluations
 *   tol          target relative l2 error, > 0
 *   n_vec        vectors per timed eval (>= 1)
 *   leaf_sizes   [host] candidate leaf sizes (n_leaf entries), or NULL for {24, 32, 40, 48, 64, 96}
 *   sample       targets in the accuracy sample, 1..n (0 selects min(n, 256))
 *   best         [host] receives the chosen options (p, leaf_size, and the launch shape
 *                near_walk, near_groups timed on the chosen plan, six shapes (walks 1, 2 and 4 on
 *                two to eight workgroups per CU) in turn over three rounds; a shape other than the
 *                default needs to be more than 2% faster; then the FP64 M2L form: the other of
 *                FMMHP_FLAG_M2L_VECTOR and FMMHP_FLAG_M2L_MFMA when more than 2% faster; then
 *                flags gets FMMHP_FLAG_M2L_FP32 when the FP32 matrix-core M2L on that plan and
 *                shape still meets tol against the direct sum and is more than 2% faster;
 *                max_level 0)
 *   err, eval_ms [host, may be NULL] the chosen pair's measured error and median eval time
 * Returns FMMHP_EUNSUPPORTED if no candidate reaches tol at p = 40.  Synchronises the stream;
 * allocates and frees its own temporaries. */
fmmhp_status fmmhp_tune(int64_t n, const double *x, const double *y, const double *q,
                        double lambda_re, double lambda_im, double tol, int n_vec,
                        const int *leaf_sizes, int n_leaf, int sample, fmmhp_opts *best,
                        double *err, double *eval_ms, hipStream_t stream);

const char *fmmhp_status_string(fmmhp_status s);
const char *fmmhp_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* FMMHP_H */
