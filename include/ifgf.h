/*
 * ifgf.h - C ABI of the MI355X (gfx950) IFGF-accelerated apply of the
 * discrete 3-D Helmholtz combined-field operator.
 *
 * The operation (paper Section 3, eq. (field1), with the combined-field
 * kernel of Section 2.2, eqs. (CombinedLayer), (GreenFunction),
 * (double_layer)):
 *
 *     u_i = sum_{j != i} w_j sigma_j K(x_i, x_j),
 *     K(x, y) = dPhi(x, y)/dnu(y) - i eta Phi(x, y),
 *     Phi(x, y) = exp(i k |x - y|) / (4 pi |x - y|),
 *
 * for pairwise distinct surface points x_j with normals nu(x_j) and
 * quadrature weights w_j.  eta is the coupling parameter (called gamma in
 * the paper).  The sum is approximated by the Interpolated Factored Green
 * Function method (Section 3, Algorithm 1): level-D neighbour interactions
 * are summed directly, all others are obtained from tensor Chebyshev
 * interpolants of the factored field on cone segments of an octree.
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] must point to device memory of the current
 *     HIP device; [host] pointers to host memory.  Arrays are row-major and
 *     tightly packed.  Complex values are interleaved (re, im) pairs, i.e.
 *     the layout of C99 complex / torch.complex64 / torch.complex128.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; entry points return once enqueued unless
 *     stated otherwise.
 *   - Nothing throws across this ABI.  Every fallible call returns an
 *     ifgf_status; ifgf_last_error() returns a message for the last failure
 *     on the calling thread.
 *   - Point order: all per-point arrays (points, normals, weights, sigma,
 *     u) are in the caller's order.  The library sorts internally and
 *     scatters results back.
 */
#ifndef IFGF_H
#define IFGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifgf_plan_s *ifgf_plan;
typedef struct ifgf_batch_s *ifgf_batch;

typedef enum {
    IFGF_OK = 0,
    IFGF_EINVAL = 1,        /* invalid argument (null pointer, size, option) */
    IFGF_EDUPLICATE = 2,    /* two points coincide (eq. field1 needs distinct points) */
    IFGF_ENOMEM = 3,        /* device allocation failed */
    IFGF_EHIP = 4,          /* a HIP runtime call failed; see ifgf_last_error() */
    IFGF_EUNSUPPORTED = 5,  /* option combination not compiled in */
    IFGF_EBUSY = 6,         /* another apply on the same plan is in progress */
    IFGF_EINTERNAL = 7      /* internal consistency check failed */
} ifgf_status;

/* Arithmetic of the interpolation stages. */
enum {
    IFGF_PREC_FP64 = 0,         /* every stage in IEEE double                          */
    IFGF_PREC_FP32_INTERP = 1   /* factors, interpolation, propagation and near field in
                                   FP32 complex; target distances, k|x - y|, its
                                   reduction modulo 2 pi and the centred factor in FP64 */
};

/* Element type of sigma / u / v arrays. */
enum { IFGF_C64 = 0, IFGF_C128 = 1 };

/* Kernel selector.  IFGF_KERNEL_CONSTANT (K = 1) is a test kernel: the
 * interpolation is then exact and u_i = sum_{j != i} w_j sigma_j, which
 * checks that the octree traversal counts every pair once. */
enum { IFGF_KERNEL_COMBINED = 0, IFGF_KERNEL_CONSTANT = 1 };

typedef struct {
    /* Compiled orders (p_s, p_ang): (3, 5) and (4, 6) in both precisions; (8, 8)
       with IFGF_PREC_FP64 only (relative error about 4e-7, the FP64 accuracy
       setting, with ns0 = 1, nc0 = 4).  Others return IFGF_EUNSUPPORTED.           */
    int32_t p_s;            /* Chebyshev points per cone segment along s (paper P_s); default 4 */
    int32_t p_ang;          /* ... along theta and along phi (paper P_ang); default 6      */
    int32_t ns0;            /* radial cone intervals at the finest level (paper n_S,0); default 2  */
    int32_t nc0;            /* polar cone intervals at the finest level (paper n_C,0); default 4;
                               azimuthal intervals are 2 * nc0 (eq. deltas)              */
    int32_t depth;          /* number of octree levels D, root = level 1 (Sec. 3.4); 0 = choose
                               D so that the finest box side is closest to leaf_h_lambda
                               wavelengths; 1 <= D <= 11                                   */
    double leaf_h_lambda;   /* finest box side in wavelengths for depth = 0; default 0.5 */
    int32_t precision;      /* IFGF_PREC_*; default IFGF_PREC_FP32_INTERP                  */
    int32_t max_rhs;        /* largest nrhs accepted by the apply calls; default 1         */
    int32_t kernel;         /* IFGF_KERNEL_*; default IFGF_KERNEL_COMBINED                  */
    int32_t prop_kernel;    /* upward pass with one right-hand side: IFGF_PROP_AUTO
                               (default), IFGF_PROP_NODE, IFGF_PROP_CONE or
                               IFGF_PROP_PAIRS (below)                                     */
    int32_t target_kernel;  /* cousin-target stage with one right-hand side:
                               IFGF_TARGET_AUTO (default), IFGF_TARGET_WAVE,
                               IFGF_TARGET_ROWS or IFGF_TARGET_PAIRS (below)               */
    int32_t far_field;      /* 1: also make the far-field cones relevant - every level-3
                               cone whose radial interval starts at s = 0 (x at infinity,
                               any direction) and, by eq. RelevantCones' node rule, what
                               they need at the finer levels - so that ifgf_far_field can
                               evaluate the far-field pattern; adds up to about one cone
                               per angular interval and box at every level.  Default 0.  */
} ifgf_options;

/* Upward-pass formulation (nrhs = 1, FP32 or FP64; other nrhs always use
 * their own kernels).  NODE: every parent node of every relevant parent cone
 * evaluates its child interpolants (work items = a parent box and a few of
 * its cones).  CONE: all boxes of a level have the same size, so a parent
 * node's position in a child's frame depends only on (parent cone id, child
 * octant, node); the boxes holding the same parent cone id are taken
 * together and the interpolation becomes a product of their child
 * coefficients with one basis matrix, on MFMA.  The plan stores the node
 * positions in each child frame once per (parent cone id, octant), about
 * 42 KB (FP32) or 60 KB (FP64) per cone id at P = (4,6,6).  AUTO picks CONE
 * for the levels where the boxes per parent cone id fill its tiles and that
 * table stays within 2.5 times the level's coefficient storage; CONE forces
 * it on every level.  PAIRS: the plan locates every (parent node, child box)
 * pair of the pass once - child cone slot, local coordinates, kernel ratio -
 * and sorts the pairs by child slot; an apply evaluates them in that order
 * and adds each node's pairs in child order (36 bytes per pair, up to 2^28
 * pairs per level; levels with more, or whose list the device memory does
 * not hold at plan creation, use NODE).  AUTO takes PAIRS on the
 * levels without tiles.  All give the same operator up to rounding; the
 * transposed apply gathers over a level's pair list where it has one. */
enum { IFGF_PROP_AUTO = 0, IFGF_PROP_NODE = 1, IFGF_PROP_CONE = 2, IFGF_PROP_PAIRS = 3 };

/* Cousin-target formulation (Algorithm 1, target evaluation; nrhs = 1, FP32
 * or FP64 — other nrhs always use their own kernels).  WAVE: a
 * lane per target walks its box's cousin list; the wave stages each distinct
 * cone it meets in LDS and the lanes holding that cone contract against it.
 * ROWS: the 16 lanes of a row walk the merged cousin lists of their targets
 * together, load the row's current cone across the row and contract with the
 * coefficients broadcast between lanes (no LDS); levels run as separate
 * work-groups and are added afterwards, which needs n x (D - 2) complex values
 * (plan precision) of plan memory.  PAIRS: the plan lists every (target,
 * cousin box) pair of every level with its cone slot, local coordinates and
 * centred factor, sorted by cone; a row of 16 lanes then mostly holds pairs
 * of one cone, evaluates them with the row stage of ROWS, and a second pass
 * sums each target's pairs in the order ROWS uses; about 40 bytes (FP32) or
 * 72 bytes (FP64) per pair of plan memory, built for at most 2^28 pairs
 * and where the device memory holds them (else the plan keeps ROWS).
 * AUTO = PAIRS where the lists were built, else ROWS.  All give the same
 * operator up to rounding. */
enum { IFGF_TARGET_AUTO = 0, IFGF_TARGET_WAVE = 1, IFGF_TARGET_ROWS = 2, IFGF_TARGET_PAIRS = 3 };

/* Plan statistics (host struct). */
#define IFGF_MAX_LEVELS 12
typedef struct {
    int32_t depth;                          /* D                                       */
    int64_t n;                              /* number of points                         */
    double root_side;                       /* side of the level-1 box                  */
    double root_corner[3];                  /* lower corner of the level-1 box          */
    int32_t p_s, p_ang;
    int32_t precision;
    int64_t boxes[IFGF_MAX_LEVELS];         /* relevant boxes per level (index = d)     */
    int32_t ns[IFGF_MAX_LEVELS];            /* cone intervals along s per level         */
    int32_t nc[IFGF_MAX_LEVELS];            /* cone intervals along theta per level     */
    int64_t cones[IFGF_MAX_LEVELS];         /* relevant cone segments per level (d >= 3)*/
    int64_t cousin_pairs[IFGF_MAX_LEVELS];  /* (target point, source box) cousin pairs  */
    int64_t near_pairs;                     /* ordered (target, source) pairs summed
                                               directly at level D, self included      */
    int64_t prop_evals[IFGF_MAX_LEVELS];    /* child interpolations into level d-1 nodes,
                                               indexed by the child level d            */
    int64_t device_bytes;                   /* device memory held by the plan           */
    int32_t prop_kernel[IFGF_MAX_LEVELS];   /* upward pass from child level d (index d):
                                               IFGF_PROP_NODE, _CONE or _PAIRS with one
                                               right-hand side, 0 if no pass            */
    int64_t pair_rows[IFGF_MAX_LEVELS];     /* rows of 16 consecutive pairs of level d's
                                               cousin-target pair list (0: no lists)    */
    int64_t pair_row_cones[IFGF_MAX_LEVELS];/* cone slots met by those rows, summed: the
                                               row stage's passes (lane use = pairs /
                                               (16 x passes))                           */
} ifgf_plan_stats;

/* Fill *o with the defaults listed above.  o: [host], non-null. */
void ifgf_options_default(ifgf_options *o);

/*
 * Build a plan: octree of D levels over the points, Morton (Z-curve) order
 * (Sec. 3.5), neighbour and cousin lists (eq. NeighborsCousins), cone
 * counts per level (Remark cone_seg_size) and relevant cone segments
 * (eq. RelevantCones), all on the device.
 *
 *   out      [host]   receives the plan handle (NULL on failure)
 *   n        number of points, n >= 1
 *   points   [device] n x 3 doubles, the surface points x_j (pairwise distinct)
 *   normals  [device] n x 3 doubles, nu(x_j) (used as given, not normalized)
 *   weights  [device] n doubles, quadrature weights w_j
 *   k        wavenumber, k > 0
 *   eta      coupling parameter (any real; 0 gives the double layer alone)
 *   opt      [host]   options, or NULL for the defaults
 *   stream   hipStream_t on which the plan is built
 *
 * The plan copies what it needs; the inputs may be freed once the call has
 * returned.  The call synchronizes `stream` to read back sizes.
 * Errors: EINVAL (n < 1, null pointer, non-finite input, k <= 0, bad
 * option), EDUPLICATE (two bitwise-equal points), ENOMEM, EHIP,
 * EUNSUPPORTED (p_s / p_ang pair not compiled), EINTERNAL.
 */
ifgf_status ifgf_plan_create(ifgf_plan *out, int64_t n, const double *points,
                             const double *normals, const double *weights,
                             double k, double eta, const ifgf_options *opt,
                             void *stream);

/*
 * A plan whose outputs are separate target points (Sec. 5: the scattered
 * field off the surface, eq. CombinedLayer discretized as eq. field1):
 *
 *     u(t_l) = sum_j w_j sigma_j K(t_l, x_j),   l = 0 .. nt - 1,
 *
 * every source j included.  The octree, lists and relevant cones are built
 * over sources and targets together (the root box holds both; target boxes
 * get neighbours and cousins like any other), the targets carrying zero
 * density, so the targets receive the same near-field sums and cousin
 * interpolations as surface points.  Arguments as ifgf_plan_create, plus
 * nt >= 1 and targets [device] nt x 3 doubles, distinct from each other and
 * from the sources (EDUPLICATE otherwise).  For such a plan ifgf_apply takes
 * sigma with n rows and writes u with nt rows; the work of one apply is that
 * of an apply over the n + nt points.  ifgf_apply_adjoint (EUNSUPPORTED),
 * ifgf_gmres_solve and ifgf_batch_create (EINVAL) do not take such plans;
 * ifgf_far_field does.
 */
ifgf_status ifgf_plan_create_targets(ifgf_plan *out, int64_t n, const double *points, const double *normals,
                                     const double *weights, int64_t nt, const double *targets, double k,
                                     double eta, const ifgf_options *opt, void *stream);

/*
 * Forward apply: u = A sigma with A_ij = w_j K(x_i, x_j) for i != j, A_ii = 0
 * (eq. field1), approximated by Algorithm 1.
 *
 *   sigma  [device] n x nrhs complex (dtype IFGF_C64 or IFGF_C128), caller order
 *   u      [device] n x nrhs complex of the same dtype, overwritten; must not alias sigma
 *   nrhs   1 <= nrhs <= opt.max_rhs
 *
 * Errors: EINVAL, EBUSY (an apply on this plan is still being enqueued by
 * another thread), EHIP.  Applies enqueued on different streams with the
 * same plan share the plan's workspace and must be ordered by the caller.
 */
ifgf_status ifgf_apply(ifgf_plan p, const void *sigma, void *u, int32_t nrhs,
                       int32_t dtype, void *stream);

/*
 * Transposed apply through the same tree: the exact transpose of every
 * linear stage of ifgf_apply, in reverse order (near field transposed,
 * cousin anterpolation, downward pass, leaf transposed, times w at the
 * output point).  With conjugate = 0 it computes out = A~^T v; with
 * conjugate = 1 it computes out = A~^H v = conj(A~^T conj(v)), the adjoint
 * used for gradients of real losses.  Here A~ is the operator that
 * ifgf_apply implements, so <A~ s, v> = <s, A~^T v> holds to rounding.
 *
 *   v, out  [device] n x nrhs complex of dtype `dtype`, caller order; no aliasing
 * Errors as for ifgf_apply.
 */
ifgf_status ifgf_apply_adjoint(ifgf_plan p, const void *v, void *out, int32_t nrhs,
                               int32_t dtype, int32_t conjugate, void *stream);

/* Plan statistics.  st: [host]. */
ifgf_status ifgf_plan_get_stats(ifgf_plan p, ifgf_plan_stats *st);

/*
 * Test hooks (device pointers, sizes from ifgf_plan_get_stats; each call
 * synchronizes the stream before returning).
 *
 * ifgf_plan_export_order: perm[i] = caller index of the i-th point in
 *   Morton order; keys[i] = its finest-level Morton key (x bit b -> bit 3b,
 *   y -> 3b+1, z -> 3b+2).  perm: n int32, keys: n uint32.
 * ifgf_plan_export_boxes: level d boxes: start (boxes+1 int32 point ranges
 *   in Morton order) and coords (boxes x 3 int32 integer box indices).
 * ifgf_plan_export_lists: level d neighbour (kind 0) or cousin (kind 1)
 *   lists as CSR: off (boxes+1 int32) and idx (off[boxes] int32).  Pass
 *   idx = NULL to query the length through *len ([host]).
 * ifgf_plan_export_cones: level d relevant cones: box (cones int32) and
 *   cone id (cones int32), cone id = (i_s * n_C + i_theta) * 2 n_C + i_phi.
 * ifgf_plan_export_field: after an apply, the level-d field of the last
 *   call, as node values (what = 0, finest level d = D only, recovered
 *   from its coefficients by the inverse Chebyshev transform: equal to
 *   rounding to the values the coefficients were made from) or Chebyshev
 *   coefficients (what = 1):
 *   cones x P x nrhs complex of the plan precision (double or float pairs),
 *   P = p_s * p_ang^2, node (a, b, c) or coefficient (i, j, l) at index
 *   (a * p_ang + b) * p_ang + c.
 */
ifgf_status ifgf_plan_export_order(ifgf_plan p, int32_t *perm, uint32_t *keys);
ifgf_status ifgf_plan_export_boxes(ifgf_plan p, int32_t d, int32_t *start, int32_t *coords);
ifgf_status ifgf_plan_export_lists(ifgf_plan p, int32_t d, int32_t kind, int32_t *off,
                                   int32_t *idx, int64_t *len);
ifgf_status ifgf_plan_export_cones(ifgf_plan p, int32_t d, int32_t *box, int32_t *cone);
ifgf_status ifgf_plan_export_field(ifgf_plan p, int32_t d, int32_t what, void *dst);

/*
 * Apply with a stage mask, for stage-by-stage parity tests: bit 0 = near
 * field, bit 1 = cousin-target interpolation; level_lo..level_hi restricts
 * the cousin-target stage to those levels.  The upward pass always runs in
 * full.  Arguments otherwise as ifgf_apply.
 */
ifgf_status ifgf_apply_stages(ifgf_plan p, const void *sigma, void *u, int32_t nrhs,
                              int32_t dtype, int32_t stage_mask, int32_t level_lo,
                              int32_t level_hi, void *stream);

/*
 * Device-side consistency flags accumulated since the plan was built:
 * bit 1 = an upward-pass node fell outside the relevant cones of a child,
 * bit 2 = a cousin point fell outside the relevant cones of a box,
 * bit 3 = a far-field direction fell outside the level-3 relevant cones.
 * All mean a plan/apply mismatch and are 0 in a correct build.  flags: [host].
 * Synchronizes the device.
 */
ifgf_status ifgf_plan_check(ifgf_plan p, int32_t *flags);

/*
 * Per-kernel timing with HIP events recorded on the apply's stream.
 * Stages: IFGF_STAGE_GATHER (a = w sigma), NEAR (near field), LEAF (leaf
 * factors), COEFFS (node values -> coefficients), PROP (upward pass,
 * node formulation), PROP_CONE (upward pass, cone-major formulation),
 * TARGETS (cousin interpolation + scatter), plus the transposed stages of
 * ifgf_apply_adjoint (ADJ_*).
 *
 * ifgf_plan_set_profiling: max_launches > 0 enables timing of up to that
 *   many kernel launches (events are created here, on the host), 0 disables.
 * ifgf_plan_read_profile: synchronizes the recorded events, writes the
 *   summed milliseconds and the launch count per stage into ms[] and
 *   launches[] (IFGF_NSTAGES entries each, [host]) and resets the record.
 *   Launches beyond max_launches are not timed and not counted.
 */
enum {
    IFGF_STAGE_GATHER = 0, IFGF_STAGE_NEAR = 1, IFGF_STAGE_LEAF = 2, IFGF_STAGE_COEFFS = 3,
    IFGF_STAGE_PROP = 4, IFGF_STAGE_TARGETS = 5, IFGF_STAGE_ADJ_TARGETS = 6, IFGF_STAGE_ADJ_PROP = 7,
    IFGF_STAGE_ADJ_COEFFS = 8, IFGF_STAGE_ADJ_LEAF = 9, IFGF_STAGE_ADJ_NEAR = 10, IFGF_STAGE_ADJ_OUT = 11,
    IFGF_STAGE_PROP_CONE = 12, IFGF_NSTAGES = 13
};
ifgf_status ifgf_plan_set_profiling(ifgf_plan p, int32_t max_launches);
ifgf_status ifgf_plan_read_profile(ifgf_plan p, double *ms, int64_t *launches);

/* Release the plan and its device memory (after its work has completed).
 * NULL is ignored. */
void ifgf_plan_destroy(ifgf_plan p);

/*
 * Autotuner of the plan's one-right-hand-side formulations, by measurement
 * on the plan's own data and this device.  For every level of the upward
 * pass (prop_kernel AUTO only) it times the node formulation, the
 * cone-major MFMA tiles of 8, 16 and 32 boxes per tile (those the order,
 * the precision - FP64 tiles hold at most 16 boxes - and the node-record
 * memory rule allow) and the pair list (where the level's pairs stay within
 * 2^28; built if the plan has none), `reps` passes each with HIP events, and
 * keeps the fastest (a pair list stays where the node formulation wins, for
 * the transposed apply); then (target_kernel AUTO, orders with row-broadcast targets) it
 * times `reps` whole applies with row-broadcast, per-wave and (where the plan
 * holds them) pair-list cousin targets and keeps the fastest; the pair lists
 * are released when they lose.  The choices persist in the plan and every
 * later apply uses them; results change only by rounding.  A plan with a
 * ragged batch built over it cannot be tuned (EBUSY: the batch's queue
 * points into the buffers the tuner rebuilds); tune before creating
 * batches.  report [host, may be NULL] receives the measurements.  Runs
 * 1 + about (5 x levels + 2) x (reps + 1) passes or applies, synchronizes
 * `stream`.  Errors: EINVAL (reps < 1), EBUSY, ENOMEM, EHIP.
 */
typedef struct {
    int32_t nlevels;                        /* upward-pass levels tuned (entries below)       */
    int32_t parent_level[IFGF_MAX_LEVELS];  /* level d - 1 of the pass d -> d - 1             */
    int32_t choice[IFGF_MAX_LEVELS];        /* 0: node formulation; 8, 16, 32: boxes per tile;
                                               1: pair list                                   */
    double ms[IFGF_MAX_LEVELS][5];          /* ms per pass: node, 8-, 16-, 32-box tiles, pair
                                               list; -1 if not a candidate                    */
    int32_t target_choice;                  /* IFGF_TARGET_ROWS, _WAVE or _PAIRS; 0 if not tuned */
    double target_ms[3];                    /* ms per apply with row, wave, pair-list targets;
                                               -1 if not a candidate                          */
} ifgf_tune_report;
ifgf_status ifgf_plan_autotune(ifgf_plan p, int32_t reps, ifgf_tune_report *report, void *stream);

/*
 * Far-field pattern (Sec. 5, eq. FarField) of the combined-field potential
 * (eq. CombinedLayer, coupling eta) with density sigma:
 *
 *   u_inf(xh) = 1/(4 pi) sum_j w_j sigma_j exp(-i k xh.x_j) (-i k <xh, nu_j> - i eta),
 *
 * through the plan's tree: the leaf factors and the upward pass run as in
 * ifgf_apply, and since for x = R xh, R -> infinity, s = h / |x - y_B| -> 0
 * and |x - y_B| = R - xh.y_B + O(1/R), the field of level-3 box B tends to
 * exp(ikR)/(4 pi R) exp(-ik xh.y_B) F_B(0, xh):
 *
 *   u_inf(xh) = 1/(4 pi) sum_B exp(-ik xh.y_B) F_B(0, theta(xh), phi(xh)),
 *
 * with F_B's interpolant taken at s = 0 (FP64 phase and box sum).  The plan
 * must have been created with far_field = 1 (EINVAL otherwise), except for
 * D <= 2, where the sum over the points is evaluated directly (exact).
 * sigma [device] n x 1 complex of `dtype`, caller's order; dirs [device]
 * ndir x 3 float64 unit vectors (used as given); uinf [device] ndir complex
 * of `dtype`.  Allocates a workspace of n complex128 values for the call and
 * synchronizes `stream` before returning.  Errors: EINVAL, EBUSY, ENOMEM,
 * EUNSUPPORTED, EHIP.
 */
ifgf_status ifgf_far_field(ifgf_plan p, const void *sigma, int64_t ndir, const double *dirs, void *uinf,
                           int32_t dtype, void *stream);

/*
 * GMRES solution of the combined-field integral equation (Sec. 2.2, eq.
 * CombLayIE, solved in Sec. 5 with complex GMRES):
 *
 *     (alpha I + A) sigma = f,
 *
 * where A is the plan's operator (the sum of ifgf_apply, without singular
 * corrections), alpha = 1/2 and f = -u^i for eq. CombLayIE.  Restarted
 * GMRES(restart) with classical Gram-Schmidt applied twice.  The Krylov
 * vectors, inner products, norms and updates are complex FP64 whatever the
 * plan's precision (the applies take and return complex128); inner products
 * are reduced in a fixed order, so a solve is deterministic.
 *
 * ifgf_gmres_solve: f [device] n complex128 right-hand side, sigma [device]
 *   n complex128 solution, caller's point order; with use_guess = 1 sigma
 *   holds the initial iterate on entry, else it starts from zero.  f and
 *   sigma must not alias.  iters [host]: operator applies of the Krylov
 *   iterations; rel_res [host]: ||f - (alpha I + A) sigma|| / ||f|| of the
 *   returned sigma (recomputed from sigma, not the recurrence); history
 *   [host, may be NULL]: max_iter + 1 doubles, the relative residual before
 *   the first iteration and the recurrence estimate after each.  Iterates
 *   until the residual is at most tol or max_iter iterations have run.  The
 *   library allocates (restart + 2) n complex128 values of workspace for
 *   the call.  Enqueues on `stream` and synchronizes it many times (the
 *   Hessenberg problem is solved on the host); returns when sigma is
 *   written.  Errors: EINVAL, EBUSY, ENOMEM, EHIP.
 */
typedef struct {
    int32_t restart;        /* Krylov dimension per cycle; default 30                    */
    int32_t max_iter;       /* maximum iterations (operator applies); default 300         */
    double tol;             /* relative residual target; default 1e-4 (Sec. 5.1)          */
    double alpha_re;        /* identity coefficient alpha; default 1/2 (eq. CombLayIE)    */
    double alpha_im;
    int32_t use_guess;      /* 1: start from sigma's content; default 0 (zero)            */
} ifgf_gmres_options;
void ifgf_gmres_options_default(ifgf_gmres_options *o);
ifgf_status ifgf_gmres_solve(ifgf_plan p, const void *f, void *sigma, const ifgf_gmres_options *opt,
                             int32_t *iters, double *rel_res, double *history, void *stream);

/*
 * Ragged batch: the forward apply (as ifgf_apply, one right-hand side) of
 * several plans - different geometries, sizes, depths and wavenumbers - in
 * ONE kernel launch (one work-group per queue item, not a persistent
 * kernel).  Algorithm 1 of every geometry is cut into
 * work items (gather chunks, near-field boxes, leaf boxes, coefficient
 * chunks, upward-pass items of each level, target chunks) held in one
 * queue in data-flow order; work-groups take items from the queue and wait
 * on per-geometry completion counters before items whose inputs other
 * work-groups produce (the leaf coefficients before the upward pass, level
 * d before level d-1, every level and the near field before the targets).
 * Small geometries thereby share the device with large ones instead of
 * leaving it idle between launches.  The result of each geometry is the
 * same as ifgf_apply on its plan with nrhs = 1.
 *
 * ifgf_batch_create: plans [host] array of nplans handles, 1 <= nplans <=
 *   IFGF_BATCH_MAX, pairwise distinct, all with the same precision, p_s and
 *   p_ang (the kernel and everything else may differ).  The batch does not
 *   own the plans: they must outlive it.  It holds a small device queue
 *   description.  Synchronizes the device.  Errors: EINVAL, EUNSUPPORTED,
 *   ENOMEM, EHIP.
 * ifgf_batch_apply: sigma, u [host] arrays of nplans [device] pointers, each
 *   an n_g x 1 complex array of dtype `dtype` in the caller's order of plan
 *   g; u[g] is overwritten and must not alias any sigma.  The applies use
 *   the plans' own workspaces: no apply on any of these plans may run
 *   concurrently (EBUSY while one is being enqueued).  Errors: EINVAL,
 *   EBUSY, EHIP.
 * ifgf_batch_check: [host] *flags = bit 0 set if, in some batch apply since
 *   the batch was created, a work item's wait for its inputs exceeded the
 *   poll limit and the item went ahead without them (results then invalid),
 *   OR the consistency flags of the plans (ifgf_plan_check).  Synchronizes
 *   the device.
 * ifgf_batch_set_spin_limit: polls of a completion counter before a wait is
 *   abandoned (default 4194304, each about 0.3 us apart; 0 = never wait).
 *   A test hook for the bounded wait.
 * ifgf_batch_get_info: [host] outputs, each may be NULL: queue items,
 *   queue segments, work-groups of the launch, threads per
 *   work-group.
 * ifgf_batch_destroy: releases the batch (not the plans).  NULL is ignored.
 */
#define IFGF_BATCH_MAX 64
ifgf_status ifgf_batch_create(ifgf_batch *out, int32_t nplans, const ifgf_plan *plans);
ifgf_status ifgf_batch_apply(ifgf_batch b, const void *const *sigma, void *const *u, int32_t dtype,
                             void *stream);

/*
 * ifgf_batch_apply_noalloc: ifgf_batch_apply for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results, ownership and errors as
 * ifgf_batch_apply; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine, on the device or through torch).  The launch's
 * completion counters (queue head and 32 per geometry) come from one fixed
 * device array of IFGF_BATCH_NOALLOC_COUNTERS ints (8,196 bytes) per GPU,
 * held by the library until the process ends, instead of the batch's own
 * buffer; a fill kernel clears them at the start of every call.  The batch
 * must have been created with the current device current (EINVAL otherwise).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or on
 * different batches) race on the counters and must be serialized by the
 * caller.  The first call on a device looks the array's address up once.
 * Errors: EINVAL (also a batch needing more counters than the array holds),
 * EBUSY, EHIP.
 */
#define IFGF_BATCH_NOALLOC_COUNTERS (1 + 32 * IFGF_BATCH_MAX)
ifgf_status ifgf_batch_apply_noalloc(ifgf_batch b, const void *const *sigma, void *const *u, int32_t dtype,
                                     void *stream);
ifgf_status ifgf_batch_check(ifgf_batch b, int32_t *flags);
ifgf_status ifgf_batch_set_spin_limit(ifgf_batch b, int32_t limit);
ifgf_status ifgf_batch_get_info(ifgf_batch b, int64_t *items, int32_t *segments, int32_t *grid,
                                int32_t *block);
void ifgf_batch_destroy(ifgf_batch b);

/* Static text for a status code. */
const char *ifgf_status_string(ifgf_status st);

/* Message describing the last failure on the calling thread ("" if none). */
const char *ifgf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IFGF_H */
