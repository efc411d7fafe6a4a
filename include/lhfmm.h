/*
 * lhfmm.h -- C ABI of the MI355X Lamb-Helmholtz vortex FMM library (liblhfmm.so).
 *
 * One call evaluates, for N vortex elements (x_i, omega_i), the Biot-Savart
 * velocity v_j = sum_{i != j} K(r;a)/r^3 omega_i x r  (r = x_j - x_i, eq. 1 with
 * the smoothing kernel of eq. 2 and the Gaussian core of eq. vem1) and the
 * stretching term s_j = (omega_j . grad) v at x_j (eq. s1.1), by a fast
 * multipole method that carries the far field in the two scalar potentials
 * (phi, chi) of the Lamb-Helmholtz decomposition v = grad phi + curl(r chi)
 * (eq. 4), translated by rotation / coaxial shift / back-rotation with the
 * conversion operators of eq. rcr1 (Sec. 4.4).  The near field (elements in
 * adjacent leaf boxes) is summed directly with the Gaussian core; the far
 * field uses the singular kernel, as eq. 2 allows.  No 1/(4 pi) factor is
 * applied (eq. 7 absorbs it into omega).
 *
 * Conventions shared by every entry point
 *  - x, omega, v, s are DEVICE pointers to [N][3] row-major arrays of double
 *    (LHF_FP64) or float (LHF_FP32); outputs are written in input order.
 *  - Truncation number p keeps orders n = 0..p-1 (p^2 terms per potential,
 *    Sec. 5.1).  FP64: 1 <= p <= 24.  FP32: 1 <= p <= 16.
 *  - Octree: the cube [lo, lo+L]^3; element i has integer coordinates
 *    q = min(floor((x-lo) * 2^21/L), 2^21-1) computed in FP64 (FP32 inputs
 *    are promoted first); a level-l box is q >> (21-l).  Uniform depth d:
 *    leaves are the non-empty level-d boxes; M2L runs on levels 2..d.
 *    Adaptive (max_per_leaf > 0): a box belongs to the tree iff it is the root
 *    or its parent holds more than max_per_leaf elements, and is a leaf iff it
 *    holds at most max_per_leaf elements or is on level d.  Lists after
 *    Carrier, Greengard & Rokhlin: M2L over V-lists as in the uniform tree;
 *    the near field of a leaf covers its adjacent leaves of any size (U,
 *    smoothed kernel) and its W and X interactions, which are summed directly
 *    with the singular kernel (the far-field kernel; eq. 2).
 *  - Streams: all device work is enqueued on the caller's HIP stream.
 *    lhf_plan_create synchronises that stream once (to read the tree sizes);
 *    lhf_execute never synchronises and allocates nothing.
 *  - Errors: a negative status means nothing was written; lhf_last_error()
 *    returns a thread-local message.  Argument checks run on the host before
 *    any launch.  A positive status is a warning with valid outputs.
 *  - Ownership: the caller owns x, omega, v, s, grad_v.  The plan owns its own device
 *    buffers (sorted elements, tree, expansions, operator tables) and copies
 *    what it needs from x, so x may be freed after lhf_plan_create.
 */
#ifndef LHFMM_H
#define LHFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lhf_plan lhf_plan;   /* opaque, owned by the library */
typedef struct lhf_batch lhf_batch; /* opaque, owned by the library */
typedef struct lhf_filament lhf_filament; /* opaque, owned by the library */

typedef enum {
    LHF_OK = 0,
    LHF_WARN_CORE_SPLIT = 1,  /* 1 - K(r_far_min; a) > tol: the far field's singular kernel
                                 differs from the smoothed one by more than tol */
    LHF_WARN_TOL_UNMET = 2,   /* p = 0 was requested and no order this library offers reaches tol
                                 by the calibration table (the largest order is used) */
    LHF_ERR_ARG = -1,         /* invalid argument (N, p, a, depth, pointers, precision) */
    LHF_ERR_DOMAIN = -2,      /* an element lies outside [lo, lo+L]^3 */
    LHF_ERR_NONFINITE = -3,   /* non-finite coordinate */
    LHF_ERR_WORKSPACE = -4,   /* the problem does not fit a fixed-size device buffer */
    LHF_ERR_HIP = -5,         /* a HIP runtime call failed */
    LHF_ERR_UNSUPPORTED = -6, /* valid but not supported by this library version */
    LHF_ERR_STATE = -7        /* plan used inconsistently */
} lhf_status;

typedef enum { LHF_FP64 = 0, LHF_FP32 = 1 } lhf_precision;

/* flags */
#define LHF_SINGULAR 0x1u      /* ignore a: singular kernel everywhere (a = 0 means the same) */
#define LHF_DETERMINISTIC 0x2u /* every kernel accumulates in a fixed order: two executes of one plan
                                  on the same input give bitwise-identical outputs (may select a
                                  slower M2L kernel) */
#define LHF_OUT_GRAD 0x4u      /* the plan keeps room for the velocity gradient: lhf_execute may then
                                  be given a grad_v output */
#define LHF_WX_EXPANSIONS 0x8u /* adaptive tree: the W-list boxes of a leaf (levels >= 2) act on its
                                  elements through their multipole expansions (M2P), and the
                                  elements of its X-list leaves, and of its ancestors' X-lists,
                                  enter its local expansion (P2L) before L2P, instead of the
                                  singular direct sums over those pairs (Carrier, Greengard and
                                  Rokhlin's W/X treatment with the (phi, chi) operators of App. A,
                                  eqs. dt3 and drt5-drt7).  Adds the truncation error of order p to
                                  those pairs; pays off where W boxes hold many more elements than
                                  the leaves they act on.  No effect on a uniform tree. */

/* translation scheme (lhf_desc.translation) */
#define LHF_TRANS_RCR 0        /* rotation - coaxial shift - back-rotation with the conversion
                                  operators of eq. rcr1 (Sec. 4.4); the only scheme built */
#define LHF_TRANS_DIRECT 1     /* full O(p^4) translation matrices of eq. mr3 (a debugging scheme):
                                  not built, rejected with LHF_ERR_UNSUPPORTED */

/* M2L kernel (lhf_desc.m2l_kernel).  AUTO picks the fastest kernel measured for (precision, p);
 * the others force one and return LHF_ERR_UNSUPPORTED where it has no instantiation. */
#define LHF_M2L_AUTO 0
#define LHF_M2L_HALF 1         /* batched VALU, each coefficient vector split over two lanes by the
                                  parity of m: p = 8, 10, 12, 16 (FP64 also 20, 22, 23, 24) */
#define LHF_M2L_TILE 2         /* batched VALU, one lane per coefficient vector (two schedule rows
                                  per batch at FP32 p = 8, 10): p = 4..12 even (FP32 also 16) */
#define LHF_M2L_TILE1 3        /* as TILE with one schedule row per batch */
#define LHF_M2L_MFMA 4         /* batched matrix-core (16x16x4 MFMA) kernel: p = 4..12 even (FP32
                                  also 16) */
#define LHF_M2L_GENERIC 5      /* one wavefront per target box over its stored V-list: any p */
#define LHF_M2L_QUARTER 6      /* batched VALU, each coefficient vector split over four lanes by m mod 4
                                  (two wavefronts per SIMD at high orders): FP64 p = 8, 10, 12, 16, 20,
                                  22, 23, 24 */
#define LHF_M2L_QMFMA 7        /* batched matrix-core (16x16x4 FP64 MFMA) kernel with the coefficient vectors
                                  in registers in the instruction's operand layout (residue m mod 4 per
                                  lane, both parts, eight translations per wavefront): FP64 p = 20, 22,
                                  23, 24 */

/* M2M / L2L kernel (lhf_desc.mm_kernel) */
#define LHF_MM_AUTO 0
#define LHF_MM_HALF 1          /* batched, eight child shifts per wavefront: p = 8, 10, 12, 16 */
#define LHF_MM_GENERIC 2       /* one wavefront per parent (M2M) or child (L2L): any p */
#define LHF_MM_QUARTER 3       /* batched, four child shifts per wavefront, each vector over four lanes
                                  by m mod 4: FP64 p = 20, 22, 23, 24 (the default there) */

typedef struct {
    int32_t p;            /* truncation number, orders n = 0..p-1 (Sec. 5.1); 0: the smallest order
                             whose calibrated error (relative L2 of v and of s against the direct
                             sum, measured per input class: uniform tree / adaptive tree) is <= tol */
    double tol;           /* target accuracy: drives p = 0 and the CORE_SPLIT warning */
    int32_t depth;        /* uniform octree depth d, or the deepest level of an adaptive tree; 2..10 */
    int32_t max_per_leaf; /* 0: uniform tree of depth d.  > 0: adaptive tree -- a box is split
                             while it holds more than max_per_leaf elements, down to level d */
    double domain_lo[3];  /* cube origin */
    double domain_len;    /* cube side, > 0 (every element must lie in the cube) */
    int32_t precision;    /* lhf_precision */
    uint32_t flags;       /* LHF_SINGULAR | LHF_DETERMINISTIC | LHF_OUT_GRAD | LHF_WX_EXPANSIONS */
    int32_t translation;  /* LHF_TRANS_RCR */
    int32_t m2l_kernel;   /* LHF_M2L_* */
    int32_t mm_kernel;    /* LHF_MM_* */
    int32_t reserved;     /* must be 0 */
} lhf_desc;

typedef struct {
    int64_t n;                 /* elements */
    int32_t depth, p;
    int64_t boxes[11];         /* non-empty boxes per level 0..depth */
    int64_t n_m2l;             /* multipole-to-local translations (V-list pairs) */
    int64_t n_m2m, n_l2l;      /* child-parent translations */
    int64_t n_p2p_pairs;       /* near-field pairs (ordered, self excluded) */
    int32_t n_theta_classes;   /* distinct polar angles of the translation directions */
    int32_t max_level;         /* deepest level holding a box */
    int64_t n_leaves;          /* leaf boxes */
    int64_t n_wx_pairs;        /* adaptive tree: element pairs of W/X interactions summed directly
                                  with the singular kernel (ordered; those not taken by M2P / P2L) */
    int32_t m2l_kernel;        /* the M2L kernel the plan runs (LHF_M2L_*, never AUTO) */
    int32_t mm_kernel;         /* the M2M/L2L kernel (LHF_MM_HALF, LHF_MM_GENERIC or LHF_MM_QUARTER) */
    int32_t deterministic;     /* 1 if every kernel of the plan accumulates in a fixed order */
    int32_t p_from_tol;        /* 1 if p was chosen from tol */
    double calib_err_v;        /* calibrated relative L2 error of v and of s at the plan's p for its */
    double calib_err_s;        /*   input class (uniform / adaptive tree), FP64 arithmetic */
    int32_t warnings;          /* bit 0: LHF_WARN_CORE_SPLIT applies, bit 1: LHF_WARN_TOL_UNMET applies
                                  (a creation status carries one of them: TOL_UNMET first) */
    int32_t wx_expansions;     /* 1 if the adaptive plan treats W/X by M2P / P2L (LHF_WX_EXPANSIONS) */
    int64_t n_m2p;             /* (W box, target element) pairs evaluated by M2P */
    int64_t n_p2l;             /* (source element, target leaf) pairs expanded by P2L */
} lhf_stats;

/* Fill *d with the defaults: p = 12, tol = 1e-6, depth = 4, cube [0,1]^3, FP64, RCR, AUTO kernels. */
void lhf_desc_default(lhf_desc *d);

/* Build a plan for the elements at x (device, [n][3], dtype by d->precision),
 * core radius a >= 0 (Gaussian core of eq. vem1; 0 = singular kernel).
 * Sorts the elements along the Morton curve, builds the octree and its
 * interaction lists, and computes the rotation / coaxial / conversion tables
 * (FP64 on the device).  Synchronises 'stream' once.  Returns LHF_OK or
 * LHF_WARN_CORE_SPLIT (plan valid) or a negative status (*out = NULL). */
lhf_status lhf_plan_create(lhf_plan **out, const lhf_desc *d, int64_t n, const void *x, double a,
                           void *stream);

/* Plan over several independent systems evaluated together at one depth
 * d->depth: system s owns elements sys_offsets[s] .. sys_offsets[s+1]-1 of x
 * (host array of n_systems + 1 non-decreasing offsets, sys_offsets[0] = 0, empty
 * systems allowed), lies in its own cube [sys_lo[3s..3s+2], + sys_len[s]]^3 and
 * has core radius sys_a[s] (host arrays; LHF_SINGULAR sets every radius to 0).
 * d->domain_lo and d->domain_len are ignored.  No element of one system sees
 * another.  The system index is prefixed to the Morton key, so one sort and one
 * launch per phase and level serve every system.  Otherwise as lhf_plan_create
 * (the CORE_SPLIT warning is returned if any system triggers it). */
lhf_status lhf_plan_create_multi(lhf_plan **out, const lhf_desc *d, int32_t n_systems,
                                 const int64_t *sys_offsets, const void *x, const double *sys_lo,
                                 const double *sys_len, const double *sys_a, void *stream);

/* One FMM evaluation with strengths omega (device, [n][3]) for the plan's
 * elements: writes v and s (device, [n][3], input order) and, if grad_v is not
 * NULL, the velocity gradient grad_v[i][3k + l] = d v_k / d x_l (device, [n][9],
 * input order; eqs. evf4-evf6 for the far field, the derivative of the
 * near-field kernel sum for the near field; s_k = sum_l omega_l grad_v[3k+l]).
 * grad_v needs a plan created with LHF_OUT_GRAD (else LHF_ERR_STATE).
 * Enqueued on 'stream'; no host synchronisation, no allocation (graph-capturable). */
lhf_status lhf_execute(lhf_plan *plan, const void *omega, void *v, void *s, void *grad_v, void *stream);

/* Same as lhf_execute, but writes only the near field (what = 2), only the far
 * field (what = 1) or both (what = 3); for stage-level testing. */
lhf_status lhf_execute_parts(lhf_plan *plan, const void *omega, void *v, void *s, void *grad_v,
                             int32_t what, void *stream);

/* Inputs and outputs of one evaluation (lhf_execute_io); device pointers, input order.
 * With monopole strengths q (divergence sources, eqs. 5-7), every element also adds
 * -grad(q_i / |y - x_i|) to the velocity: the potential phi gains the sources' monopole terms
 * (P2M: phi_n^m -= q g_n^m with the expansion of eq. rsbf5), the near field gains q_i f r with
 * the same smoothing kernel f = K/r^3 as the vortex part, and s, grad v follow. */
typedef struct {
    const void *omega; /* [N][3] vortex strengths (required) */
    const void *q;     /* [N] monopole strengths, or NULL (divergence-free field) */
    void *v;           /* [N][3] velocity (required) */
    void *s;           /* [N][3] stretching (omega . grad) v (required) */
    void *grad_v;      /* [N][9], [3k + l] = d v_k / d x_l, or NULL (needs LHF_OUT_GRAD) */
    void *beta;        /* [N] beta = grad v : grad v = sum_kl (d v_k / d x_l)^2 (Sec. 4.5; for
                          compressible flows), or NULL (needs LHF_OUT_GRAD) */
    int32_t what;      /* 3: whole field; 1: far field only; 2: near field only */
    int32_t reserved;  /* must be 0 */
} lhf_io;

/* The general evaluation: as lhf_execute_parts with the optional monopole input and the
 * beta output of lhf_io.  LHF_ERR_STATE if grad_v or beta is asked of a plan created without
 * LHF_OUT_GRAD.  Enqueued on 'stream'; no host synchronisation, no allocation. */
lhf_status lhf_execute_io(lhf_plan *plan, const lhf_io *io, void *stream);

/* Scalar harmonic FMM on the plan's tree (the paper's single-potential comparison workload,
 * Sec. 5.2): with the plan's elements as sources of strength q and as receivers,
 *   phi_j = sum_{i != j} q_i / |x_j - x_i|,   grad_phi_j = -sum_{i != j} q_i (x_j - x_i) / |x_j - x_i|^3
 * with the singular kernel (the plan's core radius is not used).  The expansions carry the single
 * potential phi: P2M of the sources, the plan's M2M / M2L / L2L on phi alone (the half-vector M2L
 * translates phi without conversion at p = 8, 10, 12, 16; the other kernels on (phi, chi = 0)),
 * L2P of phi and grad phi, near field over the adjacent leaves.  q [N], phi [N], grad_phi [N][3]
 * (may be NULL): device pointers of the plan's precision, input order.  Uniform single-system plans
 * only (else LHF_ERR_UNSUPPORTED).  Enqueued on 'stream'; no host synchronisation, no allocation. */
lhf_status lhf_execute_scalar(lhf_plan *plan, const void *q, void *phi, void *grad_phi, void *stream);

/* Vortex filaments (Sec. 5.3, App. B): ns straight segments seg[i] = (a, b) from vertex X[a] to
 * X[b] with constant circulations, evaluated at the nv vertices.  The plan's octree (d: uniform,
 * max_per_leaf = 0; p, depth, cube, precision as for particles) is built over the segment centres
 * and the vertices.  A segment's far field is the multipole of floor((p - 1)/2) + 1 Gauss-Legendre
 * points of it (eqs. vf5-vf7), its near field at a vertex in an adjacent leaf the closed form of
 * eq. dis2; both without the factor 1/(4 pi), so that a short segment is the point vortex
 * omega = G l (l = X[b] - X[a]) of the particle path.  A segment contributes nothing at its own
 * vertices (nor at points on its line).  X: device [nv][3] of the precision, seg: device int32
 * [ns][2] (copied; indices checked on the host: LHF_ERR_ARG if out of range or a == b).
 * Synchronises 'stream'.  lhf_filament_destroy releases everything. */
lhf_status lhf_filament_create(lhf_filament **out, const lhf_desc *d, int64_t nv, const void *X, int64_t ns,
                               const int32_t *seg, void *stream);
/* Velocity at the vertices for circulations G (device [ns]) into v (device [nv][3]), both of the
 * filament's precision.  Enqueued on 'stream'; no host synchronisation, no allocation. */
lhf_status lhf_filament_execute(lhf_filament *f, const void *G, void *v, void *stream);
/* The filament's plan (for lhf_plan_stats and the profiling calls; owned by the filament). */
lhf_plan *lhf_filament_plan(lhf_filament *f);
lhf_status lhf_filament_destroy(lhf_filament *f);

/* One-shot: plan_create + execute + destroy (synchronises the stream; allocates and frees the
 * plan's device buffers).  p = 0 chooses the order from tol as in lhf_plan_create. */
lhf_status lhf_evaluate(const lhf_desc *d, int64_t n, const void *x, const void *omega, double a,
                        void *v, void *s, void *stream);

/* One-shot evaluation that allocates no device memory, for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, results and errors as lhf_evaluate; every device buffer of its plan comes
 * from a fixed 256 MiB array the library holds on each device until the process ends.
 * Limits: n <= 131072, and the plan must fit the array (about 65536 FP64 elements at p = 12,
 * depth 5); otherwise LHF_ERR_WORKSPACE with nothing written.  Calls on one device share the
 * array: calls that overlap on one device (other threads, other streams) race.  Synchronises
 * 'stream'. */
lhf_status lhf_evaluate_noalloc(const lhf_desc *d, int64_t n, const void *x, const void *omega, double a,
                                void *v, void *s, void *stream);

/* Counts of the plan (boxes, translations, near-field pairs). */
lhf_status lhf_plan_stats(const lhf_plan *plan, lhf_stats *out);

/* Release the plan (synchronises the device first: executes may be queued on any stream).
 * Its device blocks stay with the library and serve the next plan that asks for the same
 * sizes (a plan rebuilt every step); LHF_NO_MEMCACHE=1 in the environment frees them at once,
 * LHF_MEMCACHE_GB bounds the idle bytes kept (default 16). */
lhf_status lhf_plan_destroy(lhf_plan *plan);

/* Return every idle device block the library keeps to the HIP runtime.  Blocks of live plans
 * and batches are not touched. */
lhf_status lhf_release_cached_memory(void);

/* Thread-local description of the last error (never NULL). */
const char *lhf_last_error(void);

/* Phase timing (HIP events recorded on the execute stream).  After
 * lhf_profile_begin(plan, k), each of the next k calls of lhf_execute records
 * events between its phases; lhf_profile_end waits for them and returns the
 * summed milliseconds per phase over those calls in phase_ms[LHF_NPHASE]:
 *   0 gather omega, 1 P2M, 2 M2M, 3 downward pass (L2L + M2L, levels 2..d),
 *   4 L2P, 5 P2P + combine + un-permute, 6 the M2L launches alone (part of 3),
 * and the number of profiled calls in *n_exec.  Recording adds no host
 * synchronisation; begin/end are called outside timed or captured regions. */
#define LHF_NPHASE 7
lhf_status lhf_profile_begin(lhf_plan *plan, int32_t max_exec);
lhf_status lhf_profile_end(lhf_plan *plan, double *phase_ms, int32_t *n_exec);

/* ---- Run-time kernel shapes of a plan (autotuner) ----
 *
 * Shapes the library can choose at run time without rebuilding the plan: the number of target
 * boxes per workgroup tile of the quarter-vector M2L kernel at every level (FP64 p = 16-24;
 * 1 .. 6 at p = 23, more at lower orders, as the LDS allows), and the number of source elements
 * staged per LDS tile by the adaptive near-field kernel (64, 128 or 256; v and s outputs only:
 * with grad_v, beta or monopoles the kernel keeps 128).  0 means the built-in choice. */
typedef struct {
    int32_t m2l_tile[9];  /* [level 0 .. 8]; 0: built-in (as many targets as fit, at least ~1024 tiles) */
    int32_t p2p_tile;     /* 0: built-in (128) */
} lhf_shapes;

/* Measure the shapes on the plan's own tree and keep the fastest in the plan: one whole
 * evaluation with omega (device [N][3], the plan's precision), then every level's M2L launched
 * once per candidate tile and the adaptive near field once per candidate source tile, timed with
 * HIP events on 'stream'.  With a non-NULL cache_path the shapes are looked up first in, and else
 * appended to, a JSON file keyed by device architecture, precision, p, tree kind, depth and N.
 * Synchronises 'stream', allocates temporary device memory (two [N][3] buffers); the plan's
 * intermediate buffers are left inconsistent, so the next lhf_execute recomputes them (outputs
 * are only ever written by lhf_execute).  out may be NULL. */
lhf_status lhf_plan_autotune(lhf_plan *plan, const void *omega, const char *cache_path, lhf_shapes *out,
                             void *stream);

/* Apply shapes (for instance those measured on an earlier plan of the same workload), or read the
 * plan's current ones.  Values outside the ranges above give LHF_ERR_ARG and change nothing. */
lhf_status lhf_plan_set_shapes(lhf_plan *plan, const lhf_shapes *shapes);
lhf_status lhf_plan_get_shapes(const lhf_plan *plan, lhf_shapes *shapes);

/* ---- Batches of independent systems with per-system depth (one HIP graph) ----
 *
 * Unit costs of the depth cost model (the paper's complexity analysis, Sec. 4.1,
 * eqs. fmm2-fmm3): far-field nanoseconds per octree box of levels 2..d (P2M, M2M,
 * M2L, L2L, L2P together) and near-field nanoseconds per ordered element pair. */
typedef struct {
    int32_t p, precision;
    double t_box_ns;
    double t_pair_ns;
} lhf_tune;

/* Built-in unit costs (host only, no device work). */
void lhf_tune_default(int32_t p, int32_t precision, lhf_tune *t);

/* Measure the unit costs on the current device: two plans over 2^17 uniform
 * points (depths 5 and 3) executed with phase timing.  With a non-NULL
 * cache_path the result is looked up first in, and else appended to, a JSON file
 * keyed by device architecture, precision and p.  Synchronises 'stream';
 * allocates temporary device memory. */
lhf_status lhf_autotune(int32_t p, int32_t precision, const char *cache_path, lhf_tune *out,
                        void *stream);

/* Depth (2..8) minimising the modelled cost of n uniform points in a cube of side
 * len among the depths whose leaf side h keeps 1 - K(h; a) <= tol (eq. vem1; any
 * depth when a = 0).  Host only.  Returns LHF_WARN_CORE_SPLIT with *depth = 2 if
 * no depth qualifies. */
lhf_status lhf_choose_depth(const lhf_tune *t, int64_t n, double len, double a, double tol,
                            int32_t *depth);

/* Batch over n_systems independent systems (arrays as in lhf_plan_create_multi).
 * Depth of system s: sys_depth[s] if sys_depth is non-NULL, else
 * lhf_choose_depth(tune or the built-in costs, ...); d->depth is ignored.  Systems
 * of equal depth share one plan; synchronises 'stream'. */
lhf_status lhf_batch_create(lhf_batch **out, const lhf_desc *d, int32_t n_systems,
                            const int64_t *sys_offsets, const void *x, const double *sys_lo,
                            const double *sys_len, const double *sys_a, const int32_t *sys_depth,
                            const lhf_tune *tune, void *stream);

/* Evaluate every system: omega, v, s are device [N][3] arrays over all systems
 * (N = sys_offsets[n_systems]).  use_graph = 1: the work of all depth groups is
 * captured once into one HIP graph (one branch per group) and replayed by later
 * calls with the same three pointers (new pointers: captured again); the graph
 * is launched on 'stream'.  use_graph = 0: direct launches on 'stream'.  No host
 * synchronisation; calls on one batch must not overlap. */
lhf_status lhf_batch_execute(lhf_batch *b, const void *omega, void *v, void *s, int32_t use_graph,
                             void *stream);

/* Number of depth groups, the depth of every system (sys_depth[n_systems]) and
 * the summed counts; any output pointer may be NULL. */
lhf_status lhf_batch_info(const lhf_batch *b, int32_t *n_groups, int32_t *sys_depth,
                          lhf_stats *total);

/* Release the batch (synchronises its streams). */
lhf_status lhf_batch_destroy(lhf_batch *b);

/* Library version string. */
const char *lhf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LHFMM_H */
