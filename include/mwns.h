/*
 * mwns.h -- C ABI of libmwns: radial-kernel integral operators applied in the modified
 * non-standard (ns) form to 3-D functions held as order-k Legendre multiwavelet coefficients
 * on adaptive dyadic trees, on one AMD Instinct MI355X (gfx950).
 *
 * Method: G. Beylkin, V. Cheruvu, F. Perez, "Fast Adaptive Algorithms in the Non-Standard Form
 * for Multidimensional Problems".  The calls follow the paper's statement of the problem:
 * compute g(x) = int K(y - x) f(y) dy for a radial kernel K given only by the exponents and
 * weights of a Gaussian sum (Sec. 3 and Sec. 5), with f and g represented on adaptive trees
 * (Sec. 2.2) at a user-supplied accuracy eps:
 *   (1) fit      mwns_fit_kernel            Gaussian sum of (-Delta+mu^2)^(-alpha)   (Sec. 3, eq. KernelApproxByGaussians)
 *   (2) operator mwns_op_create             1-D blocks F^{j;m,l} and screening plan   (eq. KernelFactor; Sec. 4)
 *   (3) project  mwns_project_gaussians     adaptive tree of a Gaussian-sum source    (Alg. 1)
 *   (4) apply    mwns_apply                 g = T f in the modified ns-form           (eq. apply_algo, Alg. 3)
 *   (5) evaluate mwns_tree_eval             g at points from its leaves               (App. A.1)
 *
 * Conventions shared by every call
 *  - Every call returns an mwns_status; MWNS_OK is 0.  No C++ exception crosses the ABI.  On a
 *    non-OK status, outputs are left untouched and no handle is created; mwns_last_error()
 *    returns a thread-local message describing the last failure on the calling thread.
 *  - The caller owns every host array passed in or out.  The library owns every handle and every
 *    device buffer; device memory comes from the context's allocator.
 *  - All device work of a context is ordered on the context's stream.  Calls that return host
 *    data synchronise that stream before returning.  A context is not thread-safe: use one
 *    context per host thread.
 *  - Orders and sizes: 1 <= k <= 10 (basis order = number of Legendre polynomials per dimension;
 *    k <= 8 runs on the one-tile contraction kernel with every precision class and tile variant,
 *    9 <= k <= 10 on the whole-brick kernel with the FP64 and FP32 classes, whose FP32 class runs
 *    the 4-row tails of the 2k = 16 + 4 split in FP64: there a routed apply takes MWNS_CLASS_F32
 *    alone and rejects the BF16 bits with EINVAL);
 *    tree levels 0..19.  Coefficient blocks are [a][b][c] with a the x degree, b the y degree and
 *    c the z degree (c fastest).  Keys are level << 57 | morton(lx, ly, lz) with the x bit lowest
 *    in each bit triple; a tree's canonical node order is ascending key.
 *  - The Gaussian source f = sum_i c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2) is a sum of unit-mass
 *    Gaussians; f is taken as zero outside the unit cube [0,1]^3 (free space).
 */
#ifndef MWNS_H
#define MWNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MWNS_OK = 0,
    MWNS_EINVAL = 1,   /* an argument is out of range or inconsistent */
    MWNS_ENOMEM = 2,   /* the allocator failed or the context's byte budget would be exceeded */
    MWNS_EDEVICE = 3,  /* a HIP runtime call or kernel launch failed */
    MWNS_ERANGE = 4,   /* a result does not fit: a caller capacity, the term cap of the fit, ... */
    MWNS_ESTATE = 5    /* a handle is used in a state that does not allow the call */
} mwns_status;

typedef struct mwns_ctx mwns_ctx;
typedef struct mwns_op mwns_op;
typedef struct mwns_tree mwns_tree;

/* Device allocator callbacks: alloc returns a device pointer of at least `bytes` bytes usable on
 * the context's device and stream (or NULL on failure); free releases it. */
typedef void* (*mwns_alloc_fn)(size_t bytes, void* user);
typedef void (*mwns_free_fn)(void* ptr, void* user);

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.
 *   stream       hipStream_t to order all work on; NULL means the device's null stream.
 *   alloc/free   device allocator; both NULL means hipMalloc/hipFree.  Both or neither.
 *   user         passed back to alloc/free unchanged.
 *   byte_budget  upper bound on device bytes the context may hold at once; 0 = unlimited.
 * The context also keeps one pinned host block (hipHostMalloc, at least 1 MiB, grown to the
 * largest host round trip of a projection or apply) for its host<->device copies; it is not part
 * of byte_budget and is freed with the context.
 * Errors: EINVAL (bad device, one of alloc/free missing), EDEVICE (HIP runtime failure). */
mwns_status mwns_ctx_create(int device, void* stream, mwns_alloc_fn alloc, mwns_free_fn free_fn, void* user,
                            size_t byte_budget, mwns_ctx** out);
/* Releases the context handle.  Trees, operators and plans made with it may outlive the call: the
 * context's memory and cached device blocks are released when the last of them is destroyed. */
void mwns_ctx_destroy(mwns_ctx* ctx);
/* Block until all work on the context's stream has completed.  Errors: EDEVICE. */
mwns_status mwns_ctx_synchronize(mwns_ctx* ctx);
/* Device bytes in live blocks of the context (handles included). */
size_t mwns_ctx_bytes_in_use(const mwns_ctx* ctx);
/* Freed device blocks are kept by the context and reused by later calls on its stream (sizes in
 * classes of a quarter octave); these count against byte_budget and are released when an
 * allocation would exceed it, by mwns_ctx_release_cache (which synchronises) and by
 * mwns_ctx_destroy.  bytes_cached reports their total. */
size_t mwns_ctx_bytes_cached(const mwns_ctx* ctx);
mwns_status mwns_ctx_release_cache(mwns_ctx* ctx);
/* Thread-local text for the last non-OK status returned on this thread ("" if none). */
const char* mwns_last_error(void);
/* Version of this interface: the entry points, their structs, and the layouts of the arrays they
 * export and import (plans of mwns_op_plan_export / mwns_op2d_plan_export, trees of
 * mwns_tree_export and its 1-D and 2-D forms).  A caller that stores such arrays stores the version
 * beside them and compares it before importing; the library returns MWNS_ABI_VERSION. */
#define MWNS_ABI_VERSION 3
int mwns_abi_version(void);

/* Tile variant of the FP64 contraction kernel used by this context for basis order k: an index in
 * [0, mwns_num_variants_for(k)), or -1 for the library's default.  For k <= 8 (the one-tile kernel,
 * mwns_num_variants() shapes, mwns_variant_shape) the default is the shape with two terms per pass
 * and a prefetched input slice for 6 <= k <= 8, variant 0 below; for k = 9, 10 (one workgroup of four
 * waves per sibling group, or two such groups on alternate terms) variant 0 is one group per
 * workgroup loading the next input slice while computing the current one, variant 1 two groups per
 * workgroup (their sums are added at the end, so it agrees with variant 0 up to rounding), variant 2
 * as 0 loading each slice when it is needed (bit for bit as 0), and variant 3, the default, as 2 with
 * one buffer for the exchanged slices instead of two, so that three workgroups share a compute unit
 * (three waves per SIMD; bit for bit as 0).  Variants
 * differ in speed only: those with one term per pass compute the same result bit for bit; those
 * with several terms per pass add the plane results of consecutive terms in another order, so they
 * agree with the others up to rounding.  mwns_tune_apply picks one by timing.
 * Errors: EINVAL (k or variant out of range). */
int mwns_num_variants(void);
int mwns_num_variants_for(int k);
/* Shape of variant v: waves per workgroup, register prefetch depth of the input slices, waves
 * per SIMD, and FP64 terms per pass over a job's cells.  Errors: EINVAL (v out of range, NULL). */
mwns_status mwns_variant_shape(int v, int* waves, int* prefetch, int* waves_per_simd, int* terms_per_pass);
mwns_status mwns_ctx_set_variant(mwns_ctx* ctx, int k, int variant);
/* The variant in use for order k (the library's default when none was set). */
mwns_status mwns_ctx_get_variant(const mwns_ctx* ctx, int k, int* variant);

/* -------------------------------------------------------------- (1) fit */

/* Exponents tau_m and weights w_m of sum_m w_m exp(-tau_m r^2) approximating `scale` times the
 * kernel of (-Delta + mu^2)^(-alpha),
 *   K_{mu,alpha}(r) = C_alpha int exp(-r^2 e^{2s} - mu^2 e^{-2s}/4 + (3 - 2 alpha) s) ds,
 * by the trapezoidal rule s_m = A + m h, m = 1..M (Sec. 3, eqs. IntegralRepr and
 * KernelApproxByGaussians), such that
 *   |K_{mu,alpha}(r) - sum w_m e^{-tau_m r^2}| <= eps K_{0,alpha}(r)   for delta <= r <= R,
 * verified on 64 points per decade (the fit targets eps/2 there).  Host FP64, no device work.
 *   mu >= 0, 0 < alpha < 3/2, 0 < eps < 1, 0 < delta < R, scale > 0.
 *   cap       capacity of tau[] and w[] (caller-owned host arrays).
 *   *M        on MWNS_OK the number of terms written; on MWNS_ERANGE the number needed.
 * Errors: EINVAL (parameters), ERANGE (M > cap; tau and w untouched). */
mwns_status mwns_fit_kernel(double mu, double alpha, double scale, double eps, double delta, double R, int cap,
                            int* M, double* tau, double* w);

/* --------------------------------------------------------- (2) operator */

typedef struct {
    /* 1 (default): every coarse displacement L gets the union of the term ranges of its set
     * Core / Boundary-1 / Boundary-2 / Boundary-3 (Sec. 4); 0: per-L ranges. */
    int group_regions;
    /* 0 (default): mwns_op_create fails with MWNS_ERANGE when the screening keeps a term at the
     * edge of the band (a coarse displacement with max |L_d| = 3, the widest the plan covers),
     * since displacements beyond the band would then still matter (the paper's remark that a
     * narrow band suffices in practice, Sec. 4); 1: build the operator anyway. */
    int allow_band_overflow;
} mwns_op_opts;

/* Build the operator for basis order k on levels 0..max_level from M Gaussian terms (host arrays
 * tau[M], w[M], copied):
 *   - the 1-D blocks F^{j;m,l}_ab = 2^-j int_{-1}^{1} exp(-tau_m (x+l)^2/4^j) Phi_ab(x) dx for
 *     j = 0..max_level, every m and l = -7..7 (eq. KernelFactor; Phi = cross-correlation of the
 *     scaling functions, App. A.4), on the device;
 *   - the screening plan: for every scale j >= 1 and coarse displacement L in [-3,3]^3, the
 *     inclusive term range R_j(L) kept after discarding terms whose cumulative estimated
 *     contribution is below eps (Sec. 4, eqs. BlockNorms and NormEstimateUsing1DBlocks).
 * opts may be NULL (defaults).  Errors: EINVAL, ENOMEM, EDEVICE, ERANGE (band overflow, see
 * mwns_op_opts; the message names the level and displacement). */
mwns_status mwns_op_create(mwns_ctx* ctx, int k, int M, const double* tau, const double* w, double eps,
                           int max_level, const mwns_op_opts* opts, mwns_op** out);
/* Plan as int32 [max_level+1][7][7][7][2] (j, L1+3, L2+3, L3+3, {m1, m2}); an empty range has
 * m2 < m1; row j = 0 holds the root (all terms at L = 0).  Two-call size query: with plan == NULL
 * only *count (number of int32) is set.  Errors: ERANGE (*count too small; *count set). */
mwns_status mwns_op_plan_export(const mwns_op* op, int32_t* plan, size_t* count);
/* Replace the plan with a caller-supplied one of the same layout (e.g. a stored band
 * structure, Sec. 4).  Errors: EINVAL (count or a range outside [0, M)). */
mwns_status mwns_op_plan_import(mwns_op* op, const int32_t* plan, size_t count);
/* F tables as double [max_level+1][M][15][k][k] (row = output degree).  Two-call size query as
 * above.  Synchronises.  Errors: ERANGE, EDEVICE. */
mwns_status mwns_op_tables_export(mwns_ctx* ctx, const mwns_op* op, double* F, size_t* count);
/* theta = eps * sum_m w_m ||F^{0;m,0}||_F^3 used by the screening (Sec. 4). */
double mwns_op_threshold(const mwns_op* op);
void mwns_op_destroy(mwns_op* op);

/* --------------------------------------------------------- (3) trees */

/* Adaptive projection (Alg. 1) of f = sum_i c_i (a_i/pi)^{3/2} exp(-a_i |x - x_i|^2), n terms,
 * host arrays xyz[n][3], a[n] > 0, c[n]: starting from every box of level j0, a box below jmax is
 * refined when, for any of its 8 children, the values interpolated from the box's coefficients
 * differ from f at the child's k^3 Gauss-Legendre nodes by more than eps * ||f||_2 (max norm);
 * leaves keep their own Gauss-Legendre coefficients (App. A.1, eq. fvals2coefs) and every
 * ancestor receives the two-scale decomposition of its children (redundant tree, Sec. 2.2.1).
 *   0 <= j0 <= jmax <= 19, eps > 0.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_project_gaussians(mwns_ctx* ctx, int k, double eps, int j0, int jmax, int n, const double* xyz,
                                   const double* a, const double* c, mwns_tree** out);
/* Tree from caller leaves: keys[nleaves] (any order, no duplicates, leaves must tile the unit cube
 * without overlap) and coeffs[nleaves][k][k][k] (host).  Ancestors are added and filled by the
 * two-scale decomposition.  Errors: EINVAL (bad keys / not a tiling), ENOMEM, EDEVICE. */
mwns_status mwns_tree_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys, const double* coeffs,
                                  mwns_tree** out);

typedef struct {
    int k;
    int depth;              /* deepest level */
    int64_t nnodes;         /* nodes of the redundant tree */
    int64_t nleaves;
    double threshold;       /* refinement threshold of the projection (0 for imported trees) */
    double min_margin;      /* min over refinement tests of |err - threshold| / threshold (projection) */
} mwns_tree_info;
mwns_status mwns_tree_get_info(const mwns_tree* t, mwns_tree_info* info);

/* Export in canonical (ascending key) order.  Two-call size query: with keys == NULL only *nnodes
 * is set.  keys[nnodes], is_leaf[nnodes] (may be NULL), coeffs[nnodes][k][k][k] (may be NULL).
 * Synchronises.  Errors: ERANGE (*nnodes too small), EDEVICE. */
mwns_status mwns_tree_export(mwns_ctx* ctx, const mwns_tree* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                             double* coeffs);
void mwns_tree_destroy(mwns_tree* t);
/* Replace the leaf coefficients of t in place (structure unchanged): coeffs[nleaves][k][k][k]
 * (host) in canonical leaf order (ascending key among the leaves, as mwns_tree_export lists
 * them); the internal nodes are recomputed by two-scale decomposition (App. A.3,
 * eq. decomp_scaling).  Errors: EINVAL, EDEVICE. */
mwns_status mwns_tree_set_leaves(mwns_ctx* ctx, mwns_tree* t, const double* coeffs);

/* ------------------------------------------------------------- (4) apply */

enum {
    MWNS_F64 = 0,             /* every contraction in FP64 (FP64 MFMA) */
    MWNS_NO_ASSEMBLY = 1 << 8, /* flag: g holds the per-scale blocks ghat before eq. g_assemble */
    MWNS_TIMES_ONLY = 1 << 9   /* flag: stats without the device passes that count contractions and
                                  sum ||g||^2 (contractions = -1, g_norm = 0); the times, flops and
                                  bounds are filled as usual */
};

typedef struct {
    int64_t contractions;     /* (node, displacement, term) triples with a non-zero coefficient */
    int64_t brick_jobs;       /* (output sibling group, region, term) contraction jobs executed */
    int64_t ghost_bricks;     /* sibling groups interpolated from coarser leaves (Alg. 3 Step 2) */
    double useful_flops;      /* FP64 flops of the executed contraction schedule, padding excluded */
    double ms_closure;        /* device time of neighbour closure and interpolation */
    double ms_contract;       /* device time of the contraction kernels */
    double ms_assemble;       /* device time of the top-down assembly */
    double err_bound;         /* a-priori bound on ||g - g_F64||_2 of the precision routing (0: all FP64) */
    double g_norm;            /* ||g||_2 over [0,1]^3 (0 with MWNS_NO_ASSEMBLY) */
    double class_flops[4];    /* useful_flops by precision class: FP64, FP32, BF16 compensated, BF16 */
    double own_flops;         /* the method's own share of useful_flops (eq. apply_algo's net coefficients):
                                 without the down-band jobs whose terms all lie in the whole band's range at
                                 every coarse displacement of their box, and, of each whole-band job at a
                                 sibling group with internal children, without the share of its (output
                                 child, L, input child, term) block pairs whose net coefficient is 0 (an
                                 internal child and a term in the finer band R_{j+1}(l)); the brick-wide
                                 whole-band job computes those because the leaf children need the same
                                 super-block products, and the down band cancels them */
    double f64_mfma_flops;    /* FP64 matrix-core flops issued by the FP64 class's contraction launches,
                                 padding of the 16 x 16 and 4 x 4 tiles included (what the hardware's
                                 FP64 MFMA operation counter reports, times 512 per operation) */
} mwns_apply_stats;

/* g = T f with T given by `op` (its F tables and plan), in the modified ns-form (eq. apply_algo;
 * Alg. 3): the output uses the redundant tree of f as its skeleton; every node b at level j
 * receives ghat_b = sum over displacements l and terms m of c_m w_m (F^{j;m,l1} (x) F^{j;m,l2}
 * (x) F^{j;m,l3}) f_{b-l} with c_m = [m in R_j(L)] - [b internal][m in R_{j+1}(l)]
 * (L = coarse displacement of the parents), missing inputs being interpolated from the deepest
 * existing ancestor (Alg. 3 Step 2), and g = ghat + up(g_parent) top-down (eq. g_assemble).
 * op->max_level must be >= depth of f.  `mode` is MWNS_F64, optionally | MWNS_NO_ASSEMBLY and
 * | MWNS_TIMES_ONLY.
 * stats may be NULL; filling it synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int mode, mwns_tree** g,
                       mwns_apply_stats* stats);

/* Precision classes of the mixed apply (bit mask of the reduced ones a call may use). */
enum {
    MWNS_CLASS_F32 = 1,       /* FP32 MFMA, FP32 inputs and accumulation (for k > 8 the 4-row tails of
                                 each mode product run in FP64) */
    MWNS_CLASS_BF16C = 2,     /* BF16 MFMA on hi/lo-split operands, all four partial products (compensated) */
    MWNS_CLASS_BF16 = 4       /* BF16 MFMA, one operand of every mode product rounded to BF16 */
};

typedef struct {
    double tol;               /* bound on ||g - g_F64||_2 the routing must keep (absolute; 0 = all FP64) */
    int classes;              /* MWNS_CLASS_* bits allowed */
} mwns_mixed_opts;

/* g = T f as mwns_apply, with every (level, displacement box, term) contraction job routed to FP64
 * or to one of the allowed reduced classes.  Not part of the paper's method: a system layer that
 * keeps the result within opts->tol of the all-FP64 apply.  A job's contribution to g over its
 * whole level, with every block taken entrywise in absolute value, is bounded by
 * beta = |w_m| ||X_level||_2 min(prod_d sum_{L_d in box} ||S_d^{m,L_d}||_F,
 * prod_d || sum_{L_d in box} |S_d^{m,L_d}| ||_2) (S_d the masked 2k x 2k super-blocks, X_level
 * every input sibling group of the level), and a class with unit rounding factor gamma computes
 * it within gamma * beta; classes are chosen so
 * that the sum of gamma * beta is at most tol (stats->err_bound), minimising modelled time.  Jobs
 * whose box holds the zero displacement keep their narrow terms in FP64 whatever the budget: the
 * terms with tau_m >= 4 k^2 4^j at level j (width 1/sqrt(tau_m) at most 1/(2k) of a level-j box).
 * A reduced class that would carry less than a tenth of the apply's work is not used (its launch
 * costs more than it saves); its jobs stay FP64.  The transforms, the
 * interpolation, the assembly and the output accumulation stay FP64.  flags: 0, MWNS_NO_ASSEMBLY,
 * MWNS_TIMES_ONLY.  Errors: EINVAL (tol < 0, unknown class or flag, a BF16 class for k > 8),
 * ENOMEM, EDEVICE. */
mwns_status mwns_apply_mixed(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, const mwns_mixed_opts* opts, int flags,
                             mwns_tree** g, mwns_apply_stats* stats);

/* Batched apply: g_i = T_i f_i for n (operator, tree) pairs, trees of any size, as one
 * persistent contraction launch per basis order present (workgroups stay resident and pull
 * output sibling groups of every tree from 8 per-XCD work queues, costliest first), with one
 * host round trip for the neighbour closure of the whole batch.  mixed: NULL for FP64, or n
 * routing options (tree i is routed with mixed[i], as mwns_apply_mixed).  gs[n] receives the
 * output handles (NULL on error).  stats (may be NULL) sums the counts over the batch; err_bound
 * is the largest per-tree bound and g_norm the root of the summed squares.  Results equal the
 * single applies bit for bit.  Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_apply_batch(mwns_ctx* ctx, int n, const mwns_op* const* ops, const mwns_tree* const* fs,
                             const mwns_mixed_opts* mixed, int flags, mwns_tree** gs, mwns_apply_stats* stats);

/* A reusable batched apply.  mwns_plan_create does everything that depends only on the trees'
 * structure and the operators -- jobs, neighbour closure, interpolation sites, routing (from
 * the inputs' norms at creation), launch orders, every buffer -- and captures the value phase
 * (interpolated inputs, reduced-precision copies, contractions, assembly) once as a hipGraph.
 * mwns_plan_execute replays it on the context's stream for the current coefficients of the input
 * trees (update them in place with mwns_tree_set_leaves); it allocates nothing and does not
 * synchronise.  The plan borrows ops and fs (keep them alive and unchanged in structure) and owns
 * its n outputs: mwns_plan_output returns a borrowed handle, valid until mwns_plan_destroy and
 * overwritten by every execute.  For routed plans the error bound holds while every level's input
 * norm stays at most its value at creation.  mwns_plan_stats synchronises.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
typedef struct mwns_plan mwns_plan;
/* Autotuner: times the FP64 contraction launch of the apply of f by op in every tile variant
 * (one warm-up and `reps` timed launches each, HIP events on the context's stream), stores the
 * fastest as the context's variant for f's k and returns it in *best; times_ms (NULL or
 * mwns_num_variants_for(k) doubles) receives the average launch time of each variant.  Synchronises.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_tune_apply(mwns_ctx* ctx, const mwns_op* op, const mwns_tree* f, int reps, int* best, double* times_ms);
mwns_status mwns_plan_create(mwns_ctx* ctx, int n, const mwns_op* const* ops, const mwns_tree* const* fs,
                             const mwns_mixed_opts* mixed, int flags, mwns_plan** out);
mwns_status mwns_plan_execute(mwns_plan* plan);
mwns_status mwns_plan_output(const mwns_plan* plan, int i, const mwns_tree** g);
mwns_status mwns_plan_stats(const mwns_plan* plan, mwns_apply_stats* stats);
void mwns_plan_destroy(mwns_plan* plan);

/* ----------------------------------------------------------- (5) evaluate */

/* Values at npts points xyz[npts][3] (host, inside [0,1]^3) from the leaves of t:
 * f(x) = 2^{3j/2} sum_abc s_abc phi_a(2^j x - l1) phi_b(2^j y - l2) phi_c(2^j z - l3) on the leaf
 * holding x (App. A.1); a point on a face belongs to the box floor(2^j x) clamped to 2^j - 1.
 * out[npts] is a host array.  Synchronises.  Errors: EINVAL (point outside the cube), ENOMEM,
 * EDEVICE. */
mwns_status mwns_tree_eval(mwns_ctx* ctx, const mwns_tree* t, int64_t npts, const double* xyz, double* out);

/* ----------------------------------------------------------- (6) details and pruning */

/* Squared l2 norm of the detail coefficients of every node (App. A.2-A.3, eq. decomp_wavelet in
 * each dimension) of the function that t's leaves represent: out[nnodes] (host, canonical order)
 * receives, for an internal node, the sum of squares of the seven detail blocks of its sibling
 * group of children (the internal nodes rebuilt from the leaves by the two-scale decomposition,
 * since an applied output holds assembled partial sums there), and 0 for a leaf.  The wavelet filters are any
 * orthonormal complement of the two-scale filters; the norms do not depend on that choice.
 * Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_tree_detail_norms(mwns_ctx* ctx, const mwns_tree* t, double* out);
/* l2 pruning (Sec. 2.2): a new tree from t with sibling groups removed, starting on the finest
 * scale, while the cumulative squared detail norm of what was removed stays <= eta^2 (eta >= 0,
 * absolute).  Candidates are internal nodes whose eight children are leaves; within a scale they
 * are taken in ascending order of their detail norm (ties by key), the first that would exceed the
 * budget ends that scale, and the rest of the budget carries to the next coarser scale.  By
 * orthonormality ||f_t - f_pruned||_2^2 equals the removed sum, returned in *removed (may be NULL).
 * Acts on the function t's leaves represent: kept leaves keep their coefficients, internal nodes
 * and new leaves hold the two-scale projections of t's leaves.  Synchronises.  Errors: EINVAL,
 * ENOMEM, EDEVICE. */
mwns_status mwns_tree_prune(mwns_ctx* ctx, const mwns_tree* t, double eta, mwns_tree** out, double* removed);
/* Alg. 3 Step 4's discard of unnecessary blocks at accuracy eps: mwns_tree_prune with
 * eta = eps ||f_t||_2 (the root block's norm and every detail norm, Parseval).  Errors: as
 * mwns_tree_prune. */
mwns_status mwns_tree_discard(mwns_ctx* ctx, const mwns_tree* t, double eps, mwns_tree** out, double* removed);

/* mwns_tree_eval for callers that cannot allocate memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation: it calls no allocator (neither hipMalloc nor the
 * context's), copies nothing between host and device and does not synchronise.  Its working memory
 * (the tree's child-brick table and a counter) is one fixed array of 16.02 MiB in device memory that
 * every GPU the library runs on holds until the process ends; its address is looked up when a context
 * is created on that GPU.
 *   xyz   DEVICE pointer, npts x 3 doubles (caller-owned, readable on the context's stream).
 *   out   DEVICE pointer, npts doubles (caller-owned); written on the context's stream.  A point outside
 *         [0,1]^3 (or NaN) and a point whose leaf is missing get NaN (no error is reported: the call does
 *         not wait for the device).
 *   The tree may have at most 4194304 nodes.
 * Every call on one GPU uses that GPU's one array, which keeps the contents of the last call: calls
 * that may overlap on one GPU (several streams or host threads) race and must be serialised by the
 * caller.  Errors: EINVAL (NULL pointers, npts < 0, tree of another context), ERANGE (more nodes than
 * the array holds), ESTATE (no array address for the device), EDEVICE (launch failure). */
mwns_status mwns_tree_eval_noalloc(mwns_ctx* ctx, const mwns_tree* t, int64_t npts, const double* xyz, double* out);

/* ---- (7) The 1-D cotangent operator (Sec. 2.4, Alg. 2; the example of Sec. 2.4.2) -----------------
 * (C f)(y) = p.v. int_0^1 cot(pi (y - x)) f(x) dx on the periodic unit interval (eq. CotangetKernel),
 * applied in the modified ns-form.  1-D keys: level << 57 | translation (translation < 2^level),
 * nodes in ascending key order; coefficient blocks are k doubles (row a = degree). */
typedef struct mwns_op1 mwns_op1;
typedef struct mwns_tree1 mwns_tree1;
/* The operator for scales 0..max_level (0 <= max_level <= 40), order k (1..16), accuracy eps > 0:
 * blocks r^{j;l}_ab = 2^-j p.v. int_{-1}^{1} cot(pi 2^-j (x + l)) Phi_ab(x) dx (eq. cot.01) for
 * l = -65..65 on every scale (the device computes them by a 64-point Gauss-Legendre rule over the
 * two polynomial pieces of the cross-correlation Phi, App. A.4), and the bands: B_j (j >= 1) is the
 * smallest B such that the Frobenius norms of the difference super-blocks S^{j;L} - [H0 H1]^T
 * r^{j-1;L} [H0 H1] (the blocks of T_j minus those of the up-sampled T_{j-1} between the children
 * of two scale-(j-1) boxes at displacement L) sum to at most eps over the coarse periodic
 * distances B < |L| <= min(32, 2^(j-2)).  The whole band of scale j holds the pairs of boxes whose
 * parents are at periodic distance <= B_j (the band b_j = 2 B_j + 1 of eq. fine_scale_band).
 * Errors: EINVAL, ENOMEM, EDEVICE, ERANGE (a band wider than 32 would be needed). */
mwns_status mwns_cot1d_op_create(mwns_ctx* ctx, int k, double eps, int max_level, mwns_op1** out);
/* bands[max_level + 2] (host): bands[j] = B_j for j = 1..max_level, bands[0] = bands[max_level+1] = 0;
 * two-call size query: bands = NULL sets *count.  Errors: EINVAL, ERANGE (*count too small). */
mwns_status mwns_cot1d_op_bands(const mwns_op1* op, int32_t* bands, int* count);
/* Replaces the bands (count = max_level + 2 entries, each 0..32; entries 0 and max_level+1 ignored):
 * any bands give an exact apply of the banded modified form.  Errors: EINVAL. */
mwns_status mwns_cot1d_op_set_bands(mwns_op1* op, const int32_t* bands, int count);
/* The blocks R[max_level + 1][131][k][k] (host, l = -65..65, row = output degree a); two-call size
 * query (R = NULL sets *count).  Synchronises.  Errors: EINVAL, ERANGE. */
mwns_status mwns_cot1d_op_blocks(mwns_ctx* ctx, const mwns_op1* op, double* R, size_t* count);
void mwns_cot1d_op_destroy(mwns_op1* op);
/* Alg. 1 in one dimension for f(x) = sum_i weights_i sum_n exp(-exps_i (x + n - centers_i)^2) (host
 * arrays of n entries; exps > 0): boxes from level j0 (0 <= j0 <= jmax <= 40) are refined while the
 * largest difference between f and the box's polynomial at both children's k Gauss-Legendre nodes
 * exceeds the absolute threshold thr (>= 0); boxes at jmax are leaves.  A leaf keeps its own
 * coefficients (eq. fvals2coefs); internal nodes hold the two-scale projections (eq.
 * decomp_scaling).  Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_cot1d_project(mwns_ctx* ctx, int k, double thr, int j0, int jmax, int n, const double* centers,
                               const double* exps, const double* weights, mwns_tree1** out);
/* A tree from leaves (host keys[nleaves], coeffs[nleaves][k]) that tile [0,1): ancestors added,
 * internal nodes by the two-scale relation.  Errors: EINVAL (keys that do not form a tree). */
mwns_status mwns_cot1d_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys, const double* coeffs,
                                   mwns_tree1** out);
/* g = C f in the modified ns-form (eq. apply_algo, Alg. 2).  The output tree is f's tree with every
 * leaf of scale j refined whose whole band holds an internal node of f of scale j, and so on for
 * the added children (a coarse leaf beside refined input then receives the finer scales' terms at
 * its children); input blocks missing from f come from
 * their nearest ancestor by zero-detail reconstruction (Step 2).  At scale j >= 1 a leaf takes the
 * pairs with parents at periodic distance <= B_j and an internal node those minus the pairs at fine
 * periodic distance <= B_{j+1}; the root takes T_0 f_0 only when it is a leaf; g is then assembled
 * top-down (eq. g_assemble): leaves hold g, internal nodes the partial sums.  *ms_contract (may be
 * NULL) receives the device time of the contraction kernel.  Synchronises.  Errors: EINVAL (orders
 * differ, tree deeper than the operator), ENOMEM, EDEVICE. */
mwns_status mwns_cot1d_apply(mwns_ctx* ctx, const mwns_op1* op, const mwns_tree1* f, mwns_tree1** g,
                             double* ms_contract);
/* Nodes of t: keys, leaf flags and coefficient blocks (host arrays of *nnodes entries, each may be
 * NULL); two-call size query with all three NULL.  Synchronises.  Errors: EINVAL, ERANGE. */
mwns_status mwns_cot1d_export(mwns_ctx* ctx, const mwns_tree1* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                              double* coeffs);
/* Values of t's leaf expansions at npts points x in [0,1] (host arrays; the leaf containing x, App.
 * A.1).  Synchronises.  Errors: EINVAL (a point outside [0,1]), ENOMEM, EDEVICE. */
mwns_status mwns_cot1d_eval(mwns_ctx* ctx, const mwns_tree1* t, int64_t npts, const double* x, double* out);
void mwns_tree1_destroy(mwns_tree1* t);

/* ---- (8) Alg. 3 in two dimensions ----------------------------------------------------------------
 * The paper writes Alg. 3 for d = 2 and notes the apply exists for d = 2; it gives no 2-D kernel.
 * The plane's kernels of (-Delta + mu^2)^(-alpha) follow from Sec. 3's representation with the
 * dimension 2: K(r) = C2 int exp(-r^2 e^{2s} - mu^2 e^{-2s}/4 + (2 - 2 alpha) s) ds, C2 = 2^{1 - 2 alpha}
 * / (pi Gamma(alpha)); alpha = 1 gives K_0(mu r) / (2 pi).  2-D keys: level << 57 | morton(x, y) with x
 * in bit 0; coefficient blocks [k][k] (a = degree in x, b = degree in y). */
typedef struct mwns_op2 mwns_op2;
typedef struct mwns_tree2 mwns_tree2;
/* Gaussian-sum fit in the plane (host FP64): the trapezoidal rule s_m = A + m h, tau_m = e^{2 s_m},
 * w_m = h C2 e^{-mu^2 e^{-2 s_m}/4 + (2 - 2 alpha) s_m}, terms whose weight underflows to zero dropped,
 * |K(r) - sum w_m e^{-tau_m r^2}| <= eps K(r) on [delta, R] (relative to K itself), checked on 64 and
 * 256 points per decade; h = pi^2 / (2 (ln(1/eps) + ln 8)), B = ln(ln(4/eps) / delta^2) / 2 + 1, A the
 * smaller of ln mu - ln(4 ln(1e30/eps)) / 2 (mu > 0) and ln(eps K(R) (2 - 2 alpha) / (C2 e)) / (2 - 2 alpha)
 * (alpha < 1); h shrinks by 0.9 and [A, B] widens by 1 until the checks pass.  Needs 0 < alpha <= 1,
 * mu >= 0 (mu > 0 when alpha = 1).  Two-call use as mwns_fit_kernel: tau = w = NULL returns *M.
 * Errors: EINVAL, ERANGE (cap too small: *M set; or no convergence). */
mwns_status mwns_fit_kernel2d(double mu, double alpha, double eps, double delta, double R, int cap, int* M, double* tau,
                              double* w);
/* The 2-D operator for scales 0..max_level (<= 19), order k (1..10): the 1-D blocks F^{j;m,l} of
 * eq. KernelFactor (the same as in 3-D; built on the device) and the 2-D plan of Sec. 4 with two
 * factors: theta = eps sum_m w_m ||F^{0;m,0}||_F^2; per |L| class the estimate
 * 1/2 sum over the orderings (p, q) of N_dif(p) N_F(q) + N_upF(p) N_dif(q) (the 2k x 2k super-block
 * norms of the 3-D plan); the range [m1, m2] after dropping the prefix and suffix whose cumulative
 * contributions stay <= theta/2 (empty when the total is <= theta); ranges grouped by the number of
 * |L_d| > 1 (Core, Boundary-1, Boundary-2).  ERANGE when a term is kept at the band's edge max |L_d| = 3
 * unless allow_band_overflow.  Errors: EINVAL, ENOMEM, EDEVICE, ERANGE. */
mwns_status mwns_op2d_create(mwns_ctx* ctx, int k, int M, const double* tau, const double* w, double eps, int max_level,
                             int allow_band_overflow, mwns_op2** out);
/* The plan as int32 [max_level + 1][7][7][2] (inclusive term ranges per scale and coarse displacement
 * L = -3..3 in each dimension; empty = (0, -1)); two-call size query.  Errors: EINVAL, ERANGE. */
mwns_status mwns_op2d_plan_export(const mwns_op2* op, int32_t* plan, size_t* count);
/* Replaces the plan (same layout; any plan gives an exact apply of its banded modified form).
 * Errors: EINVAL (size or a range outside 0..M-1). */
mwns_status mwns_op2d_plan_import(mwns_op2* op, const int32_t* plan, size_t count);
void mwns_op2d_destroy(mwns_op2* op);
/* Alg. 1 in the plane for f = sum_i c_i (a_i / pi) exp(-a_i |p - p_i|^2) (host: xy[n][2], a[n] > 0, c[n]):
 * boxes from level j0 are refined (all four children) while f and the box's polynomial differ by more
 * than eps ||f||_2 (closed-form norm) at some child's k x k Gauss-Legendre nodes; boxes at jmax
 * (<= 19) are leaves; leaves keep their own coefficients, internal nodes the two-scale projections.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_project2d(mwns_ctx* ctx, int k, double eps, int j0, int jmax, int n, const double* xy, const double* a,
                           const double* c, mwns_tree2** out);
/* A tree from leaves (host keys[nleaves], coeffs[nleaves][k][k]) that tile [0,1)^2.  Errors: EINVAL. */
mwns_status mwns_tree2d_from_leaves(mwns_ctx* ctx, int k, int64_t nleaves, const uint64_t* keys, const double* coeffs,
                                    mwns_tree2** out);
/* g = T f in the modified ns-form (eq. apply_algo, Alg. 3) on f's tree: node b of scale j >= 1 takes,
 * for each fine displacement l in [-7, 7]^2 with b - l in the square and L = floor(b/2) - floor((b-l)/2),
 * the terms of R_j(L) with + and, at internal nodes, those of R_{j+1}(l) with - (their common part
 * cancels and is skipped), each as c w_m F^{j;m,l1} X F^{j;m,l2}^T; the root takes R_0 minus R_1(0)
 * when internal; inputs missing from f's tree by zero-detail reconstruction from the nearest ancestor;
 * then the assembly from the root (eq. g_assemble): leaves hold g.  *ms_contract (may be NULL): device
 * time of the contraction kernel; *flops (may be NULL): 4 k^3 per (node, l, term).  Synchronises.
 * Errors: EINVAL (orders differ, tree deeper than the operator), ENOMEM, EDEVICE. */
mwns_status mwns_apply2d(mwns_ctx* ctx, const mwns_op2* op, const mwns_tree2* f, mwns_tree2** g, double* ms_contract,
                         double* flops);
/* Nodes of t (host arrays of *nnodes entries, each may be NULL; two-call size query).  Errors: EINVAL,
 * ERANGE. */
mwns_status mwns_tree2d_export(mwns_ctx* ctx, const mwns_tree2* t, int64_t* nnodes, uint64_t* keys, uint8_t* is_leaf,
                               double* coeffs);
/* Values at npts points (host pts[npts][2] in [0,1]^2) from the leaf containing each.  Errors: EINVAL
 * (a point outside the square), ENOMEM, EDEVICE. */
mwns_status mwns_tree2d_eval(mwns_ctx* ctx, const mwns_tree2* t, int64_t npts, const double* pts, double* out);
void mwns_tree2d_destroy(mwns_tree2* t);

/* ---- (9) The hydrogen ground state (Sec. 6.2) -----------------------------------------------------
 * phi = -2 G_mu V phi, G_mu = (-Delta + mu^2)^(-1) (kernel e^{-mu r} / (4 pi r)), V = -Z / r, with mu
 * moved to sqrt(-2 E) after each step.  The physical cube [-L, L]^3, nucleus at its centre, is the
 * unit cube scaled by s = 2 L: a tree on [0,1]^3 holds the physical function's values, physical
 * integrals are s^3 times unit-cube ones, and the kernel on the unit cube is s^2 e^{-(mu s) r} / (4 pi r). */
/* rho = c / r * f with r = s |x - (1/2,1/2,1/2)| (the physical distance to the nucleus).  The paper
 * refers to other work for products of adaptive functions; here rho lives on f's tree with every leaf
 * split once and the boxes whose closure holds the centre split further down to level jmax; each new
 * leaf's block is the k-point Gauss-Legendre rule of App. A.1 (eq. fvals2coefs) applied to c / r times
 * f's polynomial (eq. func_interp) at the leaf's nodes (the centre is a corner of boxes on every scale,
 * so no node falls on it); the ancestors hold the two-scale projections (a redundant tree).  f is not
 * changed.  *out is a new tree of ctx.  1 <= jmax <= 19, f's depth <= 18, c finite, s > 0.
 * Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
mwns_status mwns_tree_coulomb_product(mwns_ctx* ctx, const mwns_tree* f, double c, double s, int jmax,
                                      mwns_tree** out);
/* <u, v> over the unit cube as the sum, over u's leaves, of the dot product of u's block with v's block
 * of the same box (orthonormal bases): exact when v's tree holds the projection of v onto every leaf
 * box of u (a redundant tree built on a refinement of u's leaves, such as a product above, or the same
 * leaves).  The sum is formed on the device in a fixed order.  *out on the host.  Synchronises.
 * Errors: EINVAL (orders differ, a leaf box of u missing from v, trees of another context), ENOMEM,
 * EDEVICE. */
mwns_status mwns_tree_dot(mwns_ctx* ctx, const mwns_tree* u, const mwns_tree* v, double* out);
/* The iteration of Sec. 6.2 in the library, `iters` steps from phi_0 = (2/pi)^{3/4} e^{-|x|^2} (projected
 * by Alg. 1 at eps from level j0 down to at most jmax) and mu_0:
 *   rho = -2 V phi / ||phi|| (the product above, finest level jmax);
 *   each step: fit G_mu to eps on [sqrt(eps) 2^-depth, sqrt(3)] (depth of rho's tree; mwns_fit_kernel with
 *   mu s and scale s^2), build the operator at eps (mwns_op_create, default options), phi_new = G_mu rho by
 *   the modified ns-form (mwns_apply, FP64), then
 *     E = (<phi_new, rho> / 2 - mu^2 ||phi_new||^2 / 2 - ||phi_new|| <phi_new, rho_new> / 2) / ||phi_new||^2
 *   with rho_new = -2 V phi_new / ||phi_new|| formed on phi_new discarded to eps (mwns_tree_discard, Alg. 3
 *   Step 4): since (-Delta + mu^2) phi_new = rho, the kinetic term 1/2 ||grad phi_new||^2 equals
 *   <phi_new, rho> / 2 - mu^2 ||phi_new||^2 / 2 (the paper defers weak derivatives to other work);
 *   mu <- sqrt(-2 E), rho <- rho_new.
 * Outputs (host, caller-owned, iters entries): mu_out[i] = mu used by step i, E_out[i] = its energy;
 * rho_leaves[i] (may be NULL) = leaves of the rho that step i applies to; ms_apply[i] (may be NULL) =
 * device time of that apply (closure, contraction, assembly).  0 < eps < 1, L, mu0, Z > 0,
 * 0 <= j0 <= jmax <= 18, iters >= 1, 1 <= k <= 10.  Errors: EINVAL, ENOMEM, EDEVICE, ERANGE (a fit above
 * 4096 terms, a screening band overflow, or an energy E >= 0: no bound state to follow). */
mwns_status mwns_hydrogen_kalos(mwns_ctx* ctx, int k, double eps, double L, int jmax, double mu0, double Z, int j0,
                                int iters, double* mu_out, double* E_out, int64_t* rho_leaves, double* ms_apply);

#ifdef __cplusplus
}
#endif
#endif /* MWNS_H */
