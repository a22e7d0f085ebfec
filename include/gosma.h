/*
 * gosma.h -- C-ABI of libgosma, the MI355X (gfx950) implementation of the
 * branch-and-bound bound evaluation of GOSMA (Campbell, Petersson, Kneip,
 * Li, Gould, "The Alignment of the Spheres: Globally-Optimal Spherical
 * Mixture Alignment for Camera Pose Estimation", arXiv:1812.01232).
 *
 * Conventions for every entry point:
 *   - Return 0 (GOSMA_OK) on success or a negative GOSMA_E_* code.  No C++
 *     exception crosses this boundary; the message of the last failure on a
 *     context is available from gosma_last_error().
 *   - The caller owns every buffer it passes.  Functions that take host
 *     arrays copy them before returning.  Functions documented as taking
 *     device pointers read and write them asynchronously on the HIP stream
 *     passed as `stream` (NULL = the null stream) and do not synchronise.
 *   - A context is bound to one device and is not thread-safe; calls on one
 *     context must be serialised by the caller.
 *
 * Octree keys.  A cube of the rotation domain (angle-axis vectors, Section
 * 5.1) or of the translation domain is an octree cell of a root box:
 *   bits  0-18  z index      bits 19-37  y index
 *   bits 38-56  x index      bits 57-62  level L (0..19)
 * Level L splits each axis of the root box [lo, hi] into 2^L cells; cell i
 * has centre lo + (2 i + 1) (hi - lo) / 2^(L+1) and that half-width.
 * Key 0 is the root box.
 */
#ifndef GOSMA_H
#define GOSMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GOSMA_OK 0
#define GOSMA_E_INVAL (-1)          /* invalid argument (message says which) */
#define GOSMA_E_NOMEM (-2)          /* device or host allocation failed */
#define GOSMA_E_HIP (-3)            /* a HIP runtime call failed (HIP error text kept) */
#define GOSMA_E_QUEUE_OVERFLOW (-4) /* the branch-and-bound queue exceeded its capacity */
#define GOSMA_E_STATE (-5)          /* call made before the state it needs was set */

#define GOSMA_MAX_COMPONENTS 4096   /* per mixture, per problem */
#define GOSMA_MAX_LABELS 64

typedef struct gosma_ctx gosma_ctx;

/* Search domain of one pose problem (Section 5.1): the rotation box of
 * angle-axis vectors (normally [-pi, pi]^3, the cube circumscribing the
 * radius-pi ball), the translation box Omega_t', and zeta, the smallest
 * allowed distance between the camera centre and any Gaussian mean. */
typedef struct {
    double r_lo[3], r_hi[3];
    double t_lo[3], t_hi[3];
    double zeta;
} gosma_domain;

/* Flags byte written per cube by the bound evaluation. */
#define GOSMA_FLAG_SPLIT_ROT 1u     /* the cube's next split is in rotation (Section 5.1) */
#define GOSMA_FLAG_DROP_ROT 2u      /* rotation cell has no point in the radius-pi ball */
#define GOSMA_FLAG_DROP_TRANS 4u    /* every translation in the cell is within zeta of a mean */
#define GOSMA_FLAG_UB_INF 8u        /* the cell centre is not a feasible camera position */

/* Create a context on HIP device `device`.  *out receives the handle. */
int gosma_create(int device, gosma_ctx **out);

/* Release the context and all device memory it owns.  NULL is ignored. */
void gosma_destroy(gosma_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  The pointer stays
 * valid until the next call on ctx. */
const char *gosma_last_error(const gosma_ctx *ctx);

/* Set the single pose problem of the context (replacing any previous one).
 * GMM theta_1 (Section 4, eq. 7): M means mu (M x 3, row-major, metres),
 * standard deviations sigma (M, > 0) and weights phi1 (M, >= 0).  vMF mixture
 * theta_2 (eq. 9): N unit mean directions dir2 (N x 3; |d| = 1 within 1e-6),
 * concentrations kappa2 (N, > 0) and weights phi2 (N, >= 0).  Optional class
 * labels (eq. 17) label1 (M) and label2 (N) in [0, n_labels); pass NULL for
 * both to use one class.  With labels only same-class pairs contribute and
 * the objective is sum_l f_l / n_labels, the weights being renormalised
 * within each class; without labels the weights are renormalised to sum 1.
 * All arrays are host FP64/int32 and are copied.  1 <= M, N <= 4096
 * (GOSMA_E_INVAL otherwise).  A bound-kernel block stages 96 bytes per GMM
 * component in LDS plus 512 bytes per wave (and 32 bytes per vMF component
 * when several problems are set), an SMA block 44 per GMM and 24 per vMF
 * component; when that exceeds the device's LDS per block (on gfx950 beyond
 * about 1,600 components) the records go to a device buffer the context
 * allocates here (96 bytes per GMM component for each of 512 blocks, 200 MB
 * at M = N = 4096) and the kernels read them through the caches. */
int gosma_set_mixtures(gosma_ctx *ctx, int M, const double *mu, const double *sigma, const double *phi1,
                       const int32_t *label1, int N, const double *dir2, const double *kappa2,
                       const double *phi2, const int32_t *label2, int n_labels);

/* Set the search domain of the single problem (host struct, copied). */
int gosma_set_domain(gosma_ctx *ctx, const gosma_domain *domain);

/* Set n_problems independent pose problems at once (the batched form).  The
 * per-problem arrays of gosma_set_mixtures are concatenated; problem p owns
 * GMM rows gmm_off[p] .. gmm_off[p+1]-1 and vMF rows vmf_off[p] ..
 * vmf_off[p+1]-1 (offset arrays of n_problems + 1 entries, gmm_off[0] =
 * vmf_off[0] = 0).  label arrays are NULL or concatenated like the others;
 * n_labels applies to every problem.  domains holds n_problems structs.
 * Replaces any problem set before.  All host memory, copied. */
int gosma_set_problems(gosma_ctx *ctx, int n_problems, const int64_t *gmm_off, const int64_t *vmf_off,
                       const double *mu, const double *sigma, const double *phi1, const int32_t *label1,
                       const double *dir2, const double *kappa2, const double *phi2, const int32_t *label2,
                       int n_labels, const gosma_domain *domains);

/* The constant S22 of problem p (the vMF self term that eq. 10 drops from
 * the L2 distance of eq. 14).  The normalised objective used for the
 * tolerance is (f + S22) / S22, zero at perfect alignment. */
int gosma_get_S22(gosma_ctx *ctx, int problem, double *S22);

/* Theorem 1 bounds (Section 5.2) for n sub-cubes C_r x C_t.
 * All n-element arrays; each may be memory of the context's device (used in
 * place: the call is asynchronous) or host memory of any kind (copied
 * through device buffers of the context, which grow to the largest call;
 * the call then returns after the results are in place).  Device memory of
 * another device is rejected (GOSMA_E_INVAL).
 *   rkeys, tkeys  in:  octree keys of the rotation and translation cells
 *   problem       in:  uint32 problem index per cube, or NULL (all problem 0);
 *                      an index >= the number of problems gives NaN bounds
 *                      and both drop flags
 *   ub            out: upper bound, eq. 20 (objective at the centre; +inf if
 *                      the centre is infeasible or the cube is dropped)
 *   lb            out: lower bound, eq. 21 (+inf for dropped cubes); no
 *                      rounding margin is applied here
 *   flags         out: GOSMA_FLAG_* bits
 *   aux           out: NULL or n x 4 doubles {S11 at centre, S12 at centre,
 *                      S11 lower sum, S12 upper sum} (class-weighted)
 *   top8          out: NULL or n x 8 floats, the largest S12 pair terms at the
 *                      centre in descending order (zeros past the pair count)
 * Runs on `stream` (a hipStream_t, NULL = null stream).
 * n = 0 is a no-op.  Errors: GOSMA_E_STATE before mixtures and a domain are
 * set, GOSMA_E_INVAL for n < 0 or a NULL required pointer. */
int gosma_eval_bounds(gosma_ctx *ctx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *problem,
                      int64_t n, double *ub, double *lb, uint8_t *flags, double *aux, float *top8,
                      void *stream);

/* gosma_eval_bounds for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results as gosma_eval_bounds, with the
 * kernels' per-cube scratch (the S11 sums of each cube's translation cell and
 * the pair kernel's set-up record, 208 bytes per cube) in a fixed array of
 * the library, sized for GOSMA_NOALLOC_MAX_CUBES cubes (13.6 MB), that each
 * device holds from its first gosma_create until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 *   Arguments as for gosma_eval_bounds, except that every array must be
 *   device memory of the context's device (GOSMA_E_INVAL otherwise; no host
 *   staging) and n <= GOSMA_NOALLOC_MAX_CUBES (GOSMA_E_INVAL beyond).
 *   Kernel timing and work counters are not recorded.
 * Asynchronous on `stream`.  Every call on a device shares that device's
 * array (it keeps the last call's contents; this call writes every element it
 * reads before reading it, so nothing needs clearing): calls that overlap on
 * one device, on different streams or from different contexts, race and must
 * be serialised by the caller. */
#define GOSMA_NOALLOC_MAX_CUBES 65536
int gosma_eval_bounds_noalloc(gosma_ctx *ctx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *problem,
                              int64_t n, double *ub, double *lb, uint8_t *flags, double *aux, float *top8,
                              void *stream);

/* Branch-and-bound options (Algorithm 1, Section 6). */
typedef struct {
    double eps;              /* tolerance on the normalised objective (f + S22)/S22 */
    int64_t batch_parents;   /* cubes removed from the queue per iteration (8 children each) */
    int64_t max_queue;       /* queue capacity in cubes (per problem) */
    int64_t max_iters;       /* 0 = no limit */
    double time_limit_s;     /* 0 = no limit */
    int order;               /* 0: best-first by lower bound; 1: learned priority (gosma_mlp_load) */
    int log_records;         /* 1: append cube records to the sink of gosma_set_record_sink */
    int trace_every;         /* > 0: record the search state every n-th iteration (gosma_get_trace) */
    int no_graph;            /* 1: launch each iteration's kernels directly instead of replaying
                                a captured HIP graph of one iteration */
    double learned_window;   /* order = 1: the predicted rise added to a cube's normalised lower
                                bound is clamped to [0, learned_window]; <= 0: to [0, 10].  Cubes
                                whose lower bound is within eps of d* are ordered after all others
                                (by lower bound) under either setting */
    int sma_iters;           /* > 0: Algorithm 1's SMA step (Section 6): after each iteration in
                                which a bounded cube lowered d*, run SMA (gosma_refine, at most
                                sma_iters L-BFGS iterations) from the centre of the cube holding
                                d* and keep its result when it is lower; 0 = off (<= 10000) */
} gosma_opts;

typedef struct {
    double f_best;           /* best objective value d* (eq. 10 / eq. 17) */
    double lb_global;        /* certified lower bound on the minimum at exit */
    double f_norm_best;      /* (f_best + S22) / S22 */
    double lb_norm;          /* (lb_global + S22) / S22 */
    double r[3], t[3];       /* pose of d*: angle-axis rotation and camera centre */
    int64_t iters, cubes;    /* iterations run, sub-cubes bounded */
    int64_t max_queue_used;
    double seconds;          /* wall time inside the call */
    int status;              /* 0 eps-optimal, 1 queue exhausted, 2 iteration/time cap, 3 queue
                                capacity reached (f_best and lb_global still bound the optimum) */
    int64_t sma_runs;        /* SMA runs of the search, and how many of them lowered d* (r, t is */
    int64_t sma_improved;    /* then SMA's pose rather than a cube centre) */
} gosma_result;

/* Solve problem 0 to eps-optimality (Algorithm 1 without local refinement).
 * Host structs in and out; synchronous.  GOSMA_E_QUEUE_OVERFLOW if the queue
 * capacity is exceeded: the result then holds the state reached, with status
 * 3; its lb_global includes the lower bounds of the cubes that did not fit. */
int gosma_solve(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *result);

/* Search trace of the last gosma_solve with opts->trace_every > 0 (the
 * bound-evolution record of Section 7.1): rows of 6 doubles {iteration,
 * seconds since entry, cubes bounded, queue size, d*, lowest lower bound in
 * the queue}.  buf: host array of cap rows; *n receives the number of rows
 * available (at most cap are written). */
int gosma_get_trace(gosma_ctx *ctx, double *buf, int64_t cap, int64_t *n);

/* Solve every problem of gosma_set_problems together: each iteration pops
 * up to opts->batch_parents cubes from every unfinished problem's queue and
 * bounds all their children in one launch.  result: host array of
 * n_problems structs.  Synchronous.  A problem whose queue fills up stops with
 * status 3 while the others go on; the call then returns
 * GOSMA_E_QUEUE_OVERFLOW with every result filled. */
int gosma_solve_batch(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *results);

/* SMA, the local optimiser of Algorithm 1 (Section 6): L-BFGS on the
 * objective of Lemma 1 (eqs. 10-13, eq. 17) over the pose (r, t), with the
 * gradient by the chain rule.  The L-BFGS direction (5 curvature pairs,
 * initial scaling s^T y / y^T y) is followed along the path projected on the
 * problem's domain box (rotation box x translation box), with Armijo
 * backtracking (sufficient-decrease constant 1e-4, at most 40 halvings from
 * the unit step; the first direction is -g scaled to length <= 0.05); poses
 * within zeta of a Gaussian mean are infeasible.  Stops after max_iters
 * iterations, when the projected gradient's largest component is at most
 * 1e-6 of S11 + 2 S12 at the start, or when a step lowers f by at most 1e-9 of
 * |f| + S11 + 2 S12.  Pair terms are FP32 in log space, sums and the pose FP64.
 *   n          number of starts (one GPU block each)
 *   problem    host uint32 problem index per start, or NULL (all problem 0)
 *   r0, t0     host n x 3 start poses (angle-axis rotation, camera centre)
 *   max_iters  L-BFGS iterations; 0 evaluates f and its gradient at the starts
 *   r_out, t_out  host n x 3 results; f_out host n objective values there
 *   grad_out   host n x 6 gradient {d/dr, d/dt} at the result, or NULL
 *   iters_out  host n iterations taken; -1 if the start lies outside the box
 *              or within zeta of a mean (f_out = +inf) or the problem index is
 *              out of range (f_out = NaN)
 * Synchronous; allocates and frees its own device buffers.  Errors:
 * GOSMA_E_STATE before mixtures and a domain are set, GOSMA_E_INVAL for n < 0,
 * max_iters < 0 or a NULL required pointer. */
int gosma_refine(gosma_ctx *ctx, int64_t n, const uint32_t *problem, const double *r0, const double *t0,
                 int max_iters, double *r_out, double *t_out, double *f_out, double *grad_out, int32_t *iters_out);

/* Mixture generation (Section 7): the GMM theta_1 from a 3D point set by
 * DP-means clustering and the vMF mixture theta_2 from bearing vectors by
 * DP-vMF-means, with a maximum-likelihood component fitted to each cluster.
 * Both run the serial batch algorithm of their papers (Kulis and Jordan 2012;
 * Straub et al. 2015): passes over the points in index order, each point
 * joining the best cluster that exists when it is visited (ties: the cluster
 * created first) or opening a new cluster at itself when even the best is
 * beyond lambda; after each pass the centres are recomputed from their
 * points (DP-vMF-means: the normalised sum) and empty clusters are removed
 * in order; passes stop when no label changes or after max_passes.  The
 * first pass starts from one cluster at the mean of all points (DP-vMF-means:
 * their mean direction).  Scores are FP64, evaluated as |x - mu|^2 (x, y, z in
 * order) and x . mu without fused multiply-adds; centre sums are FP64
 * atomics, exact in any order when the inputs lie on a binary grid whose sums
 * do not exceed 53 bits (e.g. points on a 2^-24 m grid within 64 m, up to
 * 2^20 of them), which makes the result identical to a serial evaluation.
 *   points / dirs  device n x 3 FP64 (context's device); dirs unit vectors
 *   lambda         DP-means: squared distance beyond which a point opens a
 *                  cluster; cos_lambda: cosine below which a direction does
 *   max_clusters   1 .. GOSMA_MAX_CLUSTERS; a pass that would open more lets
 *                  the point join its best cluster and *passes is negated
 *   sigma_min      the fitted isotropic standard deviation sqrt(sum |x -
 *                  mu|^2 / (3 n)) is raised to at least this (one-point
 *                  clusters); kappa_max: the fitted concentration (root of
 *                  coth k - 1/k = |sum x| / n) is lowered to at most this
 *   labels         device n int32 out: cluster of each point
 *   centres, counts, sigma / kappa   host arrays of max_clusters (x 3) out;
 *                  the first *K entries are set (mixture weights: counts / n)
 *   K, passes      host out
 * Synchronous on `stream`; allocates and frees its own device buffers.
 * Errors: GOSMA_E_INVAL for n outside [1, 2^30], max_clusters outside
 * [1, GOSMA_MAX_CLUSTERS], max_passes < 1, a non-finite lambda, a clamp <= 0,
 * NULL pointers or points / labels that are not device memory of the context's
 * device. */
#define GOSMA_MAX_CLUSTERS 2048
int gosma_dpmeans(gosma_ctx *ctx, const double *points, int64_t n, double lambda, int max_clusters, int max_passes,
                  double sigma_min, int32_t *labels, double *centres, int64_t *counts, double *sigma, int *K,
                  int *passes, void *stream);
int gosma_dpvmf_means(gosma_ctx *ctx, const double *dirs, int64_t n, double cos_lambda, int max_clusters,
                      int max_passes, double kappa_max, int32_t *labels, double *centres, int64_t *counts,
                      double *kappa, int *K, int *passes, void *stream);

/* Checkpoint of the search (Algorithm 1's state between two iterations: the
 * queued sub-cubes with their lower bounds, d* and its pose, the counters).
 * gosma_snapshot writes the state left by the last gosma_solve or
 * gosma_solve_batch of the current problems into the caller's host buffer:
 * with buf NULL, *bytes receives the size needed; otherwise *bytes holds the
 * buffer's capacity on entry and the size written on return (25 bytes per
 * queued cube plus a few hundred per problem).  Errors: GOSMA_E_STATE if no
 * search of the current problems has finished (or the problems or domain
 * changed since), or if a problem overflowed its queue (its queue is then
 * incomplete); GOSMA_E_INVAL if the buffer is too small (*bytes receives the
 * size needed).  Synchronous.
 *
 * gosma_resume checks a snapshot against the current problems (sizes, S22
 * and domain must match: GOSMA_E_INVAL otherwise, also for a malformed or
 * truncated buffer) and copies it; the next gosma_solve / gosma_solve_batch
 * then starts from that state instead of the root cubes, under its own
 * options: a new eps (a search certified at eps can be resumed to a smaller
 * one), queue capacity (GOSMA_E_INVAL if a problem's snapshot holds more than
 * max_queue cubes), order and caps (max_iters counts the iterations of that
 * call).  The resumed search runs at least one iteration; its result counts
 * iterations and cubes from the original root.  Queue priorities restart
 * from the lower bounds.  Record logging cannot start from a snapshot
 * (GOSMA_E_STATE).  buf NULL with bytes 0 discards a pending snapshot. */
int gosma_snapshot(gosma_ctx *ctx, void *buf, size_t *bytes);
int gosma_resume(gosma_ctx *ctx, const void *buf, size_t bytes);

/* ------------------------------------------------------------------ */
/* Learned queue order (not part of the paper's method).               */
/* ------------------------------------------------------------------ */
/* A small network, 20 -> 128 -> 128 -> 128 -> 1 with GELU activations,
 * bf16 weights and FP32 accumulation, predicts for a queued cube how much
 * the lower bound of its children will exceed its own (in units of S22).
 * With gosma_opts.order = 1 the queue is ordered by the cube's normalised
 * lower bound plus that prediction; pruning and the stop test still use the
 * exact bounds, so the result keeps its eps certificate.
 *
 * Features of a cube (20 floats): rotation centre / pi (3); translation
 * centre mapped to [-1, 1] over the domain box (3); rotation level / 19;
 * translation level / 19; |rotation half-widths| / pi; |translation
 * half-widths| / |domain half-widths|; upper and lower bound normalised as
 * (f + S22) / S22 (clamped to [-10, 10]); the 8 largest S12 pair terms at
 * the centre / S22.  A training record is the 20 features of a cube followed
 * by the target: the smallest normalised lower bound of its children minus
 * its own.
 * Parameters (GOSMA_MLP_PARAMS floats, row-major): W1 [128 x 20], b1 [128],
 * W2 [128 x 128], b2, W3 [128 x 128], b3, W4 [1 x 128], b4 [1]. */
#define GOSMA_MLP_FEATURES 20
#define GOSMA_MLP_RECORD 21
#define GOSMA_MLP_PARAMS 35841

/* Random initialisation (He normal weights, zero biases), deterministic per seed. */
int gosma_mlp_init(gosma_ctx *ctx, uint64_t seed);
/* Set / read the parameters (host FP32 arrays of GOSMA_MLP_PARAMS). */
int gosma_mlp_set_params(gosma_ctx *ctx, const float *params);
int gosma_mlp_get_params(gosma_ctx *ctx, float *params);
/* Inference: x device n x 20 features, y device n outputs; async on stream. */
int gosma_mlp_predict(gosma_ctx *ctx, const float *x, int64_t n, float *y, void *stream);
/* Mean squared error over n device records (n x 21) and its gradient with
 * respect to the parameters (host array of GOSMA_MLP_PARAMS).  Synchronous. */
int gosma_mlp_loss_grad(gosma_ctx *ctx, const float *records, int64_t n, double *loss, float *grad);
/* Train with Adam on n device records: `epochs` passes in minibatches of
 * `batch` records, shuffled per epoch with `seed`.  loss_per_epoch: NULL or a
 * host array of `epochs` floats.  Synchronous. */
int gosma_mlp_train(gosma_ctx *ctx, const float *records, int64_t n, int epochs, int batch, float lr,
                    uint64_t seed, float *loss_per_epoch);
/* Record sink of the branch-and-bound (gosma_opts.log_records = 1): when a
 * cube is split and its children bounded, one record is appended to
 * `records` (device, capacity x GOSMA_MLP_RECORD floats) and *count (device
 * uint64) is advanced; records past the capacity are counted but not
 * written.  The caller owns both buffers and zeroes *count. */
int gosma_set_record_sink(gosma_ctx *ctx, float *records, int64_t capacity, unsigned long long *count);

/* ------------------------------------------------------------------ */
/* Reading of the kappa dependence of the lower bound.                  */
/* ------------------------------------------------------------------ */
/* The lower bound (eq. 21) needs, for each GMM-vMF pair, the largest value
 * of its summand over the concentrations kappa_1i(t) that the translation
 * cell allows (Theorem 1; the proof leaves this maximisation to a separate
 * step).  The default bounds it over the whole kappa interval with the
 * smaller of two second-order expansions at its ends, capped by the
 * aligned-directions and far-apart bounds.  With m pieces the interval is
 * split into m equal parts, the expansions are applied to each part and the
 * largest part bound is used (capped as before): still a valid upper bound,
 * and closer to the exact maximum over the interval as m grows.  m is 1, 2
 * or 4 (GOSMA_E_INVAL otherwise); it applies to gosma_eval_bounds,
 * gosma_eval_bounds_noalloc and the search from the next call on.  m > 1
 * needs no top-8 terms (top8 == NULL; in the search: the plain order and no
 * record logging) and mixtures whose records fit LDS (GOSMA_E_INVAL
 * otherwise).  gosma_get_kappa_pieces returns the current m (or
 * GOSMA_E_INVAL for a NULL context). */
int gosma_set_kappa_pieces(gosma_ctx *ctx, int m);
int gosma_get_kappa_pieces(const gosma_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Launch shapes of the bound kernels.                                  */
/* ------------------------------------------------------------------ */
/* Each bound kernel gives one cell (a translation cell for the GMM-GMM sums,
 * a rotation x translation cube for the GMM-vMF sums and the bounds) to one
 * block of 64 * waves threads, which stages the cell's per-component values
 * in LDS and shares its pair sums; a grid of `blocks` blocks walks the
 * cells.  Results agree between shapes up to FP64 summation order. */
typedef struct {
    int32_t waves;    /* 1, 2 or 4 */
    int32_t blocks;   /* >= 1 */
} gosma_tile;

typedef struct {
    gosma_tile s11;   /* GMM-GMM sums (GOSMA_KERNEL_S11) */
    gosma_tile s12;   /* GMM-vMF sums and bounds (GOSMA_KERNEL_S12) */
} gosma_tiles;

/* Size buckets.  The problems of a batch are grouped by their larger mixture
 * max(M, N): bucket 0 up to 64 components, 1 up to 128, 2 up to 256, 3
 * larger.  The search bounds each bucket's cubes with launches of their own,
 * in that bucket's launch shapes (gosma_get_bucket_tiles) and with LDS sized
 * for its largest problem; gosma_eval_bounds uses the shapes of
 * gosma_get_tiles for all problems at once. */
#define GOSMA_N_BUCKETS 4

/* Current shapes (host struct out).  gosma_set_problems resets them to a
 * default chosen from the largest M and N. */
int gosma_get_tiles(gosma_ctx *ctx, gosma_tiles *out);
/* Set the shapes (host struct in) for all problems and every size bucket.
 * GOSMA_E_INVAL for waves outside {1, 2, 4} or blocks < 1. */
int gosma_set_tiles(gosma_ctx *ctx, const gosma_tiles *tiles);
/* The shapes the search uses for size bucket `bucket` (0 .. GOSMA_N_BUCKETS-1)
 * and the number of current problems in it (host out; n_problems may be
 * NULL).  gosma_set_problems resets them to a default chosen from the
 * bucket's largest M and N. */
int gosma_get_bucket_tiles(gosma_ctx *ctx, int bucket, gosma_tiles *out, int *n_problems);
/* Autotuner: draws n_cubes random cubes of the current problems (levels 2-10
 * in rotation, 1-8 in translation, inside the rotation ball; deterministic
 * per seed), times every candidate shape of both kernels on them with HIP
 * events (waves 1, 2, 4 x grids of 2048 to 32768 waves in powers of 2; one
 * warm-up and three timed launches each), and keeps the fastest; then does
 * the same for each non-empty size bucket on random cubes of that bucket's
 * problems (the shapes the search uses: n_cubes cubes for the GMM-vMF kernel,
 * an eighth as many cells for the GMM-GMM kernel, which the search runs once
 * per distinct translation cell).  rows: NULL or a host array of cap x 5 doubles
 * receiving {kernel (GOSMA_KERNEL_S11 or GOSMA_KERNEL_S12), waves, blocks,
 * ms per launch, bucket (-1: all problems)} per candidate; *n_rows (if not
 * NULL) receives the number of candidates.  chosen: NULL or the shapes kept
 * for all problems.  Synchronous; allocates and frees its own device
 * buffers. */
int gosma_autotune(gosma_ctx *ctx, int64_t n_cubes, uint64_t seed, double *rows, int64_t cap, int64_t *n_rows,
                   gosma_tiles *chosen);

/* Kernel timing, for benchmarking.  While enabled, the library records a HIP
 * event pair on the launch stream around each of its kernel launches,
 * grouped by kernel kind (GOSMA_KERNEL_*).  gosma_get_timing() waits for the
 * recorded events, writes the summed milliseconds and launch counts per kind
 * into ms[GOSMA_N_KERNELS] and launches[GOSMA_N_KERNELS] (host arrays), and
 * clears the records. */
#define GOSMA_KERNEL_S11 0      /* GMM-GMM pair sums per translation cell */
#define GOSMA_KERNEL_S12 1      /* GMM-vMF pair sums and final bounds per cube */
#define GOSMA_KERNEL_SELECT 2   /* queue selection (histogram, threshold, compaction) */
#define GOSMA_KERNEL_BRANCH 3   /* children of the selected cubes */
#define GOSMA_KERNEL_PUSH 4     /* best upper bound, pruning and queue insertion */
#define GOSMA_KERNEL_MLP 5      /* learned-priority network (inference and training) */
#define GOSMA_KERNEL_SMA 6      /* SMA local refinement inside the search */
#define GOSMA_N_KERNELS 8
int gosma_set_timing(gosma_ctx *ctx, int enable);
int gosma_get_timing(gosma_ctx *ctx, double *ms, int64_t *launches);

/* Work counts of the bound kernels (Theorem 1, eqs. 20-21) in the
 * gosma_eval_bounds calls and search iterations run while timing was enabled
 * (searches launch their kernels directly then), for the roofline of the
 * kernels: counts[GOSMA_N_COUNTS] (host int64) receives
 *   [GOSMA_COUNT_CUBES]          cubes bounded that were not dropped,
 *   [GOSMA_COUNT_S12_SCREENED]   same-class GMM-vMF pairs of those cubes,
 *   [GOSMA_COUNT_S12_EVALUATED]  of those, the pairs that passed the screen of
 *                                negligible pairs and were evaluated in full,
 *   [GOSMA_COUNT_CELLS]          translation cells whose GMM-GMM sums were
 *                                evaluated (searches: once per distinct cell),
 *   [GOSMA_COUNT_S11_SCREENED]   unordered same-class GMM-GMM pairs i < i' of
 *                                those cells,
 *   [GOSMA_COUNT_S11_EVALUATED]  of those, the pairs evaluated in full.
 * The counts are cleared.  Synchronises the device.  All 0 if timing was
 * never enabled. */
#define GOSMA_COUNT_CUBES 0
#define GOSMA_COUNT_S12_SCREENED 1
#define GOSMA_COUNT_S12_EVALUATED 2
#define GOSMA_COUNT_CELLS 3
#define GOSMA_COUNT_S11_SCREENED 4
#define GOSMA_COUNT_S11_EVALUATED 5
#define GOSMA_N_COUNTS 6
int gosma_get_work_counts(gosma_ctx *ctx, int64_t *counts);

#ifdef __cplusplus
}
#endif
#endif /* GOSMA_H */
