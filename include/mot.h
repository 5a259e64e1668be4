/*
 * mot.h -- C ABI of the MI355X (gfx950) library for tree- and circle-structured
 * entropic multi-marginal optimal transport solved by Sinkhorn iterations whose
 * Gaussian-kernel products run either by direct summation or by NFFT-based
 * fast summation (Ba & Quellmalz, "Accelerating the Sinkhorn algorithm for
 * sparse multi-marginal optimal transport by fast Fourier transforms").
 *
 * Conventions shared by every call
 *   - Marginals are numbered 0..K-1; the paper's marginal 1 (the tree root and
 *     the circle's first node) is marginal 0.
 *   - Points of all marginals are passed concatenated: a row-major
 *     (sum_k n_k) x d array of doubles, marginal k occupying rows
 *     [off_k, off_k + n_k) with off_k = n_0 + ... + n_{k-1}.  Weights, scaling
 *     vectors and marginals are concatenated the same way.
 *   - ptr_kind says whether a caller buffer is host memory (MOT_HOST) or device
 *     memory of the plan's GPU (MOT_DEVICE).  The caller owns every buffer it
 *     passes; the library copies inputs and writes outputs, never keeps them.
 *   - Every call returns an int status: MOT_OK (0), MOT_MAXITER (1: stopped at
 *     the sweep limit, results valid) or a negative error code.  No exception
 *     crosses the ABI.  mot_strerror() gives a static description.
 *   - A plan is bound to one HIP stream.  All work of a call is enqueued on it;
 *     calls that return results to host memory synchronise that stream.  Two
 *     plans may be used from different threads; one plan must not be.
 */
#ifndef MOT_H
#define MOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------------- */
#define MOT_OK 0
#define MOT_MAXITER 1      /* sweep limit reached before the stopping test held        */
#define MOT_EINVAL (-1)    /* invalid argument (sizes, topology, weights, eta, ...)      */
#define MOT_EDOMAIN (-2)   /* fast-summation parameters cannot represent the points      */
#define MOT_ENOMEM (-3)    /* device allocation failed or admission budget exceeded      */
#define MOT_EDEVICE (-4)   /* HIP runtime error                                          */
#define MOT_ENUMERIC (-6)  /* a scaling vector became Inf/NaN (kernel underflow)         */
#define MOT_EUNSUPPORTED (-7) /* combination of options not provided                      */
#define MOT_ELIMIT (-8)    /* size beyond a fixed limit of an allocation-free entry point  */

/* ---- enumerations ---------------------------------------------------------------- */
#define MOT_TREE 0         /* cost decouples along a tree (Sec. 4.1)                      */
#define MOT_CIRCLE 1       /* cost decouples along a circle (Sec. 4.2)                    */

#define MOT_DIRECT 0       /* kernel products by direct O(N^2) summation, eq. (fastsum-sum) */
#define MOT_NFFT 1         /* kernel products by NFFT fast summation, Algorithm 4         */
#define MOT_DENSE 2        /* circle only: dense matrix products on MFMA                  */
#define MOT_TRUNC 3        /* tree only: direct summation truncated to the sources within
                              the kernel's cutoff radius r_c of each target, for small eta
                              (the truncation the paper suggests at the end of Sec. 6.1).
                              r_c = sqrt(eta ln(1 / eps_t)): dropped terms are below
                              eps_t v_j each.  eps_t is set from fs->target_rel_err (default
                              1e-7) times the fraction (pi eta)^(d/2) / (2^d V) of the
                              sources a corner target of a uniform cloud of bounding-box
                              volume V sees, so the relative error of such a cloud's
                              products stays near the target.  Sources are found through
                              a cell list: the a1 binning with cubic cells of side h and
                              tile edge 1, cells within r_c of the target's cell summed. */

#define MOT_PREC_FP64 0    /* direct and truncated paths: FP64 exp and accumulation       */
#define MOT_PREC_MIXED 1   /* direct and truncated paths: FP32 exp, FP32 sums over 64
                              sources, FP64 across them;
                              NFFT path: FP32 spread/FFT/interpolation                    */
#define MOT_PREC_BF16 2    /* dense circle: BF16 operands, FP32 accumulation              */
#define MOT_PREC_FP16 3    /* dense circle: FP16 operands (power-of-two scaled), FP32 acc. */
#define MOT_PREC_BF16X3 4  /* dense circle: split BF16 (hi*hi + hi*lo + lo*hi), FP32 acc.  */

#define MOT_HOST 0
#define MOT_DEVICE 1

/* Fast-summation parameters (Sec. 5, Algorithm 4).  A zero field is chosen by the
 * library's autotuner from d, eta, the point extent and the sizes.
 *   M      half bandwidth: kappa_hat is used on {-M..M-1}^d (2M coefficients per dim)
 *   n      oversampled FFT grid per dimension (power of two, 16..512)
 *   m      window cutoff: Kaiser-Bessel window supported on |s| <= m grid cells,
 *          2m taps per dimension
 *   p      smoothness of the boundary polynomial kappa_B (degree 2p)
 *   tau    half period of the periodised kernel; must exceed eps_B plus the
 *          largest distance between points of the two marginals of any edge
 *   eps_B  width of the boundary interval of the regularised kernel
 *   tile   edge (in grid cells) of the binning tiles that spreading/interpolation
 *          work on; always 17 - 2m (their patches are 16 cells wide), 0 = derive
 *   chunk  maximum points per spreading work item                              */
typedef struct {
    int32_t M, n, m, p;
    double tau, eps_B;
    int32_t tile, chunk;
    double target_rel_err; /* autotuner accuracy target for one product (0 = 1e-7) */
} mot_fastsum_params;

/* Optional device-memory provider (e.g. PyTorch's caching allocator).  NULL
 * means hipMalloc/hipFree.  alloc returns NULL on failure; a block it returns must be
 * 256-byte aligned (plan creation fails with MOT_EINVAL otherwise). */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} mot_allocator;

typedef struct mot_plan_s *mot_plan;

/* Chosen parameters and layout of a plan (for reporting and tests). */
typedef struct {
    int32_t K, d, topology, path, precision;
    int32_t M, n, m, p, tile, chunk;
    double tau, eps_B, eta;
    double scale;        /* grid cells per unit length, s = n / (2 tau)            */
    double offset[3];    /* grid coordinate of the origin per dimension, o_c       */
    int32_t box_lo[3];   /* first grid index of the active box per dimension       */
    int32_t box_len[3];  /* active box extent per dimension                        */
    int32_t depth;       /* tree depth (levels below the root)                     */
    size_t device_bytes; /* device memory held by the plan                         */
    int32_t products_per_sweep;
    double est_err;      /* autotuner's estimate of one product's relative error:
                            Fourier truncation (d x the 1-D sup error of the
                            truncated series of the regularised kernel) plus the
                            Kaiser-Bessel window bound (NFFT path); the target the
                            cutoff was set for (truncated path); 0 otherwise     */
    double trunc_radius; /* truncated path: cutoff radius r_c (0 otherwise); the
                            cell side is 1 / scale, the cells per dimension n,
                            the neighbour half-width in cells tile, and at the
                            mean density the cells per work item chunk and the
                            targets per lane m                                  */
} mot_plan_info;

/* Create a plan: copy the problem to the device and precompute everything the
 * sweeps need.  Follows the discrete problem of Secs. 2-4: K marginals
 * mu^k = sum_i mu^k_i delta_{x^k_i} with x^k_i in R^d, cost = sum over the edges
 * of the tree/circle of squared Euclidean distances, entropic regularisation eta.
 *   n        [K] sizes n_k >= 1 (host memory)
 *   points   concatenated (sum n_k) x d doubles (ptr_kind)
 *   weights  concatenated sum n_k doubles, each marginal >= 0 summing to 1 within
 *            1e-9 (ptr_kind); weights are not renormalised
 *   parent   tree only: [K] host ints, parent[0] = -1, 0 <= parent[k] < k; NULL
 *            for a circle (edges {k, k+1 mod K}, K >= 3)
 *   eta      > 0
 *   path     MOT_DIRECT, MOT_NFFT, (tree) MOT_TRUNC or (circle) MOT_DENSE
 *   precision see MOT_PREC_*; MOT_PREC_FP64 only with MOT_DIRECT and MOT_TRUNC
 *   fs       fast-summation parameters (NFFT path); NULL = all autotuned
 *   stream   hipStream_t to enqueue on; NULL = a stream the plan creates
 * Scaling vectors start at phi^(0) = 1.  On failure *out is NULL.           */
int mot_plan_create(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                    const double *weights, int32_t topology, const int32_t *parent, double eta,
                    int32_t path, int32_t precision, const mot_fastsum_params *fs,
                    int32_t ptr_kind, void *stream, const mot_allocator *alloc);

/* ---- generalised barycenters on trees (Sec. 6.2) -----------------------------------
 * Tree problems with weighted edge costs and nodes without a marginal constraint.  The
 * cost of the edge {parent[k], k} is edge_weight[k] |x - y|^2, so its kernel is
 * exp(-|x - y|^2 / (eta / edge_weight[k])).  A node k with free_node[k] != 0 has no given
 * marginal: its scaling vector is 1 in every sweep (the barycenter form of Algorithm 2's
 * phi update), and its marginal after the solve (mot_marginals) is the barycenter on the
 * node's support.  The weights passed for free nodes are not read.  The root (node 0)
 * must be constrained (MOT_EINVAL otherwise): its update fixes the common scale of the
 * scalings, without which the stale sibling messages of Algorithm 2 oscillate or grow.
 * mot_marginals reports an L1 error of 0 for free nodes.  On the NFFT path the plan's
 * grid and bandwidth serve every edge (chosen for the smallest and largest eta / w),
 * with one multiplier per distinct edge weight; on the truncated path the cutoff is
 * the one of the largest eta / w.  Other arguments as for mot_plan_create (tree). */
typedef struct {
    const double *edge_weight; /* [K] host or NULL (all 1): entry k >= 1 finite and > 0;
                                  entry 0 is not read                                  */
    const int32_t *free_node;  /* [K] host or NULL (none)                              */
} mot_tree_options;

int mot_plan_create_tree(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                         const double *weights, const int32_t *parent, const mot_tree_options *opt,
                         double eta, int32_t path, int32_t precision, const mot_fastsum_params *fs,
                         int32_t ptr_kind, void *stream, const mot_allocator *alloc);

/* ---- generalised Euler flows (Sec. 6.3) ---------------------------------------------
 * A circle whose closing edge {K, 1} compares x^K with sigma(x^1) instead of x^1: the
 * cost |x^K_{i_K} - sigma(x^1_{i_1})|^2 + sum_k |x^{k+1} - x^k|^2.  closing_points
 * (n_0 x d, ptr_kind, copied) are the mapped points sigma(x^1_i) in marginal 0's order;
 * NULL gives the plain circle.  The closing edge enters Algorithm 3 only through the
 * constant matrix beta_K = K^{(K,1)}, which is built from them.  Other arguments as for
 * mot_plan_create (circle). */
int mot_plan_create_circle(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                           const double *weights, const double *closing_points, double eta, int32_t path,
                           int32_t precision, const mot_fastsum_params *fs, int32_t ptr_kind, void *stream,
                           const mot_allocator *alloc);

/* Pair marginal at the current scaling vectors: the sum of K (.) Phi over every index
 * but two.  Circle: Pi_{1,k} of Sec. 6.3 (marginals 0 and k, 1 <= k < K),
 *   Pi[i][j] = phi^1_i lambda^{(1,k)}[i][j] alpha^{(k,1)}[j][i] phi^k_j
 * (the matrices of Theorem 4.3, recomputed at the current phi).  Tree: the edge
 * {parent[k], k} (1 <= k < K),
 *   Pi[i][j] = (phi^p gamma_p prod_{t in C_p, t != k} beta_t)_i K^{(p,k)}[i][j]
 *              (phi^k prod_{t in C_k} beta_t)_j
 * after a consistent pass as in mot_marginals.  out: n_a x n_k doubles, row-major, rows
 * = the points of marginal a (0 for the circle, parent[k] for the tree) and columns =
 * those of marginal k, both in the original order (ptr_kind).  The matrix is formed on
 * the device in FP64 from the plan's factors (FP32 with power-of-two row scales on the
 * dense circle path). */
int mot_pair_marginal(mot_plan plan, int32_t k, double *out, int32_t ptr_kind);

/* Run Sinkhorn sweeps: Algorithm 2 (tree) or Algorithm 3 (circle).  One sweep
 * updates every scaling vector once and recomputes the messages; it costs
 * 2(K-1) kernel products (tree) or 2(K-2) matrix products (circle).
 *   max_sweeps    sweep limit (>= 0)
 *   delta_S       stop when |S^(r) - S^(r-1)| < delta_S (0 = off)
 *   tol_marginal  stop when the L1 error of the first marginal after the sweep,
 *                 |P_0 - mu^0|_1, is <= tol_marginal (0 = off)
 *   check_every   stopping tests are read back every check_every sweeps (>= 1)
 *   sweeps_done, S_last, marg_err  optional outputs (host), may be NULL
 * Returns MOT_OK when a stopping test held, MOT_MAXITER at the limit,
 * MOT_ENUMERIC if a scaling vector became non-finite.  Sweeps continue from the
 * plan's current scaling vectors (warm start). */
int mot_sinkhorn(mot_plan plan, int32_t max_sweeps, double delta_S, double tol_marginal,
                 int32_t check_every, int32_t *sweeps_done, double *S_last, double *marg_err);

/* S^(r) of every sweep run so far on this plan (Algorithm 2/3, the dual
 * objective of Theorem 3.1 one sweep behind).  Writes min(count, stored) values
 * to host memory and returns the number written (>= 0) or an error. */
int mot_get_S_history(mot_plan plan, double *S_out, int32_t count);

/* Marginals P_k(K (.) Phi) at the current scaling vectors (Theorem 4.1 for a
 * tree, Theorem 4.3 for a circle), by one consistent upward and downward
 * pass.  P_out (optional) receives the concatenated marginals (ptr_kind);
 * l1_err (optional, host, [K]) receives |P_k - mu^k|_1. */
int mot_marginals(mot_plan plan, double *P_out, double *l1_err, int32_t ptr_kind);

/* Read / overwrite the scaling vectors phi^k (concatenated, original point
 * order).  Setting them warm-starts or resumes a solve. */
int mot_get_scalings(mot_plan plan, double *phi_out, int32_t ptr_kind);
int mot_set_scalings(mot_plan plan, const double *phi_in, int32_t ptr_kind);

/* One kernel product with the plan's path: out = K^{(t,s)} v, i.e.
 * out_i = sum_j v_j exp(-|x^t_i - x^s_j|^2 / eta) (Sec. 5, eq. fastsum-sum),
 * approximated by Algorithm 4 on the NFFT path.  v has n_s entries, out n_t
 * (original point order, ptr_kind).  Tree plans only (any pair (t, s));
 * MOT_EUNSUPPORTED for circle plans.  For parity tests of a single product. */
int mot_apply_kernel(mot_plan plan, int32_t t, int32_t s, const double *v, double *out,
                     int32_t ptr_kind);

int mot_plan_get_info(mot_plan plan, mot_plan_info *info);

/* Device bytes a plan with these arguments would hold (admission control).
 * fs as in mot_plan_create; parameters left zero are autotuned from eta and
 * an assumed point extent of half_width (points in [-half_width, half_width)^d). */
int mot_plan_footprint(int32_t K, int32_t d, const int64_t *n, int32_t topology, int32_t path,
                       int32_t precision, double eta, double half_width,
                       const mot_fastsum_params *fs, size_t *bytes);

/* Release the plan and all its device memory (synchronises its stream). */
int mot_plan_destroy(mot_plan plan);

const char *mot_strerror(int status);

/* Per-step device timing of the plan's sweep (tree plans): runs `sweeps` sweeps with a
 * HIP event pair around every launch of the sweep schedule on the plan's stream and
 * reports, per schedule position, the kernel kind and the mean duration.  kind:
 * 0 node update, 1 direct product, 2 spread, 3 fold, 4 FFT pass (fft_kind 0..7),
 * 5 interpolation, 6 sweep finalisation, 7 fill, 8 truncated product.  group: jobs per
 * item of a 3-D spreading launch (jobs spreading from the same points share items), else 0.
 * Returns the number of entries written (<= max_out) or an error.  The sweeps advance the
 * plan like mot_sinkhorn. */
typedef struct {
    int32_t kind, d, n, fft_kind, n_items, calls, group, reserved;
    double ms_mean;
} mot_step_timing;
int mot_plan_profile(mot_plan plan, int32_t sweeps, mot_step_timing *out, int32_t max_out);

/* ---- measured autotuner (Sec. 5 parameters) -----------------------------------------
 * With no fields fixed, the fast-summation parameters are chosen among the candidates
 * (p, eps_B, M, n, m) that meet the accuracy target by the lowest cost of one product.
 * By default that cost is an analytic model; after mot_tune_install it is read from a
 * table measured on the device:
 *   cost = n_max point_ns[d-1][m-2] / 1000 + grid_us[d-1][log2(n)-4] box / box_cells[..]
 * (microseconds; box = cells of the candidate's active box).
 * mot_tune_measure fills the table on the current GPU by creating calibration plans with
 * fixed parameters on synthetic uniform points and timing their launches
 * (mot_plan_profile):
 *   point_ns[d-1][m-2]  spreading + interpolation of one product per point, m = 2..8
 *                       (a two-marginal path of 2^15 points per marginal);
 *   grid_us[d-1][k]     fold + FFT passes of one product at n = 16 << k, k = 0..5
 *                       (a 17-marginal star of 256 points per marginal, M = n / 4),
 *                       measured on a box of box_cells[d-1][k] cells (a grid that
 *                       admits no box for that cloud, n = 16, repeats the next
 *                       grid's entry: the tuner never chooses it for such clouds).
 * It takes a few seconds, allocates and frees its own device memory, and does not install
 * the table.  mot_tune_install(table) makes every later plan creation, footprint and
 * mot_tune_resolve call of the process use it (entries must be finite and > 0, else
 * MOT_EINVAL); mot_tune_install(NULL) returns to the analytic model.  Plans already
 * created keep their parameters. */
#define MOT_TUNE_M 7 /* m = 2..8     */
#define MOT_TUNE_N 6 /* n = 16..512  */
typedef struct {
    int32_t measured, device;
    double point_ns[3][MOT_TUNE_M];
    double grid_us[3][MOT_TUNE_N];
    double box_cells[3][MOT_TUNE_N];
    double seconds; /* wall time of the measurement */
} mot_tune_table;
int mot_tune_measure(mot_tune_table *out);
int mot_tune_install(const mot_tune_table *table);

/* The parameters a plan would get (host only, no device work): d, eta, points assumed in
 * [-half_width, half_width)^d, n_max points in the largest marginal, fs as in
 * mot_plan_create (NULL = all tuned).  out receives M, n, m, p, tau, eps_B, tile, chunk
 * and the accuracy target; est_err (may be NULL) the estimate of mot_plan_info. */
int mot_tune_resolve(int32_t d, double eta, double half_width, int64_t n_max, const mot_fastsum_params *fs,
                     mot_fastsum_params *out, double *est_err);

/* ---- building block: point binning ------------------------------------------------
 * The node ordering the NFFT path uses (not in the paper):
 *   u_c = x_c * s_c + o_c   (FP64, product rounded before the add, no FMA)
 *   cell_c = clamp(floor(u_c), 0, n - 1),  tile_c = cell_c / T
 *   tile = row-major linearisation over ceil(n/T)^d tiles, coordinate 0 slowest
 *   perm = stable sort of the point indices by tile (ties by ascending index); with
 *          0 <= sub_dim < d the points of a tile are further ordered by their
 *          tile-relative cell r = cell_{sub_dim} mod T, i.e. the sort key is
 *          (tile, r, index) (requires T <= 16); sub_dim = -1 gives the plain order
 *   tile_off[t] = first sorted position of tile t; tile_off[ntiles] = npts
 * The 3-D NFFT path sorts its points with sub_dim = 1 (1-D and 2-D: -1).
 * x is npts x d (ptr_kind), s and o are [d] host arrays; cell (npts x d), perm
 * (npts) and tile_off (ceil(n/T)^d + 1) are written to ptr_kind memory.  Runs on
 * the GPU (stream may be NULL = default stream) and synchronises.  Temporary device
 * buffers are allocated and freed inside the call. */
int mot_bin_points(int32_t d, int64_t npts, const double *x, const double *s, const double *o,
                   int32_t n, int32_t T, int32_t sub_dim, int32_t *cell, int32_t *perm,
                   int32_t *tile_off, int32_t ptr_kind, void *stream);

/* Allocation-free variant of mot_bin_points, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments and results as mot_bin_points with ptr_kind = MOT_DEVICE
 * (x, cell, perm and tile_off are device pointers of the current GPU; s and o host
 * arrays of d doubles), but nothing is allocated or freed: the tile ids and the sort
 * keys live in a static device array of the library (12 MiB per GPU, held until the
 * process ends), and the call only enqueues kernels on `stream` (NULL = default stream)
 * without synchronising -- the outputs are ready when the stream reaches that point.
 * Limit: npts <= 2^20 (MOT_ELIMIT beyond it).  Every call on one GPU uses that GPU's one
 * array: calls whose work overlaps on the device (different streams, or threads without
 * ordering) race and give undefined results; calls ordered on one stream are safe.  The
 * first call on a device looks up the array's device address (outside graph capture). */
int mot_bin_points_noalloc(int32_t d, int64_t npts, const double *x, const double *s, const double *o,
                           int32_t n, int32_t T, int32_t sub_dim, int32_t *cell, int32_t *perm,
                           int32_t *tile_off, void *stream);

/* The binned order a plan keeps marginal k's points in (NFFT and truncated paths; the
 * identity otherwise): perm_out[i] = original index of the point at binned position i
 * (n_k int32, ptr_kind).  With the plan's grid scale s, offset o, grid n and tile T
 * (mot_plan_get_info) it equals mot_bin_points on the marginal's points, sub_dim 1 in
 * 3-D and -1 otherwise (truncated path: the cell grid of mot_plan_get_info, T = 1). */
int mot_plan_get_order(mot_plan plan, int32_t k, int32_t *perm_out, int32_t ptr_kind);

/* ---- batched form ------------------------------------------------------------------
 * Run `sweeps` Sinkhorn sweeps on `count` tree plans at once: every level of
 * every plan's sweep is executed by shared launches (all edges at a tree depth
 * across all plans in one set of kernels), and the whole batched sweep is
 * captured once as a HIP graph and replayed.  The plans are split into up to four lanes
 * balanced by their points; each lane's launches go to a stream of its own (the plans'
 * stream and up to three the batch creates, joined back into the plans' stream before the
 * sweep's finalisation), so the lanes' kernels overlap.  All plans must share one stream
 * and use the NFFT, direct or truncated path.  Equivalent, plan by plan, to mot_sinkhorn
 * with the same sweep count and no stopping tests (bit for bit). */
typedef struct mot_batch_s *mot_batch;
int mot_batch_create(mot_batch *out, mot_plan *plans, int32_t count);
int mot_batch_sinkhorn(mot_batch batch, int32_t sweeps, int32_t use_graph);
/* Kernel launch steps of one batched sweep (over all lanes), for reporting. */
int mot_batch_launches(mot_batch batch);
int mot_batch_destroy(mot_batch batch);

/* ---- serving form ------------------------------------------------------------------
 * A continuous-batching solver service on one GPU.  Requests (complete MOT
 * problems) are admitted in FIFO order when their device footprint fits the HBM budget
 * and a slot is free; a preparation thread builds their plans (on a stream of its own)
 * while the resident problems keep sweeping.  Resident problems stay on the device and
 * advance a few sweeps per service step -- tree problems together through one batched
 * schedule (rebuilt by the preparation thread when the resident set changes), each
 * circle problem on a stream of its own, overlapping the tree launches -- until each
 * meets its stopping test; finished ones leave and waiting ones enter between steps.
 * Plans and schedules take device memory from a pool of the server's, so finishing a
 * request frees nothing back to the runtime while others run.  A request's results do not
 * depend on which others share the device.  Requests whose footprint exceeds the
 * per-request limit are refused with MOT_ENOMEM at submission. */
typedef struct mot_server_s *mot_server;
typedef struct {
    int32_t K, d, topology;
    const int64_t *n;          /* [K] host                                            */
    const double *points;      /* host, concatenated as in mot_plan_create            */
    const double *weights;     /* host                                                */
    const int32_t *parent;     /* tree: [K] host; circle: NULL                        */
    double eta;
    int32_t path, precision;   /* as in mot_plan_create                               */
    double tol_marginal;       /* stop when |P_0 - mu^0|_1 <= tol                     */
    int32_t max_sweeps;
} mot_request;

typedef struct {
    int32_t status;            /* MOT_OK, MOT_MAXITER, MOT_ENUMERIC, ...              */
    int32_t sweeps;
    double marg_err, S_last;
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock       */
} mot_result;

/* hbm_budget: device bytes the resident problems may hold together (admission);
 * max_request_bytes: largest footprint a single request may have (0 = hbm_budget);
 * max_slots: resident problems at most; stream: the tree batch's stream (NULL = a
 * non-blocking stream the server creates). */
int mot_server_create(mot_server *out, size_t hbm_budget, size_t max_request_bytes, int32_t max_slots,
                      void *stream);
/* Queue a request (copied).  *ticket identifies it.  Thread-safe. */
int mot_server_submit(mot_server srv, const mot_request *req, uint64_t *ticket);
/* Run the service loop for at most `seconds` (or until idle when idle_exit != 0).
 * Returns the number of requests completed during the call. */
int mot_server_run(mot_server srv, double seconds, int32_t idle_exit);
/* Fetch a finished request: returns MOT_OK and fills *res (and phi_out, host,
 * concatenated, optional) once done; MOT_EINVAL for unknown tickets and 1 while
 * still pending.  A fetched result is released. */
int mot_server_fetch(mot_server srv, uint64_t ticket, mot_result *res, double *phi_out);
double mot_server_clock(mot_server srv);
int mot_server_destroy(mot_server srv);

#ifdef __cplusplus
}
#endif
#endif /* MOT_H */
