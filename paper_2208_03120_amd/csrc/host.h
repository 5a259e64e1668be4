// Host-side structures of the library: plans, launch steps, device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mot_internal.h"

#define MOT_HIP(expr)                                       \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return ::mot::hip_fail(_e, #expr, __FILE__, __LINE__); \
    } while (0)

#define MOT_TRY(expr)              \
    do {                           \
        int _rc = (expr);          \
        if (_rc < 0) return _rc;   \
    } while (0)

namespace mot {

int hip_fail(hipError_t e, const char *what, const char *file, int line);
void log_msg(const char *fmt, ...);

// ---------------------------------------------------------------------------------------
// A temporary device buffer of one C-ABI call, released on every return path (hipFree
// waits for the work still using it).
struct DevTmp {
    void *p = nullptr;
    int alloc(size_t bytes)
    {
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return MOT_ENOMEM;
        }
        return MOT_OK;
    }
    template <class T>
    T *as() const { return (T *)p; }
    ~DevTmp()
    {
        if (p) (void)hipFree(p);
    }
};

// ---------------------------------------------------------------------------------------
// Device memory of a plan.  With the caller's allocator every request is one block of
// it; otherwise requests are carved, 256-byte aligned, from slabs of hipMalloc memory that
// grow geometrically (at least kSlabMin, at least a quarter of what is held already), so a plan
// makes a handful of hipMalloc calls and, when destroyed, as many hipFree calls (each of
// which waits for the device) rather than one per buffer.
struct Arena {
    static constexpr size_t kSlabMin = (size_t)4 << 20;
    mot_allocator alloc{};
    bool custom = false;
    std::vector<void *> blocks;
    size_t bytes = 0;             // device bytes held (blocks or slabs)
    char *slab = nullptr;         // current slab and its free range
    size_t slab_used = 0, slab_size = 0;
    int get(size_t nbytes, void **out);
    template <class T>
    int get_n(size_t count, T **out)
    {
        void *p = nullptr;
        int rc = get(count * sizeof(T) + 256, &p);
        *out = (T *)p;
        return rc;
    }
    void release();
};

// ---------------------------------------------------------------------------------------
// Fast-summation parameters resolved for a plan.
struct NfftParams {
    int M = 0, n = 0, m = 0, p = 0, T = 0, chunk = 0;
    double tau = 0, eps_B = 0;
    double sigma = 0;
    double s = 0;         // grid cells per unit length
    double o[3] = {0, 0, 0};
    int lo[3] = {0, 0, 0}, L[3] = {1, 1, 1}, ntile[3] = {1, 1, 1}, tmin[3] = {0, 0, 0};
    int W = 0;
    double kb_b = 0;
    double est_err = 0;   // autotuner's error estimate for one product (relative)
};

// Cell list of the truncated path.
struct TruncParams {
    double eps = 0;        // kernel values below eps are dropped
    double rc = 0;         // cutoff radius sqrt(eta ln(1 / eps))
    double h = 0;          // cell side
    double q2 = 0;         // (rc / h)^2 (1 + 1e-6)
    double glo[3] = {0, 0, 0};  // grid origin (lower corner of the bounding box)
    int nc = 1, w = 1;     // cells per dimension; neighbour half-width in cells
    int B = 1, R = 1;      // cells per run and targets per lane at the mean density
    double box_cells[3] = {1, 1, 1};  // cells spanned by the cloud's box per dimension
    double est_err = 0;    // relative error the cutoff was set for
};

// Bounding box of all points.
struct Extent {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, ctr[3] = {0, 0, 0};
    double diag = 0, width_max = 0;
};

// params.cpp
constexpr int kTuneM = MOT_TUNE_M, kTuneN = MOT_TUNE_N;
int install_tune_table(const mot_tune_table *t);
// eta_hi > eta: the parameters must also serve kernels up to eta_hi (weighted edges)
int resolve_params(int d, double eta, const Extent &ext, const mot_fastsum_params *fs,
                   int64_t n_max, NfftParams *out, double eta_hi = 0.0);
int build_box(int d, const Extent &ext, NfftParams *P);
int resolve_trunc(int d, double eta, const Extent &ext, const mot_fastsum_params *fs,
                  double n_mean, TruncParams *out);
int64_t trunc_cells(int d, const TruncParams &T);  // nc^d
// host mirror of the kernel's neighbour rows of a run of B cells starting at cc
int trunc_row_range(int d, const TruncParams &T, const int cc[3], int B, int ri, int64_t *row_base,
                    int *xa, int *xb);
double trunc_cost(int d, const TruncParams &T, double lam_t, double lam_s, int B, int R, bool wide);
// cells per run B, targets per lane R and exponent form (wide: FP64) of the cheapest launch
// shape; lam_t / lam_s: targets / sources per grid cell; sch = sqrt(log2(e) / eta) h;
// fp64: the FP64 kernel (form fixed)
void trunc_choose_run(int d, const TruncParams &T, double lam_t, double lam_s, int max_r, double sch, bool fp64,
                      int *B, int *R, int *wide);
void kappa_B_shifted(double eta, double tau, double eps_B, int p, std::vector<double> &q);
double kappa_R(double r, double eta, double tau, double eps_B, const std::vector<double> &q);
void kappa_hat_even(int d, int M, double eta, double tau, double eps_B, int p,
                    std::vector<double> &khat);  // (M+1)^d entries, |k_c| = 0..M
void build_multiplier(int d, const NfftParams &P, double eta, std::vector<float> &D);
void build_twiddle(int n, std::vector<float2> &tw);
double kb_fourier(double k, const NfftParams &P);  // normalised window transform

// ---------------------------------------------------------------------------------------
// A launch step of a sweep schedule.  Steps reference device job and item arrays owned
// by the schedule.
enum StepKind { ST_NODE, ST_DIRECT, ST_SPREAD, ST_FOLD, ST_FFT, ST_INTERP, ST_FINAL, ST_FILL_INT,
                ST_TRUNC, ST_FORK, ST_JOIN };

struct Step {
    StepKind kind;
    int lane = 0;                 // i >= 1: runs on side stream i - 1 between ST_FORK and ST_JOIN
    int d = 0, n = 0, fft_kind = 0, precision = 0, max_patch = 0, trunc_r = 0, diff = 0;
    int group = 0;                // 3-D spreading: jobs per item (items int4)
    int max_children = 0;         // node update: most children of a node in the launch
    const void *jobs = nullptr;   // device ProdJob / NodeJob / FinalJob array
    const void *items = nullptr;  // device int2 / int4 array
    int n_items = 0;
    int n_jobs = 0;               // finalisation: jobs (plans) of the launch
    const void *items2 = nullptr; // FP64 direct: reduction items (int2), n_items2 of them
    int n_items2 = 0;
    const float2 *twiddle = nullptr;
    int32_t *fill_ptr = nullptr;
    int32_t fill_value = 0;
    int64_t fill_count = 0;
};

// Lanes of a sweep: steps of lane i >= 1 run on side[i - 1], after the ST_FORK step (which
// marks the main stream's position) and before the ST_JOIN step (from which the main stream
// waits for every side stream), so the lanes' launches can overlap on the device.
constexpr int kLanes = 4;  // the main stream and three side streams (four hardware queues)
struct Lanes {
    int n = 0;  // lanes including the main stream's; 0 until created
    hipStream_t side[kLanes - 1] = {};
    hipEvent_t fork = nullptr, join[kLanes - 1] = {};
    int create(int lanes);
    void destroy();
};

// Launch the steps on s; with lanes, lane-i steps (i >= 1) on lanes->side[i - 1].  Without
// lanes every step runs on s in order and ST_FORK / ST_JOIN do nothing.
int run_steps(const std::vector<Step> &steps, hipStream_t s, const Lanes *lanes = nullptr);

// ---------------------------------------------------------------------------------------
// Per-marginal device data (binned order).
struct MargDev {
    int64_t n = 0;
    double *pts = nullptr;   // n x d, binned order
    int32_t *perm = nullptr; // binned position -> original index
    double *mu = nullptr, *phi = nullptr, *gamma = nullptr, *beta = nullptr;
    double *down_src = nullptr, *up_src = nullptr, *marg = nullptr;
    // NFFT layout
    float *win = nullptr;    // window rows, n x d x 16
    int32_t *chunk_start = nullptr, *chunk_tile = nullptr, *tile_chunks = nullptr;
    int nchunks = 0;
    std::vector<int32_t> h_chunk_tile;
    std::vector<int32_t> h_chunk_start;  // chunk bounds, nchunks + 1 entries
    // truncated path: sorted point range of each cell
    int32_t *cell_off = nullptr;
    std::vector<int32_t> h_cell_off;
};

struct Schedule {
    std::vector<Step> sweep, init_up, marg_pass;
    Arena *arena = nullptr;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    int n_partials = 0;
    void destroy();
};

}  // namespace mot

// The opaque plan.
struct mot_plan_s {
    int K = 0, d = 0, topology = 0, path = 0, precision = 0;
    double eta = 0;
    // generalised barycenters (tree): edge weight of {parent[k], k} and free nodes
    std::vector<double> edge_w;
    std::vector<int> free_node;
    std::map<double, float *> D_of_eta;  // NFFT multiplier per distinct eta / w
    // generalised Euler flow (circle): sigma(x^1) for the closing edge, original order
    std::vector<double> closing;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    mot::Arena arena;
    std::vector<int64_t> n, off;
    std::vector<int> parent, depth;
    std::vector<std::vector<int>> children;
    int depth_max = 0;
    mot::Extent ext;
    mot::NfftParams P;
    mot::TruncParams TP;
    std::vector<mot::MargDev> marg;
    // product jobs: index 2k = down job of k (gamma_k), 2k+1 = up job of k (beta_k); slot
    // 2K is the stand-alone product used by mot_apply_kernel
    std::vector<mot::ProdJob> jobs;
    mot::ProdJob *jobs_dev = nullptr;
    int32_t *exp_slots = nullptr;  // [2K + 1] slots, kExpSlotStride ints apart
    float *D = nullptr;
    float2 *twiddle = nullptr;
    // statistics
    int32_t *sweep_ctr = nullptr, *flag = nullptr, *flag_hist = nullptr;
    double *S_hist = nullptr, *err_hist = nullptr;
    double *s_partial = nullptr, *l1_partial = nullptr;
    int hist_cap = 0;
    int host_sweeps = 0;  // sweeps run (host count)
    mot::Schedule sched;
    // circle state (circle.hip)
    void *circle = nullptr;
    // stand-alone product buffers (lazily sized)
    double *apply_in = nullptr, *apply_out = nullptr;
    // device staging of the C-ABI transfers (max(sum n_k, 2 max n_k) doubles, allocated at
    // first use): scalings in and out and the one-product call, without a hipMalloc and a
    // device-synchronising hipFree per call
    double *stage = nullptr;
    int64_t apply_cap = 0;
    float *apply_patches = nullptr;
    int apply_patch_cap = 0;
};

namespace mot {
// Per-plan host-side job tables of a tree plan (kept for batching).
struct TreeTables {
    std::vector<NodeJob> njobs;  // [0,K) down, [K,2K) up, [2K,3K) init-up, [3K,4K) marginal
    std::vector<FinalJob> fjob;
    NodeJob *njobs_dev = nullptr;
    FinalJob *fjob_dev = nullptr;
    int n_down_partials = 0, n_marg_partials = 0;
    std::vector<int> marg_block0;  // first partial slot of each node's marginal job
};
TreeTables *tables_of(const mot_plan_s *P);

// A plan inside a merged schedule: offsets of its product, node and final jobs.
struct TreeRef {
    mot_plan_s *P;
    int pbase, nbase, fbase;
};
int tree_steps(const std::vector<TreeRef> &refs, const std::vector<ProdJob> &pj, const ProdJob *pj_dev,
               const std::vector<NodeJob> &nj, const NodeJob *nj_dev, const std::vector<FinalJob> &fj,
               const FinalJob *fj_dev, Arena &arena, std::vector<Step> &sweep, std::vector<Step> &init_up,
               std::vector<Step> &marg, int max_lanes = 1, int *lanes = nullptr);
int tree_build_schedule(mot_plan_s *P);
int tree_run_sweeps(mot_plan_s *P, int sweeps, bool use_graph);
int tree_marginals(mot_plan_s *P, double *P_sorted_all);
int tree_init_up(mot_plan_s *P);
int make_prod_job(mot_plan_s *P, int t, int s, const double *v, int32_t *slot, double *out, ProdJob *J,
                  float *patches, bool alloc_buffers = true);
int product_steps(Arena &arena, const ProdJob *jobs_dev, const std::vector<ProdJob> &jobs_host,
                  const std::vector<int> &ids, std::vector<Step> &out);
int circle_create(mot_plan_s *P, const std::vector<double> &pts_h, const std::vector<double> &w_h,
                  const mot_fastsum_params *fs);
int setup_marginals(mot_plan_s *P, const std::vector<double> &pts_h, const std::vector<double> &w_h,
                    const mot_fastsum_params *fs, int64_t phi_pad_to);
int circle_run_sweeps(mot_plan_s *P, int sweeps);
int circle_marginals(mot_plan_s *P, double *P_sorted_all);
// Pi_{1,k} into out (n_0 x n_k device doubles, original orders of both marginals)
int circle_pair_marginal(mot_plan_s *P, int k, double *out);
void circle_destroy(mot_plan_s *P);
size_t circle_footprint(int K, const int64_t *n, int path, int precision);
// batch.cpp: a batch on an allocator of the caller's; sweeps enqueued without a wait
// max_lanes: streams the batched sweep may use (1: the batch's stream only)
int batch_create(mot_batch *out, mot_plan *plans, int32_t count, const mot_allocator *alloc, int max_lanes);
int batch_enqueue(mot_batch B, int sweeps);
const float2 *device_twiddle(int n);
}  // namespace mot
