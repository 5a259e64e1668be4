// Internal declarations of the MI355X multi-marginal Sinkhorn library.
// Shared by the host-side plan/scheduler code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mot.h"

namespace mot {

// ---------------------------------------------------------------------------------------
// Limits of the kernels.
constexpr int kMaxD = 3;
constexpr int kMaxTaps = 16;      // 2m taps per dimension, m <= 8
constexpr int kMaxN = 512;        // FFT grid per dimension
constexpr int kMinN = 16;
constexpr int kMaxChildren = 64;  // children per tree node handled by the node kernels
// Exponent slots (one int each, raised by atomicMax from every block of a node launch) sit
// one 128-byte line apart, so the atomics on different slots go to different L2 lines
// instead of queueing on one.
constexpr int kExpSlotStride = 32;

// ---------------------------------------------------------------------------------------
// Global-memory views of generic pointers: loads and stores through them are global
// (vector-memory counter only), so waiting for LDS results never also waits for
// outstanding global loads, as it would with flat instructions.
#define MOT_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const MOT_GLOBAL T *gp(const T *p)
{
    return (const MOT_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ MOT_GLOBAL T *gp(T *p)
{
    return (MOT_GLOBAL T *)p;
}

typedef float mot_f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld2(const float2 *p, int64_t i)  // global load of p[i]
{
    const mot_f32x2 v = ((const MOT_GLOBAL mot_f32x2 *)(const void *)p)[i];
    return make_float2(v[0], v[1]);
}
__device__ __forceinline__ void st2(float2 *p, int64_t i, float2 v)  // global store p[i] = v
{
    ((MOT_GLOBAL mot_f32x2 *)(void *)p)[i] = mot_f32x2{v.x, v.y};
}

// ---------------------------------------------------------------------------------------
// Device-side job descriptors.  Plain structs copied to device memory once per plan
// (or per batch); kernels read them through an item table of (job, sub-range) pairs.

// One Gaussian-kernel product out = K^{(t,s)} v (eq. fastsum-sum), by direct summation
// or by NFFT fast summation (Algorithm 4).  Vectors are FP64 in the marginals' binned
// (sorted) point order.
struct ProdJob {
    int32_t d, path, precision;
    int32_t diff;      // mixed direct / truncated paths: exponent formed in FP64
    // vectors
    const double *v;   // source vector, n_s entries
    int32_t *v_exp;    // slot holding max_j exponent(|v_j|) (atomicMax), reset per sweep
    double *out;       // target vector, n_t entries
    int64_t ns, nt;
    double *dpart;     // FP64 direct path: partial sums, dsplit x n_t (dsplit > 1 only)
    int32_t dsplit, pad_d;
    double eta;
    double ctr[3];     // centre of the point cloud (mixed direct path works relative to it)
    // direct path: sorted FP64 coordinates (n x d) of sources and targets
    const double *src_pts, *tgt_pts;
    // NFFT path, source and target binned layouts
    const float *src_win, *tgt_win;       // window rows, n x d x 16 (see window_rows_kernel)
    const int32_t *src_chunk_start, *tgt_chunk_start;  // point range of each chunk
    const int32_t *src_chunk_tile, *tgt_chunk_tile;    // box-relative tile of each chunk
    const int32_t *src_tile_chunks;       // [ntiles+1] chunk range of each box tile
    int32_t src_nchunks, tgt_nchunks;
    // host copies of the chunk bounds, used when launch items are built (never read on
    // the device)
    const int32_t *h_src_chunk_start, *h_tgt_chunk_start;
    // NFFT geometry
    int32_t n, M, m, T;
    int32_t L[3];      // active box extent per dimension (grid cells)
    int32_t lo[3];     // active box first grid index per dimension
    int32_t ntile[3];  // box tiles per dimension
    int32_t W;         // patch edge T + 2m - 1
    const float *D;    // multiplier on the half spectrum, layout [A2][A1][2M+1]
    const float2 *twiddle;  // exp(-2 pi i k / n), k < n/2
    // NFFT work buffers
    float *patches;    // src_nchunks * W^d
    float *grid;       // L0*L1*L2 real (box grid, coordinate 0 slowest)
    float2 *spec0, *spec1;
    int64_t spec_elems;
    // truncated path: cubic cells of side h from the origin glo, nc per dimension,
    // linearised row-major (coordinate 0 slowest); points are sorted by cell
    const int32_t *src_cell_off;            // [nc^d + 1] sorted source range of each cell
    const int32_t *h_src_cell_off, *h_tgt_cell_off;  // host copies (launch items only)
    int32_t nc, tw;    // cells per dimension; neighbour half-width in cells
    int32_t trunc_r, trunc_b;  // targets per lane and cells per run of the launch items
    double h, q2;      // cell side; (r_c / h)^2 enlarged by 1e-6 for cell rounding
    double glo[3];
};

// Node update descriptors for the tree sweep (Algorithm 2), FP64.
// DOWN: phi^k <- mu^k / (gamma_k (.) prod_{t in C_k} beta_t), S terms, and the
//       product sources u_c = phi^k (.) gamma_k (.) prod_{t in C_k \ c} beta_t.
// UP:   v_k = phi^k (.) prod_{t in C_k} beta_t (source of beta_k's product).
struct NodeJob {
    int32_t op;          // bit 0: down update, bit 1: down sources, bit 2: up source,
                         // bit 3: root (gamma = 1, extra S term), bit 4: marginal only,
                         // bit 5: free node (phi = 1, no S or error terms; Sec. 6.2)
    int32_t nchild;
    int64_t n;
    const double *mu;
    double *phi;
    const double *gamma;        // NULL for the root
    const double *const *beta;  // device array [nchild] of child beta vectors (length n)
    double *const *down_src;    // device array [nchild] of product source vectors
    int32_t *const *down_exp;   // device array [nchild] of exponent slots
    double *up_src;             // source vector of beta_k's product
    int32_t *up_exp;
    double *marg_out;           // marginal output (op bit 4)
    double *partial;            // per-item partial sums, 2 doubles per item
    int32_t *flag;              // set to 1 if an updated phi is not finite
    int32_t block0;             // first partial slot of this job
    int32_t pad;
};

// Sweep finalisation of one tree plan.
struct FinalJob {
    int64_t n0;
    const double *mu0, *phi0;
    const double *const *root_beta;  // device array [nchild]
    int32_t nchild, n_items;         // items of this job in the finalize launch
    const double *s_partial;         // node partial sums (2 per slot)
    int32_t n_partials, hist_cap;
    double *l1_partial;              // [n_items]
    int32_t *sweep_ctr, *flag, *flag_hist;
    double *S_hist, *err_hist;
    int32_t *exp_slots;
    int32_t n_exp_slots, pad;
    double eta;
};

// ---------------------------------------------------------------------------------------
// Kernel launchers (implemented in the .hip files).
int direct_targets_per_item(int precision);
// FP64 direct products: source ranges per job (partial sums added by a second kernel when
// above 1), from the target and source counts
int direct_source_split(int64_t nt, int64_t ns);
constexpr int kMaxTruncRows = 400;  // neighbour rows per truncated work item, (2w + 1)^(d-1)
// Truncated products: items int4 (job, first cell of a run of B cells of one row, first
// sorted target, count | B << 16), count <= 64 * R; R = 1, 2 or 4 (FP64: 1 or 2).
// wide != 0 (mixed precision): exponent formed in FP64 instead of FP32 coordinate differences
hipError_t launch_trunc(int d, int precision, int R, int wide, const ProdJob *jobs_dev, const int4 *items,
                        int n_items, hipStream_t s);
// diff != 0: mixed-precision pairs with the exponent formed in FP64 (small eta)
hipError_t launch_direct(int d, const ProdJob *jobs_dev, const int4 *items, int n_items, const int2 *red_items,
                         int n_red, int precision, int diff, hipStream_t s);
hipError_t launch_node(const NodeJob *jobs_dev, const int2 *items, int n_items, int max_children,
                       hipStream_t s);
hipError_t launch_finalize(const FinalJob *jobs, const int2 *items, int n_items, int n_jobs, hipStream_t s);
hipError_t launch_fill_int(int32_t *p, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_double(double *p, double value, int64_t count, hipStream_t s);
hipError_t launch_vec_exp(const double *v, int64_t n, int32_t *slot, hipStream_t s);
// Tree edge pair marginal: out[perm_a[i] * nb + perm_b[j]] = u_i exp(-|x_i - y_j|^2 / eta) w_j
hipError_t launch_tree_pair(const double *u, const double *xa, const int32_t *perm_a, int64_t na,
                            const double *w, const double *xb, const int32_t *perm_b, int64_t nb, int d,
                            double eta, double *out, hipStream_t s);
hipError_t launch_gather_rows(const double *src, const int32_t *perm, int64_t n, int d, double *dst,
                              hipStream_t s);
hipError_t launch_scatter_vec(const double *src, const int32_t *perm, int64_t n, double *dst,
                              hipStream_t s);

// Binning (a1): cells and tile ids, then a stable sort by tile.
hipError_t launch_bin_cells(int d, int64_t npts, const double *x, double s0, double s1, double s2,
                            double o0, double o1, double o2, int n, int T, int32_t *cell,
                            int32_t *tile, hipStream_t st);
size_t stable_tile_sort_scratch(int64_t npts, int64_t ntiles);
// Stable sort of points by tile; with cell != nullptr points of one tile are further
// ordered by their tile-relative cell (cell % T, T <= 16) in dimension sub_dim.
hipError_t stable_tile_sort(int64_t npts, const int32_t *tile, int64_t ntiles, int32_t *perm,
                            int32_t *tile_off, void *scratch, size_t scratch_bytes, hipStream_t st,
                            const int32_t *cell = nullptr, int d = 0, int sub_dim = 0, int T = 1);
// tile_off may be NULL (only perm is written).  After the sort, the sorted ranges of the
// tiles of an active box (t0 first tile, nt tiles per dimension, row-major) from the keys
// still in the scratch buffer: [lo[b], hi[b]).
hipError_t launch_box_tile_ranges(int64_t npts, const void *scratch, bool sub_keyed, int d, int tpd, const int *t0,
                                  const int *nt, int32_t *lo, int32_t *hi, hipStream_t st);
// Window rows of sorted points (n x d x 16 FP32), Kaiser-Bessel shape parameter b.
hipError_t launch_window_rows(int d, int64_t npts, const double *pts, double s, const double *o, int T,
                              int m, double b, float *rows, hipStream_t st);

// NFFT pipeline kernels (a2-a6).
constexpr int kNodeItemElems = 512;  // elements per node / finalisation item
constexpr int kFoldCellsPerItem = 128;  // box cells per fold item (one per thread)
// Lines of one FFT line-pass work item: one round of the block's four wavefronts, G =
// min(64, n/2) lanes per line (two real lines per complex line in the real-data passes 0
// and 4).  One round per item keeps an item's chain of loads, transforms and stores short.
constexpr int fft_lines_per_item(int kind, int n)
{
    return (kind == 0 || kind == 4 ? 2 : 1) * 4 * (64 / (n / 2 < 64 ? n / 2 : 64));
}
hipError_t launch_spread(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int max_patch_elems, hipStream_t s);  // d = 1, 2
// 3-D spreading; items int4 (job_0, .., job_{group-1}, chunk): group jobs (1..3) that spread
// from the same points.
hipError_t launch_spread3(int group, const ProdJob *jobs, const int4 *items, int n_items, hipStream_t s);
hipError_t launch_fold(int d, const ProdJob *jobs, const int2 *items, int n_items, hipStream_t s);
hipError_t launch_interp(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int max_patch_elems, hipStream_t s);
// FFT passes. kind: 0 = R2C along the fastest axis, 1 = forward C2C, 2 = fused
// forward + multiply + inverse, 3 = inverse C2C, 4 = C2R (with multiply when d == 1);
// 3-D slab chain: 6 = forward slab (R2C + C2C), 5 = fused pass on g0-major input,
// 7 = inverse slab (C2C + C2R).  Items: int4 (job, a2, a1, 0); slab items (job, g0, 0, 0).
// Twelve wavefronts per slab: a 128-point line takes one wavefront, so a slab of 46 box
// lines (23 complex) is two rounds and its 33 half-spectrum lines (M = 32) three.
constexpr int kSlabThreads = 768;
constexpr int kSlabLds = 48 * 1024;  // bytes of LDS for a slab's half spectrum L1 x (M+1)
// n = 0: the items' jobs have grids n <= 128 of several sizes (twiddle: the 128-point
// table); results equal those of the launch per size.
hipError_t launch_fft_pass(int kind, int n, const ProdJob *jobs, const int4 *items, int n_items,
                           const float2 *twiddle, hipStream_t s);

}  // namespace mot
