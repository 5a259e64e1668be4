// NFFT fast-summation kernels for gfx950: point binning, window rows, spreading into
// per-tile patches, the deterministic patch fold, and grid-to-point interpolation.
//
// Fast summation (Sec. 5, Algorithm 4) evaluates beta = F_t (kappa_hat (.) F*_s v).
// The adjoint NDFT F*_s is approximated by spreading v onto an oversampled grid of n
// cells per dimension with a Kaiser-Bessel window followed by an FFT; the NDFT F_t by an
// inverse FFT followed by interpolation with the same window.  Grid coordinates of a
// point x are u = x * s + o with s = n / (2 tau) (the 2 tau-periodic kernel becomes
// n-periodic); each point touches the 2m grid cells l = cell - m + 1 .. cell + m per
// dimension, cell = floor(u).
//
// Work decomposition: points are stable-sorted by tile (T^d cells).  A spreading work
// item is a chunk of points of one tile; it produces the tile's 16^d patch as a matrix
// product on the MFMA units and writes it once to global memory.  A fold pass sums the
// overlapping patches of neighbouring tiles into the box grid in a fixed order -- no
// atomics anywhere (gfx950 executes LDS float atomics lane by lane, far below LDS
// read rates), and the grid does not depend on which other jobs share a launch.
// Interpolation keeps a tile's patch of the result grid in registers and contracts it
// with the points' windows, again on the MFMA units.
#include "mot_internal.h"

namespace mot {

// ---------------------------------------------------------------------------------------
// Binning

__global__ void bin_cells_kernel(int d, int64_t npts, const double *__restrict__ x, double s0,
                                 double s1, double s2, double o0, double o1, double o2, int n,
                                 int T, int32_t *__restrict__ cell, int32_t *__restrict__ tile)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const double sc[3] = {s0, s1, s2}, oc[3] = {o0, o1, o2};
    int tpd = (n + T - 1) / T;
    int32_t t = 0;
    for (int c = 0; c < d; ++c) {
        // u = x*s + o with both operations rounded separately (no FMA contraction)
        double u = __dadd_rn(__dmul_rn(x[i * d + c], sc[c]), oc[c]);
        double f = floor(u);
        int ci = !(f >= 0.0) ? 0 : (f > (double)(n - 1) ? n - 1 : (int)f);
        cell[i * d + c] = ci;
        t = t * tpd + ci / T;
    }
    tile[i] = t;
}

hipError_t launch_bin_cells(int d, int64_t npts, const double *x, double s0, double s1, double s2,
                            double o0, double o1, double o2, int n, int T, int32_t *cell,
                            int32_t *tile, hipStream_t st)
{
    if (npts == 0) return hipSuccess;
    int blocks = (int)((npts + 255) / 256);
    hipLaunchKernelGGL(bin_cells_kernel, dim3(blocks), dim3(256), 0, st, d, npts, x, s0, s1, s2,
                       o0, o1, o2, n, T, cell, tile);
    return hipGetLastError();
}

// Stable sort by tile: bitonic sort of the unique 64-bit keys (tile << 32 | index).  With
// a sub-key (cell != nullptr) the key is ((tile << kSubBits | r) << 32 | index), where r
// is the point's tile-relative cell in dimension sub_dim: points of a tile then come in
// ascending r, ties in index order.
constexpr int kSubBits = 4;

__global__ void make_keys_kernel(int64_t npts, int64_t npad, const int32_t *__restrict__ tile,
                                 const int32_t *__restrict__ cell, int d, int sub_dim, int T,
                                 uint64_t *__restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    uint64_t hi = i < npts ? (uint64_t)(uint32_t)tile[i] : 0;
    if (cell != nullptr && i < npts) hi = (hi << kSubBits) | (uint64_t)(cell[i * d + sub_dim] % T);
    keys[i] = i < npts ? (hi << 32) | (uint64_t)i : ~0ull;
}

// One global compare-exchange step (k, j) of the bitonic network.
__global__ void bitonic_global_kernel(uint64_t *keys, int64_t npad, int64_t k, int64_t j)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    int64_t p = i ^ j;
    if (p > i) {
        uint64_t a = keys[i], b = keys[p];
        bool up = (i & k) == 0;
        if ((a > b) == up) {
            keys[i] = b;
            keys[p] = a;
        }
    }
}

// All steps with j < 1024 of stage k (or the full sort of 1024-element blocks when
// k_full != 0) inside LDS.
__global__ __launch_bounds__(512) void bitonic_local_kernel(uint64_t *keys, int64_t npad,
                                                            int64_t k, int k_full)
{
    __shared__ uint64_t sk[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) sk[t] = keys[base + t];
    __syncthreads();
    int64_t kk0 = k_full ? 2 : k, kk1 = k_full ? 1024 : k;
    for (int64_t kk = kk0; kk <= kk1; kk <<= 1) {
        int64_t j0 = k_full ? kk / 2 : 512;
        for (int64_t j = j0; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
                int p = t ^ (int)j;
                if (p > t) {
                    int64_t gi = base + t;
                    bool up = (gi & kk) == 0;
                    uint64_t a = sk[t], b = sk[p];
                    if ((a > b) == up) {
                        sk[t] = b;
                        sk[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) keys[base + t] = sk[t];
}

// perm[i] = index of the i-th sorted key (i < npts); tile_off[t] = first sorted position
// whose tile is >= t (t <= ntiles), by binary search over the sorted keys, so empty
// stretches of tiles cost nothing extra.
__global__ void keys_to_perm_kernel(int64_t npts, int64_t ntiles, const uint64_t *__restrict__ keys,
                                    int shift, int32_t *__restrict__ perm, int32_t *__restrict__ tile_off)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npts) perm[i] = (int32_t)(keys[i] & 0xffffffffull);
    if (tile_off != nullptr && i <= ntiles) {
        int64_t lo = 0, hi = npts;  // first position with tile >= i in [lo, hi]
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(keys[mid] >> shift) < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        tile_off[i] = (int32_t)lo;
    }
}

// Sorted ranges of the tiles of an active box after stable_tile_sort (whose sorted keys are
// still in the scratch buffer): box tile b (row-major over nt[0] x nt[1] x nt[2] tiles,
// coordinate 0 slowest, offset by t0 in the grid of tpd tiles per dimension) holds sorted
// positions [lo[b], hi[b]).  Binary searches as in keys_to_perm_kernel.
__global__ void box_tile_ranges_kernel(int64_t npts, const uint64_t *__restrict__ keys, int shift, int d, int tpd,
                                       int t00, int t01, int t02, int nt0, int nt1, int nt2, int64_t nbox,
                                       int32_t *__restrict__ lo, int32_t *__restrict__ hi)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const int t0[3] = {t00, t01, t02}, nt[3] = {nt0, nt1, nt2};
    int tc[3] = {0, 0, 0};
    int64_t rem = b;
    for (int c = d - 1; c >= 0; --c) {
        tc[c] = (int)(rem % nt[c]);
        rem /= nt[c];
    }
    int64_t gt = 0;
    for (int c = 0; c < d; ++c) gt = gt * tpd + (t0[c] + tc[c]);
    int64_t out[2];
    for (int q = 0; q < 2; ++q) {
        int64_t a = 0, e = npts;
        while (a < e) {
            const int64_t mid = (a + e) >> 1;
            if ((int64_t)(keys[mid] >> shift) < gt + q)
                a = mid + 1;
            else
                e = mid;
        }
        out[q] = a;
    }
    lo[b] = (int32_t)out[0];
    hi[b] = (int32_t)out[1];
}

hipError_t launch_box_tile_ranges(int64_t npts, const void *scratch, bool sub_keyed, int d, int tpd, const int *t0,
                                  const int *nt, int32_t *lo, int32_t *hi, hipStream_t st)
{
    int64_t nbox = 1;
    for (int c = 0; c < d; ++c) nbox *= nt[c];
    if (nbox == 0) return hipSuccess;
    hipLaunchKernelGGL(box_tile_ranges_kernel, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st, npts,
                       (const uint64_t *)scratch, sub_keyed ? 32 + kSubBits : 32, d, tpd, t0[0], d > 1 ? t0[1] : 0,
                       d > 2 ? t0[2] : 0, nt[0], d > 1 ? nt[1] : 1, d > 2 ? nt[2] : 1, nbox, lo, hi);
    return hipGetLastError();
}

size_t stable_tile_sort_scratch(int64_t npts, int64_t /*ntiles*/)
{
    int64_t npad = 1024;
    while (npad < npts) npad <<= 1;
    return (size_t)npad * sizeof(uint64_t);
}

hipError_t stable_tile_sort(int64_t npts, const int32_t *tile, int64_t ntiles, int32_t *perm,
                            int32_t *tile_off, void *scratch, size_t scratch_bytes, hipStream_t st,
                            const int32_t *cell, int d, int sub_dim, int T)
{
    int64_t npad = 1024;
    while (npad < npts) npad <<= 1;
    if (scratch_bytes < (size_t)npad * sizeof(uint64_t)) return hipErrorInvalidValue;
    if (cell != nullptr && (T > (1 << kSubBits) || sub_dim < 0 || sub_dim >= d ||
                            ntiles >= ((int64_t)1 << (32 - kSubBits))))
        return hipErrorInvalidValue;
    uint64_t *keys = (uint64_t *)scratch;
    int blocks = (int)((npad + 255) / 256);
    hipLaunchKernelGGL(make_keys_kernel, dim3(blocks), dim3(256), 0, st, npts, npad, tile, cell, d, sub_dim,
                       T, keys);
    int lblocks = (int)(npad / 1024);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(lblocks), dim3(512), 0, st, keys, npad,
                       (int64_t)0, 1);
    for (int64_t k = 2048; k <= npad; k <<= 1) {
        for (int64_t j = k / 2; j >= 1024; j >>= 1)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3(blocks), dim3(256), 0, st, keys, npad,
                               k, j);
        hipLaunchKernelGGL(bitonic_local_kernel, dim3(lblocks), dim3(512), 0, st, keys, npad, k, 0);
    }
    const int64_t nthr = std::max<int64_t>(npts, ntiles + 1);
    int pblocks = (int)((nthr + 255) / 256);
    hipLaunchKernelGGL(keys_to_perm_kernel, dim3(pblocks), dim3(256), 0, st, npts, ntiles, keys,
                       cell != nullptr ? 32 + kSubBits : 32, perm, tile_off);
    return hipGetLastError();
}

constexpr int kPatch = 16;  // patch edge T + 2m - 1 in cells

// ---------------------------------------------------------------------------------------
// Kaiser-Bessel window in grid units, normalised to 1 at s = 0:
//   psi(s) = (m / r) sinh(b r) / sinh(b m),  r = sqrt(m^2 - s^2),  |s| <= m,
// b = pi (2 - 1/sigma).  Its Fourier transform is I0(m sqrt(b^2 - w^2)), which the host
// uses for the spectral multiplier.
//
// Window rows.  A tile holds T = 17 - 2m cells per dimension, so the patch of cells its
// points touch is exactly 16 wide (T + 2m - 1).  For a point with tile-relative cell r
// and fractional offset f in dimension c, its row is the 16-vector
//   w_c[q] = psi(f + m - 1 + r - q)  if 0 <= q - r < 2m,  else 0,
// the weights of patch cells q = 0..15.  The rows depend on the points only, so they are
// evaluated once per plan in FP64 (rounded to FP32) and stored per point in binned
// order, rows[(i d + c) 16 + q]: every later product reads them instead of
// re-evaluating the window.
__global__ void window_rows_kernel(int d, int64_t npts, const double *__restrict__ pts, double s,
                                   double o0, double o1, double o2, int T, int m, double b,
                                   double inv_sinh_bm, float *__restrict__ rows)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts * d) return;
    const int64_t i = t / d;
    const int c = (int)(t - i * d);
    const double oc = c == 0 ? o0 : (c == 1 ? o1 : o2);
    // the binning's operations, so the cell is the one the point was sorted by
    const double u = __dadd_rn(__dmul_rn(pts[i * d + c], s), oc);
    const double fl = floor(u);
    const double f = u - fl;
    const int r = (int)fl % T;
    const double dm = m;
    float w[kPatch];
#pragma unroll
    for (int q = 0; q < kPatch; ++q) {
        const int j = q - r;
        float val = 0.0f;
        if (j >= 0 && j < 2 * m) {
            const double a = f + (dm - 1.0 - j);
            const double rr = sqrt(fmax(dm * dm - a * a, 0.0));
            const double br = b * rr;
            // sinh(b r) / r, with its series near r = 0 (the support edge)
            const double sr = br < 1e-4 ? b * (1.0 + br * br / 6.0) : sinh(br) / rr;
            val = (float)(dm * sr * inv_sinh_bm);
        }
        w[q] = val;
    }
    float4 *dst = reinterpret_cast<float4 *>(rows + t * kPatch);
#pragma unroll
    for (int q = 0; q < kPatch / 4; ++q) dst[q] = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

hipError_t launch_window_rows(int d, int64_t npts, const double *pts, double s, const double *o, int T,
                              int m, double b, float *rows, hipStream_t st)
{
    if (npts == 0) return hipSuccess;
    const int64_t work = npts * d;
    const int blocks = (int)((work + 255) / 256);
    hipLaunchKernelGGL(window_rows_kernel, dim3(blocks), dim3(256), 0, st, d, npts, pts, s, o[0],
                       d > 1 ? o[1] : 0.0, d > 2 ? o[2] : 0.0, T, m, b, 1.0 / sinh(b * m), rows);
    return hipGetLastError();
}

__device__ __forceinline__ int floor_div(int a, int b)  // floor(a / b) for b > 0
{
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int source_exponent(const ProdJob &J)
{
    const int e = *gp(J.v_exp);
    return e == INT32_MIN ? 0 : e;
}

// ---------------------------------------------------------------------------------------
// Spreading (a2) as a dense tile contraction on FP32 MFMA.
//
// For a chunk of points of one tile, the patch is
//   G[a][(b,c')] = sum_p X[a][p] Y[p][(b,c')],   X[a][p] = v_p w_0,p[a],
//   Y[p][(b,c')] = w_1,p[b] w_2,p[c'],
// a 16 x 256 x P product done with v_mfma_f32_16x16x4_f32: a step takes 4 points (the K
// dimension), one MFMA per b (16 output tiles of 16 x 16 over (a, c')).  Lane l holds
// A[a = l % 16][k = l / 16] and B[k = l / 16][c' = l % 16]; accumulator r of tile b holds
// G[a = 4 (l / 16) + r][b][c' = l % 16].  In 2-D the product is one 16 x 16 tile per step,
// in 1-D a plain sum over points.
//
// A block of kSpreadWaves wavefronts takes one chunk, which owns its patch: no atomics.
// In 1-D and 2-D wave w takes the 4-point steps w, w + kSpreadWaves, ... and the wave
// partials are added through LDS in a fixed order (pairwise halving); in 3-D the waves
// split the b tiles instead (spread3_kernel).  Either way a patch is the same whatever
// else shares the launch.
constexpr int kSpreadWaves = 4;
constexpr int kInterpWaves = 4;

// Points are staged through LDS kStage at a time: all threads of the block copy the
// stage's window rows (contiguous in memory for consecutive points) with 16-byte loads,
// one stage ahead of the MFMA work, so the row stream overlaps the contractions.
constexpr int kStage = 64;

// Staged 3-D window rows: a point's 48 floats are its rows for dimensions 0, 1, 2.  The
// dimension-1 row w_1[0..15] is stored transposed, position 4 i + q holding w_1[4 q + i], so
// that the four values w_1[w], w_1[w + 4], w_1[w + 8], w_1[w + 12] a wavefront w takes are
// one 16-byte read at position 4 w.  idx is the 16-byte piece (12 per point).
__device__ __forceinline__ void store_piece3(unsigned char *buf, int idx, f32x4 v)
{
    const int piece = idx % 12;
    if (piece >= 4 && piece < 8) {
        float *row = reinterpret_cast<float *>(buf) + (idx - piece + 4) * 4;
        const int q = piece - 4;
        row[q] = v[0];
        row[4 + q] = v[1];
        row[8 + q] = v[2];
        row[12 + q] = v[3];
    } else {
        reinterpret_cast<f32x4 *>(buf)[idx] = v;
    }
}

template <int D, bool WITH_V>
struct Stage {
    static constexpr int kRow4 = kStage * D * kPatch / 4;  // 16-byte row pieces per stage
    static constexpr int kPer = (kRow4 + 255) / 256;        // per thread (256 threads)
    static constexpr int kBytes = kRow4 * 16 + (WITH_V ? kStage * 4 : 0);
    f32x4 r[kPer];
    double v;  // scaled only when stored, so that the loads stay in flight

    // Registers <- global: points pb .. pb + kStage - 1 (zeros past p1), and for
    // spreading the source values.
    __device__ __forceinline__ void load(const float *rows, const double *vsrc, int64_t pb, int64_t p1)
    {
        const MOT_GLOBAL f32x4 *g = reinterpret_cast<const MOT_GLOBAL f32x4 *>(gp(rows)) + pb * (D * 4);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + 256 * i;
            r[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (idx < kRow4 && pb + idx / (D * 4) < p1) r[i] = g[idx];
        }
        if constexpr (WITH_V) {
            v = 0.0;
            const int64_t p = pb + threadIdx.x;
            if (threadIdx.x < kStage && p < p1) v = gp(vsrc)[p];
        }
    }
    // LDS <- registers; source values are stored as FP32 v 2^-e.  In 3-D the dimension-1
    // row of a point is stored transposed (see store_rows3).
    __device__ __forceinline__ void store(unsigned char *buf, int e) const
    {
        f32x4 *rl = reinterpret_cast<f32x4 *>(buf);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + 256 * i;
            if (idx < kRow4) {
                if constexpr (D == 3)
                    store_piece3(buf, idx, r[i]);
                else
                    rl[idx] = r[i];
            }
        }
        if constexpr (WITH_V)
            if (threadIdx.x < kStage) reinterpret_cast<float *>(buf + kRow4 * 16)[threadIdx.x] = (float)ldexp(v, -e);
    }
};

template <int D>
__global__ __launch_bounds__(64 * kSpreadWaves, 4) void spread_kernel(const ProdJob *__restrict__ jobs,
                                                                   const int2 *__restrict__ items,
                                                                   int n_items)
{
    static_assert(kSpreadWaves == 4, "staging assumes 256 threads");
    static_assert(D < 3, "3-D spreading is spread3_kernel");
    using St = Stage<D, true>;
    constexpr int kRed = (kSpreadWaves / 2) * 64 * 16;
    constexpr int kSmem = 2 * St::kBytes > kRed ? 2 * St::kBytes : kRed;
    __shared__ __align__(16) unsigned char smem[kSmem];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int64_t p0 = gp(J.src_chunk_start)[itm.y], p1 = gp(J.src_chunk_start)[itm.y + 1];
        const int e = source_exponent(J);
        const int nstages = (int)((p1 - p0 + kStage - 1) / kStage);
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        St stg;
        stg.load(J.src_win, J.v, p0, p1);
        stg.store(smem, e);
        __syncthreads();
        for (int k = 0; k < nstages; ++k) {
            const bool more = k + 1 < nstages;
            if (more) stg.load(J.src_win, J.v, p0 + (int64_t)(k + 1) * kStage, p1);
            const unsigned char *buf = smem + (k & 1) * St::kBytes;
            const float *rl = reinterpret_cast<const float *>(buf);
            const float *vl = reinterpret_cast<const float *>(buf + St::kRow4 * 16);
            // this wave's 4-point steps of the stage: points 4 j + lane group, j = wave + 4 i
#pragma unroll 1
            for (int i = 0; i < kStage / 16; ++i) {
                const int pi = 4 * (wave + 4 * i) + lk;
                const float *row = rl + pi * (D * kPatch);
                const float x = vl[pi] * row[li];
                if constexpr (D == 2)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x, row[kPatch + li], acc, 0, 0, 0);
                else
                    acc[0] += x;
            }
            if (more) stg.store(smem + ((k + 1) & 1) * St::kBytes, e);
            __syncthreads();
        }
        if constexpr (D == 1) {
            // sum over the four points of a step (lane groups), then over waves
            float a1 = acc[0];
            a1 += __shfl_xor(a1, 16);
            a1 += __shfl_xor(a1, 32);
            acc[0] = a1;
        }
        // wave partials: wave w < half adds wave w + half, halving until wave 0 holds the
        // patch (the staging buffers are free: the last stage ended with a barrier)
        f32x4(*red)[64] = reinterpret_cast<f32x4(*)[64]>(smem);
#pragma unroll
        for (int half = kSpreadWaves / 2; half >= 1; half >>= 1) {
            if (wave >= half && wave < 2 * half) red[wave - half][lane] = acc;
            __syncthreads();
            if (wave < half) acc += red[wave][lane];
            __syncthreads();
        }
        if (wave == 0) {
            MOT_GLOBAL float *out = gp(J.patches) + (int64_t)itm.y * (D == 2 ? 256 : 16);
            if constexpr (D == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) out[(4 * lk + r) * 16 + li] = acc[r];
            } else {
                if (lk == 0) out[li] = acc[0];
            }
        }
    }
}

// 3-D spreading: the 16 b tiles are split over the block's waves.  Wave w accumulates
// tiles b = w, w + 4, w + 8, w + 12 over every point of the chunk (one MFMA per tile and
// 4-point step, in point order), so a wave holds 4 accumulators per job rather than 16, no
// partial patches are combined, and every wave writes its own quarter of the patch.  Any
// 2m = 12 consecutive b values hold three of each wave's four, so when the points of a step
// share their window support every wave skips one step and none waits at the stage
// barrier for the others (with quarters of consecutive b values the two middle waves
// never skip).
//
// An item is (job_0, .., job_{G-1}, chunk): G jobs that spread different values from the
// same points (the down products of a node's children).  They share the chunk's window
// rows, so the rows are staged once, and the B operand w_1,p[b] w_2,p[c'] and the test for
// a zero step are formed once for G MFMAs.  Each job's patch is accumulated exactly as it
// would be on its own.
template <int G>
struct SpreadStage3 {
    static constexpr int kRow4 = kStage * 3 * kPatch / 4;  // 16-byte row pieces per stage
    static constexpr int kPer = (kRow4 + 255) / 256;        // per thread (256 threads)
    static constexpr int kBytes = kRow4 * 16 + G * kStage * 4;
    f32x4 r[kPer];
    double v;  // value of job q = threadIdx.x / kStage (the wave), scaled only when stored

    // Registers <- global: points pb .. pb + kStage - 1 (zeros past p1); wave q < G loads
    // job q's values from vq (the job's pointer, selected by the caller).
    __device__ __forceinline__ void load(const float *rows, const double *vq, int64_t pb, int64_t p1)
    {
        const MOT_GLOBAL f32x4 *g = reinterpret_cast<const MOT_GLOBAL f32x4 *>(gp(rows)) + pb * 12;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + 256 * i;
            r[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (idx < kRow4 && pb + idx / 12 < p1) r[i] = g[idx];
        }
        v = 0.0;
        const int64_t p = pb + (threadIdx.x % kStage);
        if (threadIdx.x / kStage < G && p < p1) v = gp(vq)[p];
    }
    // LDS <- registers (dimension-1 rows transposed, store_piece3); job q's values are
    // stored as FP32 v 2^-eq.
    __device__ __forceinline__ void store(unsigned char *buf, int eq) const
    {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + 256 * i;
            if (idx < kRow4) store_piece3(buf, idx, r[i]);
        }
        if (threadIdx.x / kStage < G) reinterpret_cast<float *>(buf + kRow4 * 16)[threadIdx.x] = (float)ldexp(v, -eq);
    }
};

template <int G>
__global__ __launch_bounds__(64 * kSpreadWaves, G == 1 ? 6 : (G == 2 ? 5 : 4)) void spread3_kernel(const ProdJob *__restrict__ jobs,
                                                                                 const int4 *__restrict__ items,
                                                                                 int n_items)
{
    static_assert(kSpreadWaves == 4 && kStage == 64 && G >= 1 && G <= 3,
                  "one wave per group of 4 b tiles and per job's stage values; up to 3 jobs");
    using St = SpreadStage3<G>;
    __shared__ __align__(16) unsigned char smem[2 * St::kBytes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const int c = itm.w;
        const ProdJob &J = jobs[itm.x];  // the points, shared by the item's jobs
        const int64_t p0 = gp(J.src_chunk_start)[c], p1 = gp(J.src_chunk_start)[c + 1];
        // wave q < G stages job q's values: its pointer and exponent, selected by wave
        const int jq = wave == 0 ? itm.x : (wave == 1 ? itm.y : itm.z);
        const int q_job = wave < G ? jq : itm.x;
        const double *vq = jobs[q_job].v;
        const int eq = source_exponent(jobs[q_job]);
        const int nstages = (int)((p1 - p0 + kStage - 1) / kStage);
        f32x4 acc[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[g][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        St stg;
        stg.load(J.src_win, vq, p0, p1);
        stg.store(smem, eq);
        __syncthreads();
        for (int k = 0; k < nstages; ++k) {
            const bool more = k + 1 < nstages;
            if (more) stg.load(J.src_win, vq, p0 + (int64_t)(k + 1) * kStage, p1);
            const unsigned char *buf = smem + (k & 1) * St::kBytes;
            const float *rl = reinterpret_cast<const float *>(buf);
            const float *vl = reinterpret_cast<const float *>(buf + St::kRow4 * 16);
#pragma unroll 2
            for (int j = 0; j < kStage / 4; ++j) {
                const int pi = 4 * j + lk;  // point of lane group lk in step j
                const float *row = rl + pi * (3 * kPatch);
                const float w0 = row[li];
                float x[G];
#pragma unroll
                for (int g = 0; g < G; ++g) x[g] = vl[g * kStage + pi] * w0;
                const float w2 = row[2 * kPatch + li];
                // w_1,p[b] for the wave's b = wave + 4 u (one read of the transposed row)
                const f32x4 w1 = reinterpret_cast<const f32x4 *>(row + kPatch)[wave];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    // B is zero when b = w + 4 u is outside the window of all four points:
                    // the products would add exact zeros
                    if (__any(w1[u] != 0.0f)) {
                        const float bu = w1[u] * w2;
#pragma unroll
                        for (int g = 0; g < G; ++g)
                            acc[g][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[g], bu, acc[g][u], 0, 0, 0);
                    }
            }
            if (more) stg.store(smem + ((k + 1) & 1) * St::kBytes, eq);
            __syncthreads();
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int jg = g == 0 ? itm.x : (g == 1 ? itm.y : itm.z);
            MOT_GLOBAL float *out = gp(jobs[jg].patches) + (int64_t)c * 4096;
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) out[((4 * lk + r) * 16 + wave + 4 * u) * 16 + li] = acc[g][u][r];
        }
    }
}

constexpr int kFoldMaxCover = 4;

// Fold (a2, second half): box grid cell g = sum of the patches covering it, tiles in
// ascending order and chunks in ascending order within a tile.  One thread folds one
// cell; an item is kFoldCellsPerItem consecutive cells of the box in row-major order
// (lines of the last dimension back to back, so every lane has a cell even when a line
// is shorter than a wavefront); item = (job, first cell).  The job's tile -> chunk table
// is staged in LDS when it fits, so the chunk lookups of a thread's covering tiles cost
// LDS rather than global latency.
constexpr int kFoldTab = 2048;  // tile -> chunk table entries staged in LDS

// One item of the fold; tch is the job's tile -> chunk table (in LDS when it fits).
template <int D, class Tab>
__device__ __forceinline__ void fold_item(const ProdJob &J, int f0, Tab tch)
{
    const int W = J.W, T = J.T, Ll = J.L[D - 1], ntl = J.ntile[D - 1];
    const int nl = D == 3 ? J.L[0] * J.L[1] : (D == 2 ? J.L[0] : 1);
    const int f = f0 + (int)threadIdx.x;
    if (f >= nl * Ll) return;
    const int line = f / Ll, g = f - line * Ll;
    int gu[2] = {0, 0};  // line coordinates in the leading dimensions
    if (D == 3) {
        gu[0] = line / J.L[1];
        gu[1] = line - gu[0] * J.L[1];
    } else if (D == 2) {
        gu[0] = line;
    }
    int tlo[2] = {0, 0}, thi[2] = {0, 0};
    for (int c = 0; c < D - 1; ++c) {
        tlo[c] = max(0, floor_div(gu[c] - W + T, T));  // ceil((g - W + 1) / T)
        thi[c] = min(J.ntile[c] - 1, gu[c] / T);
    }
    const int pe = D == 3 ? W * W * W : (D == 2 ? W * W : W);
    const MOT_GLOBAL float *pat = gp(J.patches);
    const int t2lo = max(0, floor_div(g - W + T, T)), t2hi = min(ntl - 1, g / T);
    float acc = 0.0f;
    if (W <= kFoldMaxCover * T) {
        // at most kFoldMaxCover covering tiles per dimension: the chunk ranges and first
        // patches of all (t1, t2) pairs of a t0 are loaded together, then added in the
        // fixed order
        constexpr int NU = D == 3 ? kFoldMaxCover : 1;
        // t0-invariant parts of the tile index and patch offset of candidate (u, k):
        //   tile = t0 nt1 ntl + tl_b + u ntl + k,
        //   loc  = (gu0 - t0 T) W^2 + loc_b - u T W - k T
        const int nt1 = D == 3 ? J.ntile[1] : 1;
        const int vu = D == 3 ? thi[1] - tlo[1] : 0, vk = t2hi - t2lo;
        const int tl_b = (D == 3 ? tlo[1] * ntl : 0) + t2lo;
        const int loc_b = (D == 3 ? (gu[1] - tlo[1] * T) * W : 0) + (g - t2lo * T);
        const int W2 = D == 1 ? 0 : (D == 2 ? W : W * W);
        for (int t0 = tlo[0]; t0 <= thi[0]; ++t0) {
            const int tl0 = t0 * nt1 * ntl + tl_b;
            const int loc0 = (gu[0] - t0 * T) * W2 + loc_b;
            int c0[NU][kFoldMaxCover], c1[NU][kFoldMaxCover];
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int k = 0; k < kFoldMaxCover; ++k) {
                    const bool ok = u <= vu && k <= vk;
                    const int tl = tl0 + u * ntl + k;
                    c0[u][k] = ok ? tch[tl] : 0;
                    c1[u][k] = ok ? tch[tl + 1] : 0;
                }
            float first[NU][kFoldMaxCover];
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int k = 0; k < kFoldMaxCover; ++k)
                    first[u][k] = c1[u][k] > c0[u][k] ? pat[(int64_t)c0[u][k] * pe + (loc0 - u * T * W - k * T)] : 0.0f;
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int k = 0; k < kFoldMaxCover; ++k) {
                    acc += first[u][k];  // +0 for an absent tile leaves the sum unchanged
                    for (int ch = c0[u][k] + 1; ch < c1[u][k]; ++ch)
                        acc += pat[(int64_t)ch * pe + (loc0 - u * T * W - k * T)];
                }
        }
    } else {
        for (int t0 = tlo[0]; t0 <= thi[0]; ++t0)
            for (int t1 = tlo[1]; t1 <= thi[1]; ++t1) {
                int lead_tile = 0, lead_loc = 0;
                if constexpr (D == 3) {
                    lead_tile = t0 * J.ntile[1] + t1;
                    lead_loc = (gu[0] - t0 * T) * W + (gu[1] - t1 * T);
                } else if constexpr (D == 2) {
                    lead_tile = t0;
                    lead_loc = gu[0] - t0 * T;
                }
                for (int t2 = t2lo; t2 <= t2hi; ++t2) {
                    const int tl = lead_tile * ntl + t2;
                    const int lc = lead_loc * W + (g - t2 * T);
                    const int ca = tch[tl], cb = tch[tl + 1];
                    for (int ch = ca; ch < cb; ++ch) acc += pat[(int64_t)ch * pe + lc];
                }
            }
    }
    gp(J.grid)[(int64_t)line * Ll + g] = acc;
}

// D = 0: every item takes its job's own d (batches of plans of several dimensions).
template <int D>
__global__ __launch_bounds__(kFoldCellsPerItem) void fold_kernel(const ProdJob *__restrict__ jobs,
                                                                 const int2 *__restrict__ items, int n_items)
{
    __shared__ int32_t s_tab[kFoldTab];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int d = D > 0 ? D : J.d;
        int ntab = 1;
        for (int c = 0; c < d; ++c) ntab *= J.ntile[c];
        ++ntab;
        const bool staged = ntab <= kFoldTab;
        if (staged) {
            __syncthreads();  // the previous item's reads of the table are done
            const MOT_GLOBAL int32_t *tg = gp(J.src_tile_chunks);
            for (int i = threadIdx.x; i < ntab; i += blockDim.x) s_tab[i] = tg[i];
            __syncthreads();
        }
        const int32_t *lt = static_cast<const int32_t *>(s_tab);
        const MOT_GLOBAL int32_t *gt = gp(J.src_tile_chunks);
        if (d == 3) {
            if (staged) fold_item<3>(J, itm.y, lt); else fold_item<3>(J, itm.y, gt);
        } else if (d == 2) {
            if (staged) fold_item<2>(J, itm.y, lt); else fold_item<2>(J, itm.y, gt);
        } else {
            if (staged) fold_item<1>(J, itm.y, lt); else fold_item<1>(J, itm.y, gt);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Interpolation (a6) as the transposed contraction on FP32 MFMA.
//
// For 16 target points of one tile and the 16^d patch G of the result grid over the
// tile, Z[a][p] = sum_{(b,c')} G[a][(b,c')] Y[(b,c')][p] with Y[(b,c')][p] =
// w_1,p[b] w_2,p[c'], then beta_p = sum_a w_0,p[a] Z[a][p].  Step s of the 64-step MFMA
// chain covers b = s / 4 and, for lane group g = l / 16, c' = 4 g + s % 4: lane l holds
// A[a = l % 16][k] = G[a][b][c'] and B[k][p = l % 16] = w_1,p[b] w_2,p[c'].  The grid
// values are the same for every point of the tile, so they stay in registers for the whole
// chunk.  Accumulator r holds Z[a = 4 g + r][p = l % 16], so each lane owns one point: the
// last contraction over a takes the lane's four a and then adds the four lane groups.  In
// 2-D the chain has 4 steps (k = b = 4 g + s); in 1-D one lane takes one point.
// out = 2^e beta, e the exponent the source was scaled by.
//
// A block of kInterpWaves wavefronts takes one chunk.  In 2-D wave w takes the 16-point
// groups w, w + kInterpWaves, ... (one per stage), in 1-D 64-point groups; 3-D
// interpolation splits the b values over the waves instead (interp3_kernel).
template <int D>
__global__ __launch_bounds__(64 * kInterpWaves, 4) void interp_kernel(const ProdJob *__restrict__ jobs,
                                                                   const int2 *__restrict__ items,
                                                                   int n_items)
{
    static_assert(kInterpWaves == 4 && kStage == 16 * kInterpWaves, "one 16-point group per wave and stage");
    static_assert(D < 3, "3-D interpolation is interp3_kernel");
    constexpr int NB = D == 2 ? 4 : 16;  // B values per lane
    using St = Stage<D, false>;
    __shared__ __align__(16) unsigned char smem[D == 1 ? 16 : 2 * St::kBytes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int T = J.T;
        int tc[3] = {0, 0, 0};
        {
            int rem = gp(J.tgt_chunk_tile)[itm.y];
#pragma unroll
            for (int c = D - 1; c >= 0; --c) {
                tc[c] = rem % J.ntile[c];
                rem /= J.ntile[c];
            }
        }
        const MOT_GLOBAL float *grid = gp(J.grid);
        float Bv[NB];
        if constexpr (D == 2) {
            const int64_t base = (int64_t)(tc[0] * T + li) * J.L[1] + tc[1] * T + 4 * lk;
#pragma unroll
            for (int s = 0; s < 4; ++s) Bv[s] = grid[base + s];
        } else {
#pragma unroll
            for (int a = 0; a < 16; ++a) Bv[a] = grid[tc[0] * T + a];
        }
        const int e = source_exponent(J);
        const int64_t p0 = gp(J.tgt_chunk_start)[itm.y], p1 = gp(J.tgt_chunk_start)[itm.y + 1];
        MOT_GLOBAL double *out = gp(J.out);
        if constexpr (D == 1) {
            const MOT_GLOBAL f32x4 *rows = reinterpret_cast<const MOT_GLOBAL f32x4 *>(gp(J.tgt_win));
            for (int64_t p = p0 + threadIdx.x; p < p1; p += 64 * kInterpWaves) {
                float s = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 w = rows[p * 4 + q];
                    s += w[0] * Bv[4 * q] + w[1] * Bv[4 * q + 1] + w[2] * Bv[4 * q + 2] + w[3] * Bv[4 * q + 3];
                }
                out[p] = ldexp((double)s, e);
            }
        } else {
            const int nstages = (int)((p1 - p0 + kStage - 1) / kStage);
            St stg;
            stg.load(J.tgt_win, nullptr, p0, p1);
            stg.store(smem, 0);
            __syncthreads();
            for (int k = 0; k < nstages; ++k) {
                const bool more = k + 1 < nstages;
                if (more) stg.load(J.tgt_win, nullptr, p0 + (int64_t)(k + 1) * kStage, p1);
                const float *rl = reinterpret_cast<const float *>(smem + (k & 1) * St::kBytes);
                // this wave's group: stage points 16 wave .. 16 wave + 15
                const float *grow = rl + (16 * wave) * (D * kPatch);
                const float *row = grow + li * (D * kPatch);  // point l % 16
                // grid values as the A operand, window values as B: acc[r] = Z[a = 4 lk + r][p]
                // for the lane's point p = l % 16
                f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                const f32x4 wb = reinterpret_cast<const f32x4 *>(row + kPatch)[lk];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[0], wb[0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[1], wb[1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[2], wb[2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[3], wb[3], acc, 0, 0, 0);
                // beta_p = sum_a w_0,p[a] Z[a][p]: the lane's four a, then the four lane groups
                const f32x4 wx = reinterpret_cast<const f32x4 *>(row)[lk];
                float z = (acc[0] * wx[0] + acc[1] * wx[1]) + (acc[2] * wx[2] + acc[3] * wx[3]);
                z += __shfl_xor(z, 16);
                z += __shfl_xor(z, 32);
                const int64_t p = p0 + (int64_t)k * kStage + 16 * wave + li;
                if (lk == 0 && p < p1) out[p] = ldexp((double)z, e);
                if (more) stg.store(smem + ((k + 1) & 1) * St::kBytes, 0);
                __syncthreads();
            }
        }
    }
}

// 3-D interpolation with the 16 b values of the contraction split over the block's waves.
// Wave w holds B only for b = w, w + 4, w + 8, w + 12 (16 registers rather than 64; a
// twelve-wide window covers three of each wave's four b, so the waves skip alike) and takes
// all four 16-point groups of a stage.  The grid values are the MFMA's A operand and the
// window products its B operand, so for group g lane l's accumulators give
// Z_w[a = 4 (l / 16) + r][p = 16 g + l % 16], the part of Z from the wave's b values, with
// the point along the lanes.  Each lane weights its four a by the point's w_0,p[a] and the
// four lane groups are added by two lane exchanges; the four waves' partial sums of a
// point are added in wave order through LDS after the stage's barrier, and wave 0 stores
// out = 2^e beta.  (With the bound of 6 blocks per CU the compiler keeps one register pair
// in scratch, stored once per wavefront and read once per item; the allocation it makes
// without that spill, under a bound of 5, measured 4 % slower.)
__global__ __launch_bounds__(64 * kInterpWaves, 6) void interp3_kernel(const ProdJob *__restrict__ jobs,
                                                                   const int2 *__restrict__ items,
                                                                   int n_items)
{
    static_assert(kInterpWaves == 4 && kStage == 64, "four 16-point groups and four b quarters per stage");
    using St = Stage<3, false>;
    __shared__ __align__(16) unsigned char smem[2 * St::kBytes];
    __shared__ float zb[2][kInterpWaves][kStage];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int T = J.T;
        int tc[3] = {0, 0, 0};
        {
            int rem = gp(J.tgt_chunk_tile)[itm.y];
#pragma unroll
            for (int c = 2; c >= 0; --c) {
                tc[c] = rem % J.ntile[c];
                rem /= J.ntile[c];
            }
        }
        // A[a = l % 16][k = (b, c')] = G[a][b][c'] for b = wave + 4 bb, c' = 4 lk + s
        const MOT_GLOBAL float *grid = gp(J.grid);
        float Bv[16];
        {
            const int64_t base =
                ((int64_t)(tc[0] * T + li) * J.L[1] + tc[1] * T + wave) * J.L[2] + tc[2] * T + 4 * lk;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
#pragma unroll
                for (int s = 0; s < 4; ++s) Bv[4 * bb + s] = grid[base + (int64_t)(4 * bb) * J.L[2] + s];
        }
        const int e = source_exponent(J);
        const int64_t p0 = gp(J.tgt_chunk_start)[itm.y], p1 = gp(J.tgt_chunk_start)[itm.y + 1];
        MOT_GLOBAL double *out = gp(J.out);
        const int nstages = (int)((p1 - p0 + kStage - 1) / kStage);
        St stg;
        stg.load(J.tgt_win, nullptr, p0, p1);
        stg.store(smem, 0);
        __syncthreads();
        for (int k = 0; k < nstages; ++k) {
            const bool more = k + 1 < nstages;
            if (more) stg.load(J.tgt_win, nullptr, p0 + (int64_t)(k + 1) * kStage, p1);
            const float *rl = reinterpret_cast<const float *>(smem + (k & 1) * St::kBytes);
#pragma unroll 1
            for (int g = 0; g < 4; ++g) {
                const float *row = rl + (16 * g + li) * (3 * kPatch);  // point 16 g + l % 16
                const f32x4 wy = reinterpret_cast<const f32x4 *>(row + kPatch)[wave];  // transposed row
                const f32x4 wz = reinterpret_cast<const f32x4 *>(row + 2 * kPatch)[lk];
                f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    // B is zero when b is outside the window of all 16 points: the four
                    // products would add exact zeros
                    if (!__any(wy[bb] != 0.0f)) continue;
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[4 * bb], wy[bb] * wz[0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[4 * bb + 1], wy[bb] * wz[1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[4 * bb + 2], wy[bb] * wz[2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[4 * bb + 3], wy[bb] * wz[3], acc, 0, 0, 0);
                }
                // acc[r] = Z_w[a = 4 lk + r][p = 16 g + l % 16]: weight by the point's own
                // w_0,p[4 lk .. 4 lk + 3], then add the four lane groups (lanes l ^ 16, l ^ 32)
                const f32x4 wx = reinterpret_cast<const f32x4 *>(row)[lk];
                float z = (acc[0] * wx[0] + acc[1] * wx[1]) + (acc[2] * wx[2] + acc[3] * wx[3]);
                z += __shfl_xor(z, 16);
                z += __shfl_xor(z, 32);
                if (lk == 0) zb[k & 1][wave][16 * g + li] = z;
            }
            if (more) stg.store(smem + ((k + 1) & 1) * St::kBytes, 0);
            __syncthreads();
            if (wave == 0) {
                const int64_t p = p0 + (int64_t)k * kStage + lane;
                const float s = ((zb[k & 1][0][lane] + zb[k & 1][1][lane]) + zb[k & 1][2][lane]) + zb[k & 1][3][lane];
                if (p < p1) out[p] = ldexp((double)s, e);
            }
        }
    }
}

static int nfft_grid(int n_items)
{
    return n_items < 65535 ? n_items : 65535;
}

hipError_t launch_spread3(int group, const ProdJob *jobs, const int4 *items, int n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid(nfft_grid(n_items)), block(64 * kSpreadWaves);
    if (group == 3)
        hipLaunchKernelGGL(spread3_kernel<3>, grid, block, 0, s, jobs, items, n_items);
    else if (group == 2)
        hipLaunchKernelGGL(spread3_kernel<2>, grid, block, 0, s, jobs, items, n_items);
    else if (group == 1)
        hipLaunchKernelGGL(spread3_kernel<1>, grid, block, 0, s, jobs, items, n_items);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_spread(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int /*max_patch_elems*/, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid(nfft_grid(n_items)), block(64 * kSpreadWaves);
    if (d == 3)
        return hipErrorInvalidValue;  // 3-D items are grouped: launch_spread3
    else if (d == 2)
        hipLaunchKernelGGL(spread_kernel<2>, grid, block, 0, s, jobs, items, n_items);
    else
        hipLaunchKernelGGL(spread_kernel<1>, grid, block, 0, s, jobs, items, n_items);
    return hipGetLastError();
}

hipError_t launch_fold(int d, const ProdJob *jobs, const int2 *items, int n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (d == 0)
        hipLaunchKernelGGL(fold_kernel<0>, dim3(nfft_grid(n_items)), dim3(kFoldCellsPerItem), 0, s, jobs, items,
                           n_items);
    else if (d == 3)
        hipLaunchKernelGGL(fold_kernel<3>, dim3(nfft_grid(n_items)), dim3(kFoldCellsPerItem), 0, s, jobs, items,
                           n_items);
    else if (d == 2)
        hipLaunchKernelGGL(fold_kernel<2>, dim3(nfft_grid(n_items)), dim3(kFoldCellsPerItem), 0, s, jobs, items,
                           n_items);
    else
        hipLaunchKernelGGL(fold_kernel<1>, dim3(nfft_grid(n_items)), dim3(kFoldCellsPerItem), 0, s, jobs, items,
                           n_items);
    return hipGetLastError();
}

hipError_t launch_interp(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int /*max_patch_elems*/, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid(nfft_grid(n_items)), block(64 * kInterpWaves);
    if (d == 3)
        hipLaunchKernelGGL(interp3_kernel, grid, block, 0, s, jobs, items, n_items);
    else if (d == 2)
        hipLaunchKernelGGL(interp_kernel<2>, grid, block, 0, s, jobs, items, n_items);
    else
        hipLaunchKernelGGL(interp_kernel<1>, grid, block, 0, s, jobs, items, n_items);
    return hipGetLastError();
}

}  // namespace mot
