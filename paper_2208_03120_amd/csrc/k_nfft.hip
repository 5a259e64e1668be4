// NFFT fast-summation kernels for gfx950: point binning, window spreading into LDS
// patches, the deterministic patch fold, and grid-to-point interpolation.
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
// Interpolation loads a tile's patch of the result grid into LDS and contracts it with
// the points' windows, again on the MFMA units.
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

// Stable sort by tile: bitonic sort of the unique 64-bit keys (tile << 32 | index).
__global__ void make_keys_kernel(int64_t npts, int64_t npad, const int32_t *__restrict__ tile,
                                 uint64_t *__restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    keys[i] = i < npts ? (((uint64_t)(uint32_t)tile[i]) << 32) | (uint64_t)i : ~0ull;
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

__global__ void keys_to_perm_kernel(int64_t npts, int64_t ntiles, const uint64_t *__restrict__ keys,
                                    int32_t *__restrict__ perm, int32_t *__restrict__ tile_off)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > npts) return;
    int64_t t_prev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> 32);
    int64_t t_cur = i == npts ? ntiles : (int64_t)(keys[i] >> 32);
    if (i < npts) perm[i] = (int32_t)(keys[i] & 0xffffffffull);
    for (int64_t t = t_prev + 1; t <= t_cur; ++t) tile_off[t] = (int32_t)i;
}

size_t stable_tile_sort_scratch(int64_t npts, int64_t /*ntiles*/)
{
    int64_t npad = 1024;
    while (npad < npts) npad <<= 1;
    return (size_t)npad * sizeof(uint64_t);
}

hipError_t stable_tile_sort(int64_t npts, const int32_t *tile, int64_t ntiles, int32_t *perm,
                            int32_t *tile_off, void *scratch, size_t scratch_bytes, hipStream_t st)
{
    int64_t npad = 1024;
    while (npad < npts) npad <<= 1;
    if (scratch_bytes < (size_t)npad * sizeof(uint64_t)) return hipErrorInvalidValue;
    uint64_t *keys = (uint64_t *)scratch;
    int blocks = (int)((npad + 255) / 256);
    hipLaunchKernelGGL(make_keys_kernel, dim3(blocks), dim3(256), 0, st, npts, npad, tile, keys);
    int lblocks = (int)(npad / 1024);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(lblocks), dim3(512), 0, st, keys, npad,
                       (int64_t)0, 1);
    for (int64_t k = 2048; k <= npad; k <<= 1) {
        for (int64_t j = k / 2; j >= 1024; j >>= 1)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3(blocks), dim3(256), 0, st, keys, npad,
                               k, j);
        hipLaunchKernelGGL(bitonic_local_kernel, dim3(lblocks), dim3(512), 0, st, keys, npad, k, 0);
    }
    int pblocks = (int)((npts + 1 + 255) / 256);
    hipLaunchKernelGGL(keys_to_perm_kernel, dim3(pblocks), dim3(256), 0, st, npts, ntiles, keys,
                       perm, tile_off);
    return hipGetLastError();
}

// Binned layout of sorted points: tile-relative cell (10 bits per dimension) and the
// fractional offset u - cell as FP32.  u is recomputed with the binning's operations,
// so the cell is the one the point was sorted by.
__global__ void point_layout_kernel(int d, int64_t npts, const double *__restrict__ pts, double s0,
                                    double s1, double s2, double o0, double o1, double o2, int T,
                                    uint32_t *__restrict__ cellpk, float *__restrict__ frac)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const double sc[3] = {s0, s1, s2}, oc[3] = {o0, o1, o2};
    uint32_t pk = 0;
    for (int c = 0; c < d; ++c) {
        double u = __dadd_rn(__dmul_rn(pts[i * d + c], sc[c]), oc[c]);
        double f = floor(u);
        int ci = (int)f;
        pk |= (uint32_t)(ci % T) << (10 * c);
        frac[i * d + c] = (float)(u - f);
    }
    cellpk[i] = pk;
}

hipError_t launch_point_layout_s(int d, int64_t npts, const double *pts, const double *s,
                                 const double *o, int T, uint32_t *cellpk, float *frac,
                                 hipStream_t st)
{
    if (npts == 0) return hipSuccess;
    int blocks = (int)((npts + 255) / 256);
    hipLaunchKernelGGL(point_layout_kernel, dim3(blocks), dim3(256), 0, st, d, npts, pts, s[0],
                       d > 1 ? s[1] : 0.0, d > 2 ? s[2] : 0.0, o[0], d > 1 ? o[1] : 0.0,
                       d > 2 ? o[2] : 0.0, T, cellpk, frac);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Kaiser-Bessel window in grid units, normalised to 1 at s = 0:
//   psi(s) = (m / r) sinh(b r) / sinh(b m),  r = sqrt(m^2 - s^2),  |s| <= m,
// b = pi (2 - 1/sigma).  Its Fourier transform is I0(m sqrt(b^2 - w^2)) (used on the host
// for the spectral multiplier).  On the device it is evaluated from 2m degree-9
// polynomials, one per unit interval of s, fitted on the host in FP64.
__device__ __forceinline__ int floor_div(int a, int b)  // floor(a / b) for b > 0
{
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------
// Spreading and interpolation as dense tile contractions on FP32 MFMA.
//
// A tile holds T = 17 - 2m cells per dimension, so the patch of cells its points touch
// is exactly 16 wide (T + 2m - 1).  For a point p with tile-relative cell r and
// fractional offset f, the "shifted window" of dimension c is the 16-vector
//   w_c[q] = psi(f + m - 1 + r - q)  if 0 <= q - r < 2m,  else 0,
// so that the point's contribution to patch cell (a, b, c') is v w_0[a] w_1[b] w_2[c'].
// Spreading a chunk of points is then the contraction
//   G[a][(b,c')] = sum_p X[a][p] Y[p][(b,c')],   X[a][p] = v_p w_0[a],
//   Y[p][(b,c')] = w_1[b] w_2[c'],
// a 16 x 256 x P matrix product done with v_mfma_f32_16x16x4_f32 (4 points per step,
// 16 output tiles, one per b).  Interpolation contracts the other way:
//   Z[p][a] = sum_{(b,c')} Y[p][(b,c')] G[a][(b,c')],  beta_p = sum_a w_0[a] Z[p][a].
// No atomics: each chunk owns its patch (spreading), each point its sum (interpolation).
// One wavefront per work item; points are taken 16 at a time.
constexpr int kPatch = 16;

// Per-lane data of one (point, dimension) row of a 16-point batch, prefetched a batch
// ahead: lane t < 16 D holds row t = p D + c.
struct RowData {
    uint32_t cell;
    float frac;
    double v;
};

template <int D>
__device__ __forceinline__ void load_rows(const uint32_t *cellpk, const float *frac, const double *v,
                                          int64_t pb, int np, RowData &rd)
{
    const int t = threadIdx.x, p = t / D, c = t - p * D;
    rd.cell = 0u;
    rd.frac = 0.0f;
    rd.v = 0.0;
    if (t < 16 * D && p < np) {
        const int64_t gi = pb + p;
        rd.cell = (cellpk[gi] >> (10 * c)) & 1023u;
        rd.frac = frac[gi * D + c];
        if (c == 0 && v) rd.v = v[gi];
    }
}

// Fill win[p][c][0..15] with the shifted windows of the batch: lane t owns row t, zeroes
// it and writes its 2m taps at positions r + j, tap j evaluated by Horner's rule at
// t = f - 1/2 on interval 2m - 1 - j (coefficients read from LDS, the same address on
// every lane).
template <int D>
__device__ __forceinline__ void shifted_windows(const ProdJob &J, const float *cf_lds, const RowData &rd,
                                                int np, bool scale_v, int e, float (*win)[D][kPatch])
{
    const int t = threadIdx.x, p = t / D, c = t - p * D;
    if (t < 16 * D) {
        float4 *row4 = reinterpret_cast<float4 *>(&win[p][c][0]);
#pragma unroll
        for (int q = 0; q < kPatch / 4; ++q) row4[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (p < np) {
            const int taps = 2 * J.m;
            const float x = rd.frac - 0.5f;
            const float sc = (c == 0 && scale_v) ? (float)ldexp(rd.v, -e) : 1.0f;
            float *row = &win[p][c][rd.cell];
            for (int j = 0; j < taps; ++j) {
                const float *cf = cf_lds + (taps - 1 - j) * (kWinDeg + 1);
                float w = cf[kWinDeg];
#pragma unroll
                for (int i = kWinDeg - 1; i >= 0; --i) w = fmaf(w, x, cf[i]);
                row[j] = sc * w;
            }
        }
    }
}

__device__ __forceinline__ void load_poly_lds(const ProdJob &J, float *cf_lds)
{
    const int n = 2 * J.m * (kWinDeg + 1);
    for (int i = threadIdx.x; i < n; i += blockDim.x) cf_lds[i] = J.winpoly[i];
}

template <int D>
__global__ __launch_bounds__(64) void spread_kernel(const ProdJob *__restrict__ jobs,
                                                    const int2 *__restrict__ items, int n_items)
{
    __shared__ float win[16][D][kPatch];
    __shared__ float cf_lds[2 * (kMaxTaps / 2) * (kWinDeg + 1)];
    const int l = threadIdx.x, li = l & 15, lk = l >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int p0 = J.src_chunk_start[itm.y], p1 = J.src_chunk_start[itm.y + 1];
        int e = *J.v_exp;
        if (e == INT32_MIN) e = 0;
        load_poly_lds(J, cf_lds);
        RowData rd;
        load_rows<D>(J.src_cell, J.src_frac, J.v, p0, min(16, p1 - p0), rd);
        __syncthreads();
        constexpr int NT = D == 3 ? 16 : 1;
        f32x4 acc[NT];
        float acc1 = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int pb = p0; pb < p1; pb += 16) {
            const int np = min(16, p1 - pb);
            shifted_windows<D>(J, cf_lds, rd, np, true, e, win);
            if (pb + 16 < p1) load_rows<D>(J.src_cell, J.src_frac, J.v, pb + 16, min(16, p1 - pb - 16), rd);
            __syncthreads();
            if constexpr (D == 3) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int pk = 4 * s + lk;
                    const float x = win[pk][0][li];
                    const float wz = win[pk][2][li];
                    float wy[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) wy[q] = win[pk][1][q];
#pragma unroll
                    for (int bt = 0; bt < 16; ++bt)
                        acc[bt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wy[bt] * wz, acc[bt], 0, 0, 0);
                }
            } else if constexpr (D == 2) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int pk = 4 * s + lk;
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(win[pk][0][li], win[pk][1][li], acc[0],
                                                                 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) acc1 += win[4 * s + lk][0][li];
            }
            __syncthreads();
        }
        float *out = J.patches + (int64_t)itm.y * (D == 3 ? 4096 : (D == 2 ? 256 : 16));
        if constexpr (D == 3) {
#pragma unroll
            for (int bt = 0; bt < 16; ++bt)
#pragma unroll
                for (int r = 0; r < 4; ++r) out[((4 * lk + r) * 16 + bt) * 16 + li] = acc[bt][r];
        } else if constexpr (D == 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[(4 * lk + r) * 16 + li] = acc[0][r];
        } else {
            acc1 += __shfl_xor(acc1, 16);
            acc1 += __shfl_xor(acc1, 32);
            if (lk == 0) out[li] = acc1;
        }
    }
}

// Fold (a2, second half): box grid cell g = sum of the patches covering it, tiles in
// ascending order and chunks in ascending order within a tile.
// item = (job, first cell of a run of 256 consecutive box cells).
template <int D>
__global__ __launch_bounds__(256) void fold_kernel(const ProdJob *__restrict__ jobs,
                                                   const int2 *__restrict__ items, int n_items)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        int64_t total = J.L[0];
        for (int c = 1; c < D; ++c) total *= J.L[c];
        const int64_t g = (int64_t)itm.y + threadIdx.x;
        if (g >= total) continue;
        int gc[3] = {0, 0, 0};
        int64_t rem = g;
        for (int c = D - 1; c >= 0; --c) {
            gc[c] = (int)(rem % J.L[c]);
            rem /= J.L[c];
        }
        const int W = J.W, T = J.T;
        int tlo[3] = {0, 0, 0}, thi[3] = {0, 0, 0};
        for (int c = 0; c < D; ++c) {
            tlo[c] = max(0, floor_div(gc[c] - W + T, T));  // ceil((g - W + 1) / T)
            thi[c] = min(J.ntile[c] - 1, gc[c] / T);
        }
        int patch_elems = W;
        for (int c = 1; c < D; ++c) patch_elems *= W;
        float acc = 0.0f;
        for (int t0 = tlo[0]; t0 <= thi[0]; ++t0)
            for (int t1 = tlo[1]; t1 <= thi[1]; ++t1)
                for (int t2 = tlo[2]; t2 <= thi[2]; ++t2) {
                    int tl = t0, loc = gc[0] - t0 * T;
                    if constexpr (D > 1) {
                        tl = tl * J.ntile[1] + t1;
                        loc = loc * W + (gc[1] - t1 * T);
                    }
                    if constexpr (D > 2) {
                        tl = tl * J.ntile[2] + t2;
                        loc = loc * W + (gc[2] - t2 * T);
                    }
                    const int c0 = J.src_tile_chunks[tl], c1 = J.src_tile_chunks[tl + 1];
                    for (int ch = c0; ch < c1; ++ch) acc += J.patches[(int64_t)ch * patch_elems + loc];
                }
        J.grid[g] = acc;
    }
}

// Interpolation (a6): item = (job, chunk of target points).  out = 2^e * beta with beta
// the window-weighted sum of the grid around each point (FP32, written as FP64), where e
// is the exponent the source vector was scaled by before spreading.
// The MFMA B operand, G[a][(b,c')] for this lane's a = lane % 16 and c' = 4q + lane / 16,
// is the same for every point of the chunk: it is loaded once into registers.
template <int D>
__global__ __launch_bounds__(64) void interp_kernel(const ProdJob *__restrict__ jobs,
                                                    const int2 *__restrict__ items, int n_items)
{
    constexpr int NB = D == 3 ? 64 : (D == 2 ? 4 : 1);  // B values per lane
    __shared__ float win[16][D][kPatch];
    __shared__ float cf_lds[2 * (kMaxTaps / 2) * (kWinDeg + 1)];
    __shared__ float G1[16];
    const int l = threadIdx.x, li = l & 15, lk = l >> 4;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int T = J.T;
        int tc[3] = {0, 0, 0};
        {
            int rem = J.tgt_chunk_tile[itm.y];
            for (int c = D - 1; c >= 0; --c) {
                tc[c] = rem % J.ntile[c];
                rem /= J.ntile[c];
            }
        }
        float Bv[NB];
        if constexpr (D == 3) {
            // K index s = 4(b) + q  <->  (b = s >> 2, c' = 4 (s & 3) + lk)
            const int64_t base = ((int64_t)(tc[0] * T + li) * J.L[1] + tc[1] * T) * J.L[2] + tc[2] * T;
#pragma unroll
            for (int s = 0; s < 64; ++s)
                Bv[s] = J.grid[base + (int64_t)(s >> 2) * J.L[2] + 4 * (s & 3) + lk];
        } else if constexpr (D == 2) {
            const int64_t base = (int64_t)(tc[0] * T + li) * J.L[1] + tc[1] * T;
#pragma unroll
            for (int s = 0; s < 4; ++s) Bv[s] = J.grid[base + 4 * s + lk];
        } else {
            if (l < 16) G1[l] = J.grid[tc[0] * T + l];
        }
        int e = *J.v_exp;
        if (e == INT32_MIN) e = 0;
        load_poly_lds(J, cf_lds);
        const int p0 = J.tgt_chunk_start[itm.y], p1 = J.tgt_chunk_start[itm.y + 1];
        RowData rd;
        load_rows<D>(J.tgt_cell, J.tgt_frac, nullptr, p0, min(16, p1 - p0), rd);
        __syncthreads();
        for (int pb = p0; pb < p1; pb += 16) {
            const int np = min(16, p1 - pb);
            shifted_windows<D>(J, cf_lds, rd, np, false, 0, win);
            if (pb + 16 < p1) load_rows<D>(J.tgt_cell, J.tgt_frac, nullptr, pb + 16, min(16, p1 - pb - 16), rd);
            __syncthreads();
            if constexpr (D == 1) {
                if (l < np) {
                    float s = 0.0f;
#pragma unroll
                    for (int a = 0; a < 16; ++a) s += G1[a] * win[l][0][a];
                    J.out[pb + l] = ldexp((double)s, e);
                }
            } else {
                f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                if constexpr (D == 3) {
                    float wy[16], wzk[4];
#pragma unroll
                    for (int q = 0; q < 16; ++q) wy[q] = win[li][1][q];
#pragma unroll
                    for (int q = 0; q < 4; ++q) wzk[q] = win[li][2][4 * q + lk];
#pragma unroll
                    for (int s = 0; s < 64; ++s)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wy[s >> 2] * wzk[s & 3], Bv[s], acc, 0, 0, 0);
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(win[li][1][4 * s + lk], Bv[s], acc, 0, 0, 0);
                }
                // acc[r] = Z[p = 4 lk + r][a = li]; beta_p = sum_a w_0[a] Z[p][a]
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int p = 4 * lk + r;
                    float z = acc[r] * win[p][0][li];
                    z += __shfl_xor(z, 1);
                    z += __shfl_xor(z, 2);
                    z += __shfl_xor(z, 4);
                    z += __shfl_xor(z, 8);
                    if (li == 0 && p < np) J.out[pb + p] = ldexp((double)z, e);
                }
            }
            __syncthreads();
        }
    }
}

static int nfft_grid(int n_items)
{
    return n_items < 65535 ? n_items : 65535;
}

hipError_t launch_spread(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int /*max_patch_elems*/, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (d == 3)
        hipLaunchKernelGGL(spread_kernel<3>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    else if (d == 2)
        hipLaunchKernelGGL(spread_kernel<2>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    else
        hipLaunchKernelGGL(spread_kernel<1>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    return hipGetLastError();
}

hipError_t launch_fold(int d, const ProdJob *jobs, const int2 *items, int n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (d == 3)
        hipLaunchKernelGGL(fold_kernel<3>, dim3(nfft_grid(n_items)), dim3(256), 0, s, jobs, items,
                           n_items);
    else if (d == 2)
        hipLaunchKernelGGL(fold_kernel<2>, dim3(nfft_grid(n_items)), dim3(256), 0, s, jobs, items,
                           n_items);
    else
        hipLaunchKernelGGL(fold_kernel<1>, dim3(nfft_grid(n_items)), dim3(256), 0, s, jobs, items,
                           n_items);
    return hipGetLastError();
}

hipError_t launch_interp(int d, const ProdJob *jobs, const int2 *items, int n_items,
                         int /*max_patch_elems*/, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (d == 3)
        hipLaunchKernelGGL(interp_kernel<3>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    else if (d == 2)
        hipLaunchKernelGGL(interp_kernel<2>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    else
        hipLaunchKernelGGL(interp_kernel<1>, dim3(nfft_grid(n_items)), dim3(64), 0, s, jobs, items,
                           n_items);
    return hipGetLastError();
}

}  // namespace mot
