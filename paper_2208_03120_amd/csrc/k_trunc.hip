// Truncated direct products for small eta (the truncation suggested at the end of
// Sec. 6.1):
//   out_i = sum over sources j in the cells near target i's cell of v_j exp(-|x_i - y_j|^2 / eta).
// Both point sets are sorted by cubic cells of side h (the a1 binning with tile edge 1).
// The sources summed for a target are those of every cell whose box distance to the
// target's cell is at most r_c, so every source within r_c of the target is included and
// the terms left out are below exp(-r_c^2 / eta) v_j.  In the row-major cell order the
// cells of one row of the neighbourhood (fixed leading coordinates, a range along the last
// one) are one contiguous range of sorted sources.
//
// One wavefront takes one item: up to 64 R targets, R per lane, from a run of B
// consecutive cells of one row (consecutive in the sorted order; B > 1 fills the lanes
// when cells hold few points).  The neighbourhood rows of a run are those of its first
// cell, widened by B - 1 cells along the row.  The wave first lists the item's non-empty
// rows in LDS with the prefix sum of their lengths, so its sources form one list; it then
// stages that list 64 entries at a time through its own LDS slice (every stage full but
// the last), and every lane sums a stage against its R targets while the next stage's
// sources are loaded.  The waves of a block take different items and synchronise only
// within themselves.
//
// Mixed precision, two forms of the exponent (c = log2(e) / eta):
//  * short runs: coordinates relative to the centre of the item's run of cells (in FP64),
//    scaled by sqrt(c) and rounded to FP32; a term is exp2(-|x'' - y''|^2).  The host takes
//    this form only when sqrt(c) times the run's half-diagonal is at most 3, so the targets
//    and every source that contributes more than a rounding error have |x''|, |y''| of a
//    few units and their FP32 rounding moves the exponent by ~1e-7;
//  * long runs (sparse cells): -c|x|^2 - c|y|^2 + 2c x.y formed in FP64 (coordinates
//    relative to the cloud's centre), rounded to FP32 for v_exp_f32.  On gfx950 the FP64
//    adds and FMAs issue at half the FP32 rate, so this form costs ~1.6x per pair.
// (The expanded form in FP32 would cancel terms of size c r^2.)  Values are scaled by
// 2^-e (e = exponent of max v); sums over 64 sources are FP32 and are added into FP64
// accumulators.
// FP64: plain exp(-|x - y|^2 / eta) with FP64 sums in source order.
#include <type_traits>

#include "mot_internal.h"

namespace mot {

// Sorted source range [a, b) of neighbour row ri of the run of B cells starting at cc;
// false when the row lies outside the grid or farther than r_c from the run.
template <int D>
__device__ __forceinline__ bool trunc_row(const ProdJob &J, const int cc[3], int B, int ri, int64_t &a,
                                          int64_t &b)
{
    const int w = J.tw, nc = J.nc, span = 2 * w + 1;
    int del[2] = {0, 0};
    if (D == 3) {
        del[0] = ri / span - w;
        del[1] = ri % span - w;
    } else if (D == 2) {
        del[0] = ri - w;
    }
    double used = 0.0;
    int64_t base = 0;
#pragma unroll
    for (int c = 0; c < D - 1; ++c) {
        const int x = cc[c] + del[c];
        if (x < 0 || x >= nc) return false;
        const int e = abs(del[c]) - 1;
        if (e > 0) used += (double)e * e;
        base = base * nc + x;
    }
    const double rem = J.q2 - used;
    if (rem < 0.0) return false;
    const int wl = min(w, 1 + (int)floor(sqrt(rem)));
    const int xa = max(cc[D - 1] - wl, 0), xb = min(cc[D - 1] + B - 1 + wl, nc - 1);
    const MOT_GLOBAL int32_t *off = gp(J.src_cell_off);
    a = off[base * nc + xa];
    b = off[base * nc + xb + 1];
    return b > a;
}

template <int D>
__device__ __forceinline__ void trunc_cell(const ProdJob &J, int cell, int cc[3])
{
    cc[0] = cc[1] = cc[2] = 0;
    int rem = cell;
#pragma unroll
    for (int c = D - 1; c >= 0; --c) {
        cc[c] = rem % J.nc;
        rem /= J.nc;
    }
}

__device__ __forceinline__ int trunc_rows(int D, int w)
{
    const int span = 2 * w + 1;
    return D == 1 ? 1 : (D == 2 ? span : span * span);
}

// Wavefront-local ordering of LDS accesses: the waves of a block work on different items
// and never wait for each other; a wave's own LDS operations execute in issue order, so
// only the compiler has to be kept from moving accesses across this point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kTruncWaves = 4;  // independent wavefronts per block, one item each

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

template <int D, int R, bool WIDE>
__global__ __launch_bounds__(64 * kTruncWaves) void trunc_mixed_kernel(const ProdJob *__restrict__ jobs,
                                                                       const int4 *__restrict__ items,
                                                                       int n_items)
{
    // FP32 form: float4 sqrt(c) (y - run centre), 2^-e v;  FP64 form: 2c (y - cloud
    // centre), -c |y - cloud centre|^2 and the value in its own array
    __shared__ double sbuf_all[kTruncWaves][64][4];
    __shared__ float sv_all[kTruncWaves][64];
    __shared__ int32_t ra_all[kTruncWaves][kMaxTruncRows];      // first sorted source of each row
    __shared__ int32_t rp_all[kTruncWaves][kMaxTruncRows + 1];  // sources before each row
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float4 *sy = reinterpret_cast<float4 *>(sbuf_all[wave]);
    double(*sw)[4] = sbuf_all[wave];
    float *sv = sv_all[wave];
    int32_t *ra = ra_all[wave], *rp = rp_all[wave];
    for (int it = blockIdx.x * kTruncWaves + wave; it < n_items; it += gridDim.x * kTruncWaves) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int cnt = itm.w & 0xffff, B = itm.w >> 16;
        int cc[3];
        trunc_cell<D>(J, itm.y, cc);
        const double c2 = 1.4426950408889634 / J.eta;  // log2(e) / eta
        const double sc = sqrt(c2);
        double ctr[3] = {0.0, 0.0, 0.0};  // centre of the run (FP32 form), of the cloud (FP64)
#pragma unroll
        for (int c = 0; c < D; ++c)
            ctr[c] = WIDE ? J.ctr[c] : J.glo[c] + (cc[c] + (c == D - 1 ? 0.5 * B : 0.5)) * J.h;
        int e = *gp(J.v_exp);
        if (e == INT32_MIN) e = 0;
        const MOT_GLOBAL double *tgt = gp(J.tgt_pts);
        const MOT_GLOBAL double *src = gp(J.src_pts);
        const MOT_GLOBAL double *vv = gp(J.v);
        // the item's non-empty neighbour rows, compacted in row order with the prefix of
        // their lengths: the sources to sum are one list of `total` entries
        int nr = 0, total = 0;
        const int nrows = trunc_rows(D, J.tw);
        wave_sync();
        for (int r0 = 0; r0 < nrows; r0 += 64) {
            int64_t a = 0, b = 0;
            const bool ok = r0 + lane < nrows && trunc_row<D>(J, cc, B, r0 + lane, a, b);
            const int len = ok ? (int)(b - a) : 0;
            const int f = len > 0 ? 1 : 0;
            const int fpos = wave_incl_scan(f, lane), lpos = wave_incl_scan(len, lane);
            if (f) {
                ra[nr + fpos - 1] = (int32_t)a;
                rp[nr + fpos - 1] = total + lpos - len;
            }
            nr += __shfl(fpos, 63);
            total += __shfl(lpos, 63);
        }
        if (lane == 0) rp[nr] = total;
        wave_sync();
        typedef typename std::conditional<WIDE, double, float>::type real;
        real xs[R][3];
        double ax[R], acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool act = lane + 64 * r < cnt;
            const int64_t i = (int64_t)itm.z + lane + 64 * r;
            double nrm = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double dx = (c < D && act) ? tgt[i * D + c] - ctr[c] : 0.0;
                xs[r][c] = WIDE ? (real)dx : (real)(dx * sc);
                nrm += dx * dx;
            }
            ax[r] = -c2 * nrm;
            acc[r] = 0.0;
        }
        // stages of 64 consecutive list entries; each lane follows its entry's row with a
        // pointer that only moves forward, and loads its source one stage ahead
        int row = 0;
        double ly[3] = {0.0, 0.0, 0.0}, lv = 0.0;
        auto fetch = [&](int q) {
            if (q < total) {
                while (rp[row + 1] <= q) ++row;
                const int64_t j = (int64_t)ra[row] + (q - rp[row]);
#pragma unroll
                for (int c = 0; c < D; ++c) ly[c] = src[j * D + c];
                lv = vv[j];
            }
        };
        fetch(lane);
        for (int s0 = 0; s0 < total; s0 += 64) {
            const int nj = min(64, total - s0);
            wave_sync();
            if (lane < nj) {
                if constexpr (WIDE) {
                    double nrm = 0.0;
                    sw[lane][0] = sw[lane][1] = sw[lane][2] = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const double dy = ly[c] - ctr[c];
                        sw[lane][c] = 2.0 * c2 * dy;
                        nrm += dy * dy;
                    }
                    sw[lane][3] = -c2 * nrm;
                    sv[lane] = (float)ldexp(lv, -e);
                } else {
                    float y[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int c = 0; c < D; ++c) y[c] = (float)((ly[c] - ctr[c]) * sc);
                    sy[lane] = make_float4(y[0], y[1], y[2], (float)ldexp(lv, -e));
                }
            }
            wave_sync();
            fetch(s0 + 64 + lane);
            float part[R];
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = 0.0f;
            if constexpr (WIDE) {
#pragma unroll 2
                for (int jj = 0; jj < nj; ++jj) {
                    const double s0v = sw[jj][0], s1 = sw[jj][1], s2 = sw[jj][2], s3 = sw[jj][3];
                    const float w = sv[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        double arg = ax[r] + s3;
                        arg = fma(xs[r][0], s0v, arg);
                        if (D > 1) arg = fma(xs[r][1], s1, arg);
                        if (D > 2) arg = fma(xs[r][2], s2, arg);
                        part[r] = fmaf(w, __builtin_amdgcn_exp2f((float)arg), part[r]);
                    }
                }
            } else {
#pragma unroll 2
                for (int jj = 0; jj < nj; ++jj) {
                    const float4 y = sy[jj];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float dx = xs[r][0] - y.x;
                        float q = dx * dx;
                        if (D > 1) {
                            const float dy = xs[r][1] - y.y;
                            q = fmaf(dy, dy, q);
                        }
                        if (D > 2) {
                            const float dz = xs[r][2] - y.z;
                            q = fmaf(dz, dz, q);
                        }
                        part[r] = fmaf(y.w, __builtin_amdgcn_exp2f(-q), part[r]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (double)part[r];
        }
        MOT_GLOBAL double *out = gp(J.out);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = (int64_t)itm.z + lane + 64 * r;
            if (lane + 64 * r < cnt) out[i] = ldexp(acc[r], e);
        }
    }
}

template <int D, int R>
__global__ __launch_bounds__(64) void trunc_fp64_kernel(const ProdJob *__restrict__ jobs,
                                                        const int4 *__restrict__ items, int n_items)
{
    __shared__ double sy[64][4];
    const int lane = threadIdx.x;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int cnt = itm.w & 0xffff, B = itm.w >> 16;
        int cc[3];
        trunc_cell<D>(J, itm.y, cc);
        const double inv_eta = 1.0 / J.eta;
        const MOT_GLOBAL double *tgt = gp(J.tgt_pts);
        const MOT_GLOBAL double *src = gp(J.src_pts);
        const MOT_GLOBAL double *vv = gp(J.v);
        double xs[R][3], acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool act = lane + 64 * r < cnt;
            const int64_t i = (int64_t)itm.z + lane + 64 * r;
#pragma unroll
            for (int c = 0; c < 3; ++c) xs[r][c] = (c < D && act) ? tgt[i * D + c] : 0.0;
            acc[r] = 0.0;
        }
        const int nrows = trunc_rows(D, J.tw);
        for (int ri = 0; ri < nrows; ++ri) {
            int64_t a, b;
            if (!trunc_row<D>(J, cc, B, ri, a, b)) continue;
            for (int64_t j0 = a; j0 < b; j0 += 64) {
                const int nj = (int)min((int64_t)64, b - j0);
                __syncthreads();
                if (lane < nj) {
                    const int64_t j = j0 + lane;
#pragma unroll
                    for (int c = 0; c < D; ++c) sy[lane][c] = src[j * D + c];
                    sy[lane][3] = vv[j];
                }
                __syncthreads();
                for (int jj = 0; jj < nj; ++jj) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        double d2 = 0.0;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const double df = xs[r][c] - sy[jj][c];
                            d2 += df * df;
                        }
                        acc[r] += sy[jj][3] * exp(-d2 * inv_eta);
                    }
                }
            }
        }
        MOT_GLOBAL double *out = gp(J.out);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = (int64_t)itm.z + lane + 64 * r;
            if (lane + 64 * r < cnt) out[i] = acc[r];
        }
    }
}

template <int D>
static void launch_trunc_d(int precision, int R, int wide, const ProdJob *jobs, const int4 *items, int n_items,
                           hipStream_t s)
{
    if (precision == MOT_PREC_FP64) {
        const dim3 grid(n_items < (1 << 20) ? n_items : (1 << 20)), block(64);
        if (R == 1) hipLaunchKernelGGL((trunc_fp64_kernel<D, 1>), grid, block, 0, s, jobs, items, n_items);
        if (R == 2) hipLaunchKernelGGL((trunc_fp64_kernel<D, 2>), grid, block, 0, s, jobs, items, n_items);
    } else {
        const int blocks = (n_items + kTruncWaves - 1) / kTruncWaves;
        const dim3 grid(blocks < (1 << 20) ? blocks : (1 << 20)), block(64 * kTruncWaves);
        if (wide) {
            if (R == 1) hipLaunchKernelGGL((trunc_mixed_kernel<D, 1, true>), grid, block, 0, s, jobs, items, n_items);
            if (R == 2) hipLaunchKernelGGL((trunc_mixed_kernel<D, 2, true>), grid, block, 0, s, jobs, items, n_items);
            if (R == 4) hipLaunchKernelGGL((trunc_mixed_kernel<D, 4, true>), grid, block, 0, s, jobs, items, n_items);
        } else {
            if (R == 1) hipLaunchKernelGGL((trunc_mixed_kernel<D, 1, false>), grid, block, 0, s, jobs, items, n_items);
            if (R == 2) hipLaunchKernelGGL((trunc_mixed_kernel<D, 2, false>), grid, block, 0, s, jobs, items, n_items);
            if (R == 4) hipLaunchKernelGGL((trunc_mixed_kernel<D, 4, false>), grid, block, 0, s, jobs, items, n_items);
        }
    }
}

hipError_t launch_trunc(int d, int precision, int R, int wide, const ProdJob *jobs_dev, const int4 *items,
                        int n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (R != 1 && R != 2 && R != 4) return hipErrorInvalidValue;
    if (precision == MOT_PREC_FP64 && R == 4) return hipErrorInvalidValue;
    if (d == 1) launch_trunc_d<1>(precision, R, wide, jobs_dev, items, n_items, s);
    if (d == 2) launch_trunc_d<2>(precision, R, wide, jobs_dev, items, n_items, s);
    if (d == 3) launch_trunc_d<3>(precision, R, wide, jobs_dev, items, n_items, s);
    return hipGetLastError();
}

}  // namespace mot
