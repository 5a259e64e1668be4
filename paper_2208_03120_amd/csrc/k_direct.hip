// Direct Gaussian-kernel products (a7), the plain O(n_t n_s) path:
//   out_i = sum_j v_j exp(-|x_i - y_j|^2 / eta)      (Sec. 5, eq. fastsum-sum)
//
// FP64 variant: one target per lane, a block's four wavefronts summing quarters of a
// source range in ascending source order, the quarters (and ranges) then added in order
// (details at direct_fp64_kernel).
//
// Mixed variant: FP32 transcendental with FP64 accumulation across tiles.  With
// c = log2(e) / eta and coordinates taken relative to the point cloud's centre,
//   exp(-|x - y|^2 / eta) = exp2(a_x + a_y + x'.y'),  a_x = -c|x|^2, a_y = -c|y|^2,
//   y' = 2 c y,
// so each pair costs d FMAs, one add, one v_exp_f32 and one FMA.  The exponent is a sum
// of terms up to c r^2 (r the cloud's radius) that cancel to -c|x - y|^2, so its FP32
// rounding error grows like 6e-8 c r^2; when c r^2 exceeds 8 (small eta) the kernel
// forms the same exponent in FP64 (gfx950 issues FP64 adds and FMAs at the unpacked FP32
// rate) and rounds only the result to FP32 for v_exp_f32: one conversion more per pair,
// and the error is the rounding of the exponent itself.  Source values are scaled by
// 2^-e (e = exponent of max v) so FP32 never under- or overflows; partial sums over 64
// sources are added into FP64 accumulators.  Each thread owns R targets to reuse every
// LDS read R times.  This kernel is bound by the transcendental and vector issue rates.
#include <algorithm>
#include <type_traits>

#include "mot_internal.h"

namespace mot {

// FP64 variant: an item is 64 targets (one per lane) and one of the job's dsplit equal
// source ranges; the block's four wavefronts take the four quarters of that range, each
// summing its sources in ascending order, and the quarters are added in order.  With
// dsplit > 1 the item writes its partial sums to the job's partial buffer and
// direct_fp64_reduce_kernel adds the ranges in order; dsplit grows as the targets get
// fewer, so that small products still spread over the chip.
constexpr int kDirectT = 64;

int direct_source_split(int64_t nt, int64_t ns)
{
    const int64_t groups = (nt + kDirectT - 1) / kDirectT;
    const int64_t want = (1024 + groups - 1) / groups;  // about a thousand items per launch
    const int64_t most = (ns + 63) / 64;               // at least 16 sources per wavefront
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(want, most), 64));
}

template <int D>
__global__ __launch_bounds__(256) void direct_fp64_kernel(const ProdJob *__restrict__ jobs,
                                                          const int4 *__restrict__ items, int n_items)
{
    __shared__ double red[3][kDirectT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int64_t i = (int64_t)itm.y + lane;
        const bool act = i < J.nt;
        double x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = act ? J.tgt_pts[i * D + c] : 0.0;
        const double eta = J.eta;
        const int64_t per = (J.ns + J.dsplit - 1) / J.dsplit;
        const int64_t a = (int64_t)itm.z * per, b = min(J.ns, a + per);
        const int64_t q = (b - a + 3) / 4;
        const int64_t ja = min(b, a + wave * q), jb = min(b, ja + q);
        double acc = 0.0;
        for (int64_t j = ja; j < jb; ++j) {
            double d2 = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const double df = x[c] - J.src_pts[j * D + c];
                d2 += df * df;
            }
            acc += J.v[j] * exp(-d2 / eta);
        }
        __syncthreads();  // the previous item's reads of red are done
        if (wave > 0) red[wave - 1][lane] = acc;
        __syncthreads();
        if (wave == 0 && act) {
            const double sum = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
            if (J.dsplit > 1)
                J.dpart[(int64_t)itm.z * J.nt + i] = sum;
            else
                J.out[i] = sum;
        }
    }
}

// out_i = sum over the job's source ranges, in range order, of the partial sums.
__global__ __launch_bounds__(256) void direct_fp64_reduce_kernel(const ProdJob *__restrict__ jobs,
                                                                 const int2 *__restrict__ items, int n_items)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const int64_t i = (int64_t)itm.y + threadIdx.x;
        if (i >= J.nt) continue;
        double acc = 0.0;
        for (int r = 0; r < J.dsplit; ++r) acc += J.dpart[(int64_t)r * J.nt + i];
        J.out[i] = acc;
    }
}

constexpr int kDirectR = 4;

// Source staging of the mixed kernel: FP32 (2 c y, -c|y|^2) or the same in FP64.
template <bool WIDE>
struct DirectSrc;
template <>
struct DirectSrc<false> {
    float4 y;
};
template <>
struct DirectSrc<true> {
    double y[4];
};

template <int D, bool WIDE>
__global__ __launch_bounds__(256) void direct_mixed_kernel(const ProdJob *__restrict__ jobs,
                                                           const int4 *__restrict__ items, int n_items)
{
    typedef typename std::conditional<WIDE, double, float>::type real;
    __shared__ DirectSrc<WIDE> sy[256];
    __shared__ float sv[256];
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        const double c2 = 1.4426950408889634 / J.eta;  // log2(e) / eta
        int e = *J.v_exp;
        if (e == INT32_MIN) e = 0;
        real xs[kDirectR][3], ax[kDirectR];
        double acc[kDirectR];
#pragma unroll
        for (int r = 0; r < kDirectR; ++r) {
            const int64_t i = (int64_t)itm.y + tid + 256 * r;
            double nrm = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double dx = 0.0;
                if (c < D && i < J.nt) dx = J.tgt_pts[i * D + c] - J.ctr[c];
                xs[r][c] = (real)dx;
                nrm += dx * dx;
            }
            ax[r] = (real)(-c2 * nrm);
            acc[r] = 0.0;
        }
        for (int64_t j0 = 0; j0 < J.ns; j0 += 256) {
            const int nj = (int)min((int64_t)256, J.ns - j0);
            __syncthreads();
            if (tid < nj) {
                double dy[3] = {0.0, 0.0, 0.0}, nrm = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    dy[c] = J.src_pts[(j0 + tid) * D + c] - J.ctr[c];
                    nrm += dy[c] * dy[c];
                }
                if constexpr (WIDE) {
                    sy[tid].y[0] = 2.0 * c2 * dy[0];
                    sy[tid].y[1] = 2.0 * c2 * dy[1];
                    sy[tid].y[2] = 2.0 * c2 * dy[2];
                    sy[tid].y[3] = -c2 * nrm;
                } else {
                    sy[tid].y = make_float4((float)(2.0 * c2 * dy[0]), (float)(2.0 * c2 * dy[1]),
                                            (float)(2.0 * c2 * dy[2]), (float)(-c2 * nrm));
                }
                sv[tid] = (float)ldexp(J.v[j0 + tid], -e);
            }
            __syncthreads();
            for (int jb = 0; jb < nj; jb += 64) {
                const int je = min(nj, jb + 64);
                float part[kDirectR];
#pragma unroll
                for (int r = 0; r < kDirectR; ++r) part[r] = 0.0f;
                for (int jj = jb; jj < je; ++jj) {
                    real s[4];
                    if constexpr (WIDE) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) s[q] = sy[jj].y[q];
                    } else {
                        const float4 f = sy[jj].y;
                        s[0] = f.x;
                        s[1] = f.y;
                        s[2] = f.z;
                        s[3] = f.w;
                    }
                    const float w = sv[jj];
#pragma unroll
                    for (int r = 0; r < kDirectR; ++r) {
                        real arg = ax[r] + s[3];
                        arg = fma(xs[r][0], s[0], arg);
                        if (D > 1) arg = fma(xs[r][1], s[1], arg);
                        if (D > 2) arg = fma(xs[r][2], s[2], arg);
                        part[r] = fmaf(w, __builtin_amdgcn_exp2f((float)arg), part[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < kDirectR; ++r) acc[r] += (double)part[r];
            }
        }
#pragma unroll
        for (int r = 0; r < kDirectR; ++r) {
            const int64_t i = (int64_t)itm.y + tid + 256 * r;
            if (i < J.nt) J.out[i] = ldexp(acc[r], e);
        }
    }
}

int direct_targets_per_item(int precision) { return precision == MOT_PREC_FP64 ? kDirectT : 256 * kDirectR; }

hipError_t launch_direct(int d, const ProdJob *jobs_dev, const int4 *items, int n_items, const int2 *red_items,
                         int n_red, int precision, int diff, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const int grid = n_items < 16384 ? n_items : 16384;
    if (precision == MOT_PREC_FP64) {
        if (d == 1) hipLaunchKernelGGL(direct_fp64_kernel<1>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 2) hipLaunchKernelGGL(direct_fp64_kernel<2>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 3) hipLaunchKernelGGL(direct_fp64_kernel<3>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (n_red > 0)
            hipLaunchKernelGGL(direct_fp64_reduce_kernel, dim3(n_red < 16384 ? n_red : 16384), dim3(256), 0, s, jobs_dev,
                               red_items, n_red);
    } else if (diff) {
        if (d == 1) hipLaunchKernelGGL((direct_mixed_kernel<1, true>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 2) hipLaunchKernelGGL((direct_mixed_kernel<2, true>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 3) hipLaunchKernelGGL((direct_mixed_kernel<3, true>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
    } else {
        if (d == 1) hipLaunchKernelGGL((direct_mixed_kernel<1, false>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 2) hipLaunchKernelGGL((direct_mixed_kernel<2, false>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
        if (d == 3) hipLaunchKernelGGL((direct_mixed_kernel<3, false>), dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
    }
    return hipGetLastError();
}

}  // namespace mot
