// Pruned multi-dimensional FFTs of the fast summation (a3-a5) for gfx950.
//
// Between spreading and interpolation, fast summation multiplies the grid's spectrum by
// D(k) = kappa_hat(k) w(k) / prod_c Psi(k_c)^2 on the band |k_c| <= M (kappa_hat: eq. fft;
// Psi: the window's Fourier transform; w: weights 1/2 at the unpaired band edge so that
// the real part of eq. (fastsum1) is produced).  The grid is nonzero only on the active
// box (L_c cells) and only the band survives the multiply, so every 1-D transform loads
// only box or band entries and stores only band or box entries.
//
// Each pass transforms lines along the fastest axis of its input.  A line of N points is
// held by G = min(64, N/2) lanes with E = N/G complex values each (value q in lane q % G,
// slot q / G).  Radix-2 stages whose butterfly partners sit in the same lane work in
// registers; the others exchange values with wavefront shuffles.  Forward transforms are
// decimation-in-frequency (natural order in, bit-reversed out) and inverse transforms
// decimation-in-time (bit-reversed in, natural out), so no reordering pass exists: the
// bit reversal is folded into the index arithmetic of the loads and stores.  Outputs are
// staged in LDS and written with the line index fastest (coalesced), which rotates the
// axes for the next pass.
//
// Pass chain, 3-D (axes 0,1,2; 2 fastest; H = M+1, B = 2M+1):
//   0 R2C  grid[L0][L1][L2] real -> spec0[H][L0][L1]     (axis 2, two real lines per FFT)
//   1 FWD  spec0[H][L0][L1]      -> spec1[H][B][L0]      (axis 1)
//   2 FUSE spec1[H][B][L0]       -> spec0[L0][H][B]      (axis 0: forward, multiply, inverse)
//   3 INV  spec0[L0][H][B]       -> spec1[L0][L1][H]     (axis 1)
//   4 C2R  spec1[L0][L1][H]      -> grid[L0][L1][L2]     (axis 2, Hermitian half spectrum)
// 2-D uses 0, 2, 4 and 1-D uses 0 and 4 (which then applies the multiplier).
//
// When a box slab's half spectrum fits in LDS, 3-D uses three passes instead:
//   6 SLAB grid[L0][L1][L2]  -> spec1[L0][H][B]   (per slab g0: R2C axis 2, FWD axis 1)
//   5 FUSE spec1[L0][H][B]   -> spec0[L0][H][B]   (axis 0 as pass 2, reading g0-major input)
//   7 SLAB spec0[L0][H][B]   -> grid[L0][L1][L2]  (per slab g0: INV axis 1, C2R axis 2)
#include "mot_internal.h"

namespace mot {


template <int N>
struct FftShape {
    static constexpr int G = N / 2 < 64 ? N / 2 : 64;
    static constexpr int E = N / G;
    static constexpr int LW = 64 / G;
    static constexpr int LOG = N == 16 ? 4 : N == 32 ? 5 : N == 64 ? 6 : N == 128 ? 7 : N == 256 ? 8 : 9;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// tw holds the twiddles of a TWS N-point transform: exp(-2 pi i j / N) = tw[j TWS]
template <int N, int TWS>
__device__ __forceinline__ void fft_dif(float2 (&x)[FftShape<N>::E], int g, const float2 *tw)
{
    constexpr int G = FftShape<N>::G, E = FftShape<N>::E;
#pragma unroll
    for (int h = N / 2; h >= 1; h >>= 1) {
        const int tstride = N / (2 * h);
        if (h >= G) {
            const int eb = h / G;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e & eb) continue;
                const int q = g + G * e;
                const float2 w = tw[(q & (h - 1)) * tstride * TWS];
                const float2 a = x[e], b = x[e + eb];
                x[e] = cadd(a, b);
                x[e + eb] = cmul(csub(a, b), w);
            }
        } else {
            // the same operations on every lane, so the wavefront does not split: the top
            // lane of a pair forms x + y, the bottom lane (y - x) w, as s x + y with s = +-1
            // times w or 1 (exact for the top lane)
            const bool bottom = (g & h) != 0;
            const float2 w = bottom ? tw[(g & (h - 1)) * tstride * TWS] : make_float2(1.0f, 0.0f);
            const float sg = bottom ? -1.0f : 1.0f;
            float2 y[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                y[e].x = __shfl_xor(x[e].x, h);
                y[e].y = __shfl_xor(x[e].y, h);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float2 t = make_float2(fmaf(sg, x[e].x, y[e].x), fmaf(sg, x[e].y, y[e].y));
                x[e] = cmul(t, w);
            }
        }
    }
}

template <int N, int TWS>
__device__ __forceinline__ void fft_dit_inv(float2 (&x)[FftShape<N>::E], int g, const float2 *tw)
{
    constexpr int G = FftShape<N>::G, E = FftShape<N>::E;
#pragma unroll
    for (int h = 1; h <= N / 2; h <<= 1) {
        const int tstride = N / (2 * h);
        if (h >= G) {
            const int eb = h / G;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e & eb) continue;
                const int q = g + G * e;
                const float2 w = tw[(q & (h - 1)) * tstride * TWS];
                const float2 a = x[e], b = cmulc(x[e + eb], w);
                x[e] = cadd(a, b);
                x[e + eb] = csub(a, b);
            }
        } else {
            // branch-free: with a the top lane's value and b the bottom lane's, the top lane
            // forms a + b conj(w) and the bottom lane a - b conj(w).  Every lane first
            // multiplies its own value by conj(w) (the top lane by 1, exactly) and the
            // products are exchanged, so each lane ends with s z + y, s = +-1.
            const bool bottom = (g & h) != 0;
            const float2 w = bottom ? tw[(g & (h - 1)) * tstride * TWS] : make_float2(1.0f, 0.0f);
            const float sg = bottom ? -1.0f : 1.0f;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float2 z = cmulc(x[e], w);
                float2 y;
                y.x = __shfl_xor(z.x, h);
                y.y = __shfl_xor(z.y, h);
                x[e] = make_float2(fmaf(sg, z.x, y.x), fmaf(sg, z.y, y.y));
            }
        }
    }
}

struct PassGeom {
    int A2, A1, LA, lo_in, Kout, lo_out;
    const float *in_r;
    const float2 *in_c;
    float *out_r;
    float2 *out_c;
};

template <int KIND>
__device__ __forceinline__ PassGeom pass_geom(const ProdJob &J)
{
    PassGeom P;
    const int H = J.M + 1, B = 2 * J.M + 1;
    P.in_r = J.grid;
    P.out_r = J.grid;
    P.lo_in = 0;
    P.lo_out = 0;
    if (J.d == 3) {
        if (KIND == 0) { P.A2 = J.L[0]; P.A1 = J.L[1]; P.LA = J.L[2]; P.lo_in = J.lo[2]; P.Kout = H; P.out_c = J.spec0; }
        if (KIND == 1) { P.A2 = H; P.A1 = J.L[0]; P.LA = J.L[1]; P.lo_in = J.lo[1]; P.Kout = B; P.in_c = J.spec0; P.out_c = J.spec1; }
        if (KIND == 2 || KIND == 5) { P.A2 = H; P.A1 = B; P.LA = J.L[0]; P.lo_in = J.lo[0]; P.Kout = J.L[0]; P.lo_out = J.lo[0]; P.in_c = J.spec1; P.out_c = J.spec0; }
        if (KIND == 3) { P.A2 = J.L[0]; P.A1 = H; P.LA = B; P.Kout = J.L[1]; P.lo_out = J.lo[1]; P.in_c = J.spec0; P.out_c = J.spec1; }
        if (KIND == 4) { P.A2 = J.L[0]; P.A1 = J.L[1]; P.LA = H; P.Kout = J.L[2]; P.lo_out = J.lo[2]; P.in_c = J.spec1; }
    } else if (J.d == 2) {
        if (KIND == 0) { P.A2 = 1; P.A1 = J.L[0]; P.LA = J.L[1]; P.lo_in = J.lo[1]; P.Kout = H; P.out_c = J.spec0; }
        if (KIND == 2) { P.A2 = 1; P.A1 = H; P.LA = J.L[0]; P.lo_in = J.lo[0]; P.Kout = J.L[0]; P.lo_out = J.lo[0]; P.in_c = J.spec0; P.out_c = J.spec1; }
        if (KIND == 4) { P.A2 = 1; P.A1 = J.L[0]; P.LA = H; P.Kout = J.L[1]; P.lo_out = J.lo[1]; P.in_c = J.spec1; }
    } else {
        if (KIND == 0) { P.A2 = 1; P.A1 = 1; P.LA = J.L[0]; P.lo_in = J.lo[0]; P.Kout = H; P.out_c = J.spec0; }
        if (KIND == 4) { P.A2 = 1; P.A1 = 1; P.LA = H; P.Kout = J.L[0]; P.lo_out = J.lo[0]; P.in_c = J.spec0; }
    }
    return P;
}

// One work item of a pass (kTL = fft_lines_per_item lines of one job), all threads of the
// block.  stage holds kTL rows of N and zl (KIND 0) 4 LW rows of N; tw the twiddles
// (stride TWS).
template <int N, int KIND, int TWS>
__device__ __forceinline__ void fft_pass_item(const ProdJob &J, const int4 itm, const float2 *tw,
                                              float2 (*stage)[N], float2 (*zl)[N])
{
    using S = FftShape<N>;
    constexpr int G = S::G, E = S::E, LW = S::LW, LOG = S::LOG;
    constexpr int LPR = 4 * LW;  // complex lines per round (4 waves)
    constexpr int kTL = fft_lines_per_item(KIND, N);
    constexpr bool FWD = KIND <= 2 || KIND == 5, MUL = KIND == 2 || KIND == 5, INV = KIND >= 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane % G, slot = wave * LW + lane / G;
    {
        const PassGeom P = pass_geom<KIND>(J);
        const int M = J.M, B = 2 * M + 1;
        const int a2 = itm.y, a10 = itm.z;
        const int nl = min(kTL, P.A1 - a10);
        const bool paired = (KIND == 0 || KIND == 4);
        const int ncl = paired ? (nl + 1) / 2 : nl;
        const int rounds = (ncl + LPR - 1) / LPR;
        for (int r = 0; r < rounds; ++r) {
            const int li = r * LPR + slot;
            const bool act = li < ncl;
            float2 x[E];
            // ---- load
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int q = g + G * e;
                float2 v = make_float2(0.0f, 0.0f);
                if (act) {
                    if (KIND == 0) {
                        const int i = q - P.lo_in;
                        if (i >= 0 && i < P.LA) {
                            const int la = a10 + 2 * li, lb = la + 1;
                            v.x = gp(P.in_r)[((int64_t)a2 * P.A1 + la) * P.LA + i];
                            if (lb < a10 + nl) v.y = gp(P.in_r)[((int64_t)a2 * P.A1 + lb) * P.LA + i];
                        }
                    } else if (KIND == 1 || KIND == 2) {
                        const int i = q - P.lo_in;
                        if (i >= 0 && i < P.LA) v = ld2(P.in_c, ((int64_t)a2 * P.A1 + a10 + li) * P.LA + i);
                    } else if (KIND == 5) {  // g0-major input: line elements H B apart
                        const int i = q - P.lo_in;
                        if (i >= 0 && i < P.LA) v = ld2(P.in_c, ((int64_t)i * P.A2 + a2) * P.A1 + a10 + li);
                    } else {
                        const int f = (int)(__brev((unsigned)q) >> (32 - LOG));
                        const int fs = f < N / 2 ? f : f - N;
                        if (KIND == 3) {
                            if (fs >= -M && fs <= M)
                                v = ld2(P.in_c, ((int64_t)a2 * P.A1 + a10 + li) * P.LA + fs + M);
                        } else {  // KIND 4: Hermitian half spectra of two real lines
                            const int la = a10 + 2 * li, lb = la + 1;
                            const int fa = fs >= 0 ? fs : -fs;
                            if (fa <= M) {
                                float2 A = ld2(P.in_c, ((int64_t)a2 * P.A1 + la) * P.LA + fa);
                                float2 Bv = lb < a10 + nl ? ld2(P.in_c, ((int64_t)a2 * P.A1 + lb) * P.LA + fa)
                                                          : make_float2(0.0f, 0.0f);
                                if (J.d == 1) {
                                    const float dm = gp(J.D)[fa];
                                    A.x *= dm; A.y *= dm; Bv.x *= dm; Bv.y *= dm;
                                }
                                if (fa == 0) {
                                    v = make_float2(A.x, Bv.x);
                                } else if (fs > 0) {
                                    v = make_float2(A.x - Bv.y, A.y + Bv.x);
                                } else {
                                    v = make_float2(A.x + Bv.y, Bv.x - A.y);
                                }
                            }
                        }
                    }
                }
                x[e] = v;
            }
            // ---- transform
            if (FWD) fft_dif<N, TWS>(x, g, tw);
            if (MUL) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int q = g + G * e;
                    const int f = (int)(__brev((unsigned)q) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    float dm = 0.0f;
                    if (act && fs >= -M && fs <= M)
                        dm = gp(J.D)[((int64_t)a2 * P.A1 + a10 + li) * B + fs + M];
                    x[e].x *= dm;
                    x[e].y *= dm;
                }
            }
            if (INV) fft_dit_inv<N, TWS>(x, g, tw);
            // ---- store
            if (KIND == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int q = g + G * e;
                    const int f = (int)(__brev((unsigned)q) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    if (fs >= -M && fs <= M) zl[slot][fs + M] = x[e];
                }
                __syncthreads();
                // unpack A(k) = (Z(k) + conj Z(-k)) / 2, B(k) = (Z(k) - conj Z(-k)) / (2i)
                for (int t = tid; t < LPR * (M + 1); t += blockDim.x) {
                    const int sl = t / (M + 1), k = t - sl * (M + 1);
                    const int lj = r * LPR + sl;
                    if (lj >= ncl) continue;
                    const float2 z = zl[sl][k + M], zm = zl[sl][M - k];
                    const int ta = 2 * lj, tb = ta + 1;
                    stage[ta][k] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
                    if (tb < nl) stage[tb][k] = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
                }
                __syncthreads();
            } else if (KIND == 1) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int q = g + G * e;
                    const int f = (int)(__brev((unsigned)q) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    if (act && fs >= -M && fs <= M) stage[li][fs + M] = x[e];
                }
            } else if (KIND == 2 || KIND == 3 || KIND == 5) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int q = g + G * e;
                    const int i = q - P.lo_out;
                    if (act && i >= 0 && i < P.Kout) stage[li][i] = x[e];
                }
            } else {  // KIND 4: real outputs, contiguous along the line
                const int la = a10 + 2 * li, lb = la + 1;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int q = g + G * e;
                    const int i = q - P.lo_out;
                    if (act && i >= 0 && i < P.Kout) {
                        gp(P.out_r)[((int64_t)a2 * P.A1 + la) * P.Kout + i] = x[e].x;
                        if (lb < a10 + nl) gp(P.out_r)[((int64_t)a2 * P.A1 + lb) * P.Kout + i] = x[e].y;
                    }
                }
            }
        }
        if (KIND <= 3 || KIND == 5) {
            __syncthreads();
            // out layout: KIND 0, 2, 5: [k][a2][a1];  KIND 1, 3: [a2][k][a1]
            for (int t = tid; t < P.Kout * nl; t += blockDim.x) {
                const int k = t / nl, l = t - k * nl;
                int64_t o;
                if (KIND == 0 || KIND == 2 || KIND == 5)
                    o = ((int64_t)k * P.A2 + a2) * P.A1 + a10 + l;
                else
                    o = ((int64_t)a2 * P.Kout + k) * P.A1 + a10 + l;
                st2(P.out_c, o, stage[l][k]);
            }
            __syncthreads();
        }
    }
}

template <int N, int KIND>
__global__ __launch_bounds__(256) void fft_pass_kernel(const ProdJob *__restrict__ jobs,
                                                       const int4 *__restrict__ items, int n_items,
                                                       const float2 *__restrict__ twiddle)
{
    constexpr int LPR = 4 * FftShape<N>::LW;
    __shared__ float2 tw[N / 2];
    __shared__ float2 stage[fft_lines_per_item(KIND, N)][N];
    __shared__ float2 zl[KIND == 0 ? LPR : 1][N];
    for (int t = threadIdx.x; t < N / 2; t += blockDim.x) tw[t] = ld2(twiddle, t);
    __syncthreads();
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        fft_pass_item<N, KIND, 1>(jobs[itm.x], itm, tw, stage, zl);
    }
}

// Mixed grid sizes n <= 128 in one launch (batches of plans): each item runs the pass of
// its job's n with the 128-point twiddles at stride 128 / n, so its values are those of
// fft_pass_kernel<n>.  For every n <= 128 an item's lines times n is 512 complex values
// (1024 in the real-data passes 0 and 4), which stage holds, and zl holds 512.
constexpr int kMixedN = 128;

template <int KIND>
__global__ __launch_bounds__(256) void fft_pass_mixed_kernel(const ProdJob *__restrict__ jobs,
                                                             const int4 *__restrict__ items, int n_items,
                                                             const float2 *__restrict__ twiddle128)
{
    __shared__ float2 tw[kMixedN / 2];
    __shared__ float2 stage[(KIND == 0 || KIND == 4 ? 2 : 1) * 4 * kMixedN];
    __shared__ float2 zl[KIND == 0 ? 512 : kMixedN];
    for (int t = threadIdx.x; t < kMixedN / 2; t += blockDim.x) tw[t] = ld2(twiddle128, t);
    __syncthreads();
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        switch (J.n) {
#define MOT_MIXED_PASS(NN)                                                                                   \
    case NN:                                                                                                 \
        fft_pass_item<NN, KIND, kMixedN / NN>(J, itm, tw, reinterpret_cast<float2(*)[NN]>(stage),            \
                                              reinterpret_cast<float2(*)[NN]>(zl));                          \
        break;
            MOT_MIXED_PASS(16)
            MOT_MIXED_PASS(32)
            MOT_MIXED_PASS(64)
            MOT_MIXED_PASS(128)
#undef MOT_MIXED_PASS
        default: break;
        }
    }
}


// ---------------------------------------------------------------------------------------
// Slab passes of the 3-D transform: one box slab g0 per work item, both in-slab axes, with
// the slab's half spectrum X[L1][H] held in LDS between them.
//   forward: grid[g0][L1][L2] --R2C axis 2--> X[L1][H] --FWD axis 1--> spec1[g0][H][B]
//   inverse: spec0[g0][H][B] --INV axis 1--> X[L1][H] --C2R axis 2--> grid[g0][L1][L2]
// Lines are transformed exactly as in passes 0, 1 (forward) and 3, 4 (inverse).
// One slab item, all threads of the block: X holds the slab's half spectrum (kSlabLds
// bytes), zl (forward) 12 LW rows of N, tw the twiddles (stride TWS).
template <int N, bool INVERSE, int TWS>
__device__ __forceinline__ void fft_slab_item(const ProdJob &J, const int4 itm, const float2 *tw,
                                              float2 *X, float2 (*zl)[N])
{
    using S = FftShape<N>;
    constexpr int G = S::G, E = S::E, LW = S::LW, LOG = S::LOG;
    constexpr int LPR = (kSlabThreads / 64) * LW;  // lines per round
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane % G, slot = wave * LW + lane / G;
    {
        const int g0 = itm.y, M = J.M, H = M + 1, B = 2 * M + 1;
        const int L1 = J.L[1], L2 = J.L[2], lo1 = J.lo[1], lo2 = J.lo[2];
        const int ncl = (L1 + 1) / 2;  // complex lines carrying two real lines of axis 2
        MOT_GLOBAL float *grid = gp(J.grid) + (int64_t)g0 * L1 * L2;
        if constexpr (!INVERSE) {
            for (int c0 = 0; c0 < ncl; c0 += LPR) {
                const int c = c0 + slot, la = 2 * c, lb = la + 1;
                const bool act = c < ncl;
                float2 x[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = g + G * e - lo2;
                    float2 v = make_float2(0.0f, 0.0f);
                    if (act && i >= 0 && i < L2) {
                        v.x = grid[(int64_t)la * L2 + i];
                        if (lb < L1) v.y = grid[(int64_t)lb * L2 + i];
                    }
                    x[e] = v;
                }
                fft_dif<N, TWS>(x, g, tw);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int f = (int)(__brev((unsigned)(g + G * e)) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    if (act && fs >= -M && fs <= M) zl[slot][fs + M] = x[e];
                }
                __builtin_amdgcn_wave_barrier();  // the line's band is read back by its own wavefront
                // unpack A(k) = (Z(k) + conj Z(-k)) / 2, B(k) = (Z(k) - conj Z(-k)) / (2i)
                if (act)
                    for (int k = g; k < H; k += G) {
                        const float2 z = zl[slot][k + M], zm = zl[slot][M - k];
                        X[la * H + k] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
                        if (lb < L1) X[lb * H + k] = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
                    }
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            for (int k0 = 0; k0 < H; k0 += LPR) {
                const int k2 = k0 + slot;
                const bool act = k2 < H;
                float2 x[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = g + G * e - lo1;
                    x[e] = (act && i >= 0 && i < L1) ? X[i * H + k2] : make_float2(0.0f, 0.0f);
                }
                fft_dif<N, TWS>(x, g, tw);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int f = (int)(__brev((unsigned)(g + G * e)) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    if (act && fs >= -M && fs <= M) st2(J.spec1, ((int64_t)g0 * H + k2) * B + fs + M, x[e]);
                }
            }
            __syncthreads();  // X is rewritten by the next item
        } else {
            for (int k0 = 0; k0 < H; k0 += LPR) {
                const int k2 = k0 + slot;
                const bool act = k2 < H;
                float2 x[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int f = (int)(__brev((unsigned)(g + G * e)) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    x[e] = (act && fs >= -M && fs <= M) ? ld2(J.spec0, ((int64_t)g0 * H + k2) * B + fs + M)
                                                        : make_float2(0.0f, 0.0f);
                }
                fft_dit_inv<N, TWS>(x, g, tw);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = g + G * e - lo1;
                    if (act && i >= 0 && i < L1) X[i * H + k2] = x[e];
                }
            }
            __syncthreads();
            for (int c0 = 0; c0 < ncl; c0 += LPR) {
                const int c = c0 + slot, la = 2 * c, lb = la + 1;
                const bool act = c < ncl;
                float2 x[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int f = (int)(__brev((unsigned)(g + G * e)) >> (32 - LOG));
                    const int fs = f < N / 2 ? f : f - N;
                    const int fa = fs >= 0 ? fs : -fs;
                    float2 v = make_float2(0.0f, 0.0f);
                    if (act && fa <= M) {
                        // Hermitian half spectra of two real lines, combined as Z = A + i B
                        const float2 A = X[la * H + fa];
                        const float2 Bv = lb < L1 ? X[lb * H + fa] : make_float2(0.0f, 0.0f);
                        if (fa == 0) {
                            v = make_float2(A.x, Bv.x);
                        } else if (fs > 0) {
                            v = make_float2(A.x - Bv.y, A.y + Bv.x);
                        } else {
                            v = make_float2(A.x + Bv.y, Bv.x - A.y);
                        }
                    }
                    x[e] = v;
                }
                fft_dit_inv<N, TWS>(x, g, tw);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = g + G * e - lo2;
                    if (act && i >= 0 && i < L2) {
                        grid[(int64_t)la * L2 + i] = x[e].x;
                        if (lb < L1) grid[(int64_t)lb * L2 + i] = x[e].y;
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int N, bool INVERSE>
__global__ __launch_bounds__(kSlabThreads) void fft_slab_kernel(const ProdJob *__restrict__ jobs,
                                                                const int4 *__restrict__ items, int n_items,
                                                                const float2 *__restrict__ twiddle)
{
    constexpr int LPR = (kSlabThreads / 64) * FftShape<N>::LW;
    __shared__ float2 tw[N / 2];
    __shared__ float2 X[kSlabLds / 8];
    __shared__ float2 zl[INVERSE ? 1 : LPR][N];
    for (int t = threadIdx.x; t < N / 2; t += blockDim.x) tw[t] = ld2(twiddle, t);
    __syncthreads();
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        fft_slab_item<N, INVERSE, 1>(jobs[itm.x], itm, tw, X, zl);
    }
}

// Mixed grid sizes n <= 128 in one slab launch, as fft_pass_mixed_kernel (zl: 12 LW rows
// of n are 1536 complex values for every n <= 128).
template <bool INVERSE>
__global__ __launch_bounds__(kSlabThreads) void fft_slab_mixed_kernel(const ProdJob *__restrict__ jobs,
                                                                      const int4 *__restrict__ items, int n_items,
                                                                      const float2 *__restrict__ twiddle128)
{
    __shared__ float2 tw[kMixedN / 2];
    __shared__ float2 X[kSlabLds / 8];
    __shared__ float2 zl[INVERSE ? kMixedN : (kSlabThreads / 64) * kMixedN];
    for (int t = threadIdx.x; t < kMixedN / 2; t += blockDim.x) tw[t] = ld2(twiddle128, t);
    __syncthreads();
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 itm = items[it];
        const ProdJob &J = jobs[itm.x];
        switch (J.n) {
#define MOT_MIXED_SLAB(NN)                                                                                     \
    case NN:                                                                                                   \
        fft_slab_item<NN, INVERSE, kMixedN / NN>(J, itm, tw, X, reinterpret_cast<float2(*)[NN]>(zl));          \
        break;
            MOT_MIXED_SLAB(16)
            MOT_MIXED_SLAB(32)
            MOT_MIXED_SLAB(64)
            MOT_MIXED_SLAB(128)
#undef MOT_MIXED_SLAB
        default: break;
        }
    }
}

template <int N>
static hipError_t launch_n(int kind, const ProdJob *jobs, const int4 *items, int n_items,
                           const float2 *tw, hipStream_t s)
{
    const int grid = n_items < 8192 ? n_items : 8192;
    switch (kind) {
    case 0: hipLaunchKernelGGL((fft_pass_kernel<N, 0>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 1: hipLaunchKernelGGL((fft_pass_kernel<N, 1>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 2: hipLaunchKernelGGL((fft_pass_kernel<N, 2>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 3: hipLaunchKernelGGL((fft_pass_kernel<N, 3>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 4: hipLaunchKernelGGL((fft_pass_kernel<N, 4>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 5: hipLaunchKernelGGL((fft_pass_kernel<N, 5>), dim3(grid), dim3(256), 0, s, jobs, items, n_items, tw); break;
    case 6: hipLaunchKernelGGL((fft_slab_kernel<N, false>), dim3(grid), dim3(kSlabThreads), 0, s, jobs, items, n_items, tw); break;
    case 7: hipLaunchKernelGGL((fft_slab_kernel<N, true>), dim3(grid), dim3(kSlabThreads), 0, s, jobs, items, n_items, tw); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_pass(int kind, int n, const ProdJob *jobs, const int4 *items, int n_items,
                           const float2 *twiddle, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (n == 0) {  // jobs with grids n <= 128 of several sizes; twiddle: the 128-point table
        const int grid = n_items < 8192 ? n_items : 8192;
        switch (kind) {
        case 0: hipLaunchKernelGGL(fft_pass_mixed_kernel<0>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 1: hipLaunchKernelGGL(fft_pass_mixed_kernel<1>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 2: hipLaunchKernelGGL(fft_pass_mixed_kernel<2>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 3: hipLaunchKernelGGL(fft_pass_mixed_kernel<3>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 4: hipLaunchKernelGGL(fft_pass_mixed_kernel<4>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 5: hipLaunchKernelGGL(fft_pass_mixed_kernel<5>, dim3(grid), dim3(256), 0, s, jobs, items, n_items, twiddle); break;
        case 6: hipLaunchKernelGGL(fft_slab_mixed_kernel<false>, dim3(grid), dim3(kSlabThreads), 0, s, jobs, items, n_items, twiddle); break;
        case 7: hipLaunchKernelGGL(fft_slab_mixed_kernel<true>, dim3(grid), dim3(kSlabThreads), 0, s, jobs, items, n_items, twiddle); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (n) {
    case 16: return launch_n<16>(kind, jobs, items, n_items, twiddle, s);
    case 32: return launch_n<32>(kind, jobs, items, n_items, twiddle, s);
    case 64: return launch_n<64>(kind, jobs, items, n_items, twiddle, s);
    case 128: return launch_n<128>(kind, jobs, items, n_items, twiddle, s);
    case 256: return launch_n<256>(kind, jobs, items, n_items, twiddle, s);
    case 512: return launch_n<512>(kind, jobs, items, n_items, twiddle, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mot
