// Circle-structured Sinkhorn (a9, Algorithm 3) on gfx950.
//
// Algorithm 3 keeps the matrices beta_k = alpha^{(k,1)} (n_k x n_1) and
// gamma_k = lambda^{(1,k)} (n_1 x n_k).  Both are stored here as n_1 x n_k row-major
// matrices: Yb_k = beta_k^T and Yg_k = gamma_k.  With Kmat(a, b)[i][j] =
// exp(-|x^a_i - x^b_j|^2 / eta) the recursions read
//   Yb_k = Yb_{k+1} diag(phi^{k+1}) Kmat(k, k+1)^T      (k = K-2 .. 1, Yb_{K-1} = Kmat(0, K-1))
//   Yg_k = Yg_{k-1} diag(phi^{k-1}) Kmat(k, k-1)^T      (k = 2 .. K-1, Yg_1 = Kmat(0, 1))
// -- one GEMM shape C = A diag(phi) B^T with a constant kernel matrix B -- and the
// row-wise inner products of Theorem 4.3 become
//   phi^k_j = mu^k_j / sum_i Yb_k[i][j] phi^0_i Yg_k[i][j]                   (column sums)
//   phi^0_i = mu^0_i / sum_j Kmat(0,1)[i][j] phi^1_j Yb_1[i][j]               (row sums)
//
// Dense path: each product forms A' = diag(2^-rexp) A diag(phi) in FP64 and rounds it to
// the 16-bit operand (scale_rows16_kernel); C = A' B^T is then a 16-bit GEMM with FP32
// accumulation and output on the MFMA units (v_mfma_f32_32x32x16_bf16 / _f16):
// gemm_big_kernel / gemm_big_split_kernel for products whose dimensions are multiples of
// 256 with enough 256 x 256 tiles to fill the chip, gemm_kernel (64 x 64 tiles) otherwise.
// Precision modes: BF16, FP16 and split BF16 (A' = Ah + Al, B = Bh + Bl,
// C = Ah Bh + Ah Bl + Al Bh).  The
// FP32 matrices carry a power-of-two scale per row: before each product the rows of
// A diag(phi) are normalised (exponent of their largest entry, taken in FP64) and the
// exponent is added to the row's scale, so long chains of products (K up to thousands of
// times n_k growth per step) stay in range.  The reductions apply the scales in FP64.
// NFFT path: every row of a product is one fast summation (column by column in the
// paper's words), run by the tree path's spreading / FFT / interpolation kernels with
// one job per row; matrices are FP64.
#include <algorithm>
#include <cmath>

#include "host.h"

namespace mot {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kBK = 32, kLdsK = kBK + 8;  // K step and padded LDS row (elements) of gemm_kernel

__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    __bf16 h = (__bf16)x;  // round to nearest even
    return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_value(unsigned short b)
{
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ __forceinline__ unsigned short f16_bits(float x)
{
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}


// C[M x N] (row-major, ldc) = A'[M x K] B[N x K]^T with A' from scale_rows16_kernel (lda)
// and B the 16-bit kernel matrix (ldb), all dimensions padded to the tile sizes by the
// caller (zero padding).  MODE: 0 BF16, 1 FP16, 2 split BF16 (hi hi + hi lo + lo hi), the
// three products accumulated in one FP32 accumulator.  A group of four wavefronts owns a
// BT x BT tile of C, wave w the (BT/2) x (BT/2) block (w / 2, w % 2).  BT = 64: a 128 x 128
// tile (64 x 64 per wave) ran slower at every measured shape, from 512 to 2304 rows (fewer
// workgroups to hide the latency of the register-staged loads).
//
// A workgroup holds KS such groups that split the K steps of its tile: group g takes the
// contiguous steps [g S / KS, (g + 1) S / KS) of the S = K / kBK, and the groups'
// accumulators are added in group order through LDS at the end.  Each K step waits on a
// round trip of its operand loads and holds little MFMA work, so a product with few tiles
// (a few hundred rows) is bound by that chain; KS > 1 shortens it without another launch
// and keeps the sum order fixed for a given shape.
constexpr int kSmallT = 64;
template <int MODE, int KS>
__global__ __launch_bounds__(256 * KS) void gemm_kernel(const unsigned short *__restrict__ Ah,
                                                        const unsigned short *__restrict__ Al, int lda,
                                                        const unsigned short *__restrict__ Bh,
                                                        const unsigned short *__restrict__ Bl, int ldb,
                                                        float *__restrict__ C, int ldc, int K)
{
    constexpr int BT = kSmallT, WT = BT / 2, FR = WT / 32;  // wave tile, 32 x 32 fragments per dimension
    constexpr int TPR = 256 / BT, NU = 4 / TPR;  // threads per staged row, 16-byte loads each
    constexpr int TS = BT * kLdsK;               // one staged operand tile (elements)
    constexpr int NOP = MODE == 2 ? 4 : 2;       // staged operands: Ah, Bh (, Al, Bl)
    // the LDS holds the groups' staged tiles, and at the end the partial accumulators of
    // groups 1 .. KS-1 (16 floats per lane)
    constexpr int kPart = (KS - 1) * 4 * 64 * 16 * 2, kStaged = KS * NOP * TS;
    static_assert(FR == 1, "one 32 x 32 accumulator per wave");
    __shared__ __align__(16) unsigned short lds[kStaged > kPart ? kStaged : kPart];
    const int grp = KS == 1 ? 0 : (int)(threadIdx.x >> 8), tid = threadIdx.x & 255, lane = tid & 63, wave = tid >> 6;
    unsigned short *As = lds + grp * NOP * TS, *Bs = As + TS, *Asl = As + 2 * TS, *Bsl = As + 3 * TS;
    const int wm = (wave >> 1) * WT, wn = (wave & 1) * WT;
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    const int steps = K / kBK, s_lo = grp * steps / KS, s_hi = (grp + 1) * steps / KS;
    const int s_max = (steps + KS - 1) / KS;  // every group runs s_max rounds (barriers are block-wide)
    f32x16 acc[FR][FR];
#pragma unroll
    for (int i = 0; i < FR; ++i)
#pragma unroll
        for (int j = 0; j < FR; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    // global staging assignment: row tid / TPR of each operand tile, 8 NU k values from
    // (tid % TPR) 8 NU; the next K step's tiles are fetched into registers while the current
    // one is multiplied
    const int ar = tid / TPR, ac = (tid % TPR) * 8 * NU;
    const unsigned short *pa = Ah + (int64_t)(m0 + ar) * lda + ac, *pb = Bh + (int64_t)(n0 + ar) * ldb + ac;
    const unsigned short *pal = MODE == 2 ? Al + (int64_t)(m0 + ar) * lda + ac : nullptr;
    const unsigned short *pbl = MODE == 2 ? Bl + (int64_t)(n0 + ar) * ldb + ac : nullptr;
    uint4 ga[NU], gb[NU], gal[NU], gbl[NU];
    auto fetch = [&](int step) {
        const int kn = step * kBK;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            ga[u] = reinterpret_cast<const uint4 *>(pa + kn)[u];
            gb[u] = reinterpret_cast<const uint4 *>(pb + kn)[u];
            if (MODE == 2) {
                gal[u] = reinterpret_cast<const uint4 *>(pal + kn)[u];
                gbl[u] = reinterpret_cast<const uint4 *>(pbl + kn)[u];
            }
        }
    };
    if (s_lo < s_hi) fetch(s_lo);
    for (int it = 0; it < s_max; ++it) {
        const bool active = s_lo + it < s_hi;
        if (active) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                reinterpret_cast<uint4 *>(&As[ar * kLdsK + ac])[u] = ga[u];
                reinterpret_cast<uint4 *>(&Bs[ar * kLdsK + ac])[u] = gb[u];
                if (MODE == 2) {
                    reinterpret_cast<uint4 *>(&Asl[ar * kLdsK + ac])[u] = gal[u];
                    reinterpret_cast<uint4 *>(&Bsl[ar * kLdsK + ac])[u] = gbl[u];
                }
            }
        }
        __syncthreads();
        if (s_lo + it + 1 < s_hi) fetch(s_lo + it + 1);
        if (active) {
#pragma unroll
            for (int ks = 0; ks < kBK; ks += 16) {
                const int kk = ks + 8 * (lane >> 5);
#pragma unroll
                for (int i = 0; i < FR; ++i) {
                    const int ra = wm + 32 * i + (lane & 31);
                    const uint4 a_h = *reinterpret_cast<const uint4 *>(&As[ra * kLdsK + kk]);
                    uint4 a_l;
                    if (MODE == 2) a_l = *reinterpret_cast<const uint4 *>(&Asl[ra * kLdsK + kk]);
#pragma unroll
                    for (int j = 0; j < FR; ++j) {
                        const int rb = wn + 32 * j + (lane & 31);
                        const uint4 b_h = *reinterpret_cast<const uint4 *>(&Bs[rb * kLdsK + kk]);
                        if (MODE == 1) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(f16x8, a_h), __builtin_bit_cast(f16x8, b_h), acc[i][j], 0, 0, 0);
                        } else {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, a_h), __builtin_bit_cast(bf16x8, b_h), acc[i][j], 0, 0, 0);
                            if (MODE == 2) {
                                const uint4 b_l = *reinterpret_cast<const uint4 *>(&Bsl[rb * kLdsK + kk]);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    __builtin_bit_cast(bf16x8, a_h), __builtin_bit_cast(bf16x8, b_l), acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    __builtin_bit_cast(bf16x8, a_l), __builtin_bit_cast(bf16x8, b_h), acc[i][j], 0, 0, 0);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if constexpr (KS > 1) {
        // groups 1 .. KS-1 leave their accumulators in the (now idle) staging LDS; group 0
        // adds them in group order
        f32x16 *part = reinterpret_cast<f32x16 *>(lds);
        if (grp > 0) part[((grp - 1) * 4 + wave) * 64 + lane] = acc[0][0];
        __syncthreads();
        if (grp > 0) return;
#pragma unroll
        for (int g = 1; g < KS; ++g) {
            const f32x16 v = part[((g - 1) * 4 + wave) * 64 + lane];
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[0][0][r] += v[r];
        }
    }
    // epilogue: acc[i][j][r] -> row wm + 32i + 8(r/4) + 4(lane/32) + r%4, col wn + 32j + lane%32
#pragma unroll
    for (int i = 0; i < FR; ++i)
#pragma unroll
        for (int j = 0; j < FR; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn + 32 * j + (lane & 31);
                C[(int64_t)row * ldc + col] = acc[i][j][r];
            }
}

// ---------------------------------------------------------------------------------------
// Large products, C[M x N] = A'[M x K] B[N x K]^T with M and N multiples of 256 and K of
// 128 (the dense matrices of at least 2048 points are padded to 256).  A workgroup of 16
// wavefronts owns a 256 x 256 tile of C, wave w the 64 x 64 block (w / 4, w % 4): per k16
// step two A and two B fragments from LDS and four 32x32x16 MFMAs.  Operand tiles of 256
// rows x 32 k move from global memory straight into LDS with global_load_lds_dwordx4 (no
// register staging): one such instruction writes each lane's 16 bytes at LDS base + 16 lane,
// so a wavefront fills 16 rows of 64 bytes.  Rows are not padded; the 16-byte chunk c of
// row r is stored at chunk c ^ ((r >> 1) & 3), which puts the 8 lanes of an LDS read phase
// (8 consecutive rows, one chunk) on 8 different bank groups.
typedef __attribute__((address_space(3))) void lds_void;
constexpr int kBigT = 256, kBigK = 32, kBigWaves = 16;

__device__ __forceinline__ int big_swizzle(int r) { return (r >> 1) & 3; }

// Tile (m0, n0) of block b: groups of four tile rows, consecutive blocks down a group's
// columns, so the blocks running together share A rows and B rows in L2.
__device__ __forceinline__ void big_tile(int b, int tiles_m, int tiles_n, int *m0, int *n0)
{
    const int group = b / (4 * tiles_n), first = group * 4;
    const int gm = min(4, tiles_m - first);
    const int rem = b % (4 * tiles_n);
    *m0 = (first + rem % gm) * kBigT;
    *n0 = (rem / gm) * kBigT;
}

// Loads of one operand part for k step kt into a stage: wave w fills row group w (rows
// 16 w .. 16 w + 15 of the A tile and of the B tile).
__device__ __forceinline__ void big_issue(const unsigned short *A, int lda, const unsigned short *B, int ldb, int m0,
                                          int n0, int k0, unsigned short *sA, unsigned short *sB, int wave, int lane)
{
    const int r = 16 * wave + (lane >> 2);
    const int c = (lane & 3) ^ big_swizzle(r);
    __builtin_amdgcn_global_load_lds((const void *)(A + (int64_t)(m0 + r) * lda + k0 + 8 * c),
                                     (lds_void *)(sA + wave * 512), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void *)(B + (int64_t)(n0 + r) * ldb + k0 + 8 * c),
                                     (lds_void *)(sB + wave * 512), 16, 0, 0);
}

// Fragment of the lane for rows (base + lane % 32) and the lane's 8 k values of step ks.
__device__ __forceinline__ uint4 big_frag(const unsigned short *s, int base, int ks, int lane)
{
    const int r = base + (lane & 31);
    const int cl = ks / 8 + (lane >> 5);
    return *reinterpret_cast<const uint4 *>(s + r * kBigK + 8 * (cl ^ big_swizzle(r)));
}

__device__ __forceinline__ void big_store(const f32x16 (&acc)[2][2], float *C, int ldc, int m0, int n0, int wm,
                                          int wn, int lane)
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn + 32 * j + (lane & 31);
                C[(int64_t)row * ldc + col] = acc[i][j][r];
            }
}

// BF16 (MODE 0) and FP16 (MODE 1).  Four stages, each its own LDS object: the compiler
// then sees that the stage being loaded is not the stage being read and does not wait for
// the loads in flight before reading LDS.  Stages are taken two per barrier: after the
// barrier of pair (s0, s1) every wavefront has finished reading (s2, s3), whose next tiles
// are requested while (s0, s1) are multiplied.
template <int MODE>
__global__ __launch_bounds__(64 * kBigWaves, 1) void gemm_big_kernel(const unsigned short *__restrict__ A, int lda,
                                                                      const unsigned short *__restrict__ B, int ldb,
                                                                      float *__restrict__ C, int ldc, int K, int tiles_m,
                                                                      int tiles_n)
{
    constexpr int TILE = kBigT * kBigK;
    __shared__ __align__(16) unsigned short s0[2 * TILE], s1[2 * TILE], s2[2 * TILE], s3[2 * TILE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 2) * 64, wn = (wave & 3) * 64;
    int m0, n0;
    big_tile(blockIdx.x, tiles_m, tiles_n, &m0, &n0);
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    auto mult = [&](const unsigned short *sA) {
        const unsigned short *sB = sA + TILE;
#pragma unroll
        for (int ks = 0; ks < kBigK; ks += 16) {
            const uint4 a0 = big_frag(sA, wm, ks, lane), a1 = big_frag(sA, wm + 32, ks, lane);
            const uint4 b0 = big_frag(sB, wn, ks, lane), b1 = big_frag(sB, wn + 32, ks, lane);
            if constexpr (MODE == 1) {
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a0), __builtin_bit_cast(f16x8, b0), acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a0), __builtin_bit_cast(f16x8, b1), acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a1), __builtin_bit_cast(f16x8, b0), acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a1), __builtin_bit_cast(f16x8, b1), acc[1][1], 0, 0, 0);
            } else {
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0), acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b1), acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1), __builtin_bit_cast(bf16x8, b0), acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1), __builtin_bit_cast(bf16x8, b1), acc[1][1], 0, 0, 0);
            }
        }
    };
    // s_waitcnt with vmcnt(0) only (expcnt and lgkmcnt left at their maxima)
    constexpr int kWaitLoads = (7 << 4) | (15 << 8);
    const int nk = K / kBigK;  // a multiple of 4
    big_issue(A, lda, B, ldb, m0, n0, 0, s0, s0 + TILE, wave, lane);
    big_issue(A, lda, B, ldb, m0, n0, kBigK, s1, s1 + TILE, wave, lane);
    for (int kt = 0; kt < nk; kt += 4) {
        __builtin_amdgcn_s_waitcnt(kWaitLoads);  // this wave's part of tiles kt, kt + 1
        __builtin_amdgcn_s_barrier();            // everybody's part; (s2, s3) no longer read
        if (kt + 2 < nk) {
            big_issue(A, lda, B, ldb, m0, n0, (kt + 2) * kBigK, s2, s2 + TILE, wave, lane);
            big_issue(A, lda, B, ldb, m0, n0, (kt + 3) * kBigK, s3, s3 + TILE, wave, lane);
        }
        mult(s0);
        mult(s1);
        if (kt + 2 < nk) {
            __builtin_amdgcn_s_waitcnt(kWaitLoads);
            __builtin_amdgcn_s_barrier();
            if (kt + 4 < nk) {
                big_issue(A, lda, B, ldb, m0, n0, (kt + 4) * kBigK, s0, s0 + TILE, wave, lane);
                big_issue(A, lda, B, ldb, m0, n0, (kt + 5) * kBigK, s1, s1 + TILE, wave, lane);
            }
            mult(s2);
            mult(s3);
        }
    }
    big_store(acc, C, ldc, m0, n0, wm, wn, lane);
}

// Split BF16: Ah Bh + Ah Bl + Al Bh in one accumulator per block (three MFMAs per fragment
// pair).  A stage holds four operand tiles (64 KB), so two stages, each its own __shared__
// object as in gemm_big_kernel (with both in one array the compiler waits for the next
// tile's loads before every read of the current one): tile kt + 1 is requested while tile
// kt is multiplied, and the barrier (with its wait for every load of the wave) separates the
// steps.  K is a multiple of 4 kBigK.
__global__ __launch_bounds__(64 * kBigWaves, 1) void gemm_big_split_kernel(
    const unsigned short *__restrict__ Ah, const unsigned short *__restrict__ Al, int lda,
    const unsigned short *__restrict__ Bh, const unsigned short *__restrict__ Bl, int ldb, float *__restrict__ C,
    int ldc, int K, int tiles_m, int tiles_n)
{
    constexpr int TILE = kBigT * kBigK, STAGE = 4 * TILE;  // Ah, Bh, Al, Bl
    __shared__ __align__(16) unsigned short t0[STAGE], t1[STAGE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 2) * 64, wn = (wave & 3) * 64;
    int m0, n0;
    big_tile(blockIdx.x, tiles_m, tiles_n, &m0, &n0);
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    auto issue = [&](int kt, unsigned short *s) {
        big_issue(Ah, lda, Bh, ldb, m0, n0, kt * kBigK, s, s + TILE, wave, lane);
        big_issue(Al, lda, Bl, ldb, m0, n0, kt * kBigK, s + 2 * TILE, s + 3 * TILE, wave, lane);
    };
    auto mult = [&](const unsigned short *sAh) {
        const unsigned short *sBh = sAh + TILE, *sAl = sAh + 2 * TILE, *sBl = sAh + 3 * TILE;
#pragma unroll
        for (int ks = 0; ks < kBigK; ks += 16) {
            uint4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ah[i] = big_frag(sAh, wm + 32 * i, ks, lane);
                al[i] = big_frag(sAl, wm + 32 * i, ks, lane);
                bh[i] = big_frag(sBh, wn + 32 * i, ks, lane);
                bl[i] = big_frag(sBl, wn + 32 * i, ks, lane);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]), __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]), __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[i]), __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
                }
        }
    };
    // a wave multiplying runs at raised priority, so the arbiter prefers the MFMA stream of
    // waves past the barrier over waves still issuing their loads (split BF16 at N = 4000:
    // 422 -> 444 sweeps/s; no gain for the one-product kernel)
    const int nk = K / kBigK;  // even
    issue(0, t0);
    for (int kt = 0; kt < nk; kt += 2) {
        __syncthreads();  // tile kt in t0 for every wave; t1 no longer read
        issue(kt + 1, t1);
        __builtin_amdgcn_s_setprio(1);
        mult(t0);
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();  // tile kt + 1 in t1; t0 no longer read
        if (kt + 2 < nk) issue(kt + 2, t0);
        __builtin_amdgcn_s_setprio(1);
        mult(t1);
        __builtin_amdgcn_s_setprio(0);
    }
    big_store(acc, C, ldc, m0, n0, wm, wn, lane);
}

// One row of a product's left operand per block: rexp = exponent of max_l |A[i][l] phi_l|
// (in FP64; 0 for a zero row), the row scale s_out[i] = s_in[i] + rexp, and the 16-bit
// operand A'[i][l] = A[i][l] phi_l 2^-rexp (formed in FP64, rounded to FP32, then to FP16
// (MODE 1) or BF16 (MODE 0), or split into BF16 high and low parts (MODE 2)).  The row is
// read twice, the second time from cache.  Kp is a multiple of 8.
template <int MODE>
__global__ __launch_bounds__(256) void scale_rows16_kernel(const float *__restrict__ A, int lda, int Kp,
                                                           const double *__restrict__ phi,
                                                           const int32_t *__restrict__ s_in, int32_t *s_out,
                                                           unsigned short *__restrict__ Ah,
                                                           unsigned short *__restrict__ Al)
{
    __shared__ double red[4];
    const int i = blockIdx.x;
    const float *row = A + (int64_t)i * lda;
    double m = 0.0;
    for (int l = 4 * (int)threadIdx.x; l < Kp; l += 4 * 256) {
        const float4 a4 = *reinterpret_cast<const float4 *>(row + l);
        m = fmax(m, fabs((double)a4.x * phi[l]));
        m = fmax(m, fabs((double)a4.y * phi[l + 1]));
        m = fmax(m, fabs((double)a4.z * phi[l + 2]));
        m = fmax(m, fabs((double)a4.w * phi[l + 3]));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double mm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const int e = (mm > 0.0 && mm < INFINITY) ? ilogb(mm) : 0;
    if (threadIdx.x == 0) s_out[i] = s_in[i] + e;
    const double rowscale = ldexp(1.0, -e);
    for (int l0 = 8 * (int)threadIdx.x; l0 < Kp; l0 += 8 * 256) {
        const float4 *src = reinterpret_cast<const float4 *>(row + l0);
        unsigned short hv[8], lv[8];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float4 a4 = src[q];
            const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float x = (float)((double)av[u] * phi[l0 + 4 * q + u] * rowscale);
                if (MODE == 1) {
                    hv[4 * q + u] = f16_bits(x);
                } else {
                    hv[4 * q + u] = bf16_bits(x);
                    if (MODE == 2) lv[4 * q + u] = bf16_bits(x - bf16_value(hv[4 * q + u]));
                }
            }
        }
        *reinterpret_cast<uint4 *>(Ah + (int64_t)i * lda + l0) = *reinterpret_cast<uint4 *>(&hv[0]);
        if (MODE == 2) *reinterpret_cast<uint4 *>(Al + (int64_t)i * lda + l0) = *reinterpret_cast<uint4 *>(&lv[0]);
    }
}

// Kernel matrix in 16-bit form: Bh[i][j] = round(K(x^a_i, x^b_j)), Bl = round(rest) (split
// mode), zero padding.  grid: rows of 256 columns.
__global__ void kernel_matrix16_kernel(const double *__restrict__ xa, int64_t na, const double *__restrict__ xb,
                                       int64_t nb, int d, double eta, int ld, int64_t rows_pad, int mode,
                                       unsigned short *__restrict__ Bh, unsigned short *__restrict__ Bl)
{
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_pad || j >= ld) return;
    double v = 0.0;
    if (i < na && j < nb) {
        double d2 = 0.0;
        for (int c = 0; c < d; ++c) {
            const double df = xa[i * d + c] - xb[j * d + c];
            d2 += df * df;
        }
        v = exp(-d2 / eta);
    }
    const float vf = (float)v;
    if (mode == 1) {
        Bh[i * ld + j] = f16_bits(vf);
    } else {
        const unsigned short h = bf16_bits(vf);
        Bh[i * ld + j] = h;
        if (Bl) Bl[i * ld + j] = bf16_bits(vf - bf16_value(h));
    }
}

// FP32 or FP64 kernel matrix (the constant first matrices of both recursions).
template <class T>
__global__ void kernel_matrix_kernel(const double *__restrict__ xa, int64_t na, const double *__restrict__ xb,
                                     int64_t nb, int d, double eta, int ld, int64_t rows_pad, T *__restrict__ out)
{
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_pad || j >= ld) return;
    double v = 0.0;
    if (i < na && j < nb) {
        double d2 = 0.0;
        for (int c = 0; c < d; ++c) {
            const double df = xa[i * d + c] - xb[j * d + c];
            d2 += df * df;
        }
        v = exp(-d2 / eta);
    }
    out[i * ld + j] = (T)v;
}

// Column sums with FP64 accumulation (Theorem 4.3's row-wise inner products, stored
// transposed): part[ch][j] = sum_{i in chunk ch} Yb[i][j] w_i Yg[i][j] over the chunk's
// chunk_rows rows (at most kColRows), ascending, with w_i = phi^0_i 2^(sb[i] + sg[i]) formed
// here (sb, sg: the two matrices' row scales on the dense path; NULL on the NFFT path).
// One column per thread.
constexpr int kColRows = 64, kColRowsMin = 16;
template <class T>
__global__ __launch_bounds__(256) void colsum_kernel(const T *__restrict__ Yb, const T *__restrict__ Yg, int ld,
                                                     int64_t n1, int64_t nk, const double *__restrict__ phi0,
                                                     const int32_t *__restrict__ sb, const int32_t *__restrict__ sg,
                                                     int chunk_rows, double *__restrict__ part)
{
    __shared__ double w[kColRows];
    const int64_t i0 = (int64_t)blockIdx.y * chunk_rows;
    const int rows = (int)min((int64_t)chunk_rows, n1 - i0);
    if ((int)threadIdx.x < rows) {
        const int64_t i = i0 + threadIdx.x;
        w[threadIdx.x] = sb ? ldexp(phi0[i], sb[i] + sg[i]) : phi0[i];
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nk) return;
    const T *yb = Yb + i0 * ld + j, *yg = Yg + i0 * ld + j;
    double acc = 0.0;
#pragma unroll 8
    for (int r = 0; r < rows; ++r) acc += (double)yb[(int64_t)r * ld] * w[r] * (double)yg[(int64_t)r * ld];
    part[blockIdx.y * nk + j] = acc;
}

// Row sums for phi^0 from the resident kernel matrix Yg_1 = K^{(1,2)}:
// den_i = 2^rs[i] sum_j Yg_1[i][j] phi^1_j Yb_1[i][j] (Theorem 4.3's first inner product;
// rs: Yb_1's row scale on the dense path, NULL on the NFFT path), one block per row.
template <class T>
__global__ __launch_bounds__(256) void rowsum_k_kernel(const T *__restrict__ Yg1, const T *__restrict__ Yb1, int ld,
                                                       int64_t n1c, const double *__restrict__ phi1,
                                                       const int32_t *__restrict__ rs, double *__restrict__ den)
{
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n1c; j += blockDim.x)
        s += (double)Yg1[i * ld + j] * phi1[j] * (double)Yb1[i * ld + j];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        den[i] = rs ? ldexp(t, rs[i]) : t;
    }
}

// phi update from a denominator (column sums: nparts > 0 partial rows to add in order;
// row sums: nparts == 0 and den given directly).  Writes S terms to part_out[2 * block].
__global__ __launch_bounds__(256) void circle_phi_kernel(const double *__restrict__ part, int nparts,
                                                         int64_t n, const double *__restrict__ mu,
                                                         double *__restrict__ phi, int root,
                                                         double *__restrict__ s_out, int32_t *flag,
                                                         double *__restrict__ marg_out, int marg_only)
{
    __shared__ double red[2][4];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s1 = 0.0, s2 = 0.0;
    if (j < n) {
        double den = 0.0;
        if (nparts > 0) {
#pragma unroll 8
            for (int p = 0; p < nparts; ++p) den += part[p * n + j];
        } else
            den = part[j];
        const double m = mu[j], old = phi[j];
        if (marg_only) {
            const double P = old * den;
            marg_out[j] = P;
            s1 = fabs(P - m);
        } else {
            const double nv = m / den;
            if (m > 0.0) {
                s1 = m * log(old);
                if (root) s2 = (m / nv) * old;
            }
            if (!isfinite(nv)) atomicOr(flag, 1);
            phi[j] = nv;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s1;
        red[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_out[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        s_out[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Sweep finalisation: S^(r) from the phi-update partials, L1 error of the first marginal
// from P_0 = phi^0 den0 (partials written by circle_phi_kernel in marginal mode).
__global__ __launch_bounds__(256) void circle_final_kernel(const double *__restrict__ s_part, int ns,
                                                           const double *__restrict__ e_part, int ne,
                                                           double eta, int32_t *ctr, int hist_cap,
                                                           double *S_hist, double *err_hist, int32_t *flag,
                                                           int32_t *flag_hist)
{
    __shared__ double red[3][4];
    double s1 = 0.0, s2 = 0.0, e = 0.0;
    for (int p = threadIdx.x; p < ns; p += blockDim.x) {
        s1 += s_part[2 * p];
        s2 += s_part[2 * p + 1];
    }
    for (int p = threadIdx.x; p < ne; p += blockDim.x) e += e_part[2 * p];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
        e += __shfl_xor(e, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s1;
        red[1][threadIdx.x >> 6] = s2;
        red[2][threadIdx.x >> 6] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double S1 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double S2 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const double E = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
        const int r = *ctr, slot = r % hist_cap;
        S_hist[slot] = eta * (S1 - S2);
        err_hist[slot] = E;
        flag_hist[slot] = *flag;
        *ctr = r + 1;
    }
}

// Pair marginal Pi_{1,k}[i][j] = phi^0_i Yg_k[i][j] Yb_k[i][j] phi^k_j (times the rows'
// power-of-two scales on the dense path), written in the original orders of both
// marginals.  Rows strided over blockIdx.y, columns across threads.
template <class T>
__global__ void circle_pair_kernel(const T *__restrict__ Yg, const T *__restrict__ Yb, int ld, int64_t n1,
                                   int64_t nk, const double *__restrict__ phi0, const double *__restrict__ phik,
                                   const int32_t *__restrict__ sg, const int32_t *__restrict__ sb,
                                   const int32_t *__restrict__ perm0, const int32_t *__restrict__ permk,
                                   double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nk) return;
    for (int64_t i = blockIdx.y; i < n1; i += gridDim.y) {
        double v = ((phi0[i] * (double)Yg[i * ld + j]) * (double)Yb[i * ld + j]) * phik[j];
        if (sg) v = ldexp(v, sg[i] + sb[i]);
        out[(int64_t)perm0[i] * nk + permk[j]] = v;
    }
}

// NFFT path: src[i][l] = A[i][l] phi_l and the row's max exponent (one block per row).
__global__ __launch_bounds__(256) void scale_rows_kernel(const double *__restrict__ A, int64_t nl,
                                                         const double *__restrict__ phi, double *__restrict__ src,
                                                         int32_t *__restrict__ rexp)
{
    __shared__ int red[4];
    const int64_t i = blockIdx.x;
    int m = INT32_MIN;
    for (int64_t l = threadIdx.x; l < nl; l += blockDim.x) {
        const double v = A[i * nl + l] * phi[l];
        src[i * nl + l] = v;
        if (v > 0.0 && v < INFINITY) m = max(m, ilogb(v));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) rexp[i] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// ---------------------------------------------------------------------------------------
// Host side

static int pad_to(int64_t n, int q) { return (int)((n + q - 1) / q * q); }

struct CircleState {
    bool nfft = false;
    int mode = 0;                  // GEMM mode (dense path)
    int64_t n1 = 0;
    int n1p = 0;                   // rows of every matrix (padded on the dense path)
    std::vector<int> ld;           // leading dimension (columns) of the matrices of marginal k
    std::vector<void *> Yb;        // [K] Yb_k, k = 1..K-1 (Yb_{K-1} constant)
    void *Yg[2] = {nullptr, nullptr};
    void *Yg1 = nullptr;           // Yg_1 = Kmat(0, 1) (constant)
    std::vector<unsigned short *> Kb_h, Kb_l, Kg_h, Kg_l;  // dense: Kmat(k,k+1), Kmat(k,k-1)
    int32_t *rexp = nullptr;
    // dense path: the scaled left operand of a product in 16-bit form (n1p x ldmax each;
    // Al only for split BF16)
    unsigned short *Ah = nullptr, *Al = nullptr;
    // dense path: power-of-two scale of every row of each matrix (see the file comment)
    int K = 0;
    std::vector<int32_t *> sb;     // [K] row scales of Yb_k
    int32_t *sg[2] = {nullptr, nullptr};
    int32_t *szero = nullptr;      // the constant matrices Yg_1, Yb_{K-1}
    double *part = nullptr;        // column-sum partials [chunk][j]
    double *den0 = nullptr;
    double *s_part = nullptr;      // phi-update partials
    std::vector<int> s_slot;       // first partial slot of marginal k's phi update
    int ns = 0;
    double *e_part = nullptr;      // first-marginal L1 partials
    double *m_part = nullptr;      // scratch partials of marginal-only evaluations
    // NFFT path: per-row product jobs for each product position
    double *src = nullptr;
    int32_t *rowexp = nullptr;
    std::vector<std::vector<Step>> steps_g, steps_b;  // [k]
};

static void *Ymat(CircleState &C, int which_gamma, int k)
{
    if (which_gamma) return k == 1 ? C.Yg1 : C.Yg[k & 1];
    return C.Yb[k];
}

static int32_t *Yscale(CircleState &C, int which_gamma, int k)  // dense path only
{
    if (which_gamma) return k == 1 ? C.szero : C.sg[k & 1];
    return k == C.K - 1 ? C.szero : C.sb[k];
}

// Rows and columns of the dense path's matrices: multiples of 256 from 2048 points on (the
// shapes gemm_big can take), of 64 (gemm_kernel's tile) below.
static int dense_pad(int64_t n) { return n >= 2048 ? pad_to(n, 256) : pad_to(n, 64); }

// A dense product's GEMM runs on gemm_big_kernel / gemm_big_split_kernel when M, N and K
// are multiples of 256, 256 and 128 and the product has at least kBigMinTiles tiles of
// 256 x 256, else on the 64 x 64 tiles of gemm_kernel.  Below about 96 tiles the large
// kernel leaves most compute units idle: at 81 tiles (2304 rows) split BF16 ran 857 sweeps/s
// on it and 1095 on the small tiles; at 121 tiles (2816 rows) 692 against 617.
constexpr int kBigMinTiles = 96;
static bool gemm_big(int Mp, int Np, int Kp)
{
    return Mp % kBigT == 0 && Np % kBigT == 0 && Kp % (4 * kBigK) == 0 &&
           (Mp / kBigT) * (Np / kBigT) >= kBigMinTiles;
}

// K split of gemm_kernel by the product's count of 64 x 64 tiles: 1 from kSplitK1Tiles
// tiles on, 2 from kSplitK2Tiles, else 4.
constexpr int kSplitK1Tiles = 512, kSplitK2Tiles = 128;

template <int MODE>
static void launch_gemm_small(int ks, dim3 grid, const unsigned short *Ah, const unsigned short *Al, int lda,
                              const unsigned short *Bh, const unsigned short *Bl, int ldb, float *Cm, int ldc, int Kp,
                              hipStream_t s)
{
    if (ks == 4)
        hipLaunchKernelGGL((gemm_kernel<MODE, 4>), grid, dim3(1024), 0, s, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp);
    else if (ks == 2)
        hipLaunchKernelGGL((gemm_kernel<MODE, 2>), grid, dim3(512), 0, s, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp);
    else
        hipLaunchKernelGGL((gemm_kernel<MODE, 1>), grid, dim3(256), 0, s, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp);
}

// One product of the recursions on the dense path: the row scales and the scaled left
// operand A' = diag(2^-rexp) A diag(phi) in 16-bit form in one pass, then C = A' B^T with 16-bit
// operands and FP32 accumulation and output in one GEMM launch (tile chosen by gemm_big).
static hipError_t launch_gemm(const CircleState &C, const float *A, int lda, const double *phi,
                              const unsigned short *Bh, const unsigned short *Bl, int ldb, float *Cm,
                              int ldc, int Mp, int Np, int Kp, const int32_t *s_in, int32_t *s_out,
                              hipStream_t s)
{
    if (C.mode == 1)
        hipLaunchKernelGGL(scale_rows16_kernel<1>, dim3(Mp), dim3(256), 0, s, A, lda, Kp, phi, s_in, s_out, C.Ah, C.Al);
    else if (C.mode == 2)
        hipLaunchKernelGGL(scale_rows16_kernel<2>, dim3(Mp), dim3(256), 0, s, A, lda, Kp, phi, s_in, s_out, C.Ah, C.Al);
    else
        hipLaunchKernelGGL(scale_rows16_kernel<0>, dim3(Mp), dim3(256), 0, s, A, lda, Kp, phi, s_in, s_out, C.Ah, C.Al);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned short *Ah = C.Ah, *Al = C.Al;
    if (gemm_big(Mp, Np, Kp)) {
        const int tm = Mp / kBigT, tn = Np / kBigT;
        const dim3 grid((unsigned)(tm * tn)), block(64 * kBigWaves);
        if (C.mode == 2)
            hipLaunchKernelGGL(gemm_big_split_kernel, grid, block, 0, s, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp, tm, tn);
        else if (C.mode == 1)
            hipLaunchKernelGGL(gemm_big_kernel<1>, grid, block, 0, s, Ah, lda, Bh, ldb, Cm, ldc, Kp, tm, tn);
        else
            hipLaunchKernelGGL(gemm_big_kernel<0>, grid, block, 0, s, Ah, lda, Bh, ldb, Cm, ldc, Kp, tm, tn);
        return hipGetLastError();
    }
    const dim3 grid(Np / kSmallT, Mp / kSmallT);
    const int tiles = (Np / kSmallT) * (Mp / kSmallT);
    const int ks = tiles >= kSplitK1Tiles ? 1 : (tiles >= kSplitK2Tiles ? 2 : 4);
    if (C.mode == 1)
        launch_gemm_small<1>(ks, grid, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp, s);
    else if (C.mode == 2)
        launch_gemm_small<2>(ks, grid, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp, s);
    else
        launch_gemm_small<0>(ks, grid, Ah, Al, lda, Bh, Bl, ldb, Cm, ldc, Kp, s);
    return hipGetLastError();
}

// One matrix product of the recursions: gamma (k from k-1) or beta (k from k+1).
static int circle_product(mot_plan_s *P, CircleState &C, int gamma, int k)
{
    const int l = gamma ? k - 1 : k + 1;
    hipStream_t st = P->stream;
    if (!C.nfft) {
        const float *A = (const float *)Ymat(C, gamma, l);
        float *Cm = (float *)Ymat(C, gamma, k);
        const unsigned short *Bh = gamma ? C.Kg_h[k] : C.Kb_h[k];
        const unsigned short *Bl = gamma ? C.Kg_l[k] : C.Kb_l[k];
        MOT_HIP(launch_gemm(C, A, C.ld[l], P->marg[l].phi, Bh, Bl, C.ld[l], Cm, C.ld[k], C.n1p, C.ld[k], C.ld[l],
                            Yscale(C, gamma, l), Yscale(C, gamma, k), st));
        return MOT_OK;
    }
    const double *A = (const double *)Ymat(C, gamma, l);
    hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)C.n1), dim3(256), 0, st, A, (int64_t)P->n[l],
                       (const double *)P->marg[l].phi, C.src, C.rowexp);
    MOT_HIP(hipGetLastError());
    return run_steps(gamma ? C.steps_g[k] : C.steps_b[k], st);
}

// Rows per chunk of a column sum: kColRows, halved down to kColRowsMin while the launch
// has fewer than 512 workgroups (small products are bound by the latency of the chunk's
// sequential loads, not by bandwidth).
static int colsum_rows(int64_t n1, int64_t nk)
{
    int rows = kColRows;
    while (rows > kColRowsMin && ((nk + 255) / 256) * ((n1 + rows - 1) / rows) < 512) rows /= 2;
    return rows;
}

static int colsum_phi(mot_plan_s *P, CircleState &C, int k, bool marg_only)
{
    hipStream_t st = P->stream;
    const int64_t n1 = C.n1, nk = P->n[k];
    const int rows = colsum_rows(n1, nk);
    const int chunks = (int)((n1 + rows - 1) / rows);
    const dim3 g((unsigned)((nk + 255) / 256), (unsigned)chunks);
    const void *Yb = C.Yb[k], *Yg = Ymat(C, 1, k);
    if (C.nfft)
        hipLaunchKernelGGL(colsum_kernel<double>, g, dim3(256), 0, st, (const double *)Yb, (const double *)Yg, C.ld[k],
                           n1, nk, (const double *)P->marg[0].phi, (const int32_t *)nullptr, (const int32_t *)nullptr,
                           rows, C.part);
    else
        hipLaunchKernelGGL(colsum_kernel<float>, g, dim3(256), 0, st, (const float *)Yb, (const float *)Yg, C.ld[k],
                           n1, nk, (const double *)P->marg[0].phi, (const int32_t *)Yscale(C, 0, k),
                           (const int32_t *)Yscale(C, 1, k), rows, C.part);
    MOT_HIP(hipGetLastError());
    const unsigned blocks = (unsigned)((nk + 255) / 256);
    double *sout = marg_only ? C.m_part : C.s_part + 2 * C.s_slot[k];
    hipLaunchKernelGGL(circle_phi_kernel, dim3(blocks), dim3(256), 0, st, (const double *)C.part, chunks, nk,
                       (const double *)P->marg[k].mu, P->marg[k].phi, 0, sout, P->flag, P->marg[k].marg,
                       marg_only ? 1 : 0);
    return hipGetLastError() == hipSuccess ? MOT_OK : MOT_EDEVICE;
}

static int rowsum_den0(mot_plan_s *P, CircleState &C)
{
    hipStream_t st = P->stream;
    if (C.nfft)
        hipLaunchKernelGGL(rowsum_k_kernel<double>, dim3((unsigned)C.n1), dim3(256), 0, st, (const double *)C.Yg1,
                           (const double *)C.Yb[1], C.ld[1], (int64_t)P->n[1], (const double *)P->marg[1].phi,
                           (const int32_t *)nullptr, C.den0);
    else
        hipLaunchKernelGGL(rowsum_k_kernel<float>, dim3((unsigned)C.n1), dim3(256), 0, st, (const float *)C.Yg1,
                           (const float *)C.Yb[1], C.ld[1], (int64_t)P->n[1], (const double *)P->marg[1].phi,
                           (const int32_t *)Yscale(C, 0, 1), C.den0);
    return hipGetLastError() == hipSuccess ? MOT_OK : MOT_EDEVICE;
}

// Upward recursion Yb_{K-2} .. Yb_1 at the current phi, then den0 (Algorithm 3 step 4).
static int circle_up(mot_plan_s *P, CircleState &C)
{
    for (int k = P->K - 2; k >= 1; --k) MOT_TRY(circle_product(P, C, 0, k));
    return rowsum_den0(P, C);
}

template <class T>
static int kmat(mot_plan_s *P, int a, int b, int ld, int rows_pad, T *out, const double *xa = nullptr)
{
    dim3 g((unsigned)((ld + 255) / 256), (unsigned)rows_pad);
    hipLaunchKernelGGL(kernel_matrix_kernel<T>, g, dim3(256), 0, P->stream,
                       xa ? xa : (const double *)P->marg[a].pts, (int64_t)P->n[a], (const double *)P->marg[b].pts,
                       (int64_t)P->n[b], P->d, P->eta, ld, (int64_t)rows_pad, out);
    return hipGetLastError() == hipSuccess ? MOT_OK : MOT_EDEVICE;
}

static int kmat16(mot_plan_s *P, CircleState &C, int a, int b, unsigned short **h, unsigned short **l)
{
    const int ld = C.ld[b], rows = C.ld[a];
    MOT_TRY(P->arena.get_n((size_t)rows * ld, h));
    *l = nullptr;
    if (C.mode == 2) MOT_TRY(P->arena.get_n((size_t)rows * ld, l));
    dim3 g((unsigned)((ld + 255) / 256), (unsigned)rows);
    hipLaunchKernelGGL(kernel_matrix16_kernel, g, dim3(256), 0, P->stream, (const double *)P->marg[a].pts,
                       (int64_t)P->n[a], (const double *)P->marg[b].pts, (int64_t)P->n[b], P->d, P->eta, ld,
                       (int64_t)rows, C.mode == 1 ? 1 : 0, *h, *l);
    return hipGetLastError() == hipSuccess ? MOT_OK : MOT_EDEVICE;
}

// NFFT path: n1 product jobs (one per matrix row) for out = K^{(t,s)} rows.
static int nfft_position(mot_plan_s *P, CircleState &C, int t, int s, double *out, std::vector<ProdJob> &tmpl,
                         std::vector<Step> &steps)
{
    const int64_t n1 = C.n1;
    std::vector<ProdJob> jobs(n1);
    for (int64_t i = 0; i < n1; ++i) {
        ProdJob &J = jobs[i];
        MOT_TRY(make_prod_job(P, t, s, C.src + i * P->n[s], C.rowexp + i, out + i * P->n[t], &J, nullptr, false));
        J.patches = tmpl[i].patches;
        J.grid = tmpl[i].grid;
        J.spec0 = tmpl[i].spec0;
        J.spec1 = tmpl[i].spec1;
    }
    ProdJob *dev = nullptr;
    MOT_TRY(P->arena.get_n(jobs.size(), &dev));
    MOT_HIP(hipMemcpy(dev, jobs.data(), jobs.size() * sizeof(ProdJob), hipMemcpyHostToDevice));
    std::vector<int> ids(n1);
    for (int64_t i = 0; i < n1; ++i) ids[i] = (int)i;
    return product_steps(P->arena, dev, jobs, ids, steps);
}

int circle_create(mot_plan_s *P, const std::vector<double> &pts_h, const std::vector<double> &w_h,
                  const mot_fastsum_params *fs)
{
    const int K = P->K;
    CircleState *Cp = new CircleState();
    P->circle = Cp;
    CircleState &C = *Cp;
    C.nfft = P->path == MOT_NFFT;
    if (!C.nfft) {
        if (P->path != MOT_DENSE) return MOT_EUNSUPPORTED;
        if (P->precision == MOT_PREC_BF16) C.mode = 0;
        else if (P->precision == MOT_PREC_FP16) C.mode = 1;
        else if (P->precision == MOT_PREC_BF16X3) C.mode = 2;
        else return MOT_EUNSUPPORTED;
    }
    MOT_TRY(setup_marginals(P, pts_h, w_h, fs, C.nfft ? 0 : 256));
    hipStream_t st = P->stream;
    C.n1 = P->n[0];
    C.n1p = C.nfft ? (int)C.n1 : dense_pad(C.n1);
    C.ld.resize(K);
    for (int k = 0; k < K; ++k) C.ld[k] = C.nfft ? (int)P->n[k] : dense_pad(P->n[k]);
    const size_t esz = C.nfft ? 8 : 4;
    int ldmax = 0;
    int64_t nmax = 0;
    for (int k = 0; k < K; ++k) {
        ldmax = std::max(ldmax, C.ld[k]);
        nmax = std::max(nmax, P->n[k]);
    }
    C.Yb.assign(K, nullptr);
    for (int k = 1; k < K; ++k) MOT_TRY(P->arena.get((size_t)C.n1p * C.ld[k] * esz, &C.Yb[k]));
    MOT_TRY(P->arena.get((size_t)C.n1p * ldmax * esz, &C.Yg[0]));
    MOT_TRY(P->arena.get((size_t)C.n1p * ldmax * esz, &C.Yg[1]));
    MOT_TRY(P->arena.get((size_t)C.n1p * C.ld[1] * esz, &C.Yg1));
    // the closing edge {K, 1}: x^1 or, for a generalised Euler flow, sigma(x^1) in
    // marginal 0's binned order
    const double *xclose = nullptr;
    if (!P->closing.empty()) {
        double *orig = nullptr, *sorted = nullptr;
        MOT_TRY(P->arena.get_n(P->closing.size(), &orig));
        MOT_TRY(P->arena.get_n(P->closing.size(), &sorted));
        MOT_HIP(hipMemcpy(orig, P->closing.data(), P->closing.size() * sizeof(double), hipMemcpyHostToDevice));
        MOT_HIP(launch_gather_rows(orig, P->marg[0].perm, P->n[0], P->d, sorted, st));
        xclose = sorted;
    }
    if (C.nfft) {
        MOT_TRY(kmat<double>(P, 0, 1, C.ld[1], C.n1p, (double *)C.Yg1));
        MOT_TRY(kmat<double>(P, 0, K - 1, C.ld[K - 1], C.n1p, (double *)C.Yb[K - 1], xclose));
    } else {
        MOT_TRY(kmat<float>(P, 0, 1, C.ld[1], C.n1p, (float *)C.Yg1));
        MOT_TRY(kmat<float>(P, 0, K - 1, C.ld[K - 1], C.n1p, (float *)C.Yb[K - 1], xclose));
        // padding of the ping-pong buffers must be zero (they become GEMM operands)
        MOT_HIP(launch_fill_int((int32_t *)C.Yg[0], 0, (int64_t)C.n1p * ldmax, st));
        MOT_HIP(launch_fill_int((int32_t *)C.Yg[1], 0, (int64_t)C.n1p * ldmax, st));
        for (int k = 1; k < K - 1; ++k) MOT_HIP(launch_fill_int((int32_t *)C.Yb[k], 0, (int64_t)C.n1p * C.ld[k], st));
        C.Kb_h.assign(K, nullptr);
        C.Kb_l.assign(K, nullptr);
        C.Kg_h.assign(K, nullptr);
        C.Kg_l.assign(K, nullptr);
        for (int k = 1; k <= K - 2; ++k) MOT_TRY(kmat16(P, C, k, k + 1, &C.Kb_h[k], &C.Kb_l[k]));
        for (int k = 2; k <= K - 1; ++k) MOT_TRY(kmat16(P, C, k, k - 1, &C.Kg_h[k], &C.Kg_l[k]));
        MOT_TRY(P->arena.get_n((size_t)C.n1p, &C.rexp));
        MOT_TRY(P->arena.get_n((size_t)C.n1p * ldmax, &C.Ah));
        if (C.mode == 2) MOT_TRY(P->arena.get_n((size_t)C.n1p * ldmax, &C.Al));
        C.K = K;
        C.sb.assign(K, nullptr);
        for (int k = 1; k < K - 1; ++k) MOT_TRY(P->arena.get_n((size_t)C.n1p, &C.sb[k]));
        MOT_TRY(P->arena.get_n((size_t)C.n1p, &C.sg[0]));
        MOT_TRY(P->arena.get_n((size_t)C.n1p, &C.sg[1]));
        MOT_TRY(P->arena.get_n((size_t)C.n1p, &C.szero));
        MOT_HIP(launch_fill_int(C.szero, 0, C.n1p, st));
    }
    const int chunks = (int)((C.n1 + kColRowsMin - 1) / kColRowsMin);  // at most, for any rows per chunk
    MOT_TRY(P->arena.get_n((size_t)chunks * nmax, &C.part));
    MOT_TRY(P->arena.get_n((size_t)C.n1, &C.den0));
    C.s_slot.assign(K, 0);
    int slot = 0;
    for (int k = 0; k < K; ++k) {
        C.s_slot[k] = slot;
        slot += (int)((P->n[k] + 255) / 256);
    }
    C.ns = slot;
    MOT_TRY(P->arena.get_n(2 * (size_t)slot, &C.s_part));
    MOT_TRY(P->arena.get_n(2 * (size_t)((C.n1 + 255) / 256), &C.e_part));
    MOT_TRY(P->arena.get_n(2 * (size_t)((nmax + 255) / 256), &C.m_part));
    if (C.nfft) {
        MOT_TRY(P->arena.get_n((size_t)C.n1 * nmax, &C.src));
        MOT_TRY(P->arena.get_n((size_t)C.n1, &C.rowexp));
        // work buffers per row, shared by all product positions
        std::vector<ProdJob> tmpl(C.n1);
        int maxc = 0;
        for (auto &g : P->marg) maxc = std::max(maxc, g.nchunks);
        int64_t pe = 1;
        for (int c = 0; c < P->d; ++c) pe *= P->P.W;
        float *patches = nullptr;
        MOT_TRY(P->arena.get_n((size_t)C.n1 * maxc * pe, &patches));
        for (int64_t i = 0; i < C.n1; ++i)
            MOT_TRY(make_prod_job(P, 1, 0, nullptr, nullptr, nullptr, &tmpl[i], patches + (size_t)i * maxc * pe, true));
        C.steps_g.assign(K, {});
        C.steps_b.assign(K, {});
        for (int k = 2; k <= K - 1; ++k)
            MOT_TRY(nfft_position(P, C, k, k - 1, (double *)Ymat(C, 1, k), tmpl, C.steps_g[k]));
        for (int k = 1; k <= K - 2; ++k) MOT_TRY(nfft_position(P, C, k, k + 1, (double *)C.Yb[k], tmpl, C.steps_b[k]));
    }
    MOT_TRY(circle_up(P, C));
    MOT_HIP(hipStreamSynchronize(st));
    return MOT_OK;
}

int circle_run_sweeps(mot_plan_s *P, int sweeps)
{
    CircleState &C = *(CircleState *)P->circle;
    hipStream_t st = P->stream;
    const int K = P->K;
    if (sweeps == 0) {  // re-initialise after new scaling vectors
        MOT_TRY(circle_up(P, C));
        MOT_HIP(hipStreamSynchronize(st));
        return MOT_OK;
    }
    for (int r = 0; r < sweeps; ++r) {
        // phi^1 <- mu^1 / <K^{(1,2)}, (phi^2 (.) beta_2)^T>  (Algorithm 3, first update)
        hipLaunchKernelGGL(circle_phi_kernel, dim3((unsigned)((C.n1 + 255) / 256)), dim3(256), 0, st,
                           (const double *)C.den0, 0, C.n1, (const double *)P->marg[0].mu, P->marg[0].phi, 1,
                           C.s_part + 2 * C.s_slot[0], P->flag, P->marg[0].marg, 0);
        MOT_HIP(hipGetLastError());
        for (int k = 1; k < K; ++k) {
            if (k >= 2) MOT_TRY(circle_product(P, C, 1, k));
            MOT_TRY(colsum_phi(P, C, k, false));
        }
        MOT_TRY(circle_up(P, C));
        // first marginal after the sweep, P_0 = phi^0 den0, and S^(r)
        hipLaunchKernelGGL(circle_phi_kernel, dim3((unsigned)((C.n1 + 255) / 256)), dim3(256), 0, st,
                           (const double *)C.den0, 0, C.n1, (const double *)P->marg[0].mu, P->marg[0].phi, 1,
                           C.e_part, P->flag, P->marg[0].marg, 1);
        hipLaunchKernelGGL(circle_final_kernel, dim3(1), dim3(256), 0, st, (const double *)C.s_part, C.ns,
                           (const double *)C.e_part, (int)((C.n1 + 255) / 256), P->eta, P->sweep_ctr, P->hist_cap,
                           P->S_hist, P->err_hist, P->flag, P->flag_hist);
        MOT_HIP(hipGetLastError());
    }
    P->host_sweeps += sweeps;
    return MOT_OK;
}

// Marginals at the current phi (Theorem 4.3): P_0 = phi^0 den0 and, through the gamma
// recursion, P_k = phi^k <beta_k, (phi^1 (.) gamma_k)^T>.
int circle_marginals(mot_plan_s *P, double *)
{
    CircleState &C = *(CircleState *)P->circle;
    hipStream_t st = P->stream;
    hipLaunchKernelGGL(circle_phi_kernel, dim3((unsigned)((C.n1 + 255) / 256)), dim3(256), 0, st,
                       (const double *)C.den0, 0, C.n1, (const double *)P->marg[0].mu, P->marg[0].phi, 1, C.m_part,
                       P->flag, P->marg[0].marg, 1);
    MOT_HIP(hipGetLastError());
    for (int k = 1; k < P->K; ++k) {
        if (k >= 2) MOT_TRY(circle_product(P, C, 1, k));
        MOT_TRY(colsum_phi(P, C, k, true));
    }
    return MOT_OK;
}

// Pi_{1,k} at the current phi: the gamma recursion up to k (beta is current after every
// sweep and after new scaling vectors), then the elementwise product of Theorem 4.3's
// factors.
int circle_pair_marginal(mot_plan_s *P, int k, double *out)
{
    CircleState &C = *(CircleState *)P->circle;
    hipStream_t st = P->stream;
    for (int q = 2; q <= k; ++q) MOT_TRY(circle_product(P, C, 1, q));
    const int64_t n1 = C.n1, nk = P->n[k];
    const dim3 g((unsigned)((nk + 255) / 256), (unsigned)(n1 < 32768 ? n1 : 32768));
    if (C.nfft)
        hipLaunchKernelGGL(circle_pair_kernel<double>, g, dim3(256), 0, st, (const double *)Ymat(C, 1, k),
                           (const double *)C.Yb[k], C.ld[k], n1, nk, (const double *)P->marg[0].phi,
                           (const double *)P->marg[k].phi, (const int32_t *)nullptr, (const int32_t *)nullptr,
                           (const int32_t *)P->marg[0].perm, (const int32_t *)P->marg[k].perm, out);
    else
        hipLaunchKernelGGL(circle_pair_kernel<float>, g, dim3(256), 0, st, (const float *)Ymat(C, 1, k),
                           (const float *)C.Yb[k], C.ld[k], n1, nk, (const double *)P->marg[0].phi,
                           (const double *)P->marg[k].phi, (const int32_t *)Yscale(C, 1, k),
                           (const int32_t *)Yscale(C, 0, k), (const int32_t *)P->marg[0].perm,
                           (const int32_t *)P->marg[k].perm, out);
    return hipGetLastError() == hipSuccess ? MOT_OK : MOT_EDEVICE;
}

void circle_destroy(mot_plan_s *P)
{
    delete (CircleState *)P->circle;
    P->circle = nullptr;
}

size_t circle_footprint(int K, const int64_t *n, int path, int precision)
{
    size_t b = 0;
    const bool nfft = path == MOT_NFFT;
    const int64_t n1 = nfft ? n[0] : dense_pad(n[0]);
    int64_t ldmax = 0;
    for (int k = 0; k < K; ++k) ldmax = std::max<int64_t>(ldmax, nfft ? n[k] : dense_pad(n[k]));
    const size_t esz = nfft ? 8 : 4;
    b += (size_t)n1 * ldmax * esz * (K + 2);
    if (!nfft) {
        const size_t parts = precision == MOT_PREC_BF16X3 ? 2 : 1;
        b += (size_t)ldmax * ldmax * 2 * (2 * (K - 2)) * parts;  // kernel matrices
        b += (size_t)n1 * ldmax * 2 * parts;                       // scaled left operand
    }
    else b += (size_t)n1 * ldmax * 8 + (size_t)n1 * 8;  // product sources, row exponents
    b += (size_t)((n[0] + kColRowsMin - 1) / kColRowsMin) * ldmax * 8;  // column-sum partials
    return b;
}

}  // namespace mot
