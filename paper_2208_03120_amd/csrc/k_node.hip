// FP64 node updates of the tree sweep (a8, a10) and small utility kernels.
//
// Algorithm 2 in terms of per-node elementwise work (cp = prod_{t in C_k} beta_t, the
// children's messages multiplied in ascending child order starting from 1):
//   update:    phi^k <- mu^k / (gamma_k * cp)            (gamma_root = 1)
//              S terms: sum mu^k log phi^k_old, and for the root
//              sum (mu / phi_new) phi_old (the last term of S^(r))
//   down src:  u_c = (phi^k * gamma_k) * prod_{t in C_k, t != c} beta_t   for every child c
//              (the vector whose transposed kernel product gives gamma_c, eq. gamma_tree)
//   up src:    v_k = phi^k * cp                             (beta_k = K^{(p,k)} v_k)
//   marginal:  P_k = (phi^k * gamma_k) * cp               (Theorem 4.1), and |P_k - mu^k|
//   free node (generalised barycenter, Sec. 6.2): phi^k = 1 instead of the update, no S
//              term and no marginal error (mu^k is not given)
// Every product vector also records max_i exponent(value) in the job's slot so the
// product kernels can scale it into FP32 range without loss.
// Per-item partial sums go to distinct slots (no floating-point atomics): reductions
// are deterministic.
#include "mot_internal.h"

namespace mot {

constexpr int kNodeElems = kNodeItemElems;   // elements per node item
constexpr int kNodeEPT = kNodeElems / 256;     // elements per thread (256 threads)
constexpr int kRegChildren = 16;  // children held in registers (more: read from memory)
constexpr int kFewChildren = 4;   // the same, for launches of nodes with at most 4 children

__device__ __forceinline__ int exp_of(double v)
{
    return (v > 0.0 && v < INFINITY) ? ilogb(v) : INT32_MIN;
}

__device__ __forceinline__ int wave_max_int(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// One node item: up to kNodeItemElems elements of one node.  The messages of up to RC
// children are held in registers (loaded before any output is written); a node with more
// children reads them from memory for every product and records the exponent maxima of its
// down sources with one atomic per element.
template <int RC>
__global__ __launch_bounds__(256) void node_kernel(const NodeJob *__restrict__ jobs,
                                                   const int2 *__restrict__ items, int n_items)
{
    __shared__ double red[4];
    __shared__ int emx[4][RC + 1];
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const NodeJob &J = jobs[itm.x];
        const int op = J.op;
        const bool upd = op & 1, dsrc = op & 2, usrc = op & 4, root = op & 8, marg = op & 16;
        const bool freen = op & 32;
        const int nch = J.nchild;
        const bool regs = nch <= RC;
        double s1 = 0.0, s2 = 0.0;
        int em_up = INT32_MIN;
        int em[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) em[c] = INT32_MIN;
        bool bad = false;
        // the inputs of all of this thread's elements (children's messages too, when they
        // fit in registers) are loaded before any output is written, so that the loads
        // are in flight together
        double mu_k[kNodeEPT], ph_k[kNodeEPT], g_k[kNodeEPT];
        double b[RC][kNodeEPT];
#pragma unroll
        for (int k = 0; k < kNodeEPT; ++k) {
            const int64_t i = (int64_t)itm.y + tid + 256 * k;
            mu_k[k] = ph_k[k] = g_k[k] = 1.0;
#pragma unroll
            for (int t = 0; t < RC; ++t) b[t][k] = 1.0;
            if (i < J.n) {
                mu_k[k] = gp(J.mu)[i];
                ph_k[k] = gp(J.phi)[i];
                if (!root) g_k[k] = gp(J.gamma)[i];
                if (regs)
#pragma unroll
                    for (int t = 0; t < RC; ++t)
                        if (t < nch) b[t][k] = gp(gp(J.beta)[t])[i];
            }
        }
#pragma unroll
        for (int k = 0; k < kNodeEPT; ++k) {
            const int64_t i = (int64_t)itm.y + tid + 256 * k;
            if (i >= J.n) break;
            double cp = 1.0;
            if (regs) {
#pragma unroll
                for (int t = 0; t < RC; ++t)
                    if (t < nch) cp *= b[t][k];
            } else {
                for (int t = 0; t < nch; ++t) cp *= gp(gp(J.beta)[t])[i];
            }
            const double g = g_k[k];
            const double mu = mu_k[k];
            double ph = ph_k[k];
            if (upd && freen) {
                gp(J.phi)[i] = 1.0;  // no marginal constraint: phi^k = 1 in every sweep
                ph = 1.0;
            } else if (upd) {
                const double nv = mu / (g * cp);
                if (mu > 0.0) {
                    s1 += mu * log(ph);
                    if (root) s2 += (mu / nv) * ph;
                }
                if (!isfinite(nv)) bad = true;
                gp(J.phi)[i] = nv;
                ph = nv;
            }
            if (marg) {
                const double P = (ph * g) * cp;
                gp(J.marg_out)[i] = P;
                if (!freen) s1 += fabs(P - mu);
            }
            if (usrc) {
                const double v = ph * cp;
                gp(J.up_src)[i] = v;
                em_up = max(em_up, exp_of(v));
            }
            if (dsrc) {
                const double pg = ph * g;
                if (regs) {
#pragma unroll
                    for (int c = 0; c < RC; ++c) {
                        if (c >= nch) break;
                        double w = 1.0;
#pragma unroll
                        for (int t = 0; t < RC; ++t)
                            if (t < nch && t != c) w *= b[t][k];
                        const double u = pg * w;
                        gp(gp(J.down_src)[c])[i] = u;
                        em[c] = max(em[c], exp_of(u));
                    }
                } else {
                    for (int c = 0; c < nch; ++c) {
                        double w = 1.0;
                        for (int t = 0; t < nch; ++t)
                            if (t != c) w *= gp(gp(J.beta)[t])[i];
                        const double u = pg * w;
                        gp(gp(J.down_src)[c])[i] = u;
                        atomicMax(J.down_exp[c], exp_of(u));
                    }
                }
            }
        }
        if (bad) atomicOr(J.flag, 1);
        // exponent maxima: wave max, then block max, then one atomic per block and vector
        if (usrc || dsrc) {
            const int wave = tid >> 6, lane = tid & 63;
            __syncthreads();
            if (usrc) {
                const int m = wave_max_int(em_up);
                if (lane == 0) emx[wave][RC] = m;
            }
            if (dsrc && regs) {
#pragma unroll
                for (int c = 0; c < RC; ++c) {
                    if (c < nch) {  // nch is uniform over the block
                        const int m = wave_max_int(em[c]);
                        if (lane == 0) emx[wave][c] = m;
                    }
                }
            }
            __syncthreads();
            if (tid <= RC) {
                const bool is_up = tid == RC;
                if ((is_up && usrc) || (!is_up && dsrc && regs && tid < nch)) {
                    int m = emx[0][tid];
                    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, emx[w][tid]);
                    if (m != INT32_MIN) atomicMax(is_up ? J.up_exp : J.down_exp[tid], m);
                }
            }
        }
        if (upd || marg) {
            const double t1 = block_sum(s1, red);
            const double t2 = block_sum(s2, red);
            if (tid == 0) {
                const int slot = J.block0 + (int)(itm.y / kNodeElems);
                gp(J.partial)[2 * slot] = t1;
                gp(J.partial)[2 * slot + 1] = t2;
            }
        }
    }
}

hipError_t launch_node(const NodeJob *jobs_dev, const int2 *items, int n_items, int max_children, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const int grid = n_items < 8192 ? n_items : 8192;
    // the register copies of the children's messages set the kernel's register count, and
    // with it how many blocks run at once: launches whose nodes have at most one or at most
    // kFewChildren children take the smaller forms
    if (max_children <= 1)  // leaves and the nodes of a path
        hipLaunchKernelGGL(node_kernel<1>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
    else if (max_children <= kFewChildren)
        hipLaunchKernelGGL(node_kernel<kFewChildren>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
    else
        hipLaunchKernelGGL(node_kernel<kRegChildren>, dim3(grid), dim3(256), 0, s, jobs_dev, items, n_items);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Sweep finalisation, two launches.
//   finalize_l1_kernel, item = (job, first root element): the root marginal
//     P_0 = phi^0 * prod_{t in C_0} beta_t after the upward pass and the L1 error of the
//     item's elements, one partial per item;
//   finalize_reduce_kernel, one block per job: the partial sums in a fixed order,
//     S^(r) = eta * (sum mu log phi_old - sum (mu / phi_new) phi_old)
//     and the error recorded at the plan's sweep counter, the exponent slots re-armed for
//     the next sweep.
// The kernel boundary orders the partials before their reduction, so no block waits on
// another and no device-scope fence is needed.
__global__ __launch_bounds__(256) void finalize_l1_kernel(const FinalJob *__restrict__ jobs,
                                                          const int2 *__restrict__ items, int n_items)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 itm = items[it];
        const FinalJob &J = jobs[itm.x];
        double l1 = 0.0;
        {
            // child products of all of this thread's elements, children in ascending order
            double cp[kNodeEPT];
            bool ok[kNodeEPT];
#pragma unroll
            for (int k = 0; k < kNodeEPT; ++k) {
                cp[k] = 1.0;
                ok[k] = (int64_t)itm.y + tid + 256 * k < J.n0;
            }
            if (J.nchild <= kRegChildren) {
                // all children's messages loaded before the products, so the loads are in
                // flight together; multiplied in ascending child order
                double b[kRegChildren][kNodeEPT];
#pragma unroll
                for (int t = 0; t < kRegChildren; ++t)
#pragma unroll
                    for (int k = 0; k < kNodeEPT; ++k)
                        b[t][k] = (t < J.nchild && ok[k]) ? gp(gp(J.root_beta)[t])[(int64_t)itm.y + tid + 256 * k]
                                                          : 1.0;
#pragma unroll
                for (int t = 0; t < kRegChildren; ++t)
#pragma unroll
                    for (int k = 0; k < kNodeEPT; ++k)
                        if (t < J.nchild) cp[k] *= b[t][k];
            } else {
                for (int t = 0; t < J.nchild; ++t) {
                    const MOT_GLOBAL double *bt = gp(gp(J.root_beta)[t]);
#pragma unroll
                    for (int k = 0; k < kNodeEPT; ++k)
                        if (ok[k]) cp[k] *= bt[(int64_t)itm.y + tid + 256 * k];
                }
            }
#pragma unroll
            for (int k = 0; k < kNodeEPT; ++k) {
                const int64_t i = (int64_t)itm.y + tid + 256 * k;
                if (ok[k]) l1 += fabs(gp(J.phi0)[i] * cp[k] - gp(J.mu0)[i]);
            }
        }
        const double tot = block_sum(l1, red);
        if (tid == 0) J.l1_partial[itm.y / kNodeElems] = tot;
    }
}

__global__ __launch_bounds__(256) void finalize_reduce_kernel(const FinalJob *__restrict__ jobs, int n_jobs)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    for (int j = blockIdx.x; j < n_jobs; j += gridDim.x) {
        const FinalJob &J = jobs[j];
        // every thread sums a fixed strided subset; block_sum combines them in a fixed
        // order.  Eight strided partials are loaded before they are added (in the same
        // order), so the loads of a thread are in flight together.
        constexpr int U = 8;
        double s1 = 0.0, s2 = 0.0, e1 = 0.0;
        for (int p0 = tid; p0 < J.n_partials; p0 += U * (int)blockDim.x) {
            double a[U], b[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int p = p0 + q * (int)blockDim.x;
                a[q] = p < J.n_partials ? J.s_partial[2 * p] : 0.0;
                b[q] = p < J.n_partials ? J.s_partial[2 * p + 1] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < U; ++q)
                if (p0 + q * (int)blockDim.x < J.n_partials) {
                    s1 += a[q];
                    s2 += b[q];
                }
        }
        for (int p = tid; p < J.n_items; p += blockDim.x) e1 += J.l1_partial[p];
        s1 = block_sum(s1, red);
        s2 = block_sum(s2, red);
        e1 = block_sum(e1, red);
        if (tid == 0) {
            const int r = *J.sweep_ctr;
            const int slot = r % J.hist_cap;
            J.S_hist[slot] = J.eta * (s1 - s2);
            J.err_hist[slot] = e1;
            J.flag_hist[slot] = *J.flag;
            *J.sweep_ctr = r + 1;
        }
        for (int s = tid; s < J.n_exp_slots; s += blockDim.x) J.exp_slots[s] = INT32_MIN;
        __syncthreads();  // red is reused by the next job
    }
}

hipError_t launch_finalize(const FinalJob *jobs, const int2 *items, int n_items, int n_jobs, hipStream_t s)
{
    if (n_items == 0 || n_jobs == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_l1_kernel, dim3(n_items < 8192 ? n_items : 8192), dim3(256), 0, s, jobs, items,
                       n_items);
    hipLaunchKernelGGL(finalize_reduce_kernel, dim3(n_jobs < 8192 ? n_jobs : 8192), dim3(256), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Utilities

__global__ void fill_int_kernel(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_double_kernel(double *p, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t launch_fill_int(int32_t *p, int32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                       value, count);
    return hipGetLastError();
}
hipError_t launch_fill_double(double *p, double value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_double_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       p, value, count);
    return hipGetLastError();
}

// dst[i] = src[perm[i]] for rows of d doubles (original -> binned order)
__global__ void gather_rows_kernel(const double *__restrict__ src, const int32_t *__restrict__ perm,
                                   int64_t n, int d, double *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    for (int c = 0; c < d; ++c) dst[i * d + c] = src[j * d + c];
}
// dst[perm[i]] = src[i] (binned -> original order)
__global__ void scatter_vec_kernel(const double *__restrict__ src, const int32_t *__restrict__ perm,
                                   int64_t n, double *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}
hipError_t launch_gather_rows(const double *src, const int32_t *perm, int64_t n, int d, double *dst,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       perm, n, d, dst);
    return hipGetLastError();
}
hipError_t launch_scatter_vec(const double *src, const int32_t *perm, int64_t n, double *dst,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_vec_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       perm, n, dst);
    return hipGetLastError();
}

// Pair marginal of a tree edge (Theorem 4.1 applied to two adjacent marginals): one
// row i of the parent per block, columns across the threads; written in original order.
__global__ void tree_pair_kernel(const double *__restrict__ u, const double *__restrict__ xa,
                                 const int32_t *__restrict__ perm_a, const double *__restrict__ w,
                                 const double *__restrict__ xb, const int32_t *__restrict__ perm_b,
                                 int64_t na, int64_t nb, int d, double inv_eta, double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    for (int64_t i = blockIdx.y; i < na; i += gridDim.y) {
        double d2 = 0.0;
        for (int c = 0; c < d; ++c) {
            const double df = xa[i * d + c] - xb[j * d + c];
            d2 += df * df;
        }
        out[(int64_t)perm_a[i] * nb + perm_b[j]] = (u[i] * exp(-d2 * inv_eta)) * w[j];
    }
}

hipError_t launch_tree_pair(const double *u, const double *xa, const int32_t *perm_a, int64_t na,
                            const double *w, const double *xb, const int32_t *perm_b, int64_t nb, int d,
                            double eta, double *out, hipStream_t s)
{
    if (na <= 0 || nb <= 0) return hipSuccess;
    const unsigned gy = (unsigned)(na < 32768 ? na : 32768);
    hipLaunchKernelGGL(tree_pair_kernel, dim3((unsigned)((nb + 255) / 256), gy), dim3(256), 0, s, u, xa, perm_a,
                       w, xb, perm_b, na, nb, d, 1.0 / eta, out);
    return hipGetLastError();
}

// max exponent of a vector into a slot (for products requested outside a sweep)
__global__ void vec_exp_kernel(const double *__restrict__ v, int64_t n, int32_t *slot)
{
    int m = INT32_MIN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, exp_of(v[i]));
    m = wave_max_int(m);
    if ((threadIdx.x & 63) == 0 && m != INT32_MIN) atomicMax(slot, m);
}
hipError_t launch_vec_exp(const double *v, int64_t n, int32_t *slot, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(vec_exp_kernel, dim3(blocks), dim3(256), 0, s, v, n, slot);
    return hipGetLastError();
}

}  // namespace mot
