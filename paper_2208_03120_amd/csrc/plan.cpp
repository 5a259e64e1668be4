// Plans, the tree sweep scheduler and the C ABI (tree topology; the circle driver lives
// in circle.hip, batching in batch.cpp, serving in server.cpp).
//
// Tree sweeps follow Algorithm 2 level by level.  Algorithm 2 computes gamma_k and
// phi^k for k = 1..K and then beta_k for k = K..2; gamma_k reads only its parent's new
// values and the previous sweep's beta, and beta_k reads only its children's new beta,
// so all nodes at one depth are independent and run in the same launches:
//   DOWN(0) PROD_DOWN(1) DOWN(1) ... DOWN(D) PROD_UP(D) UP(D-1) PROD_UP(D-1) ... UP(1)
//   PROD_UP(1) FINAL
// DOWN(l): phi update of the nodes at depth l and the product sources of their
// children (and the beta source of leaves); UP(l): beta sources of the inner nodes at
// depth l; PROD_*: the kernel products of the edges into depth l; FINAL: S^(r) and the
// first marginal's error.  The sequence is captured once as a HIP graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "host.h"

namespace mot {

static bool log_enabled()
{
    static int on = -1;
    if (on < 0) on = getenv("MOT_LOG") ? 1 : 0;
    return on == 1;
}

void log_msg(const char *fmt, ...)
{
    if (!log_enabled()) return;
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "[mot] ");
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what, const char *file, int line)
{
    fprintf(stderr, "[mot] HIP error %d (%s) at %s:%d: %s\n", (int)e, hipGetErrorString(e), file,
            line, what);
    return e == hipErrorOutOfMemory ? MOT_ENOMEM : MOT_EDEVICE;
}

int Arena::get(size_t nbytes, void **out)
{
    void *p = nullptr;
    if (nbytes == 0) nbytes = 256;
    if (custom) {
        p = alloc.alloc(nbytes, alloc.ctx);
        if (!p) return MOT_ENOMEM;
        if ((uintptr_t)p % 256 != 0) {  // kernels use 16-byte vector accesses
            alloc.free(p, alloc.ctx);
            return MOT_EINVAL;
        }
        blocks.push_back(p);
        bytes += nbytes;
        *out = p;
        return MOT_OK;
    }
    nbytes = (nbytes + 255) / 256 * 256;
    if (!slab || slab_size - slab_used < nbytes) {
        const size_t size = std::max(nbytes, std::max(kSlabMin, bytes / 4));
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, size);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return MOT_ENOMEM;
        }
        blocks.push_back(q);
        bytes += size;
        slab = (char *)q;
        slab_used = 0;
        slab_size = size;
    }
    *out = slab + slab_used;
    slab_used += nbytes;
    return MOT_OK;
}

void Arena::release()
{
    for (void *p : blocks) {
        if (custom)
            alloc.free(p, alloc.ctx);
        else
            (void)hipFree(p);
    }
    blocks.clear();
    bytes = 0;
    slab = nullptr;
    slab_used = slab_size = 0;
}

int Lanes::create(int lanes)
{
    if (n) return MOT_OK;
    n = std::max(1, std::min(lanes, kLanes));
    MOT_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (int i = 0; i + 1 < n; ++i) {
        // default priority (streams of different priorities are not used)
        MOT_HIP(hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking));
        MOT_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
    }
    return MOT_OK;
}

void Lanes::destroy()
{
    for (int i = 0; i + 1 < kLanes; ++i) {
        if (side[i]) (void)hipStreamSynchronize(side[i]);
        if (join[i]) (void)hipEventDestroy(join[i]);
        if (side[i]) (void)hipStreamDestroy(side[i]);
        side[i] = nullptr;
        join[i] = nullptr;
    }
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
    n = 0;
}

void Schedule::destroy()
{
    if (graph) (void)hipGraphExecDestroy(graph);
    if (graph_def) (void)hipGraphDestroy(graph_def);
    graph = nullptr;
    graph_def = nullptr;
    sweep.clear();
    init_up.clear();
    marg_pass.clear();
}

// Twiddle tables exp(-2 pi i k / n), one per (device, n), kept for the process lifetime.
const float2 *device_twiddle(int n)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, float2 *> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair(dev, n);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<float2> tw;
    build_twiddle(n, tw);
    float2 *d = nullptr;
    if (hipMalloc(&d, tw.size() * sizeof(float2)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    cache[key] = d;
    return d;
}

int run_steps(const std::vector<Step> &steps, hipStream_t s0, const Lanes *lanes)
{
    for (const Step &st : steps) {
        const hipStream_t s = lanes && st.lane ? lanes->side[st.lane - 1] : s0;
        switch (st.kind) {
        case ST_FORK:
            if (lanes) {
                MOT_HIP(hipEventRecord(lanes->fork, s0));
                for (int i = 0; i + 1 < lanes->n; ++i) MOT_HIP(hipStreamWaitEvent(lanes->side[i], lanes->fork, 0));
            }
            break;
        case ST_JOIN:
            if (lanes)
                for (int i = 0; i + 1 < lanes->n; ++i) {
                    MOT_HIP(hipEventRecord(lanes->join[i], lanes->side[i]));
                    MOT_HIP(hipStreamWaitEvent(s0, lanes->join[i], 0));
                }
            break;
        case ST_NODE:
            MOT_HIP(launch_node((const NodeJob *)st.jobs, (const int2 *)st.items, st.n_items, st.max_children, s));
            break;
        case ST_DIRECT:
            MOT_HIP(launch_direct(st.d, (const ProdJob *)st.jobs, (const int4 *)st.items, st.n_items,
                                  (const int2 *)st.items2, st.n_items2, st.precision, st.diff, s));
            break;
        case ST_SPREAD:
            if (st.group > 0)
                MOT_HIP(launch_spread3(st.group, (const ProdJob *)st.jobs, (const int4 *)st.items, st.n_items, s));
            else
                MOT_HIP(launch_spread(st.d, (const ProdJob *)st.jobs, (const int2 *)st.items, st.n_items,
                                      st.max_patch, s));
            break;
        case ST_FOLD:
            MOT_HIP(launch_fold(st.d, (const ProdJob *)st.jobs, (const int2 *)st.items, st.n_items, s));
            break;
        case ST_FFT:
            MOT_HIP(launch_fft_pass(st.fft_kind, st.n, (const ProdJob *)st.jobs, (const int4 *)st.items,
                                    st.n_items, st.twiddle, s));
            break;
        case ST_INTERP:
            MOT_HIP(launch_interp(st.d, (const ProdJob *)st.jobs, (const int2 *)st.items, st.n_items,
                                  st.max_patch, s));
            break;
        case ST_FINAL:
            MOT_HIP(launch_finalize((const FinalJob *)st.jobs, (const int2 *)st.items, st.n_items, st.n_jobs, s));
            break;
        case ST_FILL_INT:
            MOT_HIP(launch_fill_int(st.fill_ptr, st.fill_value, st.fill_count, s));
            break;
        case ST_TRUNC:
            MOT_HIP(launch_trunc(st.d, st.precision, st.trunc_r, st.diff, (const ProdJob *)st.jobs,
                                 (const int4 *)st.items, st.n_items, s));
            break;
        }
    }
    return MOT_OK;
}

// ---------------------------------------------------------------------------------------
// Step construction.

// Workgroups are dealt to the XCDs round-robin by block index (eight XCDs, each with its
// own L2), and a launch's block b takes item b first.  Items that read neighbouring data
// (consecutive line groups of an FFT pass, consecutive cells of a fold) are therefore
// placed `group` to an XCD: within every run of kXcds * group items, positions r, r + kXcds,
// ..., r + (group - 1) kXcds receive group consecutive items.  Results do not depend on the
// order of items.
constexpr int kXcds = 8;

template <class T>
static void xcd_group(std::vector<T> &v, int group)
{
    const size_t run = (size_t)kXcds * group;
    std::vector<T> out(v);
    for (size_t q = 0; q + run <= v.size(); q += run)
        for (int r = 0; r < kXcds; ++r)
            for (int j = 0; j < group; ++j) out[q + (size_t)j * kXcds + r] = v[q + (size_t)r * group + j];
    v.swap(out);
}

struct StepBuilder {
    Arena *arena;
    std::vector<Step> *out;
    int rc = MOT_OK;

    template <class T>
    const T *upload(const std::vector<T> &v)
    {
        if (rc < 0 || v.empty()) return nullptr;
        T *d = nullptr;
        rc = arena->get_n<T>(v.size(), &d);
        if (rc < 0) return nullptr;
        if (hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            rc = MOT_EDEVICE;
        return d;
    }

    void node(const NodeJob *jobs_dev, const std::vector<NodeJob> &host_jobs,
              const std::vector<int> &ids)
    {
        std::vector<int2> items;
        for (int j : ids)
            for (int64_t e = 0; e < host_jobs[j].n; e += kNodeItemElems) items.push_back(make_int2(j, (int)e));
        if (items.empty()) return;
        Step st{ST_NODE};
        for (int j : ids) st.max_children = std::max(st.max_children, host_jobs[j].nchild);
        st.jobs = jobs_dev;
        st.items = upload(items);
        st.n_items = (int)items.size();
        out->push_back(st);
    }

    void final_(const FinalJob *jobs_dev, const std::vector<FinalJob> &host_jobs)
    {
        std::vector<int2> items;
        for (size_t j = 0; j < host_jobs.size(); ++j)
            for (int64_t e = 0; e < host_jobs[j].n0; e += kNodeItemElems) items.push_back(make_int2((int)j, (int)e));
        Step st{ST_FINAL};
        st.jobs = jobs_dev;
        st.items = upload(items);
        st.n_items = (int)items.size();
        st.n_jobs = (int)host_jobs.size();
        out->push_back(st);
    }

    static void fft_dims(const ProdJob &J, int kind, int *A2, int *A1)
    {
        const int H = J.M + 1, B = 2 * J.M + 1;
        if (J.d == 3) {
            const int a2[5] = {J.L[0], H, H, J.L[0], J.L[0]};
            const int a1[5] = {J.L[1], J.L[0], B, H, J.L[1]};
            *A2 = a2[kind];
            *A1 = a1[kind];
        } else if (J.d == 2) {
            *A2 = 1;
            *A1 = kind == 2 ? H : J.L[0];
        } else {
            *A2 = 1;
            *A1 = 1;
        }
    }

    // Steps computing every product job in ids (indices into host_jobs / jobs_dev).
    void products(const ProdJob *jobs_dev, const std::vector<ProdJob> &host_jobs,
                  const std::vector<int> &ids)
    {
        std::map<std::tuple<int, int, int>, std::vector<int4>> direct;  // (d, precision, diff)
        std::map<std::tuple<int, int, int>, std::vector<int2>> direct_red;  // FP64 range sums
        std::map<std::tuple<int, int, int, int>, std::vector<std::pair<double, int4>>> trunc;  // (d, prec, R, wide)
        std::map<int, std::vector<int2>> spread, fold, interp;   // d
        // 3-D spreading: jobs by the points they spread from (a binned marginal's rows)
        std::map<const float *, std::vector<int>> spread3_src;
        std::map<int, std::vector<int32_t>> spread_pts, interp_pts;  // points of each item
        std::map<int, std::vector<int4>> fft[8];  // items per grid size n, per pass kind
        std::map<int, int> max_patch;
        for (int j : ids) {
            const ProdJob &J = host_jobs[j];
            if (J.path == MOT_DIRECT) {
                const int tpi = direct_targets_per_item(J.precision);
                const auto key = std::make_tuple(J.d, J.precision, J.diff);
                auto &v = direct[key];
                const int split = J.precision == MOT_PREC_FP64 ? std::max(1, J.dsplit) : 1;
                for (int64_t t = 0; t < J.nt; t += tpi)
                    for (int r = 0; r < split; ++r) v.push_back(make_int4(j, (int)t, r, 0));
                if (split > 1)
                    for (int64_t t = 0; t < J.nt; t += 256) direct_red[key].push_back(make_int2(j, (int)t));
                continue;
            }
            if (J.path == MOT_TRUNC) {
                // items of at most 64 R targets from a run of B consecutive cells of one
                // row (contiguous in the sorted order), costed by the sources they scan
                auto &v = trunc[std::make_tuple(J.d, J.precision, J.trunc_r, J.diff)];
                TruncParams TQ;
                TQ.nc = J.nc;
                TQ.w = J.tw;
                TQ.q2 = J.q2;
                int64_t nrow_cells = 1;
                for (int c = 0; c < J.d - 1; ++c) nrow_cells *= J.nc;
                const int cap = 64 * J.trunc_r;
                const int span = 2 * J.tw + 1;
                const int nrows = J.d == 1 ? 1 : (J.d == 2 ? span : span * span);
                for (int64_t row = 0; row < nrow_cells; ++row)
                    for (int x0 = 0; x0 < J.nc; x0 += J.trunc_b) {
                        const int B = std::min(J.trunc_b, J.nc - x0);
                        const int64_t cell = row * J.nc + x0;
                        const int a = J.h_tgt_cell_off[cell], b = J.h_tgt_cell_off[cell + B];
                        if (b <= a) continue;
                        int cc[3] = {0, 0, 0};
                        int64_t rem = cell;
                        for (int c = J.d - 1; c >= 0; --c) {
                            cc[c] = (int)(rem % J.nc);
                            rem /= J.nc;
                        }
                        double srcs = 0.0;
                        for (int ri = 0; ri < nrows; ++ri) {
                            int64_t base;
                            int xa, xb;
                            if (!trunc_row_range(J.d, TQ, cc, B, ri, &base, &xa, &xb)) continue;
                            srcs += J.h_src_cell_off[base + xb + 1] - J.h_src_cell_off[base + xa] + 64.0;
                        }
                        for (int s0 = a; s0 < b; s0 += cap)
                            v.push_back({srcs, make_int4(j, (int)cell, s0, std::min(cap, b - s0) | (B << 16))});
                    }
                continue;
            }
            if (J.d == 3) {
                spread3_src[J.src_win].push_back(j);
            } else {
                for (int c = 0; c < J.src_nchunks; ++c) spread[J.d].push_back(make_int2(j, c));
                for (int c = 0; c < J.src_nchunks; ++c)
                    spread_pts[J.d].push_back(J.h_src_chunk_start[c + 1] - J.h_src_chunk_start[c]);
            }
            const int lines = J.d == 3 ? J.L[0] * J.L[1] : (J.d == 2 ? J.L[0] : 1);
            const int cells = lines * J.L[J.d - 1];
            for (int f = 0; f < cells; f += kFoldCellsPerItem) fold[J.d].push_back(make_int2(j, f));
            for (int c = 0; c < J.tgt_nchunks; ++c) {
                interp[J.d].push_back(make_int2(j, c));
                interp_pts[J.d].push_back(J.h_tgt_chunk_start[c + 1] - J.h_tgt_chunk_start[c]);
            }
            int pe = 1;
            for (int c = 0; c < J.d; ++c) pe *= J.W;
            max_patch[J.d] = std::max(max_patch[J.d], pe);
            // 3-D boxes whose slab half spectrum fits in LDS take the three-pass chain
            const bool slab = J.d == 3 && (int64_t)J.L[1] * (J.M + 1) * 8 <= kSlabLds;
            const int kinds3[5] = {0, 1, 2, 3, 4}, kinds2[3] = {0, 2, 4}, kinds1[2] = {0, 4};
            const int *kinds = J.d == 3 ? kinds3 : (J.d == 2 ? kinds2 : kinds1);
            const int nk = J.d == 3 ? 5 : (J.d == 2 ? 3 : 2);
            if (slab) {
                for (int g0 = 0; g0 < J.L[0]; ++g0) {
                    fft[6][J.n].push_back(make_int4(j, g0, 0, 0));
                    fft[7][J.n].push_back(make_int4(j, g0, 0, 0));
                }
                int A2, A1;
                fft_dims(J, 2, &A2, &A1);
                auto &v = fft[5][J.n];
                const int per = fft_lines_per_item(5, J.n);
                for (int a2 = 0; a2 < A2; ++a2)
                    for (int a1 = 0; a1 < A1; a1 += per) v.push_back(make_int4(j, a2, a1, 0));
            } else {
                for (int q = 0; q < nk; ++q) {
                    int A2, A1;
                    fft_dims(J, kinds[q], &A2, &A1);
                    auto &v = fft[kinds[q]][J.n];
                    const int per = fft_lines_per_item(kinds[q], J.n);
                    for (int a2 = 0; a2 < A2; ++a2)
                        for (int a1 = 0; a1 < A1; a1 += per) v.push_back(make_int4(j, a2, a1, 0));
                }
            }
        }
        for (auto &kv : trunc) {
            // costliest items first, so the cheap boundary cells fill in at the end
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [](const std::pair<double, int4> &x, const std::pair<double, int4> &y) {
                                 return x.first > y.first;
                             });
            std::vector<int4> its(kv.second.size());
            for (size_t i = 0; i < its.size(); ++i) its[i] = kv.second[i].second;
            Step st{ST_TRUNC};
            st.d = std::get<0>(kv.first);
            st.precision = std::get<1>(kv.first);
            st.trunc_r = std::get<2>(kv.first);
            st.diff = std::get<3>(kv.first);
            st.jobs = jobs_dev;
            st.items = upload(its);
            st.n_items = (int)its.size();
            out->push_back(st);
        }
        for (auto &kv : direct) {
            Step st{ST_DIRECT};
            st.d = std::get<0>(kv.first);
            st.precision = std::get<1>(kv.first);
            st.diff = std::get<2>(kv.first);
            st.jobs = jobs_dev;
            st.items = upload(kv.second);
            st.n_items = (int)kv.second.size();
            auto red = direct_red.find(kv.first);
            if (red != direct_red.end()) {
                st.items2 = upload(red->second);
                st.n_items2 = (int)red->second.size();
            }
            out->push_back(st);
        }
        // largest chunks first: the blocks of a launch start roughly in item order, so the
        // short boundary chunks fill in at the end instead of forming a tail
        auto by_size = [](std::vector<int2> &v, const std::vector<int32_t> &npts) {
            std::vector<int> ord(v.size());
            for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return npts[a] > npts[b]; });
            std::vector<int2> out(v.size());
            for (size_t i = 0; i < ord.size(); ++i) out[i] = v[ord[i]];
            v.swap(out);
        };
        for (auto &kv : spread) by_size(kv.second, spread_pts[kv.first]);
        // 3-D: jobs spreading from the same points go three (or the remaining two) to an
        // item, which stages the chunk's rows once for all of them
        {
            std::vector<std::pair<int32_t, int4>> g3[4];
            for (auto &kv : spread3_src) {
                const std::vector<int> &js = kv.second;
                for (size_t a = 0; a < js.size();) {
                    const int G = (int)std::min<size_t>(3, js.size() - a);
                    const ProdJob &J = host_jobs[js[a]];
                    for (int c = 0; c < J.src_nchunks; ++c) {
                        const int4 it = make_int4(js[a], G > 1 ? js[a + 1] : -1, G > 2 ? js[a + 2] : -1, c);
                        g3[G].push_back({G * (J.h_src_chunk_start[c + 1] - J.h_src_chunk_start[c]), it});
                    }
                    a += G;
                }
            }
            for (int G = 3; G >= 1; --G) {
                if (g3[G].empty()) continue;
                std::stable_sort(g3[G].begin(), g3[G].end(),
                                 [](const std::pair<int32_t, int4> &x, const std::pair<int32_t, int4> &y) {
                                     return x.first > y.first;
                                 });
                std::vector<int4> its(g3[G].size());
                for (size_t i = 0; i < its.size(); ++i) its[i] = g3[G][i].second;
                Step st{ST_SPREAD};
                st.d = 3;
                st.group = G;
                st.max_patch = max_patch[3];
                st.jobs = jobs_dev;
                st.items = upload(its);
                st.n_items = (int)its.size();
                out->push_back(st);
            }
        }
        for (auto &kv : interp) by_size(kv.second, interp_pts[kv.first]);
        for (auto &kv : spread) {
            Step st{ST_SPREAD};
            st.d = kv.first;
            st.max_patch = max_patch[kv.first];
            st.jobs = jobs_dev;
            st.items = upload(kv.second);
            st.n_items = (int)kv.second.size();
            out->push_back(st);
        }
        // jobs of several dimensions fold in one launch (each item takes its job's d)
        if (fold.size() > 1) {
            std::vector<int2> all;
            for (auto &kv : fold) all.insert(all.end(), kv.second.begin(), kv.second.end());
            fold.clear();
            fold[0] = all;
        }
        for (auto &kv : fold) {
            xcd_group(kv.second, 4);
            Step st{ST_FOLD};
            st.d = kv.first;
            st.jobs = jobs_dev;
            st.items = upload(kv.second);
            st.n_items = (int)kv.second.size();
            out->push_back(st);
        }
        // per job the chain order holds: 0 < 1 < 2 < 3 < 4 and 6 < 5 < 7.  A pass kernel
        // serves every d; grids n <= 128 of several sizes share one launch (n = 0).
        for (int kind : {0, 6, 1, 2, 5, 3, 4, 7}) {
            std::vector<std::pair<int, std::vector<int4>>> launches;
            std::vector<int4> mixed;
            int small = 0;
            for (auto &kv : fft[kind]) small += kv.first <= 128;
            for (auto &kv : fft[kind]) {
                if (small > 1 && kv.first <= 128)
                    mixed.insert(mixed.end(), kv.second.begin(), kv.second.end());
                else
                    launches.push_back({kv.first, kv.second});
            }
            if (!mixed.empty()) launches.insert(launches.begin(), {0, mixed});
            for (auto &l : launches) {
                Step st{ST_FFT};
                st.d = kind >= 5 ? 3 : 0;
                st.n = l.first;
                st.fft_kind = kind;
                st.twiddle = device_twiddle(st.n == 0 ? 128 : st.n);
                if (!st.twiddle) rc = MOT_EDEVICE;
                st.jobs = jobs_dev;
                if (kind <= 5) xcd_group(l.second, 4);  // line passes: 4 neighbouring line groups
                st.items = upload(l.second);
                st.n_items = (int)l.second.size();
                out->push_back(st);
            }
        }
        for (auto &kv : interp) {
            Step st{ST_INTERP};
            st.d = kv.first;
            st.max_patch = max_patch[kv.first];
            st.jobs = jobs_dev;
            st.items = upload(kv.second);
            st.n_items = (int)kv.second.size();
            out->push_back(st);
        }
    }
};

int product_steps(Arena &arena, const ProdJob *jobs_dev, const std::vector<ProdJob> &jobs_host,
                  const std::vector<int> &ids, std::vector<Step> &out)
{
    StepBuilder B{&arena, &out};
    B.products(jobs_dev, jobs_host, ids);
    return B.rc;
}

// ---------------------------------------------------------------------------------------
// Tree plans

struct TreeNodeJobs {
    std::vector<NodeJob> down, up, init, marg;
};

}  // namespace mot

using namespace mot;

static std::map<const mot_plan_s *, TreeTables *> &tables_map()
{
    static std::map<const mot_plan_s *, TreeTables *> m;
    return m;
}
static std::mutex g_tables_mu;

TreeTables *mot::tables_of(const mot_plan_s *P)
{
    std::lock_guard<std::mutex> lk(g_tables_mu);
    auto it = tables_map().find(P);
    return it == tables_map().end() ? nullptr : it->second;
}

namespace mot {

// Build the per-plan node jobs, the finalize job and the three step sequences.
int tree_build_schedule(mot_plan_s *P)
{
    const int K = P->K;
    TreeTables *T = new TreeTables();
    {
        std::lock_guard<std::mutex> lk(g_tables_mu);
        tables_map()[P] = T;
    }
    T->njobs.resize(4 * K);
    int slot = 0;
    // device pointer arrays per node: child betas, child down sources, child exp slots
    for (int k = 0; k < K; ++k) {
        const auto &ch = P->children[k];
        std::vector<const double *> bptr;
        std::vector<double *> dptr;
        std::vector<int32_t *> eptr;
        for (int c : ch) {
            bptr.push_back(P->marg[c].beta);
            dptr.push_back(P->marg[c].down_src);
            eptr.push_back(P->exp_slots + (size_t)(2 * c) * kExpSlotStride);
        }
        const double **bdev = nullptr;
        double **ddev = nullptr;
        int32_t **edev = nullptr;
        if (!ch.empty()) {
            MOT_TRY(P->arena.get_n(ch.size(), &bdev));
            MOT_TRY(P->arena.get_n(ch.size(), &ddev));
            MOT_TRY(P->arena.get_n(ch.size(), &edev));
            MOT_HIP(hipMemcpy(bdev, bptr.data(), ch.size() * sizeof(void *), hipMemcpyHostToDevice));
            MOT_HIP(hipMemcpy(ddev, dptr.data(), ch.size() * sizeof(void *), hipMemcpyHostToDevice));
            MOT_HIP(hipMemcpy(edev, eptr.data(), ch.size() * sizeof(void *), hipMemcpyHostToDevice));
        }
        NodeJob base{};
        base.nchild = (int)ch.size();
        base.n = P->marg[k].n;
        base.mu = P->marg[k].mu;
        base.phi = P->marg[k].phi;
        base.gamma = k == 0 ? nullptr : P->marg[k].gamma;
        base.beta = bdev;
        base.down_src = ddev;
        base.down_exp = edev;
        base.up_src = P->marg[k].up_src;
        base.up_exp = P->exp_slots + (size_t)(2 * k + 1) * kExpSlotStride;
        base.marg_out = P->marg[k].marg;
        base.partial = P->s_partial;
        base.flag = P->flag;
        const int items = (int)((base.n + kNodeItemElems - 1) / kNodeItemElems);
        // DOWN: update (+ root) + down sources (+ up source for leaves)
        NodeJob dn = base;
        const int fr = (!P->free_node.empty() && P->free_node[k]) ? 32 : 0;
        dn.op = 1 | (ch.empty() ? 0 : 2) | ((ch.empty() && k > 0) ? 4 : 0) | (k == 0 ? 8 : 0) | fr;
        dn.block0 = slot;
        slot += items;
        T->njobs[k] = dn;
        // UP: beta source of inner non-root nodes
        NodeJob up = base;
        up.op = 4;
        T->njobs[K + k] = up;
        // INIT: beta source of every non-root node
        NodeJob in = base;
        in.op = 4;
        T->njobs[2 * K + k] = in;
        T->marg_block0.push_back(0);
    }
    T->n_down_partials = slot;
    for (int k = 0; k < K; ++k) {
        NodeJob mg = T->njobs[k];
        mg.op = 16 | (P->children[k].empty() ? 0 : 2) | (k == 0 ? 8 : 0) |
                ((!P->free_node.empty() && P->free_node[k]) ? 32 : 0);
        mg.block0 = slot;
        T->marg_block0[k] = slot;
        slot += (int)((mg.n + kNodeItemElems - 1) / kNodeItemElems);
        T->njobs[3 * K + k] = mg;
    }
    T->n_marg_partials = slot - T->n_down_partials;
    // finalize job
    {
        FinalJob F{};
        F.n0 = P->marg[0].n;
        F.mu0 = P->marg[0].mu;
        F.phi0 = P->marg[0].phi;
        F.root_beta = T->njobs[0].beta;
        F.nchild = T->njobs[0].nchild;
        F.n_items = (int)((F.n0 + kNodeItemElems - 1) / kNodeItemElems);
        F.s_partial = P->s_partial;
        F.n_partials = T->n_down_partials;
        F.hist_cap = P->hist_cap;
        F.l1_partial = P->l1_partial;
        F.sweep_ctr = P->sweep_ctr;
        F.flag = P->flag;
        F.flag_hist = P->flag_hist;
        F.S_hist = P->S_hist;
        F.err_hist = P->err_hist;
        F.exp_slots = P->exp_slots;
        F.n_exp_slots = (2 * K + 1) * kExpSlotStride;
        F.eta = P->eta;
        T->fjob.push_back(F);
    }
    MOT_TRY(P->arena.get_n(T->njobs.size(), &T->njobs_dev));
    MOT_HIP(hipMemcpy(T->njobs_dev, T->njobs.data(), T->njobs.size() * sizeof(NodeJob),
                      hipMemcpyHostToDevice));
    MOT_TRY(P->arena.get_n(1, &T->fjob_dev));
    MOT_HIP(hipMemcpy(T->fjob_dev, T->fjob.data(), sizeof(FinalJob), hipMemcpyHostToDevice));
    return MOT_OK;
}

// Steps of one sweep / the initial upward pass / the marginal pass for a set of tree
// plans whose node, product and final jobs are concatenated in the given device
// arrays (offsets per plan).
int tree_steps(const std::vector<TreeRef> &refs, const std::vector<ProdJob> &pj,
               const ProdJob *pj_dev, const std::vector<NodeJob> &nj, const NodeJob *nj_dev,
               const std::vector<FinalJob> &fj, const FinalJob *fj_dev, Arena &arena,
               std::vector<Step> &sweep, std::vector<Step> &init_up, std::vector<Step> &marg, int max_lanes,
               int *lanes_out)
{
    int maxD = 0;
    for (auto &r : refs) maxD = std::max(maxD, r.P->depth_max);
    // Lanes of a batched sweep: plans do not depend on each other, so kLanes lanes of them,
    // balanced by their points, run on their own streams between the fork and the
    // finalisation, and one lane's latency-bound passes overlap another's spreading and
    // interpolation.  (Splitting one plan's root subtrees the same way measured slower: the
    // lanes' launches hold a fraction of the jobs each.)  Plan r is in lane lane[r].
    const int nl = (int)std::min<size_t>(refs.size(), std::max(1, std::min(max_lanes, kLanes)));
    std::vector<int> lane(refs.size(), 0);
    {
        std::vector<double> load(nl, 0.0);
        for (size_t r = 0; r < refs.size(); ++r) {
            double pts = 0.0;
            for (int k = 0; k < refs[r].P->K; ++k) pts += (double)refs[r].P->marg[k].n;
            lane[r] = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[lane[r]] += pts;
        }
    }
    const bool two = nl >= 2;
    if (lanes_out) *lanes_out = nl;
    StepBuilder B{&arena, &sweep};
    // ln = -2: every lane
    auto nodes_at = [&](int level, int which, bool inner_only, bool nonroot, int ln = -2) {
        std::vector<int> ids;
        for (size_t ri = 0; ri < refs.size(); ++ri) {
            const TreeRef &r = refs[ri];
            const int K = r.P->K;
            for (int k = 0; k < K; ++k) {
                if (r.P->depth[k] != level) continue;
                if (inner_only && r.P->children[k].empty()) continue;
                if (nonroot && k == 0) continue;
                if (ln != -2 && lane[ri] != ln) continue;
                ids.push_back(r.nbase + which * K + k);
            }
        }
        return ids;
    };
    auto prods_at = [&](int level, int dir, int ln = -2) {  // dir 0: down job (gamma_k), 1: up (beta_k)
        std::vector<int> ids;
        for (size_t ri = 0; ri < refs.size(); ++ri) {
            const TreeRef &r = refs[ri];
            for (int k = 1; k < r.P->K; ++k)
                if (r.P->depth[k] == level && (ln == -2 || lane[ri] == ln)) ids.push_back(r.pbase + 2 * k + dir);
        }
        return ids;
    };
    // ---- sweep
    if (!two) {
        for (int l = 0; l <= maxD; ++l) {
            B.node(nj_dev, nj, nodes_at(l, 0, false, false));
            if (l < maxD) B.products(pj_dev, pj, prods_at(l + 1, 0));
        }
        for (int l = maxD; l >= 1; --l) {
            B.products(pj_dev, pj, prods_at(l, 1));
            if (l - 1 >= 1) B.node(nj_dev, nj, nodes_at(l - 1, 1, true, true));
        }
    } else {
        sweep.push_back(Step{ST_FORK});
        for (int ln = 0; ln < nl; ++ln) {
            const size_t first = sweep.size();
            for (int l = 0; l <= maxD; ++l) {
                B.node(nj_dev, nj, nodes_at(l, 0, false, false, ln));
                if (l < maxD) B.products(pj_dev, pj, prods_at(l + 1, 0, ln));
            }
            for (int l = maxD; l >= 1; --l) {
                B.products(pj_dev, pj, prods_at(l, 1, ln));
                if (l - 1 >= 1) B.node(nj_dev, nj, nodes_at(l - 1, 1, true, true, ln));
            }
            for (size_t i = first; i < sweep.size(); ++i) sweep[i].lane = ln;
        }
        sweep.push_back(Step{ST_JOIN});
    }
    B.final_(fj_dev, fj);
    if (B.rc < 0) return B.rc;
    // ---- initial upward pass (Algorithm 2, first loop)
    B.out = &init_up;
    for (int l = maxD; l >= 1; --l) {
        B.node(nj_dev, nj, nodes_at(l, 2, false, true));
        B.products(pj_dev, pj, prods_at(l, 1));
    }
    if (B.rc < 0) return B.rc;
    // ---- marginals: upward pass, then a downward pass that evaluates P_k
    B.out = &marg;
    for (int l = maxD; l >= 1; --l) {
        B.node(nj_dev, nj, nodes_at(l, 2, false, true));
        B.products(pj_dev, pj, prods_at(l, 1));
    }
    for (int l = 0; l <= maxD; ++l) {
        B.node(nj_dev, nj, nodes_at(l, 3, false, false));
        if (l < maxD) B.products(pj_dev, pj, prods_at(l + 1, 0));
    }
    return B.rc;
}

}  // namespace mot

// ---------------------------------------------------------------------------------------
// Plan creation helpers

static int copy_in(const double *src, size_t count, int ptr_kind, std::vector<double> &host)
{
    host.resize(count);
    if (count == 0) return MOT_OK;
    if (ptr_kind == MOT_DEVICE) {
        MOT_HIP(hipMemcpy(host.data(), src, count * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        memcpy(host.data(), src, count * sizeof(double));
    }
    return MOT_OK;
}

static int validate_common(int K, int d, const int64_t *n, double eta, const std::vector<double> &w,
                           const std::vector<double> &pts, int64_t total, const std::vector<int> &free_node)
{
    if (K < 2 || d < 1 || d > 3 || !(eta > 0.0) || !std::isfinite(eta)) return MOT_EINVAL;
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        if (n[k] < 1 || n[k] > (int64_t)1 << 30) return MOT_EINVAL;
        if (!free_node.empty() && free_node[k]) {  // weights of a free node are not read
            off += n[k];
            continue;
        }
        double s = 0.0;
        for (int64_t i = 0; i < n[k]; ++i) {
            const double v = w[off + i];
            if (!(v >= 0.0) || !std::isfinite(v)) return MOT_EINVAL;
            s += v;
        }
        if (std::fabs(s - 1.0) > 1e-9) return MOT_EINVAL;
        off += n[k];
    }
    for (int64_t i = 0; i < total * d; ++i)
        if (!std::isfinite(pts[i])) return MOT_EINVAL;
    return MOT_OK;
}

static Extent extent_of(int d, const std::vector<double> &pts, int64_t total)
{
    Extent E;
    for (int c = 0; c < d; ++c) {
        E.lo[c] = INFINITY;
        E.hi[c] = -INFINITY;
    }
    for (int64_t i = 0; i < total; ++i)
        for (int c = 0; c < d; ++c) {
            E.lo[c] = std::min(E.lo[c], pts[i * d + c]);
            E.hi[c] = std::max(E.hi[c], pts[i * d + c]);
        }
    double s2 = 0.0;
    for (int c = 0; c < d; ++c) {
        E.ctr[c] = 0.5 * (E.lo[c] + E.hi[c]);
        const double w = E.hi[c] - E.lo[c];
        s2 += w * w;
        E.width_max = std::max(E.width_max, w);
    }
    E.diag = std::sqrt(s2);
    return E;
}

// Bin one marginal's points (original order, device) and build its binned layout.  The
// temporaries (sort keys in scratch, cells, tile ids, box tile ranges) belong to the caller.
static int bin_marginal(mot_plan_s *P, int k, const double *pts_orig_dev, void *scratch,
                        size_t scratch_bytes, int32_t *cell_tmp, int32_t *tile_tmp,
                        int32_t *box_lo, int32_t *box_hi)
{
    MargDev &G = P->marg[k];
    const NfftParams &Q = P->P;
    const int d = P->d, n = Q.n, T = Q.T;
    const int tpd = (n + T - 1) / T;
    int64_t ntiles = 1;
    for (int c = 0; c < d; ++c) ntiles *= tpd;
    MOT_HIP(launch_bin_cells(d, G.n, pts_orig_dev, Q.s, Q.s, Q.s, Q.o[0], Q.o[1], Q.o[2], n, T,
                             cell_tmp, tile_tmp, P->stream));
    // In 3-D the points of a tile are ordered by their cell in dimension 1: the MFMA steps
    // of spreading and interpolation then mostly hold points with the same window support
    // in that dimension, and the steps outside it are skipped.
    const bool sub = d == 3 && T > 1 && ntiles < ((int64_t)1 << 28);
    MOT_HIP(stable_tile_sort(G.n, tile_tmp, ntiles, G.perm, nullptr, scratch, scratch_bytes,
                             P->stream, sub ? cell_tmp : nullptr, d, 1, T));
    MOT_HIP(launch_gather_rows(pts_orig_dev, G.perm, G.n, d, G.pts, P->stream));
    MOT_HIP(launch_window_rows(d, G.n, G.pts, Q.s, Q.o, T, Q.m, Q.kb_b, G.win, P->stream));
    // sorted ranges of the active box's tiles only (the box is a small part of the grid)
    int64_t nbox = 1;
    for (int c = 0; c < d; ++c) nbox *= Q.ntile[c];
    MOT_HIP(launch_box_tile_ranges(G.n, scratch, sub, d, tpd, Q.tmin, Q.ntile, box_lo, box_hi, P->stream));
    std::vector<int32_t> lo_h(nbox), hi_h(nbox);
    MOT_HIP(hipMemcpyAsync(lo_h.data(), box_lo, nbox * sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipMemcpyAsync(hi_h.data(), box_hi, nbox * sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    // Chunks over the box tiles in row-major order (coordinate 0 slowest).  Box tiles in
    // that order are a monotone subsequence of the global tile order the points are
    // sorted by, and every point lies in a box tile, so consecutive chunks are
    // consecutive ranges of the sorted points: chunk c = [starts[c], starts[c+1]).
    std::vector<int32_t> starts, tiles, tch2;
    tch2.push_back(0);
    int64_t covered = 0;
    for (int64_t bt = 0; bt < nbox; ++bt) {
        const int a = lo_h[bt], b = hi_h[bt];
        if (a != covered && b > a) return MOT_EDOMAIN;
        for (int s = a; s < b; s += Q.chunk) {
            starts.push_back(s);
            tiles.push_back((int32_t)bt);
        }
        covered += b - a;
        tch2.push_back((int32_t)starts.size());
    }
    if (covered != G.n) return MOT_EDOMAIN;  // a point outside the box tiles
    std::vector<int32_t> bounds = starts;
    bounds.push_back((int32_t)G.n);
    G.nchunks = (int)starts.size();
    G.h_chunk_tile = tiles;
    G.h_chunk_start = bounds;
    MOT_TRY(P->arena.get_n(bounds.size() + 2, &G.chunk_start));
    MOT_TRY(P->arena.get_n(tiles.size() + 1, &G.chunk_tile));
    MOT_TRY(P->arena.get_n(tch2.size() + 1, &G.tile_chunks));
    MOT_HIP(hipMemcpy(G.chunk_start, bounds.data(), bounds.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MOT_HIP(hipMemcpy(G.chunk_tile, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MOT_HIP(hipMemcpy(G.tile_chunks, tch2.data(), tch2.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return MOT_OK;
}

// eta of the kernel between marginals t and s: eta / w for a weighted tree edge
// (Sec. 6.2), eta otherwise.
static double pair_eta(const mot_plan_s *P, int t, int s)
{
    if (P->topology != MOT_TREE || P->edge_w.empty()) return P->eta;
    if (t > 0 && P->parent[t] == s) return P->eta / P->edge_w[t];
    if (s > 0 && P->parent[s] == t) return P->eta / P->edge_w[s];
    return P->eta;
}

// Fill the product job j: out(target t) = K^{(t,s)} v(source s).
int mot::make_prod_job(mot_plan_s *P, int t, int s, const double *v, int32_t *slot, double *out,
                       ProdJob *J, float *patches, bool alloc_buffers)
{
    ProdJob &Q = *J;
    Q = ProdJob{};
    Q.d = P->d;
    Q.path = P->path;
    Q.precision = P->precision;
    Q.v = v;
    Q.v_exp = slot;
    Q.out = out;
    Q.ns = P->marg[s].n;
    Q.nt = P->marg[t].n;
    Q.eta = pair_eta(P, t, s);
    for (int c = 0; c < 3; ++c) Q.ctr[c] = P->ext.ctr[c];
    // mixed direct sums: the expanded exponent cancels terms up to log2(e) r^2 / eta (r the
    // cloud's radius about its centre); above 8 it is formed in FP64
    const double half = 0.5 * P->ext.diag;
    Q.diff = P->precision == MOT_PREC_MIXED && 1.4426950408889634 * half * half / Q.eta > 8.0;
    Q.src_pts = P->marg[s].pts;
    Q.tgt_pts = P->marg[t].pts;
    Q.dsplit = 1;
    if (P->path == MOT_DIRECT && P->precision == MOT_PREC_FP64 && alloc_buffers) {
        const int split = direct_source_split(Q.nt, Q.ns);
        if (split > 1) {
            MOT_TRY(P->arena.get_n((size_t)split * Q.nt, &Q.dpart));
            Q.dsplit = split;
        }
    }
    if (P->path == MOT_TRUNC) {
        const TruncParams &T = P->TP;
        Q.src_cell_off = P->marg[s].cell_off;
        Q.h_src_cell_off = P->marg[s].h_cell_off.data();
        Q.h_tgt_cell_off = P->marg[t].h_cell_off.data();
        Q.nc = T.nc;
        Q.tw = T.w;
        Q.h = T.h;
        Q.q2 = T.q2;
        for (int c = 0; c < 3; ++c) Q.glo[c] = T.glo[c];
        // run length, targets per lane and exponent form from the cost model at this pair's
        // densities (points per grid cell)
        double cells = 1.0;  // full cells covering the cloud's box
        for (int c = 0; c < P->d; ++c) cells *= T.box_cells[c];
        const bool fp64 = P->precision == MOT_PREC_FP64;
        trunc_choose_run(P->d, T, (double)Q.nt / cells, (double)Q.ns / cells, fp64 ? 2 : 4,
                         std::sqrt(1.4426950408889634 / Q.eta) * T.h, fp64, &Q.trunc_b, &Q.trunc_r, &Q.diff);
        return MOT_OK;
    }
    if (P->path != MOT_NFFT) return MOT_OK;
    const NfftParams &N = P->P;
    const MargDev &S = P->marg[s], &Tm = P->marg[t];
    Q.src_win = S.win;
    Q.tgt_win = Tm.win;
    Q.src_chunk_start = S.chunk_start;
    Q.tgt_chunk_start = Tm.chunk_start;
    Q.src_chunk_tile = S.chunk_tile;
    Q.tgt_chunk_tile = Tm.chunk_tile;
    Q.src_tile_chunks = S.tile_chunks;
    Q.src_nchunks = S.nchunks;
    Q.tgt_nchunks = Tm.nchunks;
    Q.h_src_chunk_start = S.h_chunk_start.data();
    Q.h_tgt_chunk_start = Tm.h_chunk_start.data();
    Q.n = N.n;
    Q.M = N.M;
    Q.m = N.m;
    Q.T = N.T;
    for (int c = 0; c < 3; ++c) {
        Q.L[c] = N.L[c];
        Q.lo[c] = N.lo[c];
        Q.ntile[c] = N.ntile[c];
    }
    Q.W = N.W;
    {
        auto it = P->D_of_eta.find(Q.eta);
        Q.D = it != P->D_of_eta.end() ? it->second : P->D;
    }
    Q.twiddle = device_twiddle(N.n);
    int64_t pe = 1, cells = 1;
    for (int c = 0; c < P->d; ++c) {
        pe *= N.W;
        cells *= N.L[c];
    }
    const int H = N.M + 1, B = 2 * N.M + 1;
    int64_t spec = H;
    if (P->d == 2) spec = (int64_t)H * N.L[0];
    if (P->d == 3) spec = (int64_t)H * N.L[0] * std::max(N.L[1], B);
    Q.spec_elems = spec;
    if (!alloc_buffers) return MOT_OK;
    if (patches) {
        Q.patches = patches;
    } else {
        MOT_TRY(P->arena.get_n((size_t)S.nchunks * pe, &Q.patches));
    }
    MOT_TRY(P->arena.get_n((size_t)cells, &Q.grid));
    MOT_TRY(P->arena.get_n((size_t)spec, &Q.spec0));
    MOT_TRY(P->arena.get_n((size_t)spec, &Q.spec1));
    return MOT_OK;
}

static int plan_stats_alloc(mot_plan_s *P, int n_partials_hint)
{
    P->hist_cap = 1 << 16;
    MOT_TRY(P->arena.get_n(4, &P->sweep_ctr));
    MOT_TRY(P->arena.get_n(4, &P->flag));
    MOT_TRY(P->arena.get_n(P->hist_cap, &P->flag_hist));
    MOT_TRY(P->arena.get_n(P->hist_cap, &P->S_hist));
    MOT_TRY(P->arena.get_n(P->hist_cap, &P->err_hist));
    MOT_TRY(P->arena.get_n(2 * (size_t)n_partials_hint + 16, &P->s_partial));
    MOT_TRY(P->arena.get_n((size_t)n_partials_hint + 16, &P->l1_partial));
    MOT_HIP(launch_fill_int(P->sweep_ctr, 0, 1, P->stream));
    MOT_HIP(launch_fill_int(P->flag, 0, 1, P->stream));
    return MOT_OK;
}

// Per-marginal device state shared by both topologies: parameters (NFFT path), binned
// point layout (NFFT) or identity order, weights, phi = 1, statistics buffers.
int mot::setup_marginals(mot_plan_s *P, const std::vector<double> &pts_h, const std::vector<double> &w_h,
                         const mot_fastsum_params *fs, int64_t phi_pad_to)
{
    const int K = P->K, d = P->d;
    int64_t nmax = 0;
    for (int k = 0; k < K; ++k) nmax = std::max(nmax, P->n[k]);
    // the kernels' eta: eta itself and eta / w of every weighted tree edge
    std::vector<double> etas{P->eta};
    for (size_t k = 1; k < P->edge_w.size(); ++k) etas.push_back(P->eta / P->edge_w[k]);
    std::sort(etas.begin(), etas.end());
    etas.erase(std::unique(etas.begin(), etas.end()), etas.end());
    if (P->path == MOT_NFFT) {
        MOT_TRY(resolve_params(d, etas.front(), P->ext, fs, nmax, &P->P, etas.back()));
        for (double e : etas) {
            std::vector<float> D;
            build_multiplier(d, P->P, e, D);
            float *Dd = nullptr;
            MOT_TRY(P->arena.get_n(D.size(), &Dd));
            MOT_HIP(hipMemcpy(Dd, D.data(), D.size() * sizeof(float), hipMemcpyHostToDevice));
            P->D_of_eta[e] = Dd;
        }
        P->D = P->D_of_eta[P->eta];
        if (!device_twiddle(P->P.n)) return MOT_EDEVICE;
        log_msg("NFFT params: M=%d n=%d m=%d p=%d tau=%.6g eps_B=%.6g T=%d box=%dx%dx%d est_err=%.3g",
                P->P.M, P->P.n, P->P.m, P->P.p, P->P.tau, P->P.eps_B, P->P.T, P->P.L[0], P->P.L[1],
                P->P.L[2], P->P.est_err);
    }
    if (P->path == MOT_TRUNC) {
        double nsum = 0.0;
        for (int k = 0; k < K; ++k) nsum += (double)P->n[k];
        MOT_TRY(resolve_trunc(d, etas.back(), P->ext, fs, nsum / K, &P->TP));
        log_msg("truncation: eps=%.3g r_c=%.6g h=%.6g cells=%d^%d w=%d", P->TP.eps, P->TP.rc, P->TP.h,
                P->TP.nc, d, P->TP.w);
    }
    // temporaries of plan creation (points and weights in the caller's order, binning
    // scratch) come from an arena of their own: with the plan's allocator, released once
    // the plan's stream has finished with them, on every return path
    struct TmpArena {
        Arena a;
        hipStream_t st = nullptr;
        ~TmpArena()
        {
            if (st) (void)hipStreamSynchronize(st);
            a.release();
        }
    } tmp;
    tmp.a.alloc = P->arena.alloc;
    tmp.a.custom = P->arena.custom;
    tmp.st = P->stream;
    double *pts_dev = nullptr;
    MOT_TRY(tmp.a.get_n(pts_h.size(), &pts_dev));
    MOT_HIP(hipMemcpy(pts_dev, pts_h.data(), pts_h.size() * sizeof(double), hipMemcpyHostToDevice));
    P->marg.resize(K);
    int total_partials = 0;
    for (int k = 0; k < K; ++k) {
        MargDev &G = P->marg[k];
        G.n = P->n[k];
        const int64_t nphi = std::max<int64_t>(G.n, phi_pad_to > 0 ? (G.n + phi_pad_to - 1) / phi_pad_to * phi_pad_to : 0);
        MOT_TRY(P->arena.get_n((size_t)G.n * d, &G.pts));
        MOT_TRY(P->arena.get_n((size_t)G.n, &G.perm));
        MOT_TRY(P->arena.get_n((size_t)G.n, &G.mu));
        MOT_TRY(P->arena.get_n((size_t)nphi, &G.phi));
        MOT_TRY(P->arena.get_n((size_t)G.n, &G.gamma));
        MOT_TRY(P->arena.get_n((size_t)G.n, &G.up_src));
        MOT_TRY(P->arena.get_n((size_t)G.n, &G.marg));
        if (P->topology == MOT_TREE && k > 0) {
            MOT_TRY(P->arena.get_n((size_t)P->n[P->parent[k]], &G.beta));
            MOT_TRY(P->arena.get_n((size_t)P->n[P->parent[k]], &G.down_src));
        }
        if (P->path == MOT_NFFT) {
            MOT_TRY(P->arena.get_n((size_t)G.n * d * 16, &G.win));
        }
        if (nphi > G.n) MOT_HIP(launch_fill_double(G.phi + G.n, 0.0, nphi - G.n, P->stream));
        total_partials += 2 * (int)((G.n + kNodeItemElems - 1) / kNodeItemElems);
    }
    if (P->path == MOT_NFFT) {
        const int tpd = (P->P.n + P->P.T - 1) / P->P.T;
        int64_t ntiles = 1, nbox = 1;
        for (int c = 0; c < d; ++c) {
            ntiles *= tpd;
            nbox *= P->P.ntile[c];
        }
        const size_t sb = stable_tile_sort_scratch(nmax, ntiles);
        void *scratch = nullptr;
        int32_t *cell_tmp = nullptr, *tile_tmp = nullptr, *blo = nullptr, *bhi = nullptr;
        MOT_TRY(tmp.a.get(sb, &scratch));
        MOT_TRY(tmp.a.get_n((size_t)nmax * d, &cell_tmp));
        MOT_TRY(tmp.a.get_n((size_t)nmax, &tile_tmp));
        MOT_TRY(tmp.a.get_n((size_t)nbox, &blo));
        MOT_TRY(tmp.a.get_n((size_t)nbox, &bhi));
        for (int k = 0; k < K; ++k)
            MOT_TRY(bin_marginal(P, k, pts_dev + P->off[k] * d, scratch, sb, cell_tmp, tile_tmp, blo, bhi));
    } else if (P->path == MOT_TRUNC) {
        // a1's binning with tile edge 1: points sorted by cell, cell ranges kept
        const TruncParams &T = P->TP;
        const int64_t ncell = trunc_cells(d, T);
        const size_t sb = stable_tile_sort_scratch(nmax, ncell);
        void *scratch = nullptr;
        int32_t *cell_tmp = nullptr, *tile_tmp = nullptr;
        MOT_TRY(tmp.a.get(sb, &scratch));
        MOT_TRY(tmp.a.get_n((size_t)nmax * d, &cell_tmp));
        MOT_TRY(tmp.a.get_n((size_t)nmax, &tile_tmp));
        const double sc = 1.0 / T.h;
        double o[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < d; ++c) o[c] = -T.glo[c] * sc;
        for (int k = 0; k < K; ++k) {
            MargDev &G = P->marg[k];
            const double *src = pts_dev + P->off[k] * d;
            MOT_TRY(P->arena.get_n((size_t)ncell + 1, &G.cell_off));
            MOT_HIP(launch_bin_cells(d, G.n, src, sc, sc, sc, o[0], o[1], o[2], T.nc, 1, cell_tmp, tile_tmp,
                                     P->stream));
            MOT_HIP(stable_tile_sort(G.n, tile_tmp, ncell, G.perm, G.cell_off, scratch, sb, P->stream));
            MOT_HIP(launch_gather_rows(src, G.perm, G.n, d, G.pts, P->stream));
            G.h_cell_off.resize(ncell + 1);
            MOT_HIP(hipMemcpyAsync(G.h_cell_off.data(), G.cell_off, (ncell + 1) * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, P->stream));
        }
        MOT_HIP(hipStreamSynchronize(P->stream));
    } else {
        for (int k = 0; k < K; ++k) {
            std::vector<int32_t> id(P->n[k]);
            for (int64_t i = 0; i < P->n[k]; ++i) id[i] = (int32_t)i;
            MOT_HIP(hipMemcpy(P->marg[k].perm, id.data(), id.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            MOT_HIP(hipMemcpy(P->marg[k].pts, pts_h.data() + P->off[k] * d, P->n[k] * d * sizeof(double),
                              hipMemcpyHostToDevice));
        }
    }
    double *w_dev = nullptr;
    MOT_TRY(tmp.a.get_n(w_h.size(), &w_dev));
    MOT_HIP(hipMemcpy(w_dev, w_h.data(), w_h.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int k = 0; k < K; ++k) {
        MOT_HIP(launch_gather_rows(w_dev + P->off[k], P->marg[k].perm, P->n[k], 1, P->marg[k].mu, P->stream));
        MOT_HIP(launch_fill_double(P->marg[k].phi, 1.0, P->n[k], P->stream));
    }
    MOT_TRY(P->arena.get_n((size_t)(2 * K + 1) * kExpSlotStride, &P->exp_slots));
    MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * K + 1) * kExpSlotStride, P->stream));
    MOT_TRY(plan_stats_alloc(P, total_partials + 64 * K));
    return MOT_OK;
}

static int create_tree(mot_plan_s *P, const std::vector<double> &pts_h, const std::vector<double> &w_h,
                       const mot_fastsum_params *fs)
{
    const int K = P->K;
    // topology: children lists and depths
    P->children.assign(K, {});
    P->depth.assign(K, 0);
    for (int k = 1; k < K; ++k) {
        P->children[P->parent[k]].push_back(k);
        P->depth[k] = P->depth[P->parent[k]] + 1;
        P->depth_max = std::max(P->depth_max, P->depth[k]);
    }
    for (int k = 0; k < K; ++k)
        if ((int)P->children[k].size() > kMaxChildren) return MOT_EUNSUPPORTED;
    MOT_TRY(setup_marginals(P, pts_h, w_h, fs, 0));
    // product jobs
    P->jobs.assign(2 * K + 1, ProdJob{});
    for (int k = 1; k < K; ++k) {
        const int p = P->parent[k];
        // down: gamma_k = K^{(k,p)} u_k  (targets k, sources p)
        MOT_TRY(make_prod_job(P, k, p, P->marg[k].down_src, P->exp_slots + (size_t)(2 * k) * kExpSlotStride, P->marg[k].gamma,
                              &P->jobs[2 * k], nullptr));
        // up: beta_k = K^{(p,k)} v_k  (targets p, sources k)
        MOT_TRY(make_prod_job(P, p, k, P->marg[k].up_src, P->exp_slots + (size_t)(2 * k + 1) * kExpSlotStride, P->marg[k].beta,
                              &P->jobs[2 * k + 1], nullptr));
    }
    MOT_TRY(P->arena.get_n(P->jobs.size(), &P->jobs_dev));
    MOT_HIP(hipMemcpy(P->jobs_dev, P->jobs.data(), P->jobs.size() * sizeof(ProdJob), hipMemcpyHostToDevice));
    MOT_TRY(tree_build_schedule(P));
    TreeTables *T = tables_of(P);
    std::vector<TreeRef> refs{{P, 0, 0, 0}};
    MOT_TRY(tree_steps(refs, P->jobs, P->jobs_dev, T->njobs, T->njobs_dev, T->fjob, T->fjob_dev,
                       P->arena, P->sched.sweep, P->sched.init_up, P->sched.marg_pass));
    MOT_TRY(run_steps(P->sched.init_up, P->stream));
    MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * K + 1) * kExpSlotStride, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    return MOT_OK;
}

// ---------------------------------------------------------------------------------------
// Sweeps

namespace mot {

int tree_run_sweeps(mot_plan_s *P, int sweeps, bool use_graph)
{
    if (sweeps <= 0) return MOT_OK;
    if (use_graph && !P->sched.graph) {
        hipGraph_t g = nullptr;
        MOT_HIP(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
        int rc = run_steps(P->sched.sweep, P->stream);
        hipError_t e = hipStreamEndCapture(P->stream, &g);
        if (e == hipErrorStreamCaptureInvalidated) {
            // other work of the process invalidated the capture; none of its launches ran:
            // this call sweeps without the graph, the next one captures again
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            use_graph = false;
        } else {
            if (rc < 0) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            MOT_HIP(e);
            MOT_HIP(hipGraphInstantiate(&P->sched.graph, g, nullptr, nullptr, 0));
            P->sched.graph_def = g;
        }
    }
    for (int r = 0; r < sweeps; ++r) {
        if (use_graph) {
            MOT_HIP(hipGraphLaunch(P->sched.graph, P->stream));
        } else {
            MOT_TRY(run_steps(P->sched.sweep, P->stream));
        }
    }
    P->host_sweeps += sweeps;
    return MOT_OK;
}

int tree_init_up(mot_plan_s *P)
{
    MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
    MOT_TRY(run_steps(P->sched.init_up, P->stream));
    MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
    return MOT_OK;
}

}  // namespace mot

// ---------------------------------------------------------------------------------------
// C ABI

static bool use_graphs()
{
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("MOT_NO_GRAPH");
        v = (e && atoi(e) != 0) ? 0 : 1;
    }
    return v == 1;
}

extern "C" {

const char *mot_strerror(int s)
{
    switch (s) {
    case MOT_OK: return "ok";
    case MOT_MAXITER: return "sweep limit reached";
    case MOT_EINVAL: return "invalid argument";
    case MOT_EDOMAIN: return "fast-summation parameters cannot represent the points";
    case MOT_ENOMEM: return "out of device memory or admission budget";
    case MOT_EDEVICE: return "HIP runtime error";
    case MOT_ENUMERIC: return "a scaling vector became Inf/NaN";
    case MOT_EUNSUPPORTED: return "unsupported combination of options";
    case MOT_ELIMIT: return "size beyond the fixed limit of an allocation-free entry point";
    default: return "unknown status";
    }
}

int mot_plan_destroy(mot_plan P)
{
    if (!P) return MOT_EINVAL;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    if (P->circle) circle_destroy(P);
    P->sched.destroy();
    {
        std::lock_guard<std::mutex> lk(g_tables_mu);
        auto it = tables_map().find(P);
        if (it != tables_map().end()) {
            delete it->second;
            tables_map().erase(it);
        }
    }
    P->arena.release();
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
    return MOT_OK;
}

static int create_plan(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                       const double *weights, int32_t topology, const int32_t *parent,
                       const mot_tree_options *opt, const double *closing, double eta, int32_t path,
                       int32_t precision, const mot_fastsum_params *fs, int32_t ptr_kind, void *stream,
                       const mot_allocator *alloc)
{
    if (!out) return MOT_EINVAL;
    *out = nullptr;
    if (!n || !points || !weights || K < 2 || d < 1 || d > 3) return MOT_EINVAL;
    if (topology != MOT_TREE && topology != MOT_CIRCLE) return MOT_EINVAL;
    if (path != MOT_DIRECT && path != MOT_NFFT && path != MOT_DENSE && path != MOT_TRUNC) return MOT_EINVAL;
    if (path == MOT_DENSE && topology != MOT_CIRCLE) return MOT_EUNSUPPORTED;
    if (path == MOT_TRUNC && topology != MOT_TREE) return MOT_EUNSUPPORTED;
    if (precision == MOT_PREC_FP64 && path != MOT_DIRECT && path != MOT_TRUNC) return MOT_EUNSUPPORTED;
    if ((path == MOT_DIRECT || path == MOT_TRUNC) && precision != MOT_PREC_FP64 && precision != MOT_PREC_MIXED)
        return MOT_EUNSUPPORTED;
    if (path == MOT_NFFT && precision != MOT_PREC_MIXED) return MOT_EUNSUPPORTED;
    if (topology == MOT_TREE) {
        if (!parent || parent[0] != -1) return MOT_EINVAL;
        for (int k = 1; k < K; ++k)
            if (parent[k] < 0 || parent[k] >= k) return MOT_EINVAL;
    } else if (K < 3) {
        return MOT_EINVAL;
    }
    int64_t total = 0;
    for (int k = 0; k < K; ++k) {
        if (n[k] < 1) return MOT_EINVAL;
        total += n[k];
    }
    std::vector<double> edge_w;
    std::vector<int> free_node;
    if (opt) {
        if (topology != MOT_TREE) return MOT_EINVAL;
        if (opt->edge_weight) {
            edge_w.assign(opt->edge_weight, opt->edge_weight + K);
            edge_w[0] = 1.0;
            for (int k = 1; k < K; ++k)
                if (!(edge_w[k] > 0.0) || !std::isfinite(edge_w[k]) || !std::isfinite(eta / edge_w[k]))
                    return MOT_EINVAL;
        }
        if (opt->free_node) {
            free_node.assign(K, 0);
            for (int k = 0; k < K; ++k) free_node[k] = opt->free_node[k] != 0;
            if (free_node[0]) return MOT_EINVAL;  // the root's update fixes the common scale
        }
    }
    std::vector<double> pts_h, w_h;
    int rc = copy_in(points, (size_t)total * d, ptr_kind, pts_h);
    if (rc < 0) return rc;
    rc = copy_in(weights, (size_t)total, ptr_kind, w_h);
    if (rc < 0) return rc;
    rc = validate_common(K, d, n, eta, w_h, pts_h, total, free_node);
    if (rc < 0) return rc;
    std::vector<double> closing_h;
    if (closing) {
        if (topology != MOT_CIRCLE) return MOT_EINVAL;
        rc = copy_in(closing, (size_t)n[0] * d, ptr_kind, closing_h);
        if (rc < 0) return rc;
        for (double v : closing_h)
            if (!std::isfinite(v)) return MOT_EINVAL;
    }
    {  // free nodes carry no weights: zero them (no S term, mu is never divided)
        int64_t o = 0;
        for (int k = 0; k < K; ++k) {
            if (!free_node.empty() && free_node[k]) std::fill(w_h.begin() + o, w_h.begin() + o + n[k], 0.0);
            o += n[k];
        }
    }

    mot_plan_s *P = new mot_plan_s();
    P->K = K;
    P->d = d;
    P->topology = topology;
    P->path = path;
    P->precision = precision;
    P->eta = eta;
    P->edge_w = edge_w;
    P->free_node = free_node;
    P->closing = closing_h;
    (void)hipGetDevice(&P->device);
    if (alloc && alloc->alloc && alloc->free) {
        P->arena.alloc = *alloc;
        P->arena.custom = true;
    }
    if (stream) {
        P->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess) {
            delete P;
            return MOT_EDEVICE;
        }
        P->own_stream = true;
    }
    P->n.assign(n, n + K);
    P->off.assign(K + 1, 0);
    for (int k = 0; k < K; ++k) P->off[k + 1] = P->off[k] + n[k];
    if (topology == MOT_TREE) P->parent.assign(parent, parent + K);
    P->ext = extent_of(d, pts_h, total);
    if (topology == MOT_TREE)
        rc = create_tree(P, pts_h, w_h, fs);
    else
        rc = circle_create(P, pts_h, w_h, fs);
    if (rc < 0) {
        (void)hipStreamSynchronize(P->stream);
        mot_plan_destroy(P);
        return rc;
    }
    *out = P;
    return MOT_OK;
}

int mot_plan_create(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                    const double *weights, int32_t topology, const int32_t *parent, double eta,
                    int32_t path, int32_t precision, const mot_fastsum_params *fs, int32_t ptr_kind,
                    void *stream, const mot_allocator *alloc)
{
    return create_plan(out, K, d, n, points, weights, topology, parent, nullptr, nullptr, eta, path, precision,
                       fs, ptr_kind, stream, alloc);
}

int mot_plan_create_circle(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                           const double *weights, const double *closing_points, double eta, int32_t path,
                           int32_t precision, const mot_fastsum_params *fs, int32_t ptr_kind, void *stream,
                           const mot_allocator *alloc)
{
    return create_plan(out, K, d, n, points, weights, MOT_CIRCLE, nullptr, nullptr, closing_points, eta, path,
                       precision, fs, ptr_kind, stream, alloc);
}

int mot_pair_marginal(mot_plan P, int32_t k, double *out, int32_t ptr_kind)
{
    if (!P || !out || k < 1 || k >= P->K) return MOT_EINVAL;
    const int a = P->topology == MOT_CIRCLE ? 0 : P->parent[k];
    const size_t count = (size_t)P->n[a] * (size_t)P->n[k];
    DevTmp buf;
    double *dst = out;
    if (ptr_kind != MOT_DEVICE) {
        MOT_TRY(buf.alloc(count * sizeof(double)));
        dst = buf.as<double>();
    }
    auto body = [&]() -> int {
        if (P->topology == MOT_CIRCLE) return circle_pair_marginal(P, k, dst);
        // a consistent pass at the current phi (as in mot_marginals): the down source of k
        // at its parent and the up source of k are then the two outer factors
        MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
        MOT_TRY(run_steps(P->sched.marg_pass, P->stream));
        MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
        MOT_HIP(launch_tree_pair(P->marg[k].down_src, P->marg[a].pts, P->marg[a].perm, P->n[a], P->marg[k].up_src,
                                 P->marg[k].pts, P->marg[k].perm, P->n[k], P->d, P->jobs[2 * k + 1].eta, dst,
                                 P->stream));
        return MOT_OK;
    };
    int rc = body();
    if (rc >= 0 && ptr_kind != MOT_DEVICE &&
        hipMemcpyAsync(out, dst, count * sizeof(double), hipMemcpyDeviceToHost, P->stream) != hipSuccess)
        rc = MOT_EDEVICE;
    if (hipStreamSynchronize(P->stream) != hipSuccess && rc >= 0) rc = MOT_EDEVICE;
    return rc;
}

int mot_plan_create_tree(mot_plan *out, int32_t K, int32_t d, const int64_t *n, const double *points,
                         const double *weights, const int32_t *parent, const mot_tree_options *opt,
                         double eta, int32_t path, int32_t precision, const mot_fastsum_params *fs,
                         int32_t ptr_kind, void *stream, const mot_allocator *alloc)
{
    return create_plan(out, K, d, n, points, weights, MOT_TREE, parent, opt, nullptr, eta, path, precision, fs,
                       ptr_kind, stream, alloc);
}

int mot_plan_get_info(mot_plan P, mot_plan_info *info)
{
    if (!P || !info) return MOT_EINVAL;
    mot_plan_info I{};
    I.K = P->K;
    I.d = P->d;
    I.topology = P->topology;
    I.path = P->path;
    I.precision = P->precision;
    I.M = P->P.M;
    I.n = P->P.n;
    I.m = P->P.m;
    I.p = P->P.p;
    I.tile = P->P.T;
    I.chunk = P->P.chunk;
    I.tau = P->P.tau;
    I.eps_B = P->P.eps_B;
    I.eta = P->eta;
    I.scale = P->P.s;
    for (int c = 0; c < 3; ++c) {
        I.offset[c] = P->P.o[c];
        I.box_lo[c] = P->P.lo[c];
        I.box_len[c] = P->P.L[c];
    }
    I.depth = P->depth_max;
    I.device_bytes = P->arena.bytes;
    I.products_per_sweep = P->topology == MOT_TREE ? 2 * (P->K - 1) : 2 * (P->K - 2);
    I.est_err = P->path == MOT_NFFT ? P->P.est_err : 0.0;
    if (P->path == MOT_TRUNC) {
        const TruncParams &T = P->TP;
        I.est_err = T.est_err;
        I.trunc_radius = T.rc;
        I.n = T.nc;
        I.tile = T.w;
        I.chunk = T.B;
        I.m = T.R;
        // the scale and offsets the cell binning used (setup_marginals), bit for bit
        I.scale = 1.0 / T.h;
        for (int c = 0; c < 3; ++c) I.offset[c] = c < P->d ? -T.glo[c] * I.scale : 0.0;
    }
    *info = I;
    return MOT_OK;
}

int mot_sinkhorn(mot_plan P, int32_t max_sweeps, double delta_S, double tol_marginal,
                 int32_t check_every, int32_t *sweeps_done, double *S_last, double *marg_err)
{
    if (!P || max_sweeps < 0) return MOT_EINVAL;
    if (check_every < 1) check_every = 1;
    const bool stopping = delta_S > 0.0 || tol_marginal > 0.0;
    int done = 0, status = MOT_MAXITER;
    int32_t ctr0 = 0;
    MOT_HIP(hipMemcpyAsync(&ctr0, P->sweep_ctr, 4, hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    double lastS = NAN, lastE = NAN;
    while (done < max_sweeps) {
        const int batch = stopping ? std::min(check_every, max_sweeps - done) : max_sweeps - done;
        int rc = P->topology == MOT_TREE ? tree_run_sweeps(P, batch, use_graphs())
                                         : circle_run_sweeps(P, batch);
        if (rc < 0) return rc;
        done += batch;
        // read the last recorded values
        const int idx = (ctr0 + done - 1) % P->hist_cap;
        const int idxp = (ctr0 + done - 2 + P->hist_cap) % P->hist_cap;
        double h[2] = {0, 0}, e = 0;
        int32_t fl = 0;
        MOT_HIP(hipMemcpyAsync(&h[1], P->S_hist + idx, 8, hipMemcpyDeviceToHost, P->stream));
        MOT_HIP(hipMemcpyAsync(&h[0], P->S_hist + idxp, 8, hipMemcpyDeviceToHost, P->stream));
        MOT_HIP(hipMemcpyAsync(&e, P->err_hist + idx, 8, hipMemcpyDeviceToHost, P->stream));
        MOT_HIP(hipMemcpyAsync(&fl, P->flag, 4, hipMemcpyDeviceToHost, P->stream));
        MOT_HIP(hipStreamSynchronize(P->stream));
        lastS = h[1];
        lastE = e;
        if (fl) {
            status = MOT_ENUMERIC;
            break;
        }
        if (tol_marginal > 0.0 && e <= tol_marginal) {
            status = MOT_OK;
            break;
        }
        if (delta_S > 0.0 && (ctr0 + done) >= 2 && std::fabs(h[1] - h[0]) < delta_S) {
            status = MOT_OK;
            break;
        }
    }
    if (sweeps_done) *sweeps_done = done;
    if (S_last) *S_last = lastS;
    if (marg_err) *marg_err = lastE;
    return status;
}

int mot_plan_profile(mot_plan P, int32_t sweeps, mot_step_timing *out, int32_t max_out)
{
    if (!P || sweeps < 1 || (!out && max_out > 0)) return MOT_EINVAL;
    if (P->topology != MOT_TREE) return MOT_EUNSUPPORTED;
    // every launch of the schedule, one after another on the plan's stream (the lanes'
    // fork and join markers are not launches)
    std::vector<Step> steps;
    for (const Step &st : P->sched.sweep)
        if (st.kind != ST_FORK && st.kind != ST_JOIN) steps.push_back(st);
    const size_t ns = steps.size();
    // events destroyed on every return path
    struct Events {
        std::vector<hipEvent_t> e;
        ~Events()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    evs.e.assign(2 * ns, nullptr);
    std::vector<hipEvent_t> &ev = evs.e;
    for (auto &e : ev) MOT_HIP(hipEventCreate(&e));
    std::vector<double> acc(ns, 0.0);
    for (int r = 0; r < sweeps; ++r) {
        for (size_t i = 0; i < ns; ++i) {
            MOT_HIP(hipEventRecord(ev[2 * i], P->stream));
            std::vector<Step> one{steps[i]};
            MOT_TRY(run_steps(one, P->stream));
            MOT_HIP(hipEventRecord(ev[2 * i + 1], P->stream));
        }
        MOT_HIP(hipStreamSynchronize(P->stream));
        for (size_t i = 0; i < ns; ++i) {
            float ms = 0.f;
            MOT_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
            acc[i] += ms;
        }
    }
    P->host_sweeps += sweeps;
    const int nout = std::min((int)ns, (int)max_out);
    static const int kind_code[] = {0, 1, 2, 3, 4, 5, 6, 7, 8};
    for (int i = 0; i < nout; ++i) {
        mot_step_timing t{};
        t.kind = kind_code[steps[i].kind];
        t.d = steps[i].d;
        t.n = steps[i].n;
        t.fft_kind = steps[i].fft_kind;
        t.n_items = steps[i].n_items;
        t.group = steps[i].group;
        t.calls = sweeps;
        t.ms_mean = acc[i] / sweeps;
        out[i] = t;
    }
    return nout;
}

int mot_get_S_history(mot_plan P, double *S_out, int32_t count)
{
    if (!P || (!S_out && count > 0)) return MOT_EINVAL;
    int32_t ctr = 0;
    MOT_HIP(hipMemcpyAsync(&ctr, P->sweep_ctr, 4, hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    const int avail = std::min(ctr, P->hist_cap);
    const int nout = std::min(avail, (int)count);
    const int first = ctr - avail;
    for (int i = 0; i < nout; ++i) {
        const int slot = (first + i) % P->hist_cap;
        MOT_HIP(hipMemcpyAsync(S_out + i, P->S_hist + slot, 8, hipMemcpyDeviceToHost, P->stream));
    }
    MOT_HIP(hipStreamSynchronize(P->stream));
    return nout;
}

// The plan's staging buffer (see mot_plan_s::stage), allocated at first use.
static int plan_stage(mot_plan P, double **out)
{
    if (!P->stage) {
        int64_t nmax = 0;
        for (int k = 0; k < P->K; ++k) nmax = std::max<int64_t>(nmax, P->n[k]);
        MOT_TRY(P->arena.get_n((size_t)std::max<int64_t>(P->off[P->K], 2 * nmax), &P->stage));
    }
    *out = P->stage;
    return MOT_OK;
}

static int scatter_out(mot_plan P, double *const *src_sorted, double *dst, int ptr_kind)
{
    // binned order -> original order, concatenated
    const int64_t total = P->off[P->K];
    double *tmp = dst;
    if (ptr_kind != MOT_DEVICE) MOT_TRY(plan_stage(P, &tmp));
    for (int k = 0; k < P->K; ++k)
        MOT_HIP(launch_scatter_vec(src_sorted[k], P->marg[k].perm, P->n[k], tmp + P->off[k], P->stream));
    if (ptr_kind != MOT_DEVICE)
        MOT_HIP(hipMemcpyAsync(dst, tmp, total * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    return MOT_OK;
}

int mot_get_scalings(mot_plan P, double *phi_out, int32_t ptr_kind)
{
    if (!P || !phi_out) return MOT_EINVAL;
    std::vector<double *> src(P->K);
    for (int k = 0; k < P->K; ++k) src[k] = P->marg[k].phi;
    return scatter_out(P, src.data(), phi_out, ptr_kind);
}

int mot_set_scalings(mot_plan P, const double *phi_in, int32_t ptr_kind)
{
    if (!P || !phi_in) return MOT_EINVAL;
    const int64_t total = P->off[P->K];
    double *tmp = nullptr;
    MOT_TRY(plan_stage(P, &tmp));
    MOT_HIP(hipMemcpyAsync(tmp, phi_in, total * sizeof(double),
                           ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           P->stream));
    for (int k = 0; k < P->K; ++k)
        MOT_HIP(launch_gather_rows(tmp + P->off[k], P->marg[k].perm, P->n[k], 1, P->marg[k].phi, P->stream));
    if (P->topology == MOT_TREE) MOT_TRY(tree_init_up(P));
    MOT_HIP(hipStreamSynchronize(P->stream));
    if (P->topology == MOT_CIRCLE) return circle_run_sweeps(P, 0);
    return MOT_OK;
}

int mot_marginals(mot_plan P, double *P_out, double *l1_err, int32_t ptr_kind)
{
    if (!P) return MOT_EINVAL;
    if (P->topology == MOT_CIRCLE) {
        MOT_TRY(circle_marginals(P, nullptr));
    } else {
        MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
        MOT_TRY(run_steps(P->sched.marg_pass, P->stream));
        MOT_HIP(launch_fill_int(P->exp_slots, INT32_MIN, (2 * P->K + 1) * kExpSlotStride, P->stream));
        // the marginal pass overwrote beta with values at the current phi (the same
        // values a following sweep expects), and gamma with consistent values
    }
    MOT_HIP(hipStreamSynchronize(P->stream));
    if (l1_err) {
        if (P->topology == MOT_TREE) {
            TreeTables *T = tables_of(P);
            std::vector<double> part(2 * (size_t)(T->n_down_partials + T->n_marg_partials));
            MOT_HIP(hipMemcpy(part.data(), P->s_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int k = 0; k < P->K; ++k) {
                const int items = (int)((P->n[k] + kNodeItemElems - 1) / kNodeItemElems);
                double s = 0.0;
                for (int i = 0; i < items; ++i) s += part[2 * (T->marg_block0[k] + i)];
                l1_err[k] = s;
            }
        } else {
            std::vector<double> Pm(P->off[P->K]), mu(P->off[P->K]);
            for (int k = 0; k < P->K; ++k) {
                MOT_HIP(hipMemcpy(Pm.data() + P->off[k], P->marg[k].marg, P->n[k] * 8, hipMemcpyDeviceToHost));
                MOT_HIP(hipMemcpy(mu.data() + P->off[k], P->marg[k].mu, P->n[k] * 8, hipMemcpyDeviceToHost));
                double s = 0.0;
                for (int64_t i = 0; i < P->n[k]; ++i) s += std::fabs(Pm[P->off[k] + i] - mu[P->off[k] + i]);
                l1_err[k] = s;
            }
        }
    }
    if (P_out) {
        std::vector<double *> src(P->K);
        for (int k = 0; k < P->K; ++k) src[k] = P->marg[k].marg;
        MOT_TRY(scatter_out(P, src.data(), P_out, ptr_kind));
    }
    return MOT_OK;
}

int mot_apply_kernel(mot_plan P, int32_t t, int32_t s, const double *v, double *out, int32_t ptr_kind)
{
    if (!P || !v || !out || t < 0 || s < 0 || t >= P->K || s >= P->K) return MOT_EINVAL;
    if (P->topology != MOT_TREE) return MOT_EUNSUPPORTED;
    const int64_t cap = *std::max_element(P->n.begin(), P->n.end());
    if (!P->apply_in) {
        MOT_TRY(P->arena.get_n((size_t)cap, &P->apply_in));
        MOT_TRY(P->arena.get_n((size_t)cap, &P->apply_out));
        P->apply_cap = cap;
    }
    // v (original order) -> binned order of s
    double *tmp = nullptr;
    MOT_TRY(plan_stage(P, &tmp));  // n[s] + n[t] <= 2 max n_k doubles
    MOT_HIP(hipMemcpyAsync(tmp, v, P->n[s] * sizeof(double),
                           ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           P->stream));
    MOT_HIP(launch_gather_rows(tmp, P->marg[s].perm, P->n[s], 1, P->apply_in, P->stream));
    int32_t *slot = P->exp_slots + (size_t)(2 * P->K) * kExpSlotStride;
    MOT_HIP(launch_fill_int(slot, INT32_MIN, 1, P->stream));
    MOT_HIP(launch_vec_exp(P->apply_in, P->n[s], slot, P->stream));
    // job slot 2K: buffers sized for the largest chunk count, allocated on first use
    ProdJob &slotjob = P->jobs[2 * P->K];
    if (P->path == MOT_NFFT && !slotjob.grid) {
        int maxc = 0;
        for (auto &g : P->marg) maxc = std::max(maxc, g.nchunks);
        int64_t pe = 1;
        for (int c = 0; c < P->d; ++c) pe *= P->P.W;
        MOT_TRY(P->arena.get_n((size_t)maxc * pe, &P->apply_patches));
        MOT_TRY(make_prod_job(P, t, s, P->apply_in, slot, P->apply_out, &slotjob, P->apply_patches));
    }
    ProdJob J;
    MOT_TRY(make_prod_job(P, t, s, P->apply_in, slot, P->apply_out, &J, nullptr, false));
    J.patches = P->apply_patches;
    J.grid = slotjob.grid;
    J.spec0 = slotjob.spec0;
    J.spec1 = slotjob.spec1;
    ProdJob *jd = P->jobs_dev + 2 * P->K;
    MOT_HIP(hipMemcpyAsync(jd, &J, sizeof(ProdJob), hipMemcpyHostToDevice, P->stream));
    std::vector<Step> steps;
    StepBuilder B{&P->arena, &steps};
    std::vector<ProdJob> hj(2 * P->K + 1);
    hj[2 * P->K] = J;
    B.products(P->jobs_dev, hj, {2 * P->K});
    if (B.rc < 0) return B.rc;
    MOT_TRY(run_steps(steps, P->stream));
    MOT_HIP(launch_scatter_vec(P->apply_out, P->marg[t].perm, P->n[t], tmp + P->n[s], P->stream));
    MOT_HIP(hipMemcpyAsync(out, tmp + P->n[s], P->n[t] * sizeof(double),
                           ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    return MOT_OK;
}

int mot_bin_points(int32_t d, int64_t npts, const double *x, const double *s, const double *o,
                   int32_t n, int32_t T, int32_t sub_dim, int32_t *cell, int32_t *perm, int32_t *tile_off,
                   int32_t ptr_kind, void *stream)
{
    if (d < 1 || d > 3 || npts < 0 || !x || !s || !o || n < 1 || T < 1 || !cell || !perm || !tile_off)
        return MOT_EINVAL;
    if (sub_dim < -1 || sub_dim >= d || (sub_dim >= 0 && T > 16)) return MOT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int tpd = (n + T - 1) / T;
    int64_t ntiles = 1;
    for (int c = 0; c < d; ++c) ntiles *= tpd;
    if (ntiles > ((int64_t)1 << 30) || (sub_dim >= 0 && ntiles >= ((int64_t)1 << 28))) return MOT_EINVAL;
    const size_t sb = stable_tile_sort_scratch(npts, ntiles);
    DevTmp bx, bc, bt, bp, bo, bs;
    MOT_TRY(bx.alloc(std::max<int64_t>(npts, 1) * d * sizeof(double)));
    MOT_TRY(bc.alloc(std::max<int64_t>(npts, 1) * d * sizeof(int32_t)));
    MOT_TRY(bt.alloc(std::max<int64_t>(npts, 1) * sizeof(int32_t)));
    MOT_TRY(bp.alloc(std::max<int64_t>(npts, 1) * sizeof(int32_t)));
    MOT_TRY(bo.alloc((ntiles + 1) * sizeof(int32_t)));
    MOT_TRY(bs.alloc(sb));
    double *xd = bx.as<double>();
    int32_t *cd = bc.as<int32_t>(), *td = bt.as<int32_t>(), *pd = bp.as<int32_t>(), *od = bo.as<int32_t>();
    void *scratch = bs.p;
    const hipMemcpyKind kin = ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kout = ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (npts > 0) MOT_HIP(hipMemcpyAsync(xd, x, npts * d * sizeof(double), kin, st));
    MOT_HIP(launch_bin_cells(d, npts, xd, s[0], d > 1 ? s[1] : 0.0, d > 2 ? s[2] : 0.0, o[0],
                             d > 1 ? o[1] : 0.0, d > 2 ? o[2] : 0.0, n, T, cd, td, st));
    // the plan's binning (bin_marginal) calls the same sort with the same sub-key
    MOT_HIP(stable_tile_sort(npts, td, ntiles, pd, od, scratch, sb, st, sub_dim >= 0 ? cd : nullptr, d,
                             sub_dim >= 0 ? sub_dim : 0, T));
    if (npts > 0) {
        MOT_HIP(hipMemcpyAsync(cell, cd, npts * d * sizeof(int32_t), kout, st));
        MOT_HIP(hipMemcpyAsync(perm, pd, npts * sizeof(int32_t), kout, st));
    }
    MOT_HIP(hipMemcpyAsync(tile_off, od, (ntiles + 1) * sizeof(int32_t), kout, st));
    MOT_HIP(hipStreamSynchronize(st));
    return MOT_OK;
}

int mot_plan_get_order(mot_plan P, int32_t k, int32_t *perm_out, int32_t ptr_kind)
{
    if (!P || !perm_out || k < 0 || k >= P->K) return MOT_EINVAL;
    MOT_HIP(hipMemcpyAsync(perm_out, P->marg[k].perm, P->n[k] * sizeof(int32_t),
                           ptr_kind == MOT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, P->stream));
    MOT_HIP(hipStreamSynchronize(P->stream));
    return MOT_OK;
}

// FFT line-pass items of one product job: the step builder's count for the job's chain.
static int64_t fft_items_of(int d, int n, int M, const int L[3])
{
    const int H = M + 1, B = 2 * M + 1;
    auto items = [n](int kind, int64_t a2, int64_t a1) {
        const int per = mot::fft_lines_per_item(kind, n);
        return a2 * ((a1 + per - 1) / per);
    };
    if (d == 1) return 2;
    if (d == 2) return items(0, 1, L[0]) + items(2, 1, H) + items(4, 1, L[0]);
    if ((int64_t)L[1] * H * 8 <= mot::kSlabLds) return 2 * (int64_t)L[0] + items(5, H, B);
    return items(0, L[0], L[1]) + items(1, H, L[0]) + items(2, H, B) + items(3, L[0], H) + items(4, L[0], L[1]);
}

int mot_plan_footprint(int32_t K, int32_t d, const int64_t *n, int32_t topology, int32_t path,
                       int32_t precision, double eta, double half_width,
                       const mot_fastsum_params *fs, size_t *bytes)
{
    if (!n || !bytes || K < 2 || d < 1 || d > 3) return MOT_EINVAL;
    int64_t total = 0, nmax = 0;
    for (int k = 0; k < K; ++k) {
        total += n[k];
        nmax = std::max(nmax, n[k]);
    }
    size_t b = 0;
    // per point: points, perm, mu, phi, gamma, up/down sources, beta, marginal; window
    // rows on the NFFT path
    b += (size_t)total * (8 * d + 4 + 8 * 7 + (path == MOT_NFFT ? 64 * d : 0));
    if (topology == MOT_CIRCLE) {
        b += circle_footprint(K, n, path, precision);
        if (path == MOT_NFFT) {
            // row-by-row fast sums: every row of a product is one job with its own patches,
            // grid and spectra (shared by the product positions), and every position has
            // its job table and launch item arrays
            Extent E;
            for (int c = 0; c < d; ++c) {
                E.lo[c] = -half_width;
                E.hi[c] = half_width;
            }
            E.diag = 2.0 * half_width * std::sqrt((double)d);
            NfftParams Q;
            int rc = resolve_params(d, eta, E, fs, nmax, &Q);
            if (rc < 0) return rc;
            int64_t cells = 1, pe = 1, tiles = 1;
            for (int c = 0; c < d; ++c) {
                cells *= Q.L[c];
                pe *= Q.W;
                tiles *= Q.ntile[c];
            }
            const int H = Q.M + 1, B = 2 * Q.M + 1;
            int64_t spec = H;
            if (d == 2) spec = (int64_t)H * Q.L[0];
            if (d == 3) spec = (int64_t)H * Q.L[0] * std::max(Q.L[1], B);
            const int64_t maxc = tiles + nmax / std::max(1, Q.chunk) + 1;
            const int64_t n1 = n[0];
            b += (size_t)n1 * ((size_t)maxc * pe * 4 + (size_t)cells * 4 + (size_t)spec * 16 + 3 * 256);
            const int64_t fft_items = fft_items_of(d, Q.n, Q.M, Q.L) + 8;
            const int64_t per_job = (int64_t)sizeof(ProdJob) + 8 * 2 * maxc + 8 * (cells / kFoldCellsPerItem + 1) +
                                    16 * fft_items;
            b += (size_t)(2 * (K - 2)) * ((size_t)n1 * per_job + 16 * 256);
            b += (size_t)(2 * (K - 2) + 1) * (64 * 1024);
        }
    } else if (path == MOT_NFFT) {
        Extent E;
        for (int c = 0; c < d; ++c) {
            E.lo[c] = -half_width;
            E.hi[c] = half_width;
        }
        E.diag = 2.0 * half_width * std::sqrt((double)d);
        NfftParams Q;
        int rc = resolve_params(d, eta, E, fs, nmax, &Q);
        if (rc < 0) return rc;
        int64_t cells = 1, pe = 1;
        for (int c = 0; c < d; ++c) {
            cells *= Q.L[c];
            pe *= Q.W;
        }
        const int H = Q.M + 1, B = 2 * Q.M + 1;
        int64_t spec = H;
        if (d == 2) spec = (int64_t)H * Q.L[0];
        if (d == 3) spec = (int64_t)H * Q.L[0] * std::max(Q.L[1], B);
        int64_t tiles = 1;
        for (int c = 0; c < d; ++c) tiles *= Q.ntile[c];
        // every product job holds one patch per chunk of its source marginal: at most one
        // chunk per non-empty tile plus one per Q.chunk points
        const int64_t chunks_per_job = std::min(tiles, nmax) + nmax / std::max(1, Q.chunk) + 1;
        b += (size_t)(2 * (K - 1) + 1) * (cells * 4 + spec * 16);
        b += (size_t)(2 * (K - 1) + 1) * chunks_per_job * pe * 4;
        b += (size_t)H * B * B * 4;
        // launch items: FFT passes, spreading and interpolation chunks, fold cells
        b += (size_t)(2 * (K - 1)) * (16 * (fft_items_of(d, Q.n, Q.M, Q.L) + 8) + 8 * 2 * chunks_per_job +
                                      8 * (cells / kFoldCellsPerItem + 1));
    } else if (path == MOT_DIRECT && precision == MOT_PREC_FP64 && topology == MOT_TREE) {
        // partial sums of the source ranges: split x n_t <= 1024 x 64 + n_t + 64 per job
        b += (size_t)(2 * (K - 1)) * (size_t)(1024 * 64 + nmax + 64) * 8;
    } else if (path == MOT_TRUNC) {
        Extent E;
        for (int c = 0; c < d; ++c) {
            E.lo[c] = -half_width;
            E.hi[c] = half_width;
        }
        E.width_max = 2.0 * half_width;
        E.diag = 2.0 * half_width * std::sqrt((double)d);
        TruncParams T;
        int rc = resolve_trunc(d, eta, E, fs, (double)total / K, &T);
        if (rc < 0) return rc;
        const int64_t ncell = trunc_cells(d, T);
        b += (size_t)(K + 1) * (ncell + 1) * 4 + stable_tile_sort_scratch(nmax, ncell);
    }
    b += (size_t)(1 << 16) * 20 + (1 << 20);
    *bytes = b;
    return MOT_OK;
}

}  // extern "C"
