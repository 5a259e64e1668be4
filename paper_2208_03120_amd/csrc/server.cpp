// Serving form (a12): a continuous-batching solver service on one GPU.
//
// Requests are complete MOT problems.  They wait in FIFO order until their device
// footprint fits the HBM budget and a slot is free; a preparation thread then builds the
// plan on a stream of its own (copies, binning, window rows, precompute), off the sweep
// loop's critical path.  The service loop advances every resident problem a few sweeps per
// step: the tree problems through one batched schedule on the server's stream, each circle
// problem on a stream of its own, so circle products overlap the tree launches.  After a
// step it reads every problem's first-marginal error in one synchronisation and retires the
// problems that meet their tolerance (or fail, or reach their sweep limit).
//
// When the resident tree set changes, the preparation thread builds the batched schedule of
// the new set while the loop keeps sweeping the old one; the loop swaps it in between steps.
// Retired trees stay in the old schedule until then (their results are already copied out)
// and are released at the swap.  Plans and schedules take their device memory from a pool
// owned by the server, so releasing them calls no hipFree (which would wait for the whole
// device) while other problems run.  A problem's arithmetic does not depend on which others
// share the launches, nor on when it joins them.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>

#include "host.h"

namespace {

// Device memory pool: blocks rounded up to powers of two (at least 256 bytes), handed out
// again after release, returned to the runtime only when the server is destroyed.
struct Pool {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free_blocks;
    std::map<void *, size_t> block_size;
    size_t held = 0;

    static void *alloc(size_t bytes, void *ctx)
    {
        Pool *p = (Pool *)ctx;
        size_t cls = 256;
        while (cls < bytes) cls <<= 1;
        std::lock_guard<std::mutex> lk(p->mu);
        auto it = p->free_blocks.find(cls);
        if (it != p->free_blocks.end() && !it->second.empty()) {
            void *q = it->second.back();
            it->second.pop_back();
            return q;
        }
        void *q = nullptr;
        if (hipMalloc(&q, cls) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        p->block_size[q] = cls;
        p->held += cls;
        return q;
    }
    static void free(void *q, void *ctx)
    {
        Pool *p = (Pool *)ctx;
        std::lock_guard<std::mutex> lk(p->mu);
        auto it = p->block_size.find(q);
        if (it != p->block_size.end()) p->free_blocks[it->second].push_back(q);
    }
    void release_all()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : block_size) (void)hipFree(kv.first);
        block_size.clear();
        free_blocks.clear();
        held = 0;
    }
};

struct Req {
    uint64_t ticket = 0;
    int32_t K = 0, d = 0, topology = 0, path = 0, precision = 0, max_sweeps = 0;
    double eta = 0, tol = 0;
    std::vector<int64_t> n;
    std::vector<double> points, weights;
    std::vector<int32_t> parent;
    double t_submit = 0;
    size_t footprint = 0;
};

// A resident problem.
struct Live {
    Req req;
    mot_plan plan = nullptr;
    double t_admit = 0;
    size_t bytes = 0;        // budget charged: max(footprint estimate, device bytes held)
    int32_t sweeps = 0;
    bool retired = false;
};

struct Done {
    mot_result res{};
    std::vector<double> phi;
};

}  // namespace

struct mot_server_s {
    size_t budget = 0, max_request = 0;
    int32_t max_slots = 0;
    int32_t step_sweeps = 2;
    int device = 0;
    hipStream_t stream = nullptr;       // tree batch
    hipStream_t prep_stream = nullptr;  // plan creation
    bool own_stream = false;
    Pool pool;
    mot_allocator alloc{};
    std::mutex mu;  // guards everything below that the preparation thread touches
    std::condition_variable cv;
    size_t used = 0;
    int32_t slots_used = 0;
    int creating = 0;
    std::deque<Req> pending;
    std::vector<Live *> ready;                // built, not yet seen by the loop
    std::map<uint64_t, Done> done;
    std::set<uint64_t> in_flight;             // submitted, not yet done
    uint64_t next_ticket = 1;
    // batch rebuilds: requested by the loop, built by the preparation thread
    bool rebuild_wanted = false, rebuild_busy = false, rebuild_done = false;
    std::vector<Live *> rebuild_set;
    mot_batch rebuilt = nullptr;
    int rebuild_rc = 0;
    bool stop = false;
    std::thread prep;
    // loop state (service loop only)
    std::vector<Live *> active;               // resident, not retired
    std::vector<Live *> zombies;              // retired trees still in the current batch
    mot_batch batch = nullptr;
    std::vector<Live *> batch_set;
    double *pinned = nullptr;
    int pinned_cap = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

using namespace mot;

static double half_width_of(const Req &r)
{
    double hw = 0.0;
    const int64_t total = (int64_t)r.weights.size();
    for (int c = 0; c < r.d; ++c) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t i = 0; i < total; ++i) {
            lo = std::min(lo, r.points[i * r.d + c]);
            hi = std::max(hi, r.points[i * r.d + c]);
        }
        hw = std::max(hw, 0.5 * (hi - lo));
    }
    return hw;
}

// Preparation thread: admits waiting requests (FIFO, budget, slots) and builds their
// plans; builds the batched schedules the loop asks for.
static void prep_main(mot_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] {
            if (S->stop || S->rebuild_wanted) return true;
            return !S->pending.empty() && S->slots_used < S->max_slots &&
                   S->used + S->pending.front().footprint <= S->budget;
        });
        if (S->stop) return;
        if (S->rebuild_wanted) {
            std::vector<Live *> set = S->rebuild_set;
            S->rebuild_wanted = false;
            lk.unlock();
            std::vector<mot_plan> plans;
            for (Live *l : set) plans.push_back(l->plan);
            mot_batch B = nullptr;
            // one lane: the resident set changes often, and every rebuild would create and
            // destroy the lanes' streams (measured: capacity 34 -> 31 solves/s with four)
            const int rc = batch_create(&B, plans.data(), (int32_t)plans.size(), &S->alloc, 1);
            lk.lock();
            S->rebuilt = rc < 0 ? nullptr : B;
            S->rebuild_rc = rc;
            S->rebuild_done = true;
            continue;
        }
        Req r = std::move(S->pending.front());
        S->pending.pop_front();
        S->used += r.footprint;
        S->slots_used += 1;
        S->creating += 1;
        const double t_admit = S->now();
        lk.unlock();
        Live *l = new Live();
        l->t_admit = t_admit;
        // trees on the preparation stream (moved to the batch stream when built), circles on
        // a stream of their own
        const bool tree = r.topology == MOT_TREE;
        int rc = mot_plan_create(&l->plan, r.K, r.d, r.n.data(), r.points.data(), r.weights.data(), r.topology,
                                 tree ? r.parent.data() : nullptr, r.eta, r.path, r.precision, nullptr, MOT_HOST,
                                 tree ? S->prep_stream : nullptr, &S->alloc);
        if (rc >= 0 && tree) {
            if (hipStreamSynchronize(S->prep_stream) != hipSuccess) rc = MOT_EDEVICE;
            l->plan->stream = S->stream;  // creation is complete; the plan now lives on the batch stream
        }
        lk.lock();
        S->creating -= 1;
        if (rc < 0) {
            Done dn;
            dn.res.status = rc;
            dn.res.t_submit = r.t_submit;
            dn.res.t_admit = t_admit;
            dn.res.t_done = S->now();
            S->done[r.ticket] = std::move(dn);
            S->in_flight.erase(r.ticket);
            S->used -= r.footprint;
            S->slots_used -= 1;
            delete l;
            continue;
        }
        l->bytes = std::max(r.footprint, l->plan->arena.bytes);
        S->used += l->bytes - r.footprint;
        l->req = std::move(r);
        S->ready.push_back(l);
    }
}

// Release a plan whose work is complete (its stream is idle): memory back to the pool.
static void release_live(mot_server_s *S, Live *l)
{
    mot_plan_destroy(l->plan);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->used -= l->bytes;
    }
    S->cv.notify_all();
    delete l;
}

// Copy a finished problem's result out and free its slot.
static int retire(mot_server_s *S, Live *l, int status, double err, double Sl)
{
    Done dn;
    dn.res.status = status;
    dn.res.sweeps = l->sweeps;
    dn.res.marg_err = err;
    dn.res.S_last = Sl;
    dn.res.t_submit = l->req.t_submit;
    dn.res.t_admit = l->t_admit;
    int64_t total = 0;
    for (int64_t v : l->req.n) total += v;
    dn.phi.resize(total);
    const int rc = mot_get_scalings(l->plan, dn.phi.data(), MOT_HOST);
    dn.res.t_done = S->now();
    l->retired = true;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->done[l->req.ticket] = std::move(dn);
        S->in_flight.erase(l->req.ticket);
        S->slots_used -= 1;
    }
    S->cv.notify_all();
    return rc;
}

extern "C" {

int mot_server_create(mot_server *out, size_t hbm_budget, size_t max_request_bytes, int32_t max_slots, void *stream)
{
    if (!out || hbm_budget == 0 || max_slots < 1) return MOT_EINVAL;
    mot_server_s *S = new mot_server_s();
    S->budget = hbm_budget;
    S->max_request = max_request_bytes ? std::min(max_request_bytes, hbm_budget) : hbm_budget;
    S->max_slots = max_slots;
    S->t0 = std::chrono::steady_clock::now();
    (void)hipGetDevice(&S->device);
    if (stream) {
        S->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
            delete S;
            return MOT_EDEVICE;
        }
        S->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&S->prep_stream, hipStreamNonBlocking) != hipSuccess) {
        if (S->own_stream) (void)hipStreamDestroy(S->stream);
        delete S;
        return MOT_EDEVICE;
    }
    S->alloc.alloc = &Pool::alloc;
    S->alloc.free = &Pool::free;
    S->alloc.ctx = &S->pool;
    S->prep = std::thread(prep_main, S);
    *out = S;
    return MOT_OK;
}

double mot_server_clock(mot_server S) { return S ? S->now() : 0.0; }

int mot_server_submit(mot_server S, const mot_request *q, uint64_t *ticket)
{
    if (!S || !q || !ticket || q->K < 2 || q->d < 1 || q->d > 3 || !q->n || !q->points || !q->weights)
        return MOT_EINVAL;
    if (q->topology == MOT_TREE && !q->parent) return MOT_EINVAL;
    Req r;
    r.K = q->K;
    r.d = q->d;
    r.topology = q->topology;
    r.path = q->path;
    r.precision = q->precision;
    r.max_sweeps = q->max_sweeps > 0 ? q->max_sweeps : 10000;
    r.eta = q->eta;
    r.tol = q->tol_marginal;
    r.n.assign(q->n, q->n + q->K);
    int64_t total = 0;
    for (int64_t v : r.n) {
        if (v < 1) return MOT_EINVAL;
        total += v;
    }
    r.points.assign(q->points, q->points + total * q->d);
    r.weights.assign(q->weights, q->weights + total);
    if (q->topology == MOT_TREE) r.parent.assign(q->parent, q->parent + q->K);
    size_t fp = 0;
    int rc = mot_plan_footprint(r.K, r.d, r.n.data(), r.topology, r.path, r.precision, r.eta, half_width_of(r),
                                nullptr, &fp);
    if (rc < 0) return rc;
    if (fp > S->max_request) return MOT_ENOMEM;  // can never be admitted
    r.footprint = fp;
    r.t_submit = S->now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r.ticket = S->next_ticket++;
        *ticket = r.ticket;
        S->in_flight.insert(r.ticket);
        S->pending.push_back(std::move(r));
    }
    S->cv.notify_all();
    return MOT_OK;
}

int mot_server_run(mot_server S, double seconds, int32_t idle_exit)
{
    if (!S) return MOT_EINVAL;
    const double deadline = S->now() + seconds;
    int completed = 0;
    while (S->now() < deadline) {
        // newly built plans, and a rebuilt batch
        mot_batch nb = nullptr;
        bool swap = false;
        std::vector<Live *> nb_set;
        int rb_rc = 0;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Live *l : S->ready) S->active.push_back(l);
            S->ready.clear();
            if (S->rebuild_done) {
                swap = true;
                nb = S->rebuilt;
                nb_set = S->rebuild_set;
                rb_rc = S->rebuild_rc;
                S->rebuilt = nullptr;
                S->rebuild_done = S->rebuild_busy = false;
            }
        }
        if (swap) {
            if (rb_rc < 0) return rb_rc;
            if (S->batch) MOT_TRY(mot_batch_destroy(S->batch));  // waits for its last launches
            S->batch = nb;
            S->batch_set = nb_set;
            std::set<Live *> kept(nb_set.begin(), nb_set.end());
            std::vector<Live *> still;
            for (Live *z : S->zombies) {
                if (kept.count(z))
                    still.push_back(z);
                else
                    release_live(S, z);
            }
            S->zombies.swap(still);
        }
        // the tree set the batch should hold
        std::vector<Live *> want;
        for (Live *l : S->active)
            if (l->req.topology == MOT_TREE) want.push_back(l);
        std::vector<Live *> have;
        for (Live *l : S->batch_set)
            if (!l->retired) have.push_back(l);
        if (!S->rebuild_busy && want != have) {
            if (want.empty()) {  // nothing left to batch: drop the old schedule now
                if (S->batch) MOT_TRY(mot_batch_destroy(S->batch));
                S->batch = nullptr;
                S->batch_set.clear();
                for (Live *z : S->zombies) release_live(S, z);
                S->zombies.clear();
            } else {
                std::lock_guard<std::mutex> lk(S->mu);
                S->rebuild_set = want;
                S->rebuild_wanted = S->rebuild_busy = true;
                S->cv.notify_all();
            }
        }
        // the problems that advance this step
        std::vector<Live *> step;
        for (Live *l : S->batch_set)
            if (!l->retired) step.push_back(l);
        for (Live *l : S->active)
            if (l->req.topology == MOT_CIRCLE) step.push_back(l);
        if (step.empty()) {
            bool idle;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                idle = S->pending.empty() && S->ready.empty() && S->creating == 0 && S->active.empty() &&
                       !S->rebuild_busy;
            }
            if (idle && idle_exit) break;
            std::this_thread::sleep_for(std::chrono::microseconds(100));
            continue;
        }
        if (S->batch) MOT_TRY(batch_enqueue(S->batch, S->step_sweeps));
        for (Live *l : S->active)
            if (l->req.topology == MOT_CIRCLE) MOT_TRY(circle_run_sweeps(l->plan, S->step_sweeps));
        // every advancing problem's latest error, S and flag, read in one pass
        const int na = (int)step.size();
        if (S->pinned_cap < 3 * na) {
            if (S->pinned) (void)hipHostFree(S->pinned);
            S->pinned_cap = std::max(3 * na, 256);
            MOT_HIP(hipHostMalloc((void **)&S->pinned, S->pinned_cap * sizeof(double), hipHostMallocDefault));
        }
        for (int i = 0; i < na; ++i) {
            mot_plan P = step[i]->plan;
            const int slot = (P->host_sweeps - 1) % P->hist_cap;
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i], P->err_hist + slot, 8, hipMemcpyDeviceToHost, P->stream));
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i + 1], P->S_hist + slot, 8, hipMemcpyDeviceToHost, P->stream));
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i + 2], P->flag, 4, hipMemcpyDeviceToHost, P->stream));
        }
        MOT_HIP(hipStreamSynchronize(S->stream));
        for (Live *l : S->active)
            if (l->req.topology == MOT_CIRCLE) MOT_HIP(hipStreamSynchronize(l->plan->stream));
        std::vector<Live *> still;
        for (int i = 0; i < na; ++i) {
            Live *l = step[i];
            l->sweeps += S->step_sweeps;
            const double err = S->pinned[3 * i], Sl = S->pinned[3 * i + 1];
            int32_t flag = 0;
            memcpy(&flag, &S->pinned[3 * i + 2], 4);
            int status = -100;
            if (flag || !std::isfinite(err)) status = MOT_ENUMERIC;
            else if (err <= l->req.tol) status = MOT_OK;
            else if (l->sweeps >= l->req.max_sweeps) status = MOT_MAXITER;
            if (status == -100) continue;
            MOT_TRY(retire(S, l, status, err, Sl));
            ++completed;
            if (l->req.topology == MOT_CIRCLE)
                release_live(S, l);      // its stream is idle and no schedule holds it
            else
                S->zombies.push_back(l); // released when the batch no longer holds it
        }
        for (Live *l : S->active)
            if (!l->retired) still.push_back(l);
        S->active.swap(still);
    }
    return completed;
}

int mot_server_fetch(mot_server S, uint64_t ticket, mot_result *res, double *phi_out)
{
    if (!S) return MOT_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return S->in_flight.count(ticket) ? 1 : MOT_EINVAL;
    if (res) *res = it->second.res;
    if (phi_out) memcpy(phi_out, it->second.phi.data(), it->second.phi.size() * sizeof(double));
    S->done.erase(it);
    return MOT_OK;
}

int mot_server_destroy(mot_server S)
{
    if (!S) return MOT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->prep.joinable()) S->prep.join();
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    if (S->batch) mot_batch_destroy(S->batch);
    if (S->rebuilt) mot_batch_destroy(S->rebuilt);
    for (Live *l : S->active) {
        mot_plan_destroy(l->plan);
        delete l;
    }
    for (Live *l : S->zombies) {
        mot_plan_destroy(l->plan);
        delete l;
    }
    for (Live *l : S->ready) {
        mot_plan_destroy(l->plan);
        delete l;
    }
    S->pool.release_all();
    if (S->pinned) (void)hipHostFree(S->pinned);
    (void)hipStreamDestroy(S->prep_stream);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return MOT_OK;
}

}  // extern "C"
