// Serving form (a12): a continuous-batching solver service on one GPU.
//
// Requests are complete MOT problems.  They wait in FIFO order until their device
// footprint fits the HBM budget and a slot is free; admitted problems become resident
// plans on the server's stream.  The service loop advances every resident problem by a
// fixed number of sweeps per step -- all tree problems together through one batched
// schedule (rebuilt when the resident set changes), circle problems one by one -- then
// reads every problem's first-marginal error and retires those that meet their
// tolerance (or fail, or reach their sweep limit).  Waiting requests enter as soon as
// memory and slots free up, so work arriving while others run overlaps with them.
// A problem's arithmetic does not depend on which others share the launches.
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "host.h"

namespace {

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

struct Active {
    Req req;
    mot_plan plan = nullptr;
    double t_admit = 0;
    int32_t sweeps = 0;
};

struct Done {
    mot_result res{};
    std::vector<double> phi;
};

}  // namespace

struct mot_server_s {
    size_t budget = 0, used = 0;
    int32_t max_slots = 0;
    int32_t step_sweeps = 2;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::mutex mu;
    std::deque<Req> pending;
    std::vector<Active> active;
    std::map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    std::chrono::steady_clock::time_point t0;
    mot_batch batch = nullptr;
    bool batch_dirty = true;
    double *pinned = nullptr;
    int pinned_cap = 0;

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

static int admit(mot_server_s *S)
{
    for (;;) {
        Req r;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->pending.empty() || (int)S->active.size() >= S->max_slots) return MOT_OK;
            if (S->used + S->pending.front().footprint > S->budget) return MOT_OK;
            r = std::move(S->pending.front());
            S->pending.pop_front();
        }
        Active a;
        a.t_admit = S->now();
        int rc = mot_plan_create(&a.plan, r.K, r.d, r.n.data(), r.points.data(), r.weights.data(), r.topology,
                                 r.topology == MOT_TREE ? r.parent.data() : nullptr, r.eta, r.path, r.precision,
                                 nullptr, MOT_HOST, S->stream, nullptr);
        if (rc < 0) {
            Done dn;
            dn.res.status = rc;
            dn.res.t_submit = r.t_submit;
            dn.res.t_admit = a.t_admit;
            dn.res.t_done = S->now();
            std::lock_guard<std::mutex> lk(S->mu);
            S->done[r.ticket] = std::move(dn);
            continue;
        }
        S->used += r.footprint;
        a.req = std::move(r);
        S->active.push_back(std::move(a));
        S->batch_dirty = true;
    }
}

static int retire(mot_server_s *S, size_t idx, int status, double err, double Sl)
{
    Active &a = S->active[idx];
    Done dn;
    dn.res.status = status;
    dn.res.sweeps = a.sweeps;
    dn.res.marg_err = err;
    dn.res.S_last = Sl;
    dn.res.t_submit = a.req.t_submit;
    dn.res.t_admit = a.t_admit;
    int64_t total = 0;
    for (int64_t v : a.req.n) total += v;
    dn.phi.resize(total);
    int rc = mot_get_scalings(a.plan, dn.phi.data(), MOT_HOST);
    dn.res.t_done = S->now();
    mot_plan_destroy(a.plan);
    S->used -= a.req.footprint;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->done[a.req.ticket] = std::move(dn);
    }
    S->active.erase(S->active.begin() + idx);
    S->batch_dirty = true;
    return rc;
}

extern "C" {

int mot_server_create(mot_server *out, size_t hbm_budget, int32_t max_slots, void *stream)
{
    if (!out || hbm_budget == 0 || max_slots < 1) return MOT_EINVAL;
    mot_server_s *S = new mot_server_s();
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    S->t0 = std::chrono::steady_clock::now();
    if (stream) {
        S->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
            delete S;
            return MOT_EDEVICE;
        }
        S->own_stream = true;
    }
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
    if (fp > S->budget) return MOT_ENOMEM;  // can never be admitted
    r.footprint = fp;
    r.t_submit = S->now();
    std::lock_guard<std::mutex> lk(S->mu);
    r.ticket = S->next_ticket++;
    *ticket = r.ticket;
    S->pending.push_back(std::move(r));
    return MOT_OK;
}

int mot_server_run(mot_server S, double seconds, int32_t idle_exit)
{
    if (!S) return MOT_EINVAL;
    const double deadline = S->now() + seconds;
    int completed = 0;
    while (S->now() < deadline) {
        MOT_TRY(admit(S));
        if (S->active.empty()) {
            bool empty;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                empty = S->pending.empty();
            }
            if (idle_exit && empty) break;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        // advance every resident problem
        std::vector<mot_plan> trees;
        for (auto &a : S->active)
            if (a.req.topology == MOT_TREE) trees.push_back(a.plan);
        if (S->batch_dirty) {
            if (S->batch) mot_batch_destroy(S->batch);
            S->batch = nullptr;
            if (!trees.empty()) MOT_TRY(mot_batch_create(&S->batch, trees.data(), (int32_t)trees.size()));
            S->batch_dirty = false;
        }
        if (S->batch) MOT_TRY(mot_batch_sinkhorn(S->batch, S->step_sweeps, 0));
        for (auto &a : S->active)
            if (a.req.topology == MOT_CIRCLE) MOT_TRY(circle_run_sweeps(a.plan, S->step_sweeps));
        // read back every problem's latest error, S and flag in one synchronisation
        const int na = (int)S->active.size();
        if (S->pinned_cap < 3 * na) {
            if (S->pinned) (void)hipHostFree(S->pinned);
            S->pinned_cap = std::max(3 * na, 256);
            MOT_HIP(hipHostMalloc((void **)&S->pinned, S->pinned_cap * sizeof(double), hipHostMallocDefault));
        }
        for (int i = 0; i < na; ++i) {
            Active &a = S->active[i];
            a.sweeps += S->step_sweeps;
            mot_plan P = a.plan;
            const int slot = (P->host_sweeps - 1) % P->hist_cap;
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i], P->err_hist + slot, 8, hipMemcpyDeviceToHost, S->stream));
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i + 1], P->S_hist + slot, 8, hipMemcpyDeviceToHost, S->stream));
            MOT_HIP(hipMemcpyAsync(&S->pinned[3 * i + 2], P->flag, 4, hipMemcpyDeviceToHost, S->stream));
        }
        MOT_HIP(hipStreamSynchronize(S->stream));
        for (int i = na - 1; i >= 0; --i) {
            const Active &a = S->active[i];
            const double err = S->pinned[3 * i], Sl = S->pinned[3 * i + 1];
            int32_t flag = 0;
            memcpy(&flag, &S->pinned[3 * i + 2], 4);
            int status = -100;
            if (flag || !std::isfinite(err)) status = MOT_ENUMERIC;
            else if (err <= a.req.tol) status = MOT_OK;
            else if (a.sweeps >= a.req.max_sweeps) status = MOT_MAXITER;
            if (status != -100) {
                MOT_TRY(retire(S, (size_t)i, status, err, Sl));
                ++completed;
            }
        }
    }
    return completed;
}

int mot_server_fetch(mot_server S, uint64_t ticket, mot_result *res, double *phi_out)
{
    if (!S) return MOT_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) {
        for (auto &r : S->pending)
            if (r.ticket == ticket) return 1;
        for (auto &a : S->active)
            if (a.req.ticket == ticket) return 1;
        return MOT_EINVAL;
    }
    if (res) *res = it->second.res;
    if (phi_out) memcpy(phi_out, it->second.phi.data(), it->second.phi.size() * sizeof(double));
    S->done.erase(it);
    return MOT_OK;
}

int mot_server_destroy(mot_server S)
{
    if (!S) return MOT_EINVAL;
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    if (S->batch) mot_batch_destroy(S->batch);
    for (auto &a : S->active) mot_plan_destroy(a.plan);
    if (S->pinned) (void)hipHostFree(S->pinned);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return MOT_OK;
}

}  // extern "C"
