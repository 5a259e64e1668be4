// Batched form (a11): many tree plans advanced by shared launches.
//
// The product, node and finalisation jobs of all plans are concatenated into one set of
// device job tables; the merged sweep runs, for every tree depth, one set of launches
// covering the edges at that depth in every plan (grouped by dimension and FFT size),
// and is captured once as a HIP graph.  Each plan keeps its own buffers, statistics
// and exponent slots, so its results are those of running it alone.
#include <algorithm>

#include "host.h"

struct mot_batch_s {
    std::vector<mot_plan_s *> plans;
    hipStream_t stream = nullptr;
    mot::Lanes lanes;  // lanes of plans (created when the batch has two or more plans)
    mot::Arena arena;
    std::vector<mot::Step> sweep, init_up, marg;
    hipGraph_t graph_def = nullptr;
    hipGraphExec_t graph = nullptr;
};

using namespace mot;

static const Lanes *lanes_of(mot_batch_s *B) { return B->lanes.n > 1 ? &B->lanes : nullptr; }

extern "C" {

int mot_batch_destroy(mot_batch B)
{
    if (!B) return MOT_EINVAL;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    B->lanes.destroy();
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    if (B->graph_def) (void)hipGraphDestroy(B->graph_def);
    B->arena.release();
    delete B;
    return MOT_OK;
}

}  // extern "C"

// A batch whose device memory comes from alloc (NULL: hipMalloc slabs).
int mot::batch_create(mot_batch *out, mot_plan *plans, int32_t count, const mot_allocator *alloc, int max_lanes)
{
    if (!out || !plans || count < 1) return MOT_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || plans[i]->topology != MOT_TREE) return MOT_EINVAL;
        if (plans[i]->device != plans[0]->device) return MOT_EINVAL;
    }
    mot_batch_s *B = new mot_batch_s();
    if (alloc && alloc->alloc && alloc->free) {
        B->arena.alloc = *alloc;
        B->arena.custom = true;
    }
    B->plans.assign(plans, plans + count);
    B->stream = plans[0]->stream;
    std::vector<ProdJob> pj;
    std::vector<NodeJob> nj;
    std::vector<FinalJob> fj;
    std::vector<TreeRef> refs;
    for (mot_plan_s *P : B->plans) {
        TreeTables *T = tables_of(P);
        if (!T) {
            delete B;
            return MOT_EINVAL;
        }
        refs.push_back({P, (int)pj.size(), (int)nj.size(), (int)fj.size()});
        pj.insert(pj.end(), P->jobs.begin(), P->jobs.end());
        nj.insert(nj.end(), T->njobs.begin(), T->njobs.end());
        fj.insert(fj.end(), T->fjob.begin(), T->fjob.end());
    }
    ProdJob *pj_dev = nullptr;
    NodeJob *nj_dev = nullptr;
    FinalJob *fj_dev = nullptr;
    int rc = B->arena.get_n(pj.size(), &pj_dev);
    if (rc >= 0) rc = B->arena.get_n(nj.size(), &nj_dev);
    if (rc >= 0) rc = B->arena.get_n(fj.size(), &fj_dev);
    if (rc >= 0 && (hipMemcpy(pj_dev, pj.data(), pj.size() * sizeof(ProdJob), hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(nj_dev, nj.data(), nj.size() * sizeof(NodeJob), hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(fj_dev, fj.data(), fj.size() * sizeof(FinalJob), hipMemcpyHostToDevice) != hipSuccess))
        rc = MOT_EDEVICE;
    int lanes = 1;
    if (rc >= 0)
        rc = tree_steps(refs, pj, pj_dev, nj, nj_dev, fj, fj_dev, B->arena, B->sweep, B->init_up, B->marg, max_lanes,
                        &lanes);
    if (rc >= 0 && lanes > 1) rc = B->lanes.create(lanes);
    if (rc < 0) {
        mot_batch_destroy(B);
        return rc;
    }
    *out = B;
    return MOT_OK;
}

// Enqueue sweeps of the batch on its stream without waiting for them (no graph).
int mot::batch_enqueue(mot_batch B, int sweeps)
{
    for (int r = 0; r < sweeps; ++r) MOT_TRY(run_steps(B->sweep, B->stream, lanes_of(B)));
    for (mot_plan_s *P : B->plans) P->host_sweeps += sweeps;
    return MOT_OK;
}

extern "C" {

int mot_batch_create(mot_batch *out, mot_plan *plans, int32_t count)
{
    return batch_create(out, plans, count, nullptr, kLanes);
}

int mot_batch_launches(mot_batch B)
{
    if (!B) return MOT_EINVAL;
    int n = 0;
    for (const Step &st : B->sweep) n += st.kind != ST_FORK && st.kind != ST_JOIN;
    return n;
}

int mot_batch_sinkhorn(mot_batch B, int32_t sweeps, int32_t use_graph)
{
    if (!B || sweeps < 0) return MOT_EINVAL;
    // work queued on the plans' own streams must finish first
    for (mot_plan_s *P : B->plans)
        if (P->stream != B->stream) MOT_HIP(hipStreamSynchronize(P->stream));
    if (use_graph && !B->graph && sweeps > 0) {
        MOT_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        int rc = run_steps(B->sweep, B->stream, lanes_of(B));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(B->stream, &g);
        if (e == hipErrorStreamCaptureInvalidated) {
            // other work of the process invalidated the capture; none of its launches ran:
            // this call sweeps without the graph, the next one captures again
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            use_graph = 0;
        } else {
            if (rc < 0) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            MOT_HIP(e);
            B->graph_def = g;
            MOT_HIP(hipGraphInstantiate(&B->graph, B->graph_def, nullptr, nullptr, 0));
        }
    }
    for (int r = 0; r < sweeps; ++r) {
        if (use_graph) {
            MOT_HIP(hipGraphLaunch(B->graph, B->stream));
        } else {
            MOT_TRY(run_steps(B->sweep, B->stream, lanes_of(B)));
        }
    }
    for (mot_plan_s *P : B->plans) P->host_sweeps += sweeps;
    MOT_HIP(hipStreamSynchronize(B->stream));
    return MOT_OK;
}

}  // extern "C"
