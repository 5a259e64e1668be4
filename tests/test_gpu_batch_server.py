"""Batched and serving forms: every problem's result equals its result alone (bitwise;
all reductions run in a fixed order and no floating-point atomics are used)."""
import numpy as np
import pytest

import oracle
from paper_2208_03120_amd import workloads as W
from tests.helpers import gauge_fix, max_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mot():
    from paper_2208_03120_amd import mot as m
    return m


def small_batch_instances(count=6, extra=()):
    return [W.batched_instance(i, n_range=(300, 3000)) for i in list(range(count)) + list(extra)]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_sweeps_equal_single_plans(mot, use_graph):
    """Eight instances of d = 1, 2, 3 whose grids include several sizes n <= 128 in 1-D/2-D
    and in 3-D: the batch's launches then mix dimensions (fold) and grid sizes (FFT passes
    and slabs), and every result still equals its plan's result alone, bit for bit."""
    insts = small_batch_instances(6, extra=(7, 12))
    stream = mot.current_stream()
    plans = [mot.Plan(x.points, x.weights, W.TREE, x.parent, x.eta, path=mot.NFFT, stream=stream)
             for x in insts]
    grids = [(p.info()["d"], p.info()["n"]) for p in plans]
    assert len({n for d, n in grids if d < 3 and n <= 128}) >= 2, grids
    assert len({n for d, n in grids if d == 3 and n <= 128}) >= 2, grids
    assert len({d for d, n in grids}) == 3, grids
    batch = mot.Batch(plans)
    batch.sinkhorn(12, use_graph=use_graph)
    for x, p in zip(insts, plans):
        alone = mot.Plan(x.points, x.weights, W.TREE, x.parent, x.eta, path=mot.NFFT)
        alone.sinkhorn(12)
        for a, b in zip(p.scalings(), alone.scalings()):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(p.S_history(), alone.S_history())
        alone.close()
    batch.close()
    for p in plans:
        p.close()


def test_batched_instance_matches_oracle(mot):
    x = small_batch_instances(3)[2]
    plan = mot.Plan(x.points, x.weights, W.TREE, x.parent, x.eta, path=mot.NFFT)
    batch = mot.Batch([plan])
    batch.sinkhorn(15)
    ophi, _, _, _ = oracle.tree_sinkhorn(x.points, x.weights, x.parent, x.eta, 15)
    assert max_rel(gauge_fix(plan.scalings(), x.weights), gauge_fix(ophi, x.weights)) < 1e-5
    batch.close()
    plan.close()


def test_batched_direct_paths_equal_alone(mot):
    """A batch of a plan on the FP64 direct path (a path of 500 points per marginal, whose
    products split the sources over blocks and add the partial sums in a fixed order), one
    on the mixed direct path (d = 3) and one on NFFT: each equals its plan alone bit for bit
    (scaling vectors and S history), and the FP64 plan matches the oracle within 1e-11."""
    r = np.random.Generator(np.random.PCG64(601))
    a = W.path_fp64_direct(seed=1, N=500)
    b = W.make_instance(r, 3, [700, 650, 600], 3, W.TREE, 0.05, parent=[-1, 0, 0])
    c = W.make_instance(r, 4, [900, 800, 850, 700], 2, W.TREE, 0.05, parent=[-1, 0, 1, 1])
    cases = [(a, dict(path=mot.DIRECT, precision=mot.PREC_FP64)), (b, dict(path=mot.DIRECT, precision=mot.PREC_MIXED)),
             (c, dict(path=mot.NFFT))]
    stream = mot.current_stream()
    plans = [mot.Plan(x.points, x.weights, W.TREE, x.parent, x.eta, stream=stream, **kw) for x, kw in cases]
    batch = mot.Batch(plans)
    batch.sinkhorn(8)
    for (x, kw), p in zip(cases, plans):
        alone = mot.Plan(x.points, x.weights, W.TREE, x.parent, x.eta, **kw)
        alone.sinkhorn(8)
        for u, v in zip(p.scalings(), alone.scalings()):
            np.testing.assert_array_equal(u, v)
        np.testing.assert_array_equal(p.S_history(), alone.S_history())
        alone.close()
    ophi, _, _, _ = oracle.tree_sinkhorn(a.points, a.weights, a.parent, a.eta, 8)
    assert max_rel(plans[0].scalings(), ophi) < 1e-11
    batch.close()
    for p in plans:
        p.close()


def test_server_serves_circle_nfft_requests(mot):
    """Circle requests on the row-by-row NFFT path served beside tree requests: each equals
    its stand-alone result bit for bit, and the circles match the oracle's Algorithm 3 for the
    same sweeps (gauge-fixed, 1e-5)."""
    r = np.random.Generator(np.random.PCG64(83))
    reqs = []
    for i in range(4):
        if i % 2 == 0:
            reqs.append(W.make_instance(r, 4, [int(x) for x in r.integers(200, 400, 4)], 2, W.CIRCLE, 0.1))
        else:
            reqs.append(W.make_instance(r, 3, [int(x) for x in r.integers(300, 700, 3)], 2, W.TREE, 0.05,
                                        parent=[-1, 0, 0]))
    srv = mot.Server(hbm_budget=8 << 30, max_slots=8)
    tickets = [srv.submit(q, tol=1e-6, max_sweeps=300, path=mot.NFFT)[1] for q in reqs]
    srv.run(60.0, idle_exit=True)
    res = [srv.fetch(t, want_phi=True) for t in tickets]
    srv.close()
    assert all(x is not None and x["status"] in (mot.OK, mot.MAXITER) for x in res)
    for q, x in zip(reqs, res):
        solo = mot.Server(hbm_budget=8 << 30, max_slots=1)
        _, t = solo.submit(q, tol=1e-6, max_sweeps=300, path=mot.NFFT)
        solo.run(60.0, idle_exit=True)
        y = solo.fetch(t, want_phi=True)
        solo.close()
        assert y["sweeps"] == x["sweeps"]
        for a, b in zip(y["phi"], x["phi"]):
            np.testing.assert_array_equal(a, b)
        if q.topology == W.CIRCLE:
            ophi, _, _, _ = oracle.circle_sinkhorn(q.points, q.weights, q.eta, x["sweeps"])
            assert max_rel(gauge_fix(x["phi"], q.weights), gauge_fix(ophi, q.weights)) < 1e-5


def _requests():
    stream = W.request_stream(seed=7, count=10, n_range=(300, 2500), circle_n_max=400)
    return [inst for _, inst in stream]


def test_server_results_alone_equal_in_mix(mot):
    """40 mixed requests (trees through NFFT, circles through dense split-BF16) served
    together; 32 of them re-run alone give bitwise the same status, sweep count and
    scaling vectors, and 4 tree results match the FP64 oracle run for the same number of
    sweeps (gauge-fixed, 1e-5)."""
    stream = W.request_stream(seed=11, count=40, n_range=(200, 600), circle_n_max=300)
    reqs = [inst for _, inst in stream]

    def path(q):
        return mot.DENSE if q.topology == W.CIRCLE else mot.NFFT

    srv = mot.Server(hbm_budget=8 << 30, max_slots=16)
    tickets = [srv.submit(q, tol=1e-6, max_sweeps=300, path=path(q))[1] for q in reqs]
    while True:
        srv.run(5.0, idle_exit=True)
        res = [srv.fetch(t, want_phi=True) for t in tickets]
        if all(r is not None for r in res):
            break
    srv.close()
    assert all(r["status"] in (mot.OK, mot.MAXITER) for r in res)
    assert sum(r["status"] == mot.OK for r in res) >= 36
    for i in range(32):
        q = reqs[i]
        solo = mot.Server(hbm_budget=8 << 30, max_slots=16)
        _, t = solo.submit(q, tol=1e-6, max_sweeps=300, path=path(q))
        solo.run(60.0, idle_exit=True)
        r = solo.fetch(t, want_phi=True)
        solo.close()
        assert r["status"] == res[i]["status"] and r["sweeps"] == res[i]["sweeps"], i
        for a, b in zip(r["phi"], res[i]["phi"]):
            np.testing.assert_array_equal(a, b)
    trees = [i for i, q in enumerate(reqs) if q.topology == W.TREE][:4]
    for i in trees:
        q = reqs[i]
        ophi, _, _, _ = oracle.tree_sinkhorn(q.points, q.weights, q.parent, q.eta, res[i]["sweeps"])
        assert max_rel(gauge_fix(res[i]["phi"], q.weights), gauge_fix(ophi, q.weights)) < 1e-5, i


def test_server_admission_slots_and_footprint(mot):
    reqs = _requests()[:4]
    srv = mot.Server(hbm_budget=8 << 30, max_slots=1)   # one resident problem at a time
    tk = [srv.submit(q, tol=1e-6, max_sweeps=200,
                     path=(mot.DENSE if q.topology == W.CIRCLE else mot.NFFT))[1] for q in reqs]
    srv.run(60.0, idle_exit=True)
    res = [srv.fetch(t) for t in tk]
    assert all(r is not None for r in res)
    order = sorted(range(len(res)), key=lambda i: res[i]["t_admit"])
    assert order == list(range(len(res)))               # FIFO admission
    for a, b in zip(order, order[1:]):
        assert res[b]["t_admit"] >= res[a]["t_done"]
    srv.close()
    # a problem whose device footprint exceeds the budget is refused at submission
    tiny = mot.Server(hbm_budget=1 << 20, max_slots=2)
    rc, t = tiny.submit(reqs[0])
    assert rc == mot.ENOMEM and t is None
    tiny.close()


def test_server_serves_truncated_path_requests(mot):
    """Small-eta tree requests on the truncated path served in a mix with NFFT requests:
    each equals its stand-alone result bitwise and the oracle's Algorithm 2 for the same
    sweeps (gauge-fixed, 1e-5)."""
    r = np.random.Generator(np.random.PCG64(77))
    reqs, paths = [], []
    for i in range(6):
        small = i % 2 == 0
        eta = 2e-3 if small else 0.05
        inst = W.make_instance(r, 3, [int(x) for x in r.integers(300, 700, 3)], 2, W.TREE, eta,
                               parent=[-1, 0, 0])
        reqs.append(inst)
        paths.append(mot.TRUNC if small else mot.NFFT)
    srv = mot.Server(hbm_budget=8 << 30, max_slots=8)
    tickets = [srv.submit(q, tol=1e-6, max_sweeps=400, path=p)[1] for q, p in zip(reqs, paths)]
    srv.run(60.0, idle_exit=True)
    res = [srv.fetch(t, want_phi=True) for t in tickets]
    srv.close()
    assert all(x is not None and x["status"] in (mot.OK, mot.MAXITER) for x in res)
    for q, p, x in zip(reqs, paths, res):
        solo = mot.Server(hbm_budget=8 << 30, max_slots=1)
        _, t = solo.submit(q, tol=1e-6, max_sweeps=400, path=p)
        solo.run(60.0, idle_exit=True)
        y = solo.fetch(t, want_phi=True)
        solo.close()
        assert y["sweeps"] == x["sweeps"]
        for a, b in zip(y["phi"], x["phi"]):
            np.testing.assert_array_equal(a, b)
        if p == mot.TRUNC:
            ophi, _, _, _ = oracle.tree_sinkhorn(q.points, q.weights, q.parent, q.eta, x["sweeps"])
            assert max_rel(gauge_fix(x["phi"], q.weights), gauge_fix(ophi, q.weights)) < 1e-5


def test_footprint_bounds_plan_memory_across_the_serving_mix(mot):
    """The footprint the server admits by is at least the device memory a plan holds once
    built (plan memory from PyTorch's allocator, counted block by block), over request shapes
    of the serving mix: trees through NFFT, direct and truncated paths, circles dense and
    NFFT, d = 2 and 3, small and large eta."""
    stream = W.request_stream(seed=13, count=24, n_range=(300, 6000), circle_n_max=900)
    for _, q in stream:
        circle = q.topology == W.CIRCLE
        for path in ((mot.DENSE, mot.NFFT) if circle else (mot.NFFT, mot.DIRECT, mot.TRUNC)):
            prec = mot.PREC_BF16X3 if path == mot.DENSE else mot.PREC_MIXED
            hw = max(float(np.max(np.concatenate(q.points)[:, c]) - np.min(np.concatenate(q.points)[:, c])) / 2
                     for c in range(q.d))
            fp = mot.footprint(q.sizes, q.d, q.topology, path, prec, q.eta, half_width=hw)
            try:
                plan = mot.Plan(q.points, q.weights, q.topology, q.parent, q.eta, path=path, precision=prec)
            except mot.MotError as e:  # e.g. a bandwidth the fast summation cannot reach
                assert e.status in (mot.EDOMAIN, mot.EUNSUPPORTED), e
                continue
            held = plan.info()["device_bytes"]
            plan.close()
            assert held <= fp, (q.K, q.sizes[0], q.d, q.eta, circle, path, held, fp)


def test_server_refuses_requests_above_the_per_request_limit(mot):
    reqs = _requests()[:3]
    fps = [mot.footprint(q.sizes, q.d, q.topology, mot.DENSE if q.topology == W.CIRCLE else mot.NFFT,
                         mot.PREC_BF16X3 if q.topology == W.CIRCLE else mot.PREC_MIXED, q.eta) for q in reqs]
    cap = sorted(fps)[1]  # admits the two smallest, refuses the largest
    srv = mot.Server(hbm_budget=64 << 30, max_slots=8, max_request_bytes=cap)
    out = [srv.submit(q, tol=1e-6, max_sweeps=100, path=(mot.DENSE if q.topology == W.CIRCLE else mot.NFFT))
           for q in reqs]
    for (rc, t), fp in zip(out, fps):
        assert (rc == mot.ENOMEM) == (fp > cap)
    srv.run(60.0, idle_exit=True)
    for rc, t in out:
        if rc == mot.OK:
            assert srv.fetch(t) is not None
    srv.close()
