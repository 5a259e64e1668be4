"""Parity at the benchmark's own shapes, the binned order the products use, the paper's
stopping rule, and the boundary's device pointers and caller-supplied memory.

* The star tree of the NFFT benchmark (K = 10, d = 3, eta = 0.05, grid 128^3, m = 6,
  M = 32, tau = 1, eps_B = 1/8, p = 3) at N = 1e4 per marginal over the full 200 sweeps
  against the FP64 oracle's Algorithm 2 (Sec. 4.1), with the fixed parameters the
  benchmark uses: gauge-fixed scaling vectors within 1e-5, marginals within 1e-6 in L1,
  S^(0) within (K - 1) 2e-6 relative and S^(r >= 1) within eta (K + 2.2) 1e-5 absolute
  (the bound the scaling gate implies; derivation at the assertion).
* The binned order of every marginal, as the plan holds it, equals the oracle's binning
  definition bit for bit: the (tile, cell mod T, index) order in 3-D, the plain tile order
  in 1-D and 2-D, the cell order of the truncated path.
* The stopping rule |S^(r) - S^(r-1)| < delta (last step of Algorithm 2) stops the GPU at
  the oracle's sweep.
* A plan made from device pointers (MOT_DEVICE) and writing into device buffers equals the
  host-pointer plan bit for bit, and a plan whose memory comes from PyTorch's caching
  allocator equals one on hipMalloc memory bit for bit.
"""
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


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---- binning ------------------------------------------------------------------------

@pytest.mark.parametrize("d,npts,n,T,sub", [(3, 20000, 128, 5, 1), (3, 3001, 32, 4, 1), (3, 1, 64, 5, 1),
                                            (3, 0, 64, 5, 1), (3, 9000, 64, 7, 0), (3, 9000, 64, 7, 2),
                                            (2, 7777, 128, 16, 1), (1, 5000, 64, 8, 0)])
def test_bin_points_sub_keyed_bit_exact(mot, d, npts, n, T, sub):
    """The sub-keyed order (tile, cell_sub mod T, index) of mot_bin_points against the
    oracle's definition, including points on cell boundaries, one point and none."""
    r = rng(110 + d + npts + T)
    x = r.uniform(-0.3, 0.3, size=(npts, d))
    if npts > 10:
        x[:5] = np.round(x[:5] * 64) / 64
    s = np.full(d, n / 2.0)
    o = n / 2.0 + r.uniform(-0.5, 0.5, size=d)
    cell, perm, toff = mot.bin_points(x, s, o, n, T, sub_dim=sub)
    ocell, _, operm, otoff = oracle.bin_points(x, s, o, n, T, sub_dim=sub)
    np.testing.assert_array_equal(cell, ocell)
    np.testing.assert_array_equal(perm, operm)
    np.testing.assert_array_equal(toff, otoff)


def _check_plan_order(plan, inst, sub_dim):
    info = plan.info()
    d = inst.d
    s = np.full(d, info["scale"])
    o = np.asarray(info["offset"][:d])
    for k in range(inst.K):
        _, _, operm, _ = oracle.bin_points(inst.points[k], s, o, info["n"], info["tile"], sub_dim=sub_dim)
        np.testing.assert_array_equal(plan.order(k), operm)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_plan_binned_order_is_the_oracle_order(mot, d):
    """The order the NFFT products keep each marginal's points in (mot_plan_get_order)
    is the oracle's binning at the plan's grid: sub-keyed by dimension 1 in 3-D."""
    inst = W.make_instance(rng(120 + d), 3, [3000, 2500, 2700], d, W.TREE, 0.05, parent=[-1, 0, 0])
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT)
    _check_plan_order(plan, inst, 1 if d == 3 else -1)
    plan.close()


def test_headline_plan_binned_order(mot):
    """The benchmark's plan (N = 1e5 per marginal, 128^3, m = 6): every marginal's order."""
    inst = W.star_nfft(seed=2, N=100_000)
    fs = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125)
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, fastsum=fs)
    info = plan.info()
    assert (info["n"], info["m"], info["tile"]) == (128, 6, 5)
    _check_plan_order(plan, inst, 1)
    plan.close()


def test_truncated_plan_cell_order(mot):
    inst = W.make_instance(rng(125), 2, [4000, 3000], 3, W.TREE, 1e-3, parent=[-1, 0])
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.TRUNC)
    info = plan.info()
    d = inst.d
    for k in range(2):
        _, _, operm, _ = oracle.bin_points(inst.points[k], np.full(d, info["scale"]),
                                           np.asarray(info["offset"][:d]), info["n"], 1)
        np.testing.assert_array_equal(plan.order(k), operm)
    plan.close()


# ---- the benchmark's star at N = 1e4 over 200 sweeps -----------------------------------

SWEEPS = 200


@pytest.fixture(scope="module")
def star_1e4():
    inst = W.star_nfft(seed=2, N=10_000)
    ophi, oS, done, rc = oracle.tree_sinkhorn(inst.points, inst.weights, inst.parent, inst.eta, SWEEPS)
    assert done == SWEEPS
    oP = oracle.tree_marginals(inst.points, inst.parent, inst.eta, ophi)
    return inst, ophi, oS, oP


@pytest.mark.timeout(1200)
def test_headline_star_200_sweeps_against_oracle(mot, star_1e4):
    inst, ophi, oS, oP = star_1e4
    fs = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125)
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, fastsum=fs)
    rc, done, S_last, err = plan.sinkhorn(SWEEPS)
    assert rc == mot.MAXITER and done == SWEEPS
    phi = plan.scalings()
    rel = max_rel(gauge_fix(phi, inst.weights), gauge_fix(ophi, inst.weights))
    S = plan.S_history()
    s0_rel = abs(S[0] - oS[0]) / abs(oS[0])
    s_abs = float(np.max(np.abs(S[1:] - oS[1:])))
    P, l1 = plan.marginals()
    viol = max(float(np.sum(np.abs(a - b))) for a, b in zip(P, oP))
    print("N=1e4, 200 sweeps: gauge-fixed phi %.3e, S^(0) rel %.3e, S^(r>=1) abs %.3e, marginal L1 vs "
          "oracle %.3e, own marginal L1 %.3e" % (rel, s0_rel, s_abs, viol, max(l1)))
    assert rel < 1e-5
    # S^(r) = eta (sum_k mu^k . log phi^k(r) - (mu^1 / phi^1(r+1)) . phi^1(r)) is gauge invariant.
    # At phi = 1 (r = 0) its last sum is the unnormalised mass of the kernel tensor, the sum
    # over root points of a product of K - 1 kernel products: relative error at most K - 1
    # times a product's (2e-6, the sampled product bound).  From r = 1 on the mass is that
    # of a plan whose last-updated marginals are close to mu (the oracle gives 1.07 after the
    # first sweep of this star and 1 + 2e-4 after the third): scalings within eps move each
    # of the K log sums by at most eps and the mass term by at most 2 eps times the mass.
    assert s0_rel < (inst.K - 1) * 2e-6
    assert s_abs < inst.eta * (inst.K + 2 * 1.1) * 1e-5
    assert viol < 1e-6
    plan.close()


# ---- stopping rule ------------------------------------------------------------------

def test_delta_stop_at_the_oracle_sweep(mot):
    """Path K = 3, N = 500, FP64 direct: mot_sinkhorn's |S^(r) - S^(r-1)| < delta stops at
    the sweep where the oracle's Algorithm 2 stops, for deltas chosen between the S
    differences of consecutive sweeps (from the oracle's own history)."""
    inst = W.path_fp64_direct(seed=1, N=500)
    _, oS, _, _ = oracle.tree_sinkhorn(inst.points, inst.weights, inst.parent, inst.eta, 60)
    diffs = np.abs(np.diff(oS))
    for r_stop in (3, 5, 7):
        lo = diffs[r_stop - 2]
        hi = np.min(diffs[:r_stop - 2])
        assert lo < 0.5 * hi
        delta = float(np.sqrt(lo * hi))
        _, oS2, odone, orc = oracle.tree_sinkhorn(inst.points, inst.weights, inst.parent, inst.eta, 60,
                                                  delta=delta)
        assert orc == oracle.OK and odone == r_stop
        plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.DIRECT,
                        precision=mot.PREC_FP64)
        rc, done, S_last, err = plan.sinkhorn(60, delta_S=delta)
        assert rc == mot.OK and done == odone, (rc, done, odone)
        np.testing.assert_allclose(plan.S_history(), oS2, rtol=1e-12)
        plan.close()


# ---- boundary: device pointers and caller memory ------------------------------------

def test_device_pointers_and_torch_memory_bitwise(mot):
    import torch
    inst = W.make_instance(rng(130), 4, [2100, 1900, 2000, 1800], 3, W.TREE, 0.05, parent=[-1, 0, 0, 1])
    dev = torch.device("cuda")
    base = torch.cuda.memory_allocated()
    hplan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, allocator=None)
    assert torch.cuda.memory_allocated() == base  # library memory, not PyTorch's
    pts = [torch.from_numpy(p).to(dev) for p in inst.points]
    wts = [torch.from_numpy(w).to(dev) for w in inst.weights]
    base = torch.cuda.memory_allocated()
    dplan = mot.Plan(pts, wts, W.TREE, inst.parent, inst.eta, path=mot.NFFT)  # PyTorch's allocator
    held = torch.cuda.memory_allocated() - base
    assert held >= dplan.info()["device_bytes"] > 0
    for p in (hplan, dplan):
        p.sinkhorn(15)
    total = int(sum(inst.sizes))
    phi_d = dplan.scalings_device(torch.empty(total, dtype=torch.float64, device=dev))
    np.testing.assert_array_equal(phi_d.cpu().numpy(), np.concatenate(hplan.scalings()))
    P_d, l1_d = dplan.marginals_device(torch.empty(total, dtype=torch.float64, device=dev))
    P_h, l1_h = hplan.marginals()
    np.testing.assert_array_equal(P_d.cpu().numpy(), np.concatenate(P_h))
    np.testing.assert_array_equal(l1_d, l1_h)
    # device scalings in, then the same sweeps on both
    new = torch.from_numpy(np.concatenate([r.uniform(0.5, 2.0, n) for r, n in
                                           zip([rng(131)] * 4, inst.sizes)])).to(dev)
    dplan.set_scalings_device(new)
    hplan.set_scalings(np.split(new.cpu().numpy(), np.cumsum(inst.sizes)[:-1]))
    for p in (hplan, dplan):
        p.sinkhorn(5)
    np.testing.assert_array_equal(np.concatenate(dplan.scalings()), np.concatenate(hplan.scalings()))
    hplan.close()
    dplan.close()
    del phi_d, P_d, new
    assert torch.cuda.memory_allocated() == base  # every block returned
