"""Generalised Euler flows (a circle whose closing edge compares x^K with sigma(x^1)) and
pair marginals, on the GPU against the FP64 oracle (Sec. 6.3).

The paper's setting: N = 400 uniform points on [0, 1], eta = 0.05, 50 sweeps, sigma(x) =
1 - x or the tent map; K = 6 time steps as in its figures.  Scaling vectors are compared
with the oracle's after the same sweeps; pair marginals Pi_{1,k} at the solver's own
scaling vectors with the oracle's at those vectors, relative to their largest entry, and
their row and column sums must equal the first and k-th marginals."""
import numpy as np
import pytest

import oracle
from paper_2208_03120_amd import workloads as W
from tests.helpers import gauge_fix, max_rel, rel_to_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mot():
    from paper_2208_03120_amd import mot as m
    return m


@pytest.fixture(scope="module", params=["reverse", "tent"])
def flow(request):
    inst, closing = W.euler_flow(seed=8, N=400, K=6, eta=0.05, sigma=request.param)
    phi, S, _, rc = oracle.circle_sinkhorn(inst.points, inst.weights, inst.eta, 50, closing=closing)
    return inst, closing, phi, S


# Tolerances follow the products' error model.  The scaling vectors of this flow span
# 1e-14 .. 14, and the NFFT's error is absolute (FP32 rounding times each row product's
# total mass), so small entries of the chained products carry relative errors up to about
# 1e-4 against the largest; the dense products keep FP32 (split BF16) or FP16 / BF16
# relative accuracy entry by entry.
@pytest.mark.parametrize("path,prec,tol", [("nfft", "mixed", 3e-4), ("dense", "bf16x3", 1e-5),
                                           ("dense", "fp16", 3e-4), ("dense", "bf16", 3e-3)])
def test_euler_flow_pair_marginals(mot, flow, path, prec, tol):
    inst, closing, ophi, oS = flow
    p = mot.NFFT if path == "nfft" else mot.DENSE
    precision = {"mixed": mot.PREC_MIXED, "bf16x3": mot.PREC_BF16X3, "fp16": mot.PREC_FP16,
                 "bf16": mot.PREC_BF16}[prec]
    plan = mot.Plan(inst.points, inst.weights, W.CIRCLE, None, inst.eta, path=p, precision=precision,
                    closing_points=closing)
    plan.sinkhorn(50)
    phi = plan.scalings()
    assert max_rel(gauge_fix(phi, inst.weights), gauge_fix(ophi, inst.weights)) < tol
    np.testing.assert_allclose(plan.S_history(), oS, rtol=tol)
    P, _ = plan.marginals()
    for k in range(1, inst.K):
        # the pair marginal of the solver's own phi, against the oracle's at that phi
        pk = plan.pair_marginal(k)
        want = oracle.circle_pair_marginal(inst.points, inst.eta, phi, k, closing=closing)
        assert rel_to_max(pk, want) < tol, k
        np.testing.assert_allclose(pk.sum(axis=1), P[0], rtol=10 * tol, atol=1e-12)
        np.testing.assert_allclose(pk.sum(axis=0), P[k], rtol=10 * tol, atol=1e-12)
    plan.close()


def test_closing_map_changes_the_problem(mot):
    """Without the map the last pair marginal is concentrated near the diagonal; with
    sigma(x) = 1 - x near the anti-diagonal (particles end at 1 - x)."""
    inst, closing = W.euler_flow(seed=9, N=300, K=4, eta=0.02, sigma="reverse")
    x0, xK = inst.points[0][:, 0], inst.points[-1][:, 0]
    for cl, target in [(None, x0), (closing, 1.0 - x0)]:
        plan = mot.Plan(inst.points, inst.weights, W.CIRCLE, None, inst.eta, path=mot.DENSE,
                        precision=mot.PREC_BF16X3, closing_points=cl)
        plan.sinkhorn(100)
        Pi = plan.pair_marginal(inst.K - 1)
        mean_end = (Pi @ xK) / Pi.sum(axis=1)  # expected final position per start
        assert float(np.mean(np.abs(mean_end - target))) < 0.1
        plan.close()


def test_tree_edge_pair_marginals(mot):
    """Pi_{p(k),k} of a weighted tree at the solver's phi against the oracle's, every edge."""
    r = np.random.Generator(np.random.PCG64(501))
    parent = [-1, 0, 0, 1, 1]
    inst = W.make_instance(r, 5, [300, 250, 280, 260, 240], 2, W.TREE, 0.03, parent=parent)
    ew = [0.0, 0.5, 1.0, 2.0, 0.7]
    for path, prec, tol in [(mot.DIRECT, mot.PREC_FP64, 1e-12), (mot.NFFT, mot.PREC_MIXED, 1e-5)]:
        plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=path,
                        precision=prec, edge_weight=ew)
        plan.sinkhorn(15)
        phi = plan.scalings()
        for k in range(1, 5):
            want = oracle.tree_pair_marginal(inst.points, parent, inst.eta, phi, k, edge_weight=ew)
            assert rel_to_max(plan.pair_marginal(k), want) < tol, (path, k)
        plan.close()
