"""GPU NFFT path at its edges and at full size, against the FP64 oracle (through the C ABI).

* window cutoff m over its range (tile edge T = 17 - 2m from 11 down to 1, which moves
  the patch fold between its bounded and general loops): the error against the exact
  trigonometric sums of eq. (fastsum1) falls with m down to FP32 level;
* tiles split into many chunks (several patches per tile);
* the smallest and largest FFT grids (16 and 512 points per dimension);
* tiny and ragged marginals (1, 2, 17 points) through a whole Sinkhorn solve;
* the star tree at N = 100000 per marginal, K = 10, d = 3 with the fixed parameters of the
  benchmark (M = 32, n = 128, m = 6): sampled outputs of one product, and sampled entries
  of the root marginal, whose upward products run batched nine at a time exactly as in
  a sweep.
"""
import numpy as np
import pytest

import oracle
from oracle import fastsum
from paper_2208_03120_amd import workloads as W
from tests.helpers import gauge_fix, max_rel, rel_to_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mot():
    from paper_2208_03120_amd import mot as m
    return m


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _pair(seed, sizes, d):
    return W.make_instance(rng(seed), 2, sizes, d, W.TREE, 0.05, parent=[-1, 0])


def test_window_cutoff_range(mot):
    """d = 2, M = 16, n = 64 (sigma = 2): error vs the exact chain for m = 3..8."""
    inst = _pair(51, [700, 650], 2)
    v = rng(52).uniform(0, 1, 650)
    chain = fastsum.fastsum(inst.points[0], inst.points[1], v, 0.05, 1.0, 0.125, 3, 16)
    errs = {}
    for m in (3, 4, 5, 6, 7, 8):
        fs = mot.fastsum_params(M=16, n=64, m=m, p=3, tau=1.0, eps_B=0.125)
        plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT,
                        fastsum=fs)
        assert plan.info()["tile"] == 17 - 2 * m
        errs[m] = rel_to_max(plan.apply(0, 1, v), chain)
        plan.close()
    # the Kaiser-Bessel error decays geometrically in m; with sigma = 2 it is ~1e-5 at
    # m = 3 and already below the FP32 rounding of the pipeline (a few 1e-7) at m = 4
    assert 1e-6 < errs[3] < 1e-4, errs
    assert errs[4] < errs[3] / 10, errs
    assert max(errs[m] for m in (4, 5, 6, 7, 8)) < 1e-6, errs


def test_window_cutoff_range_3d(mot):
    """d = 3, M = 16, n = 64 (sigma = 4): every tile edge T = 17 - 2m the 3-D spreading and
    interpolation meet (11, 9, 7, 5, 3), with several chunks per tile, against the exact
    trigonometric sums of eq. (fastsum1).  The points of a tile are ordered by their cell in
    dimension 1 and the MFMA steps outside every point's window are skipped, so this also
    covers tiles whose points start at every offset."""
    inst = _pair(55, [1500, 1400], 3)
    v = rng(56).uniform(0, 1, 1400)
    chain = fastsum.fastsum(inst.points[0], inst.points[1], v, 0.05, 1.0, 0.125, 3, 16)
    errs = {}
    for m in (3, 4, 5, 6, 7):
        fs = mot.fastsum_params(M=16, n=64, m=m, p=3, tau=1.0, eps_B=0.125, chunk=40)
        plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT,
                        fastsum=fs)
        assert plan.info()["tile"] == 17 - 2 * m
        errs[m] = rel_to_max(plan.apply(0, 1, v), chain)
        # the reverse direction: sources are the 1500-point marginal
        u = rng(57).uniform(0, 1, 1500)
        back = fastsum.fastsum(inst.points[1], inst.points[0], u, 0.05, 1.0, 0.125, 3, 16)
        errs[-m] = rel_to_max(plan.apply(1, 0, u), back)
        plan.close()
    print("3-D window errors", errs)
    # the window's truncation error is ~1e-5 at m = 3 and below the FP32 rounding of the
    # pipeline (a few 1e-7) from m = 4 on, in both directions
    assert 1e-6 < errs[3] < 1e-4 and 1e-6 < errs[-3] < 1e-4, errs
    assert max(e for m, e in errs.items() if abs(m) >= 4) < 1e-6, errs


@pytest.mark.parametrize("chunk", [8, 24, 100])
def test_tiles_split_into_chunks(mot, chunk):
    """Chunks far smaller than a tile's points: several patches per tile, folded in order.
    Results equal the one-chunk-per-tile plan's to FP32 summation-order level and stay
    within the product accuracy of the direct sum."""
    inst = _pair(61, [3000, 2800], 3)
    v = rng(62).uniform(0, 1, 2800)
    base = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125)
    split = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125, chunk=chunk)
    p1 = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, fastsum=base)
    p2 = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, fastsum=split)
    a, b = p1.apply(0, 1, v), p2.apply(0, 1, v)
    want = oracle.kernel_apply(inst.points[0], inst.points[1], v, inst.eta)
    assert rel_to_max(b, a) < 1e-6
    assert float(np.max(np.abs(b - want) / want)) < 1e-5
    # and the reverse direction, sources = the 3000-point marginal
    u = rng(63).uniform(0, 1, 3000)
    c = p2.apply(1, 0, u)
    want2 = oracle.kernel_apply(inst.points[1], inst.points[0], u, inst.eta)
    assert float(np.max(np.abs(c - want2) / want2)) < 1e-5
    p1.close()
    p2.close()


@pytest.mark.parametrize("d,M,n,npts", [(1, 128, 512, [900, 800]), (2, 8, 32, [500, 400]),
                                         (3, 8, 32, [300, 250]), (1, 4, 16, [100, 90])])
def test_fft_grid_extremes(mot, d, M, n, npts):
    """Smallest and largest FFT sizes against the exact chain with the same M; m = 6
    (error at FP32 level for sigma = 2)."""
    inst = _pair(70 + d + n, npts, d)
    # tau large enough that the cloud fits the grid with its window margin: the grid
    # covers [-tau, tau) with n cells, and the box needs the points' cells plus 2m - 1
    tau = 1.0 if n >= 64 else 2.0
    v = rng(71).uniform(0, 1, npts[1])
    chain = fastsum.fastsum(inst.points[0], inst.points[1], v, 0.05, tau, 0.125, 3, M)
    fs = mot.fastsum_params(M=M, n=n, m=6, p=3, tau=tau, eps_B=0.125)
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT, fastsum=fs)
    assert plan.info()["n"] == n
    assert rel_to_max(plan.apply(0, 1, v), chain) < 3e-6
    plan.close()


def test_tiny_and_ragged_marginals(mot):
    """Path tree with 1, 2 and 17 points (d = 2): a whole NFFT solve against the oracle."""
    r = rng(81)
    inst = W.make_instance(r, 3, [1, 2, 17], 2, W.TREE, 0.1, parent=[-1, 0, 1])
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT)
    rc, done, S_last, err = plan.sinkhorn(40)
    phi = plan.scalings()
    ophi, oS, _, _ = oracle.tree_sinkhorn(inst.points, inst.weights, inst.parent, inst.eta, 40)
    assert max_rel(gauge_fix(phi, inst.weights), gauge_fix(ophi, inst.weights)) < 1e-5
    np.testing.assert_allclose(plan.S_history(), oS, rtol=1e-5)
    plan.close()


@pytest.fixture(scope="module")
def full(mot):
    inst = W.star_nfft(seed=2, N=100_000)
    fs = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125)
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT,
                    fastsum=fs)
    yield inst, plan
    plan.close()


def test_full_size_product_sampled(mot, full):
    """One product at N = 100000 (root -> leaf 3), 512 sampled targets vs the direct sum."""
    inst, plan = full
    v = rng(91).uniform(0.5, 1.5, 100_000)
    got = plan.apply(3, 0, v)
    idx = rng(92).choice(100_000, 512, replace=False)
    want = oracle.kernel_apply(inst.points[3][idx], inst.points[0], v, inst.eta)
    assert float(np.max(np.abs(got[idx] - want) / want)) < 2e-6


def test_full_size_root_marginal_sampled(mot, full):
    """After sweeps at N = 100000, the root marginal P_0 = phi^0 prod_t beta_t (Theorem
    4.1; beta_t = K^{(0,t)} phi^t for the leaves t of the star) at 256 sampled root points.
    Each of the 9 batched products carries the product error above, so P_0's relative
    error is at most 9 times it."""
    inst, plan = full
    plan.set_scalings([np.ones(n) for n in inst.sizes])
    plan.sinkhorn(3)
    phi = plan.scalings()
    P, _ = plan.marginals()
    idx = rng(93).choice(100_000, 256, replace=False)
    want = phi[0][idx].copy()
    for t in range(1, inst.K):
        want *= oracle.kernel_apply(inst.points[0][idx], inst.points[t], phi[t], inst.eta)
    assert float(np.max(np.abs(P[0][idx] - want) / want)) < 9 * 2e-6


@pytest.mark.timeout(900)
def test_full_size_leaf_marginals_sampled(mot, full):
    """The down products at N = 100000, whose spreading takes three of the root's children
    per work item: leaf marginals P_k = phi^k gamma_k with gamma_k = K^{(k,0)} (phi^0
    prod_{t != k} beta_t) (Theorem 4.1; gamma_0 = 1 at the root of the star), at 256
    sampled points of leaves 1, 5 and 9, against the oracle's direct sums at the plan's own
    phi.  The oracle's beta_t = K^{(0,t)} phi^t are full products over all root points.
    Each of the 9 products on the way carries the product error of the sampled product
    test, so the marginal's relative error is at most 9 times it."""
    inst, plan = full
    plan.set_scalings([np.ones(n) for n in inst.sizes])
    plan.sinkhorn(3)
    phi = plan.scalings()
    P, _ = plan.marginals()
    beta = [None] + [oracle.kernel_apply(inst.points[0], inst.points[t], phi[t], inst.eta)
                     for t in range(1, inst.K)]
    for k in (1, 5, 9):
        u = phi[0].copy()
        for t in range(1, inst.K):
            if t != k:
                u *= beta[t]
        idx = rng(97 + k).choice(100_000, 256, replace=False)
        want = phi[k][idx] * oracle.kernel_apply(inst.points[k][idx], inst.points[0], u, inst.eta)
        err = float(np.max(np.abs(P[k][idx] - want) / want))
        print("leaf %d marginal, sampled: max rel err %.3e" % (k, err))
        assert err < 9 * 2e-6


def test_error_vs_M_tracks_the_estimate(mot):
    """One product's error against the direct sum falls as M grows until FP32 rounding
    (a few 1e-7), and stays within a factor of the autotuner's estimate (d = 2)."""
    inst = W.make_instance(rng(95), 2, [1200, 1000], 2, W.TREE, 0.05, parent=[-1, 0])
    v = rng(96).uniform(0.5, 1.5, 1000)
    want = oracle.kernel_apply(inst.points[0], inst.points[1], v, inst.eta)
    errs, ests = [], []
    for M in (6, 8, 12, 16, 24):
        n = 16
        while n < 4 * M:
            n *= 2
        plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT,
                        fastsum=mot.fastsum_params(M=M, n=n, p=3))
        ests.append(plan.info()["est_err"])
        errs.append(float(np.max(np.abs(plan.apply(0, 1, v) - want) / want)))
        plan.close()
    print("M errors", errs, "estimates", ests)
    for a, b in zip(errs, errs[1:]):
        assert b < a or b < 2e-6, errs
    for e, est in zip(errs, ests):
        assert e <= 10 * est + 2e-6, (errs, ests)
    assert errs[-1] < 2e-6, errs
