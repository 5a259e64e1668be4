"""Seeded synthetic inputs shaped like the paper's experiments.

Holds no arithmetic of the method: it only draws points, weights, tree
topologies and request streams.  The GPU library and the FP64 oracle both take
their inputs from here, so both see bit-identical data.

The paper times only synthetic uniform point clouds (Sec. 6.1); these
generators follow that recipe: points i.i.d. uniform in [-1/4, 1/4)^d, weights
i.i.d. uniform(0,1) normalised to one (or Dirichlet(1)), drawn in FP64 from
numpy's PCG64 generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TREE, CIRCLE = 0, 1


@dataclass
class Instance:
    points: list          # K arrays (n_k, d) float64
    weights: list         # K arrays (n_k,) float64, each summing to 1
    topology: int         # TREE or CIRCLE
    parent: np.ndarray    # int32 (K,), parent[0] = -1, parent[k] < k (tree); None for circle
    eta: float
    meta: dict = field(default_factory=dict)

    @property
    def K(self):
        return len(self.points)

    @property
    def d(self):
        return self.points[0].shape[1]

    @property
    def sizes(self):
        return [p.shape[0] for p in self.points]


def uniform_points(rng, n, d, half_width=0.25):
    return rng.uniform(-half_width, half_width, size=(n, d))


def uniform_weights(rng, n):
    w = rng.uniform(0.0, 1.0, size=n)
    return w / w.sum()


def dirichlet_weights(rng, n):
    w = rng.dirichlet(np.ones(n))
    return w / w.sum()


def chain_parent(K):
    return np.array([-1] + list(range(K - 1)), dtype=np.int32)


def star_parent(K):
    return np.array([-1] + [0] * (K - 1), dtype=np.int32)


def prufer_parent(rng, K):
    """Uniform random labelled tree (Pruefer sequence of length K-2), rooted at
    node 0 and relabelled in BFS order so that parent[k] < k."""
    if K == 2:
        return np.array([-1, 0], dtype=np.int32)
    seq = rng.integers(0, K, size=K - 2)
    degree = np.ones(K, dtype=np.int64)
    for s in seq:
        degree[s] += 1
    adj = [[] for _ in range(K)]
    for s in seq:
        leaf = int(np.flatnonzero(degree == 1)[0])
        adj[leaf].append(int(s))
        adj[int(s)].append(leaf)
        degree[leaf] -= 1
        degree[s] -= 1
    u, v = [int(i) for i in np.flatnonzero(degree == 1)]
    adj[u].append(v)
    adj[v].append(u)
    order, parent_old, seen = [0], {0: -1}, {0}
    head = 0
    while head < len(order):
        a = order[head]
        head += 1
        for b in sorted(adj[a]):
            if b not in seen:
                seen.add(b)
                parent_old[b] = a
                order.append(b)
    new_id = {old: new for new, old in enumerate(order)}
    parent = np.full(K, -1, dtype=np.int32)
    for old in order[1:]:
        parent[new_id[old]] = new_id[parent_old[old]]
    return parent


def make_instance(rng, K, sizes, d, topology, eta, parent=None, weights="uniform", meta=None):
    if np.isscalar(sizes):
        sizes = [int(sizes)] * K
    wfun = uniform_weights if weights == "uniform" else dirichlet_weights
    pts = [uniform_points(rng, int(n), d) for n in sizes]
    wts = [wfun(rng, int(n)) for n in sizes]
    if topology == TREE and parent is None:
        parent = chain_parent(K)
    return Instance(pts, wts, topology, None if topology == CIRCLE else np.asarray(parent, np.int32),
                    float(eta), dict(meta or {}))


# --- the benchmark workloads ------------------------------------------------------

def path_fp64_direct(seed=1, N=500):
    """Path tree K=3, N points in d=2, eta=0.1 (FP64 direct summation, 100 sweeps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_instance(rng, 3, N, 2, TREE, 0.1, parent=chain_parent(3),
                         meta={"name": "path_K3_N%d_d2" % N, "sweeps": 100})


def star_nfft(seed=2, N=100_000):
    """Star tree K=10, N points in d=3, eta=0.05, grid 128^3, window cutoff m=6, 200 sweeps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_instance(rng, 10, N, 3, TREE, 0.05, parent=star_parent(10),
                         meta={"name": "star_K10_N%d_d3" % N, "sweeps": 200,
                               "grid": 128, "m": 6})


def star_small_eta(seed=6, N=100_000, eta=1e-3):
    """Star tree K=10, N points in d=3 with a small eta (kernel radius well below the
    cloud's extent), for the truncated direct path."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_instance(rng, 10, N, 3, TREE, eta, parent=star_parent(10),
                         meta={"name": "star_K10_N%d_d3_eta%g" % (N, eta), "sweeps": 200})


def shape_points(rng, n, shape, half_width=0.25):
    """n points drawn uniformly from a planar shape inside [-half_width, half_width)^2:
    'disk', 'ring' (annulus), 'square' (a square's frame) or 'blobs' (two discs)."""
    h = half_width
    out = np.empty((0, 2))
    while out.shape[0] < n:
        p = rng.uniform(-h, h, size=(4 * n, 2))
        r = np.hypot(p[:, 0], p[:, 1])
        if shape == "disk":
            keep = r < 0.8 * h
        elif shape == "ring":
            keep = (r > 0.5 * h) & (r < 0.8 * h)
        elif shape == "square":
            m = np.maximum(np.abs(p[:, 0]), np.abs(p[:, 1]))
            keep = (m > 0.55 * h) & (m < 0.8 * h)
        elif shape == "blobs":
            keep = (np.hypot(p[:, 0] - 0.4 * h, p[:, 1] - 0.4 * h) < 0.35 * h) | \
                   (np.hypot(p[:, 0] + 0.4 * h, p[:, 1] + 0.4 * h) < 0.35 * h)
        else:
            raise ValueError(shape)
        out = np.concatenate([out, p[keep]])
    return out[:n]


H_TREE_PARENT = np.array([-1, 0, 1, 1, 2, 4, 4], dtype=np.int32)
H_TREE_LEAVES = (0, 3, 5, 6)


def h_tree_barycenter(seed=7, N=2500, eta=5e-3, leaf_weight=0.25):
    """Generalised barycenter on the H-shaped tree of Sec. 6.2 (K = 7): leaves 0, 3, 5, 6
    carry given measures with uniform weights 1/N on synthetic planar shapes (disk,
    ring, square frame, two discs: stand-ins for the paper's dithered images); the
    inner nodes 1, 2, 4 are free, supported on the union of the leaves' points.  Edge
    {p, k} has weight leaf_weight when it touches a leaf and 1 otherwise.  Returns
    (Instance, edge weights [K], free flags [K])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    leaves = {k: shape_points(rng, N, s) for k, s in zip(H_TREE_LEAVES, ("disk", "ring", "square", "blobs"))}
    union = np.concatenate([leaves[k] for k in H_TREE_LEAVES])
    K = len(H_TREE_PARENT)
    pts, wts, free = [], [], []
    for k in range(K):
        if k in leaves:
            pts.append(leaves[k])
            wts.append(np.full(N, 1.0 / N))
            free.append(False)
        else:
            pts.append(union.copy())
            wts.append(None)
            free.append(True)
    ew = np.ones(K)
    for k in range(1, K):
        if (k in leaves) != (int(H_TREE_PARENT[k]) in leaves):
            ew[k] = leaf_weight
    inst = Instance(pts, wts, TREE, H_TREE_PARENT.copy(), float(eta),
                    {"name": "h_tree_barycenter_N%d" % N, "sweeps": 150})
    return inst, ew, np.array(free)


def sigma_map(name, x):
    """Connection maps of [0, 1] for generalised Euler flows (Sec. 6.3): 'reverse'
    x -> 1 - x and 'tent' x -> min(2x, 2 - 2x)."""
    if name == "reverse":
        return 1.0 - x
    if name == "tent":
        return np.minimum(2.0 * x, 2.0 - 2.0 * x)
    raise ValueError(name)


def euler_flow(seed=8, N=400, K=6, eta=0.05, sigma="reverse"):
    """Generalised Euler flow of Sec. 6.3: K marginals of N uniform points on [0, 1]
    (d = 1) with uniform weights 1/N, circle cost whose closing edge compares x^K with
    sigma(x^1).  Returns (Instance, closing points sigma(x^1))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [rng.uniform(0.0, 1.0, size=(N, 1)) for _ in range(K)]
    wts = [np.full(N, 1.0 / N) for _ in range(K)]
    inst = Instance(pts, wts, CIRCLE, None, float(eta),
                    {"name": "euler_flow_%s_K%d_N%d" % (sigma, K, N), "sweeps": 50})
    return inst, sigma_map(sigma, pts[0])


def cycle(seed=3, N=4000):
    """Cycle K=5, N points in d=2, eta=0.1, 100 sweeps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_instance(rng, 5, N, 2, CIRCLE, 0.1,
                         meta={"name": "cycle_K5_N%d_d2" % N, "sweeps": 100})


def batched_instance(i, n_range=(1000, 50_000)):
    """Instance i of the batched workload (seed 4+i): K ~ U{3..12}, N log-uniform,
    d ~ U{1,2,3}, uniform random Pruefer tree, eta ~ U(0.02, 0.2), Dirichlet(1) weights."""
    rng = np.random.Generator(np.random.PCG64(4 + i))
    K = int(rng.integers(3, 13))
    N = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
    d = int(rng.integers(1, 4))
    parent = prufer_parent(rng, K)
    eta = float(rng.uniform(0.02, 0.2))
    return make_instance(rng, K, N, d, TREE, eta, parent=parent, weights="dirichlet",
                         meta={"name": "batch_%d" % i})


def request_stream(seed=5, count=2000, rate=100.0, n_range=(500, 200_000), circle_frac=0.2,
                   circle_n_max=None):
    """Poisson request stream for the serving workload.  Yields (arrival_s, Instance)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        is_circle = rng.uniform() < circle_frac
        K = int(rng.integers(3, 17))
        N = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        if is_circle and circle_n_max is not None:
            N = min(N, circle_n_max)
        d = int(rng.integers(2, 4))
        eta = float(np.exp(rng.uniform(np.log(0.01), np.log(0.3))))
        topo = CIRCLE if is_circle else TREE
        parent = None if is_circle else prufer_parent(rng, K)
        inst = make_instance(rng, K, N, d, topo, eta, parent=parent, weights="dirichlet",
                             meta={"name": "req_%d" % r})
        out.append((t, inst))
    return out
