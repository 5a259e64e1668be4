"""Full-tensor brute force for tiny problems (TEST INFRASTRUCTURE).

Builds the whole cost tensor C of eq. (C) / eq. (cost_sparse), the kernel
tensor of Theorem 3.1 and the marginal projections of eq. (Pk), and runs
Algorithm 1 (generic multi-marginal Sinkhorn) on them.  Exponential in K: only
for K <= 4 and a few tens of points per marginal.
"""
from __future__ import annotations

import numpy as np


def tree_edges(parent):
    return [(int(p), k) for k, p in enumerate(parent) if p >= 0]


def circle_edges(K):
    return [(k, (k + 1) % K) for k in range(K)]


def cost_tensor(points, edges, edge_weights=None, closing=None):
    """C_i = sum_{(a,b) in edges} w_(a,b) |x^a_{i_a} - x^b_{i_b}|^2, eq. (cost_sparse), with
    the edge weights of eq. (cost_function_barycenter_tree) (default 1).  ``closing``:
    the Euler-flow cost of Sec. 6.3, where the edge between the last marginal and marginal
    0 compares x^K with sigma(x^1) = closing[i_1]."""
    K = len(points)
    shape = tuple(p.shape[0] for p in points)
    C = np.zeros(shape)
    for e, (a, b) in enumerate(edges):
        xa, xb = points[a], points[b]
        if closing is not None and {a, b} == {K - 1, 0}:
            xa, xb = (closing, xb) if a == 0 else (xa, closing)
        D = np.sum((xa[:, None, :] - xb[None, :, :]) ** 2, axis=-1)
        if edge_weights is not None:
            D = edge_weights[e] * D
        idx = [None] * K
        idx[a] = slice(None)
        idx[b] = slice(None)
        if a < b:
            C = C + D[tuple(idx)]
        else:
            C = C + D.T[tuple(idx)]
    return C


def kernel_tensor(C, eta):
    """K_i = exp(-C_i / eta) (Theorem 3.1)."""
    return np.exp(-C / eta)


def marginal(T, k):
    """P_k(T): sum over every index except the k-th, eq. (Pk)."""
    axes = tuple(a for a in range(T.ndim) if a != k)
    return T.sum(axis=axes)


def pair_marginal(T, a, b):
    """The sum of T over every index except the a-th and b-th (a < b), an n_a x n_b matrix."""
    axes = tuple(x for x in range(T.ndim) if x not in (a, b))
    return T.sum(axis=axes)


def outer(vectors):
    """Phi = phi^1 (x) ... (x) phi^K."""
    out = vectors[0]
    for v in vectors[1:]:
        out = np.multiply.outer(out, v)
    return out


def algorithm1(Kt, weights, sweeps, phi0=None, constrained=None):
    """Algorithm 1: phi^k <- (mu^k (.) phi^k) / P_k(K (.) Phi~), k = 1..K per sweep.

    One sweep updates every marginal once in order, each update using the
    newest values of the others.  Marginals without a constraint (``constrained[k]``
    false; the barycenter nodes of Sec. 6.2) keep phi^k = 1.  Returns the list of phi
    after each sweep."""
    K = Kt.ndim
    phi = [np.ones(Kt.shape[k]) for k in range(K)] if phi0 is None else [p.copy() for p in phi0]
    hist = []
    for _ in range(sweeps):
        for k in range(K):
            if constrained is not None and not constrained[k]:
                continue
            Pk = marginal(Kt * outer(phi), k)
            phi[k] = (weights[k] * phi[k]) / Pk
        hist.append([p.copy() for p in phi])
    return hist


def sinkhorn_S(Kt, weights, phi, eta, constrained=None):
    """S(phi) = eta sum_k mu^k . log phi^k - eta sum_i K_i Phi_i (Theorem 3.1); the sum
    over k runs over the constrained marginals only."""
    s = sum(float(np.sum(w[w > 0] * np.log(p[w > 0]))) for k, (w, p) in enumerate(zip(weights, phi))
            if constrained is None or constrained[k])
    return eta * (s - float(np.sum(Kt * outer(phi))))


def primal_value(Pi, C, eta):
    """<Pi, C> + eta <Pi, log Pi - 1>, eq. (MOTe)."""
    pos = Pi > 0
    return float(np.sum(Pi * C)) + eta * float(np.sum(Pi[pos] * (np.log(Pi[pos]) - 1.0)))
