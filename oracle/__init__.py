"""FP64 CPU oracle for tree/circle multi-marginal Sinkhorn (TEST INFRASTRUCTURE).

This package is the reference the GPU library is checked against.  It shares no
code with the GPU path (``paper_2208_03120_amd``) and never imports it.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path must never route through it.

Contents
  * ``mot_oracle.c`` (loaded here through ctypes): the plain Gaussian kernel
    product (Sec. 5, eq. fastsum-sum), Algorithm 2 (tree), Algorithm 3 (circle),
    the marginals of Theorems 4.1 and 4.3, and the point-binning definition.
  * ``fastsum.py``: the Fourier fast-summation chain of Sec. 5 -- the
    regularised kernel (eq. Ker-reg), its periodisation (eq. kappa_tilde), the
    Fourier coefficients (eq. fft) and the trigonometric-sum approximation
    (eq. fastsum1) evaluated directly, without any NFFT.
  * ``brute.py``: full-tensor brute force for tiny K and n (Sec. 3,
    Algorithm 1, Theorem 3.1).
  * ``kernel_apply_truncated`` (here, numpy): the direct sum restricted to the pairs
    within a cutoff radius (the truncation for small eta, end of Sec. 6.1).

Marginals are 0-based here: the paper's root / first marginal is index 0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mot_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAXITER, EINVAL, ENOMEM, ENUMERIC = 0, 1, -1, -3, -6


def build(force: bool = False) -> str:
    """Compile ``mot_oracle.c`` into ``liboracle.so`` with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_kernel_apply.argtypes = [ctypes.c_int, ctypes.c_long, dp, ctypes.c_long, dp,
                                         dp, ctypes.c_double, dp]
        lib.orc_kernel_apply.restype = None
        lib.orc_tree_sinkhorn.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp, ip,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                          dp, dp, ip]
        lib.orc_tree_sinkhorn.restype = ctypes.c_int
        lib.orc_tree_sinkhorn_ex.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp, ip, dp, ip,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                             dp, dp, ip]
        lib.orc_tree_sinkhorn_ex.restype = ctypes.c_int
        lib.orc_tree_marginals_ex.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, ip, dp,
                                              ctypes.c_double, dp, dp]
        lib.orc_tree_marginals_ex.restype = ctypes.c_int
        lib.orc_tree_marginals.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, ip,
                                           ctypes.c_double, dp, dp]
        lib.orc_tree_marginals.restype = ctypes.c_int
        lib.orc_circle_sinkhorn.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            dp, dp, ip]
        lib.orc_circle_sinkhorn.restype = ctypes.c_int
        lib.orc_circle_sinkhorn_ex.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp, dp,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                               dp, dp, ip]
        lib.orc_circle_sinkhorn_ex.restype = ctypes.c_int
        lib.orc_circle_marginals_ex.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp,
                                                ctypes.c_double, dp, dp]
        lib.orc_circle_marginals_ex.restype = ctypes.c_int
        lib.orc_circle_pair_marginal.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, dp,
                                                 ctypes.c_double, dp, ctypes.c_int, dp]
        lib.orc_circle_pair_marginal.restype = ctypes.c_int
        lib.orc_tree_pair_marginal.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp, ip, dp,
                                               ctypes.c_double, dp, ctypes.c_int, dp]
        lib.orc_tree_pair_marginal.restype = ctypes.c_int
        lib.orc_circle_marginals.argtypes = [ctypes.c_int, ctypes.c_int, lp, dp,
                                             ctypes.c_double, dp, dp]
        lib.orc_circle_marginals.restype = ctypes.c_int
        lib.orc_bin_points.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, ctypes.c_int,
                                       ctypes.c_int, ip, ip, ip, ip]
        lib.orc_bin_points.restype = ctypes.c_int
        lib.orc_bin_points_sub.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ip, ip, ip, ip]
        lib.orc_bin_points_sub.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _cat(points, weights=None):
    d = points[0].shape[1]
    off = np.zeros(len(points) + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.shape[0] for p in points])
    pts = np.ascontiguousarray(np.concatenate(points, axis=0), dtype=np.float64)
    mu = None
    if weights is not None:
        mu = np.ascontiguousarray(np.concatenate(weights), dtype=np.float64)
    return d, off, pts, mu


def _split(cat, off):
    return [cat[off[k]:off[k + 1]].copy() for k in range(len(off) - 1)]


def kernel_apply(xt, xs, v, eta):
    """out_i = sum_j v_j exp(-|xt_i - xs_j|^2 / eta) (Sec. 5, eq. fastsum-sum)."""
    lib = _load()
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    d = xt.shape[1]
    assert xs.shape[1] == d and v.shape[0] == xs.shape[0]
    out = np.empty(xt.shape[0], dtype=np.float64)
    lib.orc_kernel_apply(d, xt.shape[0], _d(xt), xs.shape[0], _d(xs), _d(v), float(eta),
                         _d(out))
    return out


def kernel_apply_truncated(xt, xs, v, eta, r_c):
    """out_i = sum over j with |xt_i - xs_j| <= r_c of v_j exp(-|xt_i - xs_j|^2 / eta):
    the direct sum of eq. fastsum-sum with every term beyond the cutoff radius dropped,
    the simple truncation the end of Sec. 6.1 suggests for small eta.  Targets in
    blocks of 32, sources in their given order."""
    xt = np.asarray(xt, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    d = xt.shape[1]
    out = np.empty(xt.shape[0])
    for i0 in range(0, xt.shape[0], 32):
        i1 = min(i0 + 32, xt.shape[0])
        d2 = np.zeros((i1 - i0, xs.shape[0]))
        for c in range(d):
            d2 += (xt[i0:i1, c, None] - xs[None, :, c]) ** 2
        terms = np.where(d2 <= r_c * r_c, np.exp(-d2 / eta), 0.0)
        out[i0:i1] = terms @ v
    return out


def tree_sinkhorn(points, weights, parent, eta, sweeps, delta=0.0, phi0=None, edge_weight=None,
                  free=None):
    """Algorithm 2.  Returns (phi list, S history, sweeps done, status).

    ``edge_weight`` ([K], entry k for the edge {parent[k], k}) and ``free`` ([K] booleans)
    give the generalised barycenter problem of Sec. 6.2: weighted edge costs, and nodes
    without a marginal constraint whose scaling vector is 1 in every sweep."""
    lib = _load()
    K = len(points)
    weights = [np.zeros(len(p)) if w is None else w for p, w in zip(points, weights)]
    d, off, pts, mu = _cat(points, weights)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    phi = np.ones(off[-1]) if phi0 is None else np.concatenate(phi0).astype(np.float64)
    phi = np.ascontiguousarray(phi)
    S = np.zeros(max(sweeps, 1))
    done = ctypes.c_int(0)
    if edge_weight is None and free is None:
        rc = lib.orc_tree_sinkhorn(K, d, _l(off), _d(pts), _d(mu), _i(par), float(eta),
                                   int(sweeps), float(delta), _d(phi), _d(S),
                                   ctypes.byref(done))
    else:
        ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, dtype=np.float64)
        fr = None if free is None else np.ascontiguousarray(np.asarray(free, dtype=bool), dtype=np.int32)
        rc = lib.orc_tree_sinkhorn_ex(K, d, _l(off), _d(pts), _d(mu), _i(par),
                                      _d(ew) if ew is not None else None,
                                      _i(fr) if fr is not None else None, float(eta),
                                      int(sweeps), float(delta), _d(phi), _d(S),
                                      ctypes.byref(done))
    return _split(phi, off), S[:done.value].copy(), done.value, rc


def tree_marginals(points, parent, eta, phi, edge_weight=None):
    """P_k(K (.) Phi) of Theorem 4.1 at fixed phi (edge costs weighted by edge_weight)."""
    lib = _load()
    K = len(points)
    d, off, pts, _ = _cat(points)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    ph = np.ascontiguousarray(np.concatenate(phi), dtype=np.float64)
    P = np.empty(off[-1])
    ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, dtype=np.float64)
    rc = lib.orc_tree_marginals_ex(K, d, _l(off), _d(pts), _i(par),
                                   _d(ew) if ew is not None else None, float(eta), _d(ph), _d(P))
    assert rc == OK, rc
    return _split(P, off)


def _closing(closing, n0, d):
    if closing is None:
        return None
    c = np.ascontiguousarray(np.asarray(closing, dtype=np.float64).reshape(n0, d))
    return c


def circle_sinkhorn(points, weights, eta, sweeps, delta=0.0, phi0=None, closing=None):
    """Algorithm 3.  Returns (phi list, S history, sweeps done, status).

    ``closing`` (n_0 x d): the points sigma(x^1) marginal 0 takes on the closing edge
    {K, 1} (generalised Euler flows, Sec. 6.3); None = x^1 itself."""
    lib = _load()
    K = len(points)
    d, off, pts, mu = _cat(points, weights)
    phi = np.ones(off[-1]) if phi0 is None else np.concatenate(phi0).astype(np.float64)
    phi = np.ascontiguousarray(phi)
    S = np.zeros(max(sweeps, 1))
    done = ctypes.c_int(0)
    cl = _closing(closing, off[1], d)
    rc = lib.orc_circle_sinkhorn_ex(K, d, _l(off), _d(pts), _d(cl) if cl is not None else None, _d(mu),
                                    float(eta), int(sweeps), float(delta), _d(phi), _d(S),
                                    ctypes.byref(done))
    return _split(phi, off), S[:done.value].copy(), done.value, rc


def circle_marginals(points, eta, phi, closing=None):
    """P_k(K (.) Phi) of Theorem 4.3 at fixed phi."""
    lib = _load()
    K = len(points)
    d, off, pts, _ = _cat(points)
    ph = np.ascontiguousarray(np.concatenate(phi), dtype=np.float64)
    P = np.empty(off[-1])
    cl = _closing(closing, off[1], d)
    rc = lib.orc_circle_marginals_ex(K, d, _l(off), _d(pts), _d(cl) if cl is not None else None,
                                     float(eta), _d(ph), _d(P))
    assert rc == OK, rc
    return _split(P, off)


def circle_pair_marginal(points, eta, phi, k, closing=None):
    """Pi_{1,k} of the circle (Sec. 6.3) at fixed phi, n_0 x n_k (k = 1..K-1, 0-based)."""
    lib = _load()
    K = len(points)
    d, off, pts, _ = _cat(points)
    ph = np.ascontiguousarray(np.concatenate(phi), dtype=np.float64)
    out = np.empty((off[1], off[k + 1] - off[k]))
    cl = _closing(closing, off[1], d)
    rc = lib.orc_circle_pair_marginal(K, d, _l(off), _d(pts), _d(cl) if cl is not None else None,
                                      float(eta), _d(ph), int(k), _d(out))
    assert rc == OK, rc
    return out


def tree_pair_marginal(points, parent, eta, phi, k, edge_weight=None):
    """Pi_{p(k),k} of a tree edge at fixed phi, n_{p(k)} x n_k."""
    lib = _load()
    K = len(points)
    d, off, pts, _ = _cat(points)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    ph = np.ascontiguousarray(np.concatenate(phi), dtype=np.float64)
    p = int(par[k])
    out = np.empty((off[p + 1] - off[p], off[k + 1] - off[k]))
    ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, dtype=np.float64)
    rc = lib.orc_tree_pair_marginal(K, d, _l(off), _d(pts), _i(par), _d(ew) if ew is not None else None,
                                    float(eta), _d(ph), int(k), _d(out))
    assert rc == OK, rc
    return out


def sinkhorn_function(weights, phi, total_mass, eta):
    """S(phi) of Theorem 3.1: eta sum_k mu^k . log phi^k - eta sum_i K_i Phi_i.

    ``total_mass`` is sum_i K_i Phi_i, i.e. the sum of any marginal of K (.) Phi.
    Terms with mu = 0 are dropped (0 log 0 := 0)."""
    s = 0.0
    for mu, ph in zip(weights, phi):
        pos = mu > 0
        s += float(np.sum(mu[pos] * np.log(ph[pos])))
    return eta * (s - total_mass)


def bin_points(x, s, o, n, T, sub_dim=-1):
    """Point binning: cells, tile ids, stable tile-sorted permutation and tile offsets.

    ``sub_dim`` >= 0 orders the points of a tile by their tile-relative cell in that
    dimension (cell mod T), ties by index: the sort key (tile, cell mod T, index)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    npts, d = x.shape
    s = np.ascontiguousarray(np.broadcast_to(np.asarray(s, dtype=np.float64), (d,)))
    o = np.ascontiguousarray(np.broadcast_to(np.asarray(o, dtype=np.float64), (d,)))
    tpd = (n + T - 1) // T
    cell = np.empty((npts, d), dtype=np.int32)
    tile = np.empty(npts, dtype=np.int32)
    perm = np.empty(npts, dtype=np.int32)
    tile_off = np.empty(tpd ** d + 1, dtype=np.int32)
    rc = lib.orc_bin_points_sub(d, npts, _d(x), _d(s), _d(o), int(n), int(T), int(sub_dim),
                                _i(cell), _i(tile), _i(perm), _i(tile_off))
    assert rc == OK, rc
    return cell, tile, perm, tile_off
