"""Thin ctypes binding of libmot.so (argument marshalling only).

Every computation runs in the library's gfx950 kernels; this module only converts
Python/numpy/torch arguments into the C ABI of include/mot.h.  PyTorch, when present,
supplies the HIP stream and (optionally) device memory through its caching allocator.
The library must be built (``paper_2208_03120_amd.build.build()``); importing this
module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmot.so")

OK, MAXITER = 0, 1
EINVAL, EDOMAIN, ENOMEM, EDEVICE, ENUMERIC, EUNSUPPORTED, ELIMIT = -1, -2, -3, -4, -6, -7, -8
TREE, CIRCLE = 0, 1
DIRECT, NFFT, DENSE, TRUNC = 0, 1, 2, 3
PREC_FP64, PREC_MIXED, PREC_BF16, PREC_FP16, PREC_BF16X3 = 0, 1, 2, 3, 4
HOST, DEVICE = 0, 1


class MotError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, _lib.mot_strerror(status).decode(), status))


class FastsumParams(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("p", ctypes.c_int32), ("tau", ctypes.c_double), ("eps_B", ctypes.c_double),
                ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("target_rel_err", ctypes.c_double)]


class TreeOptions(ctypes.Structure):
    _fields_ = [("edge_weight", ctypes.POINTER(ctypes.c_double)),
                ("free_node", ctypes.POINTER(ctypes.c_int32))]


class PlanInfo(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("d", ctypes.c_int32), ("topology", ctypes.c_int32),
                ("path", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("M", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("p", ctypes.c_int32), ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("tau", ctypes.c_double), ("eps_B", ctypes.c_double), ("eta", ctypes.c_double),
                ("scale", ctypes.c_double), ("offset", ctypes.c_double * 3),
                ("box_lo", ctypes.c_int32 * 3), ("box_len", ctypes.c_int32 * 3),
                ("depth", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
                ("products_per_sweep", ctypes.c_int32), ("est_err", ctypes.c_double),
                ("trunc_radius", ctypes.c_double)]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)),
                ("ctx", ctypes.c_void_p)]


class StepTiming(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int32), ("n", ctypes.c_int32),
                ("fft_kind", ctypes.c_int32), ("n_items", ctypes.c_int32), ("calls", ctypes.c_int32),
                ("group", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms_mean", ctypes.c_double)]


STEP_KIND = {0: "node", 1: "direct", 2: "spread", 3: "fold", 4: "fft", 5: "interp", 6: "final",
             7: "fill", 8: "trunc"}


class TuneTable(ctypes.Structure):
    _fields_ = [("measured", ctypes.c_int32), ("device", ctypes.c_int32),
                ("point_ns", (ctypes.c_double * 7) * 3), ("grid_us", (ctypes.c_double * 6) * 3),
                ("box_cells", (ctypes.c_double * 6) * 3), ("seconds", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("d", ctypes.c_int32), ("topology", ctypes.c_int32),
                ("n", ctypes.POINTER(ctypes.c_int64)), ("points", ctypes.POINTER(ctypes.c_double)),
                ("weights", ctypes.POINTER(ctypes.c_double)),
                ("parent", ctypes.POINTER(ctypes.c_int32)), ("eta", ctypes.c_double),
                ("path", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tol_marginal", ctypes.c_double), ("max_sweeps", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("marg_err", ctypes.c_double), ("S_last", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


# names declared in include/mot.h, used by the ABI export test
EXPORTED = ["mot_plan_create", "mot_plan_create_tree", "mot_plan_create_circle", "mot_pair_marginal", "mot_sinkhorn", "mot_get_S_history", "mot_marginals",
            "mot_get_scalings", "mot_set_scalings", "mot_apply_kernel", "mot_plan_get_info",
            "mot_plan_footprint", "mot_plan_destroy", "mot_strerror", "mot_bin_points",
            "mot_plan_profile", "mot_plan_get_order", "mot_bin_points_noalloc",
            "mot_batch_create", "mot_batch_sinkhorn", "mot_batch_launches", "mot_batch_destroy", "mot_server_create",
            "mot_server_submit", "mot_server_run", "mot_server_fetch", "mot_server_clock",
            "mot_server_destroy", "mot_tune_measure", "mot_tune_install", "mot_tune_resolve"]

_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_ip = _P(ctypes.c_int32)
_lp = _P(ctypes.c_int64)
_vp = ctypes.c_void_p


def _load():
    # PyTorch bundles its own HIP runtime.  Import it first so that libmot.so binds to
    # that runtime (same soname) instead of loading a second one, which would leave the
    # process with two HIP runtimes that do not share devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmot.so is not built; run paper_2208_03120_amd.build.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "mot_plan_create": (ctypes.c_int, [_P(_vp), ctypes.c_int32, ctypes.c_int32, _lp, _dp, _dp,
                                           ctypes.c_int32, _ip, ctypes.c_double, ctypes.c_int32,
                                           ctypes.c_int32, _P(FastsumParams), ctypes.c_int32, _vp,
                                           _P(Allocator)]),
        "mot_plan_create_tree": (ctypes.c_int, [_P(_vp), ctypes.c_int32, ctypes.c_int32, _lp, _dp, _dp,
                                                _ip, _P(TreeOptions), ctypes.c_double, ctypes.c_int32,
                                                ctypes.c_int32, _P(FastsumParams), ctypes.c_int32, _vp,
                                                _P(Allocator)]),
        "mot_plan_create_circle": (ctypes.c_int, [_P(_vp), ctypes.c_int32, ctypes.c_int32, _lp, _dp, _dp,
                                                  _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                                  _P(FastsumParams), ctypes.c_int32, _vp, _P(Allocator)]),
        "mot_pair_marginal": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, ctypes.c_int32]),
        "mot_sinkhorn": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, _ip, _dp, _dp]),
        "mot_get_S_history": (ctypes.c_int, [_vp, _dp, ctypes.c_int32]),
        "mot_marginals": (ctypes.c_int, [_vp, _dp, _dp, ctypes.c_int32]),
        "mot_get_scalings": (ctypes.c_int, [_vp, _dp, ctypes.c_int32]),
        "mot_set_scalings": (ctypes.c_int, [_vp, _dp, ctypes.c_int32]),
        "mot_apply_kernel": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _dp, _dp,
                                            ctypes.c_int32]),
        "mot_plan_get_info": (ctypes.c_int, [_vp, _P(PlanInfo)]),
        "mot_plan_footprint": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _lp, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_double, _P(FastsumParams),
                                              _P(ctypes.c_size_t)]),
        "mot_plan_destroy": (ctypes.c_int, [_vp]),
        "mot_plan_profile": (ctypes.c_int, [_vp, ctypes.c_int32, _P(StepTiming), ctypes.c_int32]),
        "mot_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "mot_bin_points": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _dp, _dp, _dp,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _ip, _ip,
                                          _ip, ctypes.c_int32, _vp]),
        "mot_plan_get_order": (ctypes.c_int, [_vp, ctypes.c_int32, _ip, ctypes.c_int32]),
        "mot_bin_points_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _dp, _dp, _dp,
                                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _ip, _ip,
                                                  _ip, _vp]),
        "mot_batch_create": (ctypes.c_int, [_P(_vp), _P(_vp), ctypes.c_int32]),
        "mot_batch_sinkhorn": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "mot_batch_launches": (ctypes.c_int, [_vp]),
        "mot_batch_destroy": (ctypes.c_int, [_vp]),
        "mot_server_create": (ctypes.c_int, [_P(_vp), ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int32, _vp]),
        "mot_server_submit": (ctypes.c_int, [_vp, _P(Request), _P(ctypes.c_uint64)]),
        "mot_server_run": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int32]),
        "mot_server_fetch": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(Result), _dp]),
        "mot_server_clock": (ctypes.c_double, [_vp]),
        "mot_server_destroy": (ctypes.c_int, [_vp]),
        "mot_tune_measure": (ctypes.c_int, [_P(TuneTable)]),
        "mot_tune_install": (ctypes.c_int, [_P(TuneTable)]),
        "mot_tune_resolve": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                            _P(FastsumParams), _P(FastsumParams), _dp]),
    }
    for name, (res, args) in sig.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def strerror(status):
    return _lib.mot_strerror(status).decode()


def _check(status, what):
    if status < 0:
        raise MotError(status, what)
    return status


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _concat(points, weights):
    d = int(points[0].shape[1])
    sizes = np.array([p.shape[0] for p in points], dtype=np.int64)
    pts = _f64(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1, d) for p in points]))
    # None: a free node's weights (not read by the library)
    w = _f64(np.concatenate([np.zeros(len(p)) if x is None else np.asarray(x, dtype=np.float64)
                             for p, x in zip(points, weights)]))
    return d, sizes, pts, w


def _split(cat, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)])
    return [cat[off[k]:off[k + 1]].copy() for k in range(len(sizes))]


def fastsum_params(M=0, n=0, m=0, p=0, tau=0.0, eps_B=0.0, tile=0, chunk=0, target=0.0):
    return FastsumParams(M, n, m, p, tau, eps_B, tile, chunk, target)


def current_stream():
    """The current PyTorch HIP stream handle (or None when no GPU is visible)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


_ALLOC_FN = Allocator._fields_[0][1]
_FREE_FN = Allocator._fields_[1][1]


def _torch_alloc(nbytes, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  torch.cuda.current_stream())
    except Exception:  # out of memory: the library reports MOT_ENOMEM
        return None


def _torch_free(ptr, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:  # interpreter shutdown: the process releases the memory
        pass


_TORCH_ALLOCATOR = None


def torch_allocator():
    """A mot_allocator whose blocks come from PyTorch's caching allocator (so PyTorch
    owns the plan's device memory), or None when no GPU is visible.  The library frees
    a plan's blocks only after synchronising the plan's stream."""
    global _TORCH_ALLOCATOR
    if _TORCH_ALLOCATOR is None:
        try:
            import torch
            if not torch.cuda.is_available():
                return None
        except Exception:
            return None
        _TORCH_ALLOCATOR = Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)
    return _TORCH_ALLOCATOR


def _is_device_tensor(a):
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


class Plan:
    """One multi-marginal OT problem resident on the GPU (mot_plan_create)."""

    def __init__(self, points, weights, topology=TREE, parent=None, eta=0.1, path=NFFT,
                 precision=None, fastsum=None, stream=None, edge_weight=None, free=None,
                 closing_points=None, allocator="torch"):
        """points / weights: K host arrays (n_k x d, n_k), or K device tensors (float64 on
        the plan's GPU), which are passed as MOT_DEVICE pointers.  edge_weight ([K], entry
        k for the edge {parent[k], k}) and free ([K] booleans) pose the generalised
        barycenter problem of Sec. 6.2 (mot_plan_create_tree); closing_points (n_0 x d,
        sigma(x^1)) the generalised Euler flow of Sec. 6.3 on a circle
        (mot_plan_create_circle).  allocator: "torch" (default) takes the plan's device
        memory from PyTorch's caching allocator, None lets the library use hipMalloc."""
        if precision is None:
            precision = PREC_MIXED if path != DENSE else PREC_BF16
        kind = HOST
        if _is_device_tensor(points[0]):
            import torch
            kind = DEVICE
            d = int(points[0].shape[1])
            sizes = np.array([int(p.shape[0]) for p in points], dtype=np.int64)
            self._dev_in = (torch.cat([p.reshape(-1, d) for p in points]).to(torch.float64).contiguous(),
                            torch.cat([x for x in weights]).to(torch.float64).contiguous())
            pts_p = ctypes.cast(self._dev_in[0].data_ptr(), _dp)
            w_p = ctypes.cast(self._dev_in[1].data_ptr(), _dp)
        else:
            d, sizes, pts, w = _concat(points, weights)
            pts_p, w_p = _dptr(pts), _dptr(w)
        self.sizes = sizes
        self.K = len(sizes)
        self.d = d
        self._h = ctypes.c_void_p()
        par = None
        if topology == TREE:
            par = np.ascontiguousarray(parent, dtype=np.int32)
        self._parent = par
        fs = ctypes.byref(fastsum) if fastsum is not None else None
        st = stream if stream is not None else current_stream()
        self._alloc = torch_allocator() if allocator == "torch" else None
        al = ctypes.byref(self._alloc) if self._alloc is not None else None
        if closing_points is not None:
            if topology != CIRCLE:
                raise ValueError("closing points are a circle option")
            if kind == DEVICE:
                self._dev_cl = closing_points.reshape(int(sizes[0]), d).to(closing_points.device,
                                                                             dtype=self._dev_in[0].dtype).contiguous()
                cl_p = ctypes.cast(self._dev_cl.data_ptr(), _dp)
            else:
                cl = _f64(np.asarray(closing_points, dtype=np.float64).reshape(int(sizes[0]), d))
                cl_p = _dptr(cl)
            rc = _lib.mot_plan_create_circle(ctypes.byref(self._h), self.K, d, sizes.ctypes.data_as(_lp),
                                             pts_p, w_p, cl_p, float(eta), path, precision, fs, kind, st, al)
        elif edge_weight is None and free is None:
            rc = _lib.mot_plan_create(ctypes.byref(self._h), self.K, d, sizes.ctypes.data_as(_lp),
                                      pts_p, w_p, topology,
                                      par.ctypes.data_as(_ip) if par is not None else None,
                                      float(eta), path, precision, fs, kind, st, al)
        else:
            if topology != TREE:
                raise ValueError("edge weights and free nodes are tree options")
            ew = None if edge_weight is None else _f64(edge_weight)
            fr = None if free is None else np.ascontiguousarray(np.asarray(free, dtype=bool), dtype=np.int32)
            opt = TreeOptions(_dptr(ew) if ew is not None else None,
                              fr.ctypes.data_as(_ip) if fr is not None else None)
            rc = _lib.mot_plan_create_tree(ctypes.byref(self._h), self.K, d, sizes.ctypes.data_as(_lp),
                                           pts_p, w_p, par.ctypes.data_as(_ip), ctypes.byref(opt),
                                           float(eta), path, precision, fs, kind, st, al)
        self._dev_in = None
        _check(rc, "mot_plan_create")

    def close(self):
        if self._h:
            _lib.mot_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def sinkhorn(self, max_sweeps, delta_S=0.0, tol_marginal=0.0, check_every=1):
        done = ctypes.c_int32(0)
        S = ctypes.c_double(0)
        e = ctypes.c_double(0)
        rc = _lib.mot_sinkhorn(self._h, int(max_sweeps), float(delta_S), float(tol_marginal),
                               int(check_every), ctypes.byref(done), ctypes.byref(S),
                               ctypes.byref(e))
        _check(rc, "mot_sinkhorn") if rc != ENUMERIC else None
        return rc, done.value, S.value, e.value

    def S_history(self, count=1 << 16):
        out = np.zeros(count)
        n = _check(_lib.mot_get_S_history(self._h, _dptr(out), count), "mot_get_S_history")
        return out[:n].copy()

    def scalings(self):
        out = np.zeros(int(self.sizes.sum()))
        _check(_lib.mot_get_scalings(self._h, _dptr(out), HOST), "mot_get_scalings")
        return _split(out, self.sizes)

    def set_scalings(self, phi):
        cat = _f64(np.concatenate(phi))
        _check(_lib.mot_set_scalings(self._h, _dptr(cat), HOST), "mot_set_scalings")

    def marginals(self):
        out = np.zeros(int(self.sizes.sum()))
        l1 = np.zeros(self.K)
        _check(_lib.mot_marginals(self._h, _dptr(out), _dptr(l1), HOST), "mot_marginals")
        return _split(out, self.sizes), l1

    def scalings_device(self, out):
        """Concatenated scaling vectors into a float64 device tensor (MOT_DEVICE)."""
        _check(_lib.mot_get_scalings(self._h, ctypes.cast(out.data_ptr(), _dp), DEVICE), "mot_get_scalings")
        return out

    def set_scalings_device(self, phi):
        _check(_lib.mot_set_scalings(self._h, ctypes.cast(phi.data_ptr(), _dp), DEVICE), "mot_set_scalings")

    def marginals_device(self, out):
        """Concatenated marginals into a float64 device tensor (MOT_DEVICE) and the L1
        errors (host)."""
        l1 = np.zeros(self.K)
        _check(_lib.mot_marginals(self._h, ctypes.cast(out.data_ptr(), _dp), _dptr(l1), DEVICE),
               "mot_marginals")
        return out, l1

    def order(self, k):
        """The binned order of marginal k's points (mot_plan_get_order)."""
        out = np.zeros(int(self.sizes[k]), dtype=np.int32)
        _check(_lib.mot_plan_get_order(self._h, int(k), out.ctypes.data_as(_ip), HOST), "mot_plan_get_order")
        return out

    def pair_marginal(self, k):
        """Pi between marginal a and k (circle: a = 0; tree: a = parent[k]), n_a x n_k."""
        a = 0 if self._parent is None else int(self._parent[k])
        out = np.zeros((int(self.sizes[a]), int(self.sizes[k])))
        _check(_lib.mot_pair_marginal(self._h, int(k), _dptr(out), HOST), "mot_pair_marginal")
        return out

    def apply(self, t, s, v):
        v = _f64(v)
        out = np.zeros(int(self.sizes[t]))
        _check(_lib.mot_apply_kernel(self._h, int(t), int(s), _dptr(v), _dptr(out), HOST),
               "mot_apply_kernel")
        return out

    def profile(self, sweeps):
        """Per-launch mean device time (ms) of one sweep, from HIP events."""
        arr = (StepTiming * 512)()
        n = _check(_lib.mot_plan_profile(self._h, int(sweeps), arr, 512), "mot_plan_profile")
        return [{"kind": STEP_KIND.get(arr[i].kind, "?"), "d": arr[i].d, "n": arr[i].n,
                 "fft_kind": arr[i].fft_kind, "n_items": arr[i].n_items, "group": arr[i].group,
                 "ms": arr[i].ms_mean}
                for i in range(n)]

    def info(self):
        I = PlanInfo()
        _check(_lib.mot_plan_get_info(self._h, ctypes.byref(I)), "mot_plan_get_info")
        return {f: (list(getattr(I, f)) if f in ("offset", "box_lo", "box_len") else getattr(I, f))
                for f, _ in PlanInfo._fields_}


def bin_points(x, s, o, n, T, sub_dim=-1, stream=None):
    """GPU point binning (mot_bin_points): cells, stable tile permutation (sub-keyed by
    the tile-relative cell in dimension sub_dim when sub_dim >= 0), tile offsets."""
    x = _f64(x)
    npts, d = x.shape
    s = _f64(np.broadcast_to(np.asarray(s, dtype=np.float64), (d,)))
    o = _f64(np.broadcast_to(np.asarray(o, dtype=np.float64), (d,)))
    tpd = (n + T - 1) // T
    cell = np.zeros((npts, d), dtype=np.int32)
    perm = np.zeros(npts, dtype=np.int32)
    toff = np.zeros(tpd ** d + 1, dtype=np.int32)
    st = stream if stream is not None else current_stream()
    _check(_lib.mot_bin_points(d, npts, _dptr(x), _dptr(s), _dptr(o), int(n), int(T), int(sub_dim),
                               cell.ctypes.data_as(_ip), perm.ctypes.data_as(_ip),
                               toff.ctypes.data_as(_ip), HOST, st), "mot_bin_points")
    return cell, perm, toff


def footprint(sizes, d, topology, path, precision, eta, half_width=0.25, fastsum=None):
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    out = ctypes.c_size_t(0)
    fs = ctypes.byref(fastsum) if fastsum is not None else None
    _check(_lib.mot_plan_footprint(len(sizes), d, sizes.ctypes.data_as(_lp), topology, path,
                                   precision, float(eta), float(half_width), fs,
                                   ctypes.byref(out)), "mot_plan_footprint")
    return out.value


def tune_measure():
    """Measure the autotuner's cost table on the current GPU (mot_tune_measure)."""
    t = TuneTable()
    _check(_lib.mot_tune_measure(ctypes.byref(t)), "mot_tune_measure")
    return t


def tune_install(table):
    """Make later plans use `table` (a TuneTable); None returns to the analytic model."""
    _check(_lib.mot_tune_install(ctypes.byref(table) if table is not None else None), "mot_tune_install")


def tune_table(point_ns, grid_us, box_cells):
    """A TuneTable from nested lists: point_ns [3][7], grid_us [3][6], box_cells [3][6]."""
    t = TuneTable()
    for d in range(3):
        for i in range(7):
            t.point_ns[d][i] = float(point_ns[d][i])
        for i in range(6):
            t.grid_us[d][i] = float(grid_us[d][i])
            t.box_cells[d][i] = float(box_cells[d][i])
    return t


def tune_resolve(d, eta, n_max, half_width=0.25, fastsum=None):
    """Parameters a plan would get (mot_tune_resolve): dict of M, n, m, p, tau, eps_B,
    tile, chunk, target_rel_err and est_err."""
    out = FastsumParams()
    err = ctypes.c_double(0.0)
    fs = ctypes.byref(fastsum) if fastsum is not None else None
    _check(_lib.mot_tune_resolve(d, float(eta), float(half_width), int(n_max), fs, ctypes.byref(out),
                                 ctypes.byref(err)), "mot_tune_resolve")
    r = {f: getattr(out, f) for f, _ in FastsumParams._fields_}
    r["est_err"] = err.value
    return r


class Batch:
    """Many tree plans advanced together by shared launches (mot_batch_*)."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self._h = ctypes.c_void_p()
        _check(_lib.mot_batch_create(ctypes.byref(self._h), arr, len(self.plans)),
               "mot_batch_create")

    def sinkhorn(self, sweeps, use_graph=True):
        return _check(_lib.mot_batch_sinkhorn(self._h, int(sweeps), int(bool(use_graph))),
                      "mot_batch_sinkhorn")

    def launches(self):
        """Kernel launches of one batched sweep."""
        return _check(_lib.mot_batch_launches(self._h), "mot_batch_launches")

    def close(self):
        if self._h:
            _lib.mot_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solver service (mot_server_*)."""

    def __init__(self, hbm_budget, max_slots=64, stream=None, max_request_bytes=0):
        """stream None: the server works on non-blocking streams of its own."""
        self._h = ctypes.c_void_p()
        _check(_lib.mot_server_create(ctypes.byref(self._h), int(hbm_budget), int(max_request_bytes),
                                      int(max_slots), stream), "mot_server_create")
        self._keep = {}

    def submit(self, inst, path=NFFT, precision=None, tol=1e-6, max_sweeps=2000):
        if precision is None:
            precision = PREC_MIXED if path != DENSE else PREC_BF16X3
        d, sizes, pts, w = _concat(inst.points, inst.weights)
        par = None if inst.parent is None else np.ascontiguousarray(inst.parent, dtype=np.int32)
        req = Request(len(sizes), d, inst.topology, sizes.ctypes.data_as(_lp), _dptr(pts),
                      _dptr(w), par.ctypes.data_as(_ip) if par is not None else None,
                      float(inst.eta), path, precision, float(tol), int(max_sweeps))
        t = ctypes.c_uint64(0)
        rc = _lib.mot_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc < 0:
            return rc, None
        self._keep[t.value] = sizes
        return OK, t.value

    def run(self, seconds, idle_exit=True):
        return _check(_lib.mot_server_run(self._h, float(seconds), int(bool(idle_exit))),
                      "mot_server_run")

    def fetch(self, ticket, want_phi=False):
        res = Result()
        sizes = self._keep.get(ticket)
        phi = np.zeros(int(sizes.sum())) if (want_phi and sizes is not None) else None
        rc = _lib.mot_server_fetch(self._h, ctypes.c_uint64(ticket), ctypes.byref(res),
                                   _dptr(phi) if phi is not None else None)
        if rc == 1:
            return None
        _check(rc, "mot_server_fetch")
        self._keep.pop(ticket, None)
        out = {f: getattr(res, f) for f, _ in Result._fields_}
        if phi is not None:
            out["phi"] = _split(phi, sizes)
        return out

    def clock(self):
        return _lib.mot_server_clock(self._h)

    def close(self):
        if self._h:
            _lib.mot_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
