"""Python binding of the MI355X Kemeny-constant library (``include/kc.h``).

Argument marshalling only: every step of the estimator runs in the HIP
library ``libkc_mi355x.so`` built from ``csrc/``.  PyTorch provides device
memory (output tensors) and the current HIP stream.  If the library has not
been built, importing works but every call raises ``KcError`` -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkc_mi355x.so")

KC_OK = 0
STATUS = {0: "KC_OK", 1: "KC_ERR_INVALID", 2: "KC_ERR_DISCONNECTED", 3: "KC_ERR_NOMEM",
          4: "KC_ERR_DEVICE", 5: "KC_ERR_OVERFLOW", 6: "KC_ERR_LIMIT", 7: "KC_ERR_UNSUPPORTED"}
KC_TRAV_AUTO, KC_TRAV_WALK, KC_TRAV_SWEEP = 0, 1, 2
KC_OPT_WALKERS, KC_OPT_SLOTS, KC_OPT_TRAVERSAL, KC_OPT_STEP_LIMIT, KC_OPT_MEM_BUDGET = 1, 2, 3, 4, 5
KC_OPT_START_ORDER = 6
KC_OPT_CHAINS = 7
KC_TAU0_BFS, KC_TAU0_DFS, KC_TAU0_GIVEN = 0, 1, 2
KC_OPT_MAINTENANCE = 8
KC_OPT_LEAN_LOOKS = 9
KC_MAINT_BASIC, KC_MAINT_IMPROVED = 0, 1

# every symbol include/kc.h declares
EXPORTS = ("kc_graph_create", "kc_graph_destroy", "kc_graph_get_info", "kc_set_option", "kc_set_tau0",
           "kc_reserve", "kc_trim", "kc_progress",
           "kc_samples_init", "kc_samples_query", "kc_samples_get", "kc_samples_weights", "kc_apply_updates",
           "kc_sample_trees", "kc_estimate", "kc_estimate_static", "kc_evaluate_trees", "kc_combine_results",
           "kc_batch_create", "kc_batch_launch", "kc_batch_results", "kc_batch_f", "kc_batch_destroy",
           "kc_autotune", "kc_status_string",
           "kc_last_error")


class KcError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        self.name = STATUS.get(status, "KC_ERR_%d" % status)
        super().__init__("%s: %s" % (self.name, detail) if detail else self.name)


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("two_m", ctypes.c_int64), ("root", ctypes.c_int32),
                ("depth0", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("traversal", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("tau0", ctypes.c_int32),
                ("sample_bytes", ctypes.c_int64), ("chains", ctypes.c_int32)]


class _Tune(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int32), ("slots", ctypes.c_int32), ("walkers", ctypes.c_int32),
                ("traversal", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("trials", ctypes.c_int32), ("samples_per_s", ctypes.c_double),
                ("start_samples_per_s", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("std_error", ctypes.c_double),
                ("sum_f_lo", ctypes.c_uint64), ("sum_f_hi", ctypes.c_int64),
                ("sum_f2_lo", ctypes.c_uint64), ("sum_f2_hi", ctypes.c_uint64),
                ("count", ctypes.c_int64), ("total_steps", ctypes.c_int64),
                ("sampler_iterations", ctypes.c_int64)]


_lib = None


def library() -> ctypes.CDLL:
    """Load libkc_mi355x.so (raises KcError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KcError(4, "HIP library %s is missing: run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.kc_graph_create.restype = ctypes.c_int
    lib.kc_graph_create.argtypes = [i64, p, ctypes.c_int, p, i32, p, ctypes.POINTER(p)]
    lib.kc_graph_destroy.restype = ctypes.c_int
    lib.kc_graph_destroy.argtypes = [p]
    lib.kc_graph_get_info.restype = ctypes.c_int
    lib.kc_graph_get_info.argtypes = [p, ctypes.POINTER(_Info)]
    lib.kc_set_option.restype = ctypes.c_int
    lib.kc_set_option.argtypes = [p, ctypes.c_int, i64]
    lib.kc_set_tau0.restype = ctypes.c_int
    lib.kc_set_tau0.argtypes = [p, ctypes.c_int, p, p]
    lib.kc_samples_init.restype = ctypes.c_int
    lib.kc_samples_init.argtypes = [p, u64, i32, p]
    lib.kc_samples_query.restype = ctypes.c_int
    lib.kc_samples_query.argtypes = [p, ctypes.POINTER(_Result), p]
    lib.kc_samples_weights.restype = ctypes.c_int
    lib.kc_samples_weights.argtypes = [p, p]
    lib.kc_samples_get.restype = ctypes.c_int
    lib.kc_samples_get.argtypes = [p, p, p, p, p]
    lib.kc_apply_updates.restype = ctypes.c_int
    lib.kc_apply_updates.argtypes = [p, p, p, p, i32, ctypes.POINTER(i32), p]
    lib.kc_progress.restype = ctypes.c_int
    lib.kc_progress.argtypes = [p, ctypes.POINTER(i64)]
    lib.kc_trim.restype = ctypes.c_int
    lib.kc_trim.argtypes = [p, p]
    lib.kc_reserve.restype = ctypes.c_int
    lib.kc_reserve.argtypes = [p, i32, p]
    lib.kc_sample_trees.restype = ctypes.c_int
    lib.kc_sample_trees.argtypes = [p, u64, i64, i32, p, p, p, p]
    lib.kc_estimate.restype = ctypes.c_int
    lib.kc_estimate.argtypes = [p, u64, i64, i32, ctypes.POINTER(_Result), p, p, p]
    lib.kc_combine_results.restype = ctypes.c_int
    lib.kc_combine_results.argtypes = [p, ctypes.POINTER(_Result), i32, ctypes.POINTER(_Result)]
    lib.kc_estimate_static.restype = ctypes.c_int
    lib.kc_estimate_static.argtypes = [p, u64, i64, i32, ctypes.POINTER(_Result), p, p]
    lib.kc_batch_create.restype = ctypes.c_int
    lib.kc_batch_create.argtypes = [p, i32, p, p, p, p, ctypes.POINTER(p)]
    lib.kc_batch_launch.restype = ctypes.c_int
    lib.kc_batch_launch.argtypes = [p, p]
    lib.kc_batch_results.restype = ctypes.c_int
    lib.kc_batch_results.argtypes = [p, ctypes.POINTER(_Result), ctypes.POINTER(i64), p]
    lib.kc_batch_f.restype = ctypes.c_int
    lib.kc_batch_f.argtypes = [p, i32, p, p]
    lib.kc_batch_destroy.restype = ctypes.c_int
    lib.kc_batch_destroy.argtypes = [p]
    lib.kc_autotune.restype = ctypes.c_int
    lib.kc_autotune.argtypes = [p, i32, ctypes.c_char_p, ctypes.POINTER(_Tune), p]
    lib.kc_evaluate_trees.restype = ctypes.c_int
    lib.kc_evaluate_trees.argtypes = [p, p, i32, p, p]
    lib.kc_status_string.restype = ctypes.c_char_p
    lib.kc_status_string.argtypes = [ctypes.c_int]
    lib.kc_last_error.restype = ctypes.c_char_p
    lib.kc_last_error.argtypes = []
    _lib = lib
    return lib


def _check(st: int):
    if st != KC_OK:
        detail = library().kc_last_error().decode(errors="replace")
        raise KcError(st, detail)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Estimate:
    """Theorem 3.3's estimate over `count` samples (exact integer sums)."""

    kappa: float
    std_error: float
    sum_f: int
    sum_f2: int
    count: int
    total_steps: int
    sampler_iterations: int


def _result_of(est: Estimate) -> "_Result":
    m64 = (1 << 64) - 1
    s1 = est.sum_f & ((1 << 128) - 1)
    hi = s1 >> 64
    return _Result(est.kappa, est.std_error, s1 & m64, hi - (1 << 64) if hi >> 63 else hi,
                   est.sum_f2 & m64, est.sum_f2 >> 64, est.count, est.total_steps, est.sampler_iterations)


def _estimate_of(res: "_Result") -> Estimate:
    s1 = (res.sum_f_hi << 64) | res.sum_f_lo
    s2 = (res.sum_f2_hi << 64) | res.sum_f2_lo
    return Estimate(res.kappa, res.std_error, s1, s2, res.count, res.total_steps, res.sampler_iterations)


class Graph:
    """A prepared graph resident on the current HIP device."""

    def __init__(self, offsets, indices, root: int = -1, stream=None):
        lib = library()
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        n = int(off.shape[0] - 1)
        h = ctypes.c_void_p()
        st = lib.kc_graph_create(n, ctypes.c_void_p(off.ctypes.data), 1,
                                 ctypes.c_void_p(idx.ctypes.data), int(root),
                                 _stream(stream) if n >= 2 else None, ctypes.byref(h))
        _check(st)
        self._h = h
        self.info = self._info()

    @classmethod
    def from_graph(cls, g, root: int = -1, stream=None) -> "Graph":
        return cls(g.offsets, g.indices, root, stream)

    def _info(self) -> dict:
        inf = _Info()
        _check(library().kc_graph_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    @property
    def n(self) -> int:
        return self.info["n"]

    @property
    def two_m(self) -> int:
        return self.info["two_m"]

    @property
    def root(self) -> int:
        return self.info["root"]

    def set_option(self, option: int, value: int):
        _check(library().kc_set_option(self._h, option, int(value)))
        self.info = self._info()

    def set_tau0(self, kind: int, parent=None, stream=None):
        """Rebuild tau0 by rule `kind` (KC_TAU0_BFS / KC_TAU0_DFS), or adopt the
        spanning tree `parent` (host int array, parent[root] = -1) for KC_TAU0_GIVEN."""
        arr = None
        if parent is not None:
            arr = np.ascontiguousarray(parent, dtype=np.int32)
            if arr.shape != (self.n,):
                raise ValueError("tau0 parent array must have n entries")
        _check(library().kc_set_tau0(self._h, int(kind), None if arr is None else arr.ctypes.data_as(ctypes.c_void_p),
                                     _stream(stream)))
        self.info = self._info()

    def progress(self) -> int:
        """Samples finished so far by the running (or last) sampling call; safe to
        call from another thread while that call runs."""
        out = ctypes.c_int64(0)
        _check(library().kc_progress(self._h, ctypes.byref(out)))
        return out.value

    # ---- resident sample set and updates
    def samples_init(self, seed: int, count: int, stream=None):
        """Draw samples 0..count-1 and keep them (parents and f) on the device."""
        _check(library().kc_samples_init(self._h, seed, count, _stream(stream)))
        self.res_count = count

    def samples_query(self, stream=None) -> "Estimate":
        res = _Result()
        _check(library().kc_samples_query(self._h, ctypes.byref(res), _stream(stream)))
        return _estimate_of(res)

    def samples_get(self, stream=None):
        """(parents [count, n] int32 CUDA, f [count] int64 CUDA, ids [count] numpy int64)."""
        import torch
        c = self.res_count
        par = torch.empty((c, self.n), dtype=torch.int32, device="cuda")
        f = torch.empty((c,), dtype=torch.int64, device="cuda")
        ids = np.zeros(c, dtype=np.int64)
        _check(library().kc_samples_get(self._h, _dptr(par), _dptr(f), ids.ctypes.data_as(ctypes.c_void_p),
                                        _stream(stream)))
        return par, f, ids

    def samples_weights(self) -> np.ndarray:
        """The resident trees' weights (float64 [count])."""
        w = np.zeros(self.res_count, dtype=np.float64)
        _check(library().kc_samples_weights(self._h, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def apply_updates(self, u, v, is_insert=None, stream=None) -> int:
        """Apply a batch of edge updates; returns how many resident trees were replaced."""
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        ins = None if is_insert is None else np.ascontiguousarray(is_insert, dtype=np.uint8)
        out = ctypes.c_int32(0)
        st = library().kc_apply_updates(self._h, u.ctypes.data_as(ctypes.c_void_p),
                                        v.ctypes.data_as(ctypes.c_void_p),
                                        None if ins is None else ins.ctypes.data_as(ctypes.c_void_p),
                                        int(u.shape[0]), ctypes.byref(out), _stream(stream))
        detail = library().kc_last_error().decode(errors="replace") if st != KC_OK else ""
        self.info = self._info()  # updates before a failing one stay applied
        if st != KC_OK:
            raise KcError(st, detail)
        return out.value

    def reserve(self, count: int, stream=None):
        """Allocate the workspace for estimates of up to `count` samples now."""
        _check(library().kc_reserve(self._h, count, _stream(stream)))

    def trim(self, stream=None):
        """Free the graph's workspace now (allocated again on next use)."""
        _check(library().kc_trim(self._h, _stream(stream)))

    def sample_trees(self, seed: int, first: int, count: int, popcounts: bool = True,
                     steps: bool = True, stream=None):
        """(parents [count, n] int32, draws [count, n] int32 or None, steps [count] int64 or None)
        as CUDA tensors."""
        import torch
        n = self.n
        par = torch.empty((count, n), dtype=torch.int32, device="cuda")
        cnt = torch.empty((count, n), dtype=torch.int32, device="cuda") if popcounts else None
        stp = torch.empty((count,), dtype=torch.int64, device="cuda") if steps else None
        _check(library().kc_sample_trees(self._h, seed, first, count, _dptr(par), _dptr(cnt),
                                         _dptr(stp), _stream(stream)))
        return par, cnt, stp

    def estimate(self, seed: int, first: int, count: int, per_sample: bool = False, stream=None):
        """Estimate (and, if per_sample, the f [count] and draws [count] CUDA tensors)."""
        import torch
        f = stp = None
        if per_sample:
            f = torch.empty((count,), dtype=torch.int64, device="cuda")
            stp = torch.empty((count,), dtype=torch.int64, device="cuda")
        res = _Result()
        _check(library().kc_estimate(self._h, seed, first, count, ctypes.byref(res), _dptr(f),
                                     _dptr(stp), _stream(stream)))
        est = _estimate_of(res)
        return (est, f, stp) if per_sample else est

    def estimate_static(self, seed: int, first: int, count: int, per_sample: bool = False, stream=None):
        """kc_estimate_static: the same estimate with no device allocation (the
        library's static workspace); with per_sample, also the f [count] CUDA tensor."""
        import torch
        f = torch.empty((count,), dtype=torch.int64, device="cuda") if per_sample else None
        res = _Result()
        _check(library().kc_estimate_static(self._h, seed, first, count, ctypes.byref(res), _dptr(f),
                                            _stream(stream)))
        est = _estimate_of(res)
        return (est, f) if per_sample else est

    def combine(self, estimates) -> Estimate:
        """One estimate over all samples of several estimates of this graph
        (disjoint sample ranges), pooled by the library from the exact sums."""
        parts = (_Result * len(estimates))(*[_result_of(e) for e in estimates])
        out = _Result()
        _check(library().kc_combine_results(self._h, parts, len(estimates), ctypes.byref(out)))
        return _estimate_of(out)

    def autotune(self, count: int, cache_path=None, stream=None) -> dict:
        """kc_autotune: choose and apply this graph's launch options for estimates
        of `count` samples (cached in the JSON-lines file cache_path)."""
        out = _Tune()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(library().kc_autotune(self._h, count, path, ctypes.byref(out), _stream(stream)))
        self.info = self._info()
        return {k: getattr(out, k) for k, _ in _Tune._fields_}

    def evaluate_trees(self, parents, stream=None):
        """f for given rooted parent arrays (CUDA int32 tensor [count, n])."""
        import torch
        parents = parents.contiguous()
        count = int(parents.shape[0])
        f = torch.empty((count,), dtype=torch.int64, device="cuda")
        _check(library().kc_evaluate_trees(self._h, _dptr(parents), count, _dptr(f),
                                           _stream(stream)))
        return f

    def close(self):
        if getattr(self, "_h", None):
            library().kc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """kc_batch: one captured persistent launch over the samples of several
    graphs; launch L estimates samples firsts[j] + L*counts[j] .. of graph j."""

    def __init__(self, graphs, seeds, firsts, counts, stream=None):
        lib = library()
        k = len(graphs)
        hs = (ctypes.c_void_p * k)(*[g._h.value for g in graphs])
        sd = np.ascontiguousarray(seeds, dtype=np.uint64)
        fi = np.ascontiguousarray(firsts, dtype=np.int64)
        co = np.ascontiguousarray(counts, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib.kc_batch_create(hs, k, sd.ctypes.data_as(ctypes.c_void_p), fi.ctypes.data_as(ctypes.c_void_p),
                                   co.ctypes.data_as(ctypes.c_void_p), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.k = k
        self.counts = [int(c) for c in co]
        self.graphs = list(graphs)  # the graphs must outlive the batch

    def launch(self, stream=None):
        _check(library().kc_batch_launch(self._h, _stream(stream)))

    def results(self, stream=None):
        """(per-graph Estimates of the last launch, launches done so far)."""
        res = (_Result * self.k)()
        nl = ctypes.c_int64(0)
        _check(library().kc_batch_results(self._h, res, ctypes.byref(nl), _stream(stream)))
        return [_estimate_of(r) for r in res], nl.value

    def f(self, j: int, stream=None):
        import torch
        out = torch.empty((self.counts[j],), dtype=torch.int64, device="cuda")
        _check(library().kc_batch_f(self._h, j, _dptr(out), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            library().kc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
