"""Python binding of the C ABI in include/quake.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors on the current HIP device; the current torch
stream is passed as the stream argument.  Nothing is computed in Python:
a missing library raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libquake_mi355x.so")

OK, E_INVALID, E_NOMEM, E_NOTFOUND, E_DUPLICATE, E_DEVICE, E_STATE, E_IO = 0, -1, -2, -3, -4, -5, -6, -7
L2, IP = 0, 1
F32, BF16, F16 = 0, 1, 2
PQ8 = 3   # scan_dtype of a search over product codes
SCAN_PLAIN, SCAN_BATCHED = 0, 1

_METRIC = {"l2": L2, "ip": IP}
_DTYPE = {"f32": F32, "bf16": BF16, "f16": F16}
_SCAN_DTYPE = dict(_DTYPE, pq8=PQ8)
_MODE = {"plain": SCAN_PLAIN, "batched": SCAN_BATCHED}

EXPORTED = ("quake_build", "quake_search", "quake_search_noalloc", "quake_insert", "quake_delete", "quake_stats", "quake_export",
            "quake_export_top", "quake_candidates", "quake_cap_table", "quake_profile", "quake_set_tuning",
            "quake_free", "quake_last_error", "quake_autotune", "quake_server_create", "quake_server_search", "quake_server_insert",
            "quake_server_delete", "quake_server_wait", "quake_server_stats", "quake_server_destroy",
            "quake_access_stats", "quake_maintain", "quake_profile_latency", "quake_describe", "quake_save",
            "quake_load", "quake_insert_attrs", "quake_add_level", "quake_remove_level", "quake_adjust_levels",
            "quake_export_level", "quake_level_sizes", "quake_export_pq")
PROF_KINDS = ("centroids", "select", "plan", "scan", "commit", "rerank", "scan_sets", "upper")


class QuakeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"quake error {code}: {msg}")
        self.code = code


class BuildParams(ctypes.Structure):
    _fields_ = [("metric", ctypes.c_int32), ("storage_dtype", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("kmeans_iters", ctypes.c_int32), ("nlist", ctypes.c_int64), ("nlist_top", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("centroids", ctypes.c_void_p), ("assign", ctypes.c_void_p),
                ("hbm_budget_bytes", ctypes.c_size_t), ("capacity_slack", ctypes.c_double),
                ("drop_f32_tiles", ctypes.c_int32), ("attrs", ctypes.c_void_p), ("pq_m", ctypes.c_int32),
                ("pq_codebook", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


def _torch_alloc(nbytes, ctx):
    # ctx carries the device index; memory comes from torch's caching
    # allocator on that device's current stream
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(ctx or 0))
    except Exception:
        return None


def _torch_free(ptr, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# the callbacks live as long as the module (an index may call them until it is freed)
_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)


def torch_allocator(device: int) -> Allocator:
    """quake_allocator backed by torch's caching allocator on `device`."""
    return Allocator(_TORCH_ALLOC, _TORCH_FREE, ctypes.c_void_p(device))


class SearchParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("nprobe", ctypes.c_int32), ("recall_target", ctypes.c_double),
                ("f_M", ctypes.c_double), ("tau_rho", ctypes.c_double), ("upper_recall_target", ctypes.c_double),
                ("upper_f_M", ctypes.c_double), ("scan_mode", ctypes.c_int32), ("scan_dtype", ctypes.c_int32),
                ("rerank_factor", ctypes.c_int32), ("window", ctypes.c_int32), ("estimator", ctypes.c_int32),
                ("filter", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_tiles", ctypes.c_int32), ("first_window", ctypes.c_int32), ("max_window", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("max_items", ctypes.c_int64), ("rounds_per_sync", ctypes.c_int32),
                ("no_graph", ctypes.c_int32), ("window_scale", ctypes.c_int32)]


class ServerParams(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("overlap_updates", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_size_t), ("search", SearchParams)]


class ServerReport(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("slots", ctypes.c_int64), ("max_in_flight", ctypes.c_int64), ("epochs", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("overlapped_updates", ctypes.c_int64),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("qps", ctypes.c_double)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("milliseconds", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


class Decision(ctypes.Structure):
    _fields_ = [("partition", ctypes.c_int32), ("action", ctypes.c_int32), ("committed", ctypes.c_int32),
                ("new_partition", ctypes.c_int32), ("estimate", ctypes.c_double), ("verified", ctypes.c_double)]


class MaintainParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("alpha", ctypes.c_double), ("refine_radius", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("split_iters", ctypes.c_int32), ("min_split_size", ctypes.c_int32),
                ("merge_below", ctypes.c_int64), ("lambda_points", ctypes.c_int32), ("max_decisions", ctypes.c_int32),
                ("lambda_size", ctypes.c_void_p), ("lambda_cost", ctypes.c_void_p), ("hits", ctypes.c_void_p),
                ("window", ctypes.c_int64), ("decisions", ctypes.c_void_p)]


class MaintainReport(ctypes.Structure):
    _fields_ = [("decisions", ctypes.c_int32), ("splits", ctypes.c_int32), ("deletes", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("nlist_before", ctypes.c_int64), ("nlist_after", ctypes.c_int64),
                ("vectors_moved", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2506_03437_amd.build_lib`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.quake_build.argtypes = [vp, vp, i64, i32, ctypes.POINTER(BuildParams), ctypes.POINTER(Allocator), vp,
                                ctypes.POINTER(vp)]
    lib.quake_search.argtypes = [vp, vp, i64, ctypes.POINTER(SearchParams), vp, vp, vp, vp, vp]
    lib.quake_search_noalloc.argtypes = [vp, vp, i64, ctypes.POINTER(SearchParams), vp, vp, vp, vp, vp]
    lib.quake_insert.argtypes = [vp, vp, vp, i64, vp]
    lib.quake_insert_attrs.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.quake_delete.argtypes = [vp, vp, i64, vp]
    lib.quake_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)]
    lib.quake_export.argtypes = [vp, vp, vp, vp, vp]
    lib.quake_export_pq.argtypes = [vp, ctypes.POINTER(i32), vp, vp, vp]
    lib.quake_export_top.argtypes = [vp, vp, vp, vp]
    lib.quake_describe.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
    lib.quake_save.argtypes = [vp, ctypes.c_char_p, vp]
    lib.quake_add_level.argtypes = [vp, i64, i32, ctypes.c_uint64, vp]
    lib.quake_export_level.argtypes = [vp, i32, vp, vp, vp]
    lib.quake_level_sizes.argtypes = [vp, ctypes.POINTER(i64)]
    lib.quake_remove_level.argtypes = [vp, vp]
    lib.quake_adjust_levels.argtypes = [vp, i64, i64, i64, i32, ctypes.c_uint64, vp, ctypes.POINTER(i32)]
    lib.quake_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(Allocator), ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.quake_access_stats.argtypes = [vp, i32, vp, ctypes.POINTER(i64), i32, vp]
    lib.quake_maintain.argtypes = [vp, ctypes.POINTER(MaintainParams), ctypes.POINTER(MaintainReport), vp]
    lib.quake_profile_latency.argtypes = [vp, vp, i32, i32, ctypes.POINTER(SearchParams), i32, vp, vp]
    lib.quake_candidates.argtypes = [vp, vp, i64, ctypes.POINTER(SearchParams), vp, vp, ctypes.POINTER(i32), vp]
    lib.quake_cap_table.argtypes = [i32, ctypes.POINTER(f64)]
    lib.quake_profile.argtypes = [vp, i32, i32, vp]
    lib.quake_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.quake_autotune.argtypes = [vp, vp, i64, ctypes.POINTER(SearchParams), i32, ctypes.POINTER(Tuning),
                                   ctypes.POINTER(f64), vp]
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.quake_server_create.argtypes = [vp, ctypes.POINTER(ServerParams), ctypes.POINTER(vp)]
    lib.quake_server_search.argtypes = [vp, vp, i64, u64p]
    lib.quake_server_insert.argtypes = [vp, vp, vp, i64, u64p]
    lib.quake_server_delete.argtypes = [vp, vp, i64, u64p]
    lib.quake_server_wait.argtypes = [vp, ctypes.c_uint64, f64, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.quake_server_stats.argtypes = [vp, ctypes.POINTER(ServerReport), i32]
    lib.quake_server_destroy.argtypes = [vp]
    lib.quake_server_destroy.restype = None
    lib.quake_free.argtypes = [vp]
    lib.quake_free.restype = None
    lib.quake_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("quake_free", "quake_last_error", "quake_server_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        msg = load_library().quake_last_error()
        raise QuakeError(rc, msg.decode() if msg else "")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(t, dtype):
    import torch
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), f"need a contiguous CUDA {dtype} tensor"
    return t


def _labels(t):
    """Label bits (32 per row or query): a contiguous CUDA int32 or uint32
    tensor, passed as its bit pattern."""
    import torch
    assert t.is_cuda and t.dtype in (torch.int32, torch.uint32) and t.is_contiguous(), \
        "need a contiguous CUDA int32 / uint32 tensor of label bits"
    return t


def quake_cap_table(d: int) -> np.ndarray:
    out = np.zeros(1024, dtype=np.float64)
    _check(load_library().quake_cap_table(d, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def quake_build(x, ids=None, *, metric="l2", nlist=256, storage="f32", n_levels=1, nlist_top=0, kmeans_iters=10,
                seed=0, centroids=None, assign=None, hbm_budget_bytes=0, capacity_slack=0.0,
                allocator="torch", f32_tiles=True, attrs=None, pq_m=0, pq_codebook=None) -> int:
    """allocator: "torch" (the caching allocator of x's device, the default) or "hip" (hipMalloc).
    f32_tiles=False (with a 16-bit storage copy or product codes): no FP32 tile copy.
    pq_m > 0: also keep product codes of pq_m subspaces (searched with scan_dtype="pq8"), with the
    codebook pq_codebook (device f32 [pq_m, 256, d / pq_m]) or one trained on x."""
    import torch
    _dev(x, torch.float32)
    if ids is not None:
        _dev(ids, torch.int64)
    if centroids is not None:
        _dev(centroids, torch.float32)
    if assign is not None:
        _dev(assign, torch.int32)
    if attrs is not None:
        _labels(attrs)
    if pq_codebook is not None:
        _dev(pq_codebook, torch.float32)
    p = BuildParams(_METRIC[metric], _DTYPE[storage], n_levels, kmeans_iters, nlist, nlist_top, seed,
                    _ptr(centroids), _ptr(assign), hbm_budget_bytes, capacity_slack, 0 if f32_tiles else 1,
                    _ptr(attrs), pq_m, _ptr(pq_codebook))
    if allocator not in ("torch", "hip"):
        raise ValueError(f"allocator must be 'torch' or 'hip', not {allocator!r}")
    alloc = ctypes.byref(torch_allocator(x.device.index or 0)) if allocator == "torch" else None
    h = ctypes.c_void_p()
    _check(load_library().quake_build(_ptr(x), _ptr(ids), x.shape[0], x.shape[1], ctypes.byref(p), alloc,
                                      _stream(), ctypes.byref(h)))
    return h.value


# recall estimator variants (QUAKE_EST_*): the threshold recompute from the
# table, every-partition recompute from the table, and every-partition
# recompute with the cap share evaluated directly
ESTIMATORS = {"aps": 0, "aps-r": 1, "aps-rp": 2}


def _search_params(k=10, nprobe=0, recall_target=0.0, f_M=0.0, tau_rho=0.0, upper_recall_target=0.0,
                   upper_f_M=0.0, scan_mode="plain", scan_dtype="f32", rerank_factor=0, window=0,
                   estimator="aps", filter=None) -> SearchParams:
    est = ESTIMATORS[estimator] if isinstance(estimator, str) else int(estimator)
    return SearchParams(k, nprobe, recall_target, f_M, tau_rho, upper_recall_target, upper_f_M, _MODE[scan_mode],
                        _SCAN_DTYPE[scan_dtype], rerank_factor, window, est,
                        None if filter is None else _labels(filter).data_ptr())


def quake_search(handle: int, q, *, k=10, nprobe=0, recall_target=0.0, f_M=0.0, tau_rho=0.0,
                 upper_recall_target=0.0, upper_f_M=0.0, scan_mode="plain", scan_dtype="f32", rerank_factor=0,
                 window=0, estimator="aps", filter=None, outputs=None):
    """Returns (ids int64 [nq,k], dist f32 [nq,k], nscanned int32 [nq], recall f64 [nq])."""
    import torch
    _dev(q, torch.float32)
    nq = q.shape[0]
    if outputs is None:
        dev = q.device
        outputs = (torch.empty((nq, k), dtype=torch.int64, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev),
                   torch.empty((nq,), dtype=torch.int32, device=dev),
                   torch.empty((nq,), dtype=torch.float64, device=dev))
    ids, dist, ns, rec = outputs
    p = _search_params(k, nprobe, recall_target, f_M, tau_rho, upper_recall_target, upper_f_M, scan_mode, scan_dtype,
                       rerank_factor, window, estimator, filter)
    _check(load_library().quake_search(handle, _ptr(q), nq, ctypes.byref(p), _ptr(ids), _ptr(dist), _ptr(ns),
                                       _ptr(rec), _stream()))
    return ids, dist, ns, rec


def quake_search_noalloc(handle: int, q, *, outputs, k=10, nprobe=0, recall_target=0.0, f_M=0.0, tau_rho=0.0,
                         upper_recall_target=0.0, upper_f_M=0.0, scan_mode="plain", scan_dtype="f32",
                         rerank_factor=0, window=0, estimator="aps", filter=None):
    """quake_search into caller-given outputs (ids, dist, nscanned, recall) with no allocation in the library."""
    import torch
    _dev(q, torch.float32)
    ids, dist, ns, rec = outputs
    p = _search_params(k, nprobe, recall_target, f_M, tau_rho, upper_recall_target, upper_f_M, scan_mode, scan_dtype,
                       rerank_factor, window, estimator, filter)
    _check(load_library().quake_search_noalloc(handle, _ptr(q), q.shape[0], ctypes.byref(p), _ptr(ids), _ptr(dist),
                                               _ptr(ns), _ptr(rec), _stream()))
    return ids, dist, ns, rec


def quake_insert(handle: int, x, ids):
    import torch
    _dev(x, torch.float32)
    _dev(ids, torch.int64)
    _check(load_library().quake_insert(handle, _ptr(x), _ptr(ids), x.shape[0], _stream()))


def quake_insert_attrs(handle: int, x, ids, attrs):
    import torch
    _dev(x, torch.float32)
    _dev(ids, torch.int64)
    _labels(attrs)
    _check(load_library().quake_insert_attrs(handle, _ptr(x), _ptr(ids), _ptr(attrs), x.shape[0], _stream()))


def quake_delete(handle: int, ids):
    import torch
    _dev(ids, torch.int64)
    _check(load_library().quake_delete(handle, _ptr(ids), ids.shape[0], _stream()))


def quake_stats(handle: int):
    n_live, nparts, nbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    _check(load_library().quake_stats(handle, ctypes.byref(n_live), ctypes.byref(nparts), ctypes.byref(nbytes)))
    return n_live.value, nparts.value, nbytes.value


def quake_export(handle: int, d: int):
    """(centroids f32 [nlist, d], ids int64 [n_live], partition int32 [n_live]) as torch tensors."""
    import torch
    n_live, nlist, _ = quake_stats(handle)
    dev = torch.device("cuda", torch.cuda.current_device())
    C = torch.empty((nlist, d), dtype=torch.float32, device=dev)
    ids = torch.empty((max(n_live, 1),), dtype=torch.int64, device=dev)
    part = torch.empty((max(n_live, 1),), dtype=torch.int32, device=dev)
    _check(load_library().quake_export(handle, _ptr(C), _ptr(ids), _ptr(part), _stream()))
    return C, ids[:n_live], part[:n_live]


def quake_export_pq(handle: int, d: int):
    """(codebook f32 [m, 256, d / m], codes uint8 [n_live, m]) of the index's product
    quantization, codes in quake_export's row order; (None, None) without codes."""
    import torch
    lib = load_library()
    m = ctypes.c_int32()
    _check(lib.quake_export_pq(handle, ctypes.byref(m), None, None, _stream()))
    if m.value == 0:
        return None, None
    n_live, _, _ = quake_stats(handle)
    dev = torch.device("cuda", torch.cuda.current_device())
    book = torch.empty((m.value, 256, d // m.value), dtype=torch.float32, device=dev)
    codes = torch.empty((max(n_live, 1), m.value), dtype=torch.uint8, device=dev)
    _check(lib.quake_export_pq(handle, ctypes.byref(m), _ptr(book), _ptr(codes), _stream()))
    return book, codes[:n_live]


def quake_export_top(handle: int, d: int, nlist_top: int):
    import torch
    _, nlist, _ = quake_stats(handle)
    dev = torch.device("cuda", torch.cuda.current_device())
    C1 = torch.empty((nlist_top, d), dtype=torch.float32, device=dev)
    top_of = torch.empty((nlist,), dtype=torch.int32, device=dev)
    _check(load_library().quake_export_top(handle, _ptr(C1), _ptr(top_of), _stream()))
    return C1, top_of


def quake_describe(handle: int) -> dict:
    d, metric, storage, levels = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().quake_describe(handle, ctypes.byref(d), ctypes.byref(metric), ctypes.byref(storage),
                                         ctypes.byref(levels)))
    inv_m = {v: k for k, v in _METRIC.items()}
    inv_d = {v: k for k, v in _DTYPE.items()}
    return {"d": d.value, "metric": inv_m[metric.value], "storage": inv_d[storage.value], "n_levels": levels.value}


def quake_add_level(handle: int, nlist_top: int, kmeans_iters: int = 10, seed: int = 0):
    _check(load_library().quake_add_level(handle, nlist_top, kmeans_iters, seed, _stream()))


def quake_level_sizes(handle: int) -> list:
    out = (ctypes.c_int64 * 3)()
    _check(load_library().quake_level_sizes(handle, out))
    return [int(v) for v in out]


def quake_export_level(handle: int, level: int, d: int):
    """(centroids f32 [N_level, d], parent int32 [N_{level-1}]) of upper level `level`."""
    import torch
    sizes = quake_level_sizes(handle)
    dev = torch.device("cuda", torch.cuda.current_device())
    C = torch.empty((max(sizes[level], 1), d), dtype=torch.float32, device=dev)
    parent = torch.empty((max(sizes[level - 1], 1),), dtype=torch.int32, device=dev)
    _check(load_library().quake_export_level(handle, level, _ptr(C), _ptr(parent), _stream()))
    return C[: sizes[level]], parent[: sizes[level - 1]]


def quake_remove_level(handle: int):
    _check(load_library().quake_remove_level(handle, _stream()))


def quake_adjust_levels(handle: int, add_above: int = 0, remove_below: int = 0, nlist_top: int = 0,
                        kmeans_iters: int = 10, seed: int = 0) -> int:
    """1 when a level was added, -1 when one was removed, else 0."""
    action = ctypes.c_int32()
    _check(load_library().quake_adjust_levels(handle, add_above, remove_below, nlist_top, kmeans_iters, seed,
                                              _stream(), ctypes.byref(action)))
    return action.value


def quake_save(handle: int, path: str):
    _check(load_library().quake_save(handle, os.fsencode(path), _stream()))


def quake_load(path: str, *, device: int = 0, hbm_budget_bytes: int = 0, allocator="torch") -> int:
    """A saved index in a new handle on `device` (allocator as quake_build)."""
    if allocator not in ("torch", "hip"):
        raise ValueError(f"allocator must be 'torch' or 'hip', not {allocator!r}")
    alloc = ctypes.byref(torch_allocator(device)) if allocator == "torch" else None
    h = ctypes.c_void_p()
    _check(load_library().quake_load(os.fsencode(path), alloc, hbm_budget_bytes, _stream(), ctypes.byref(h)))
    return h.value


def quake_access_stats(handle: int, level: int = 0, reset: bool = False):
    """(hits int64 [nlist] numpy, window) of the level's access statistics."""
    nlist = quake_stats(handle)[1] if level == 0 else None
    if nlist is None:
        raise ValueError("level 1 statistics: pass level=0 or read them through the C ABI")
    hits = np.zeros(nlist, dtype=np.int64)
    window = ctypes.c_int64()
    _check(load_library().quake_access_stats(handle, level, hits.ctypes.data, ctypes.byref(window), int(reset),
                                             _stream()))
    return hits, window.value


def quake_profile_latency(handle: int, sizes, nq: int = 1024, reps: int = 3, **search_kw) -> np.ndarray:
    """Microseconds per query of scanning one partition of each size (numpy float64)."""
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    out = np.zeros(sz.size, dtype=np.float64)
    kw = dict(search_kw)
    kw.setdefault("nprobe", 1)
    p = _search_params(**kw)
    _check(load_library().quake_profile_latency(handle, sz.ctypes.data, sz.size, nq, ctypes.byref(p), reps,
                                                out.ctypes.data, _stream()))
    return out


def quake_maintain(handle: int, lambda_size, lambda_cost, *, tau=0.25, alpha=0.9, refine_radius=50, refine_iters=1,
                   split_iters=8, min_split_size=2, merge_below=0, hits=None, window=0, max_decisions=4096):
    """One maintenance pass; returns (report dict, decisions list of dicts)."""
    ls = np.ascontiguousarray(lambda_size, dtype=np.float64)
    lc = np.ascontiguousarray(lambda_cost, dtype=np.float64)
    if ls.shape != lc.shape or ls.ndim != 1:
        raise ValueError("lambda_size and lambda_cost must be 1-D arrays of the same length")
    h = None if hits is None else np.ascontiguousarray(hits, dtype=np.int64)
    dec = (Decision * max(max_decisions, 1))()
    p = MaintainParams(tau, alpha, refine_radius, refine_iters, split_iters, min_split_size, merge_below, ls.size,
                       max_decisions, ls.ctypes.data, lc.ctypes.data, None if h is None else h.ctypes.data,
                       window, ctypes.cast(dec, ctypes.c_void_p))
    r = MaintainReport()
    _check(load_library().quake_maintain(handle, ctypes.byref(p), ctypes.byref(r), _stream()))
    rep = {name: getattr(r, name) for name, _ in MaintainReport._fields_ if name != "pad"}
    out = [{name: getattr(dec[i], name) for name, _ in Decision._fields_}
           for i in range(min(r.decisions, max_decisions))]
    return rep, out


def quake_candidates(handle: int, q, f_M: float, upper_recall_target=0.0, upper_f_M=0.0, tau_rho=0.0):
    """(order int32 [nq, M], h f32 [nq, M]) of adaptive scanning, without scanning level 0."""
    import torch
    _dev(q, torch.float32)
    p = _search_params(k=1, f_M=f_M, tau_rho=tau_rho, upper_recall_target=upper_recall_target,
                       upper_f_M=upper_f_M)
    M = ctypes.c_int32()
    _check(load_library().quake_candidates(handle, None, 0, ctypes.byref(p), None, None, ctypes.byref(M),
                                           _stream()))
    nq = q.shape[0]
    order = torch.empty((nq, M.value), dtype=torch.int32, device=q.device)
    h = torch.empty((nq, M.value), dtype=torch.float32, device=q.device)
    _check(load_library().quake_candidates(handle, _ptr(q), nq, ctypes.byref(p), _ptr(order), _ptr(h), None,
                                           _stream()))
    return order, h


def quake_profile(handle: int, enable: bool = True, reset: bool = False):
    """Per-kernel-class totals {name: (launches, ms, bytes, flops)} before this call."""
    out = (KernelProfile * 8)()
    _check(load_library().quake_profile(handle, int(enable), int(reset), ctypes.cast(out, ctypes.c_void_p)))
    return {n: (o.launches, o.milliseconds, o.bytes, o.flops) for n, o in zip(PROF_KINDS, out)}


def quake_set_tuning(handle: int, chunk_tiles=0, first_window=0, max_window=0, max_items=0, blocks_per_cu=0,
                     rounds_per_sync=0, no_graph=0, window_scale=0):
    t = Tuning(chunk_tiles, first_window, max_window, blocks_per_cu, max_items, rounds_per_sync, no_graph,
               window_scale)
    _check(load_library().quake_set_tuning(handle, ctypes.byref(t)))


def quake_autotune(handle: int, q, reps: int = 3, **search_kw):
    """Pick the fastest scheduling knobs for searches of q with search_kw; returns (knobs dict, median ms)."""
    import torch
    _dev(q, torch.float32)
    p = _search_params(**search_kw)
    t = Tuning()
    ms = ctypes.c_double()
    _check(load_library().quake_autotune(handle, _ptr(q), q.shape[0], ctypes.byref(p), reps, ctypes.byref(t),
                                         ctypes.byref(ms), _stream()))
    return {name: getattr(t, name) for name, _ in Tuning._fields_}, ms.value


def quake_free(handle: int):
    if handle:
        load_library().quake_free(handle)


def _host(a, dtype, ndim):
    a = np.ascontiguousarray(a, dtype=dtype)
    assert a.ndim == ndim, f"need a {ndim}-d host array"
    return a


def quake_server_create(handle: int, *, max_slots=0, hbm_budget_bytes=0, overlap_updates=False, **search_kw) -> int:
    """Start a serving loop on an index; search_kw as for quake_search."""
    p = ServerParams(max_slots, int(bool(overlap_updates)), hbm_budget_bytes, _search_params(**search_kw))
    h = ctypes.c_void_p()
    _check(load_library().quake_server_create(handle, ctypes.byref(p), ctypes.byref(h)))
    return h.value


def quake_server_search(server: int, q) -> int:
    """Queue the rows of q (host float32 [n, d]); returns the first ticket (tickets are consecutive)."""
    q = _host(q, np.float32, 2)
    t = ctypes.c_uint64()
    _check(load_library().quake_server_search(server, q.ctypes.data, q.shape[0], ctypes.byref(t)))
    return t.value


def quake_server_insert(server: int, x, ids) -> int:
    x = _host(x, np.float32, 2)
    ids = _host(ids, np.int64, 1)
    t = ctypes.c_uint64()
    _check(load_library().quake_server_insert(server, x.ctypes.data, ids.ctypes.data, ids.shape[0], ctypes.byref(t)))
    return t.value


def quake_server_delete(server: int, ids) -> int:
    ids = _host(ids, np.int64, 1)
    t = ctypes.c_uint64()
    _check(load_library().quake_server_delete(server, ids.ctypes.data, ids.shape[0], ctypes.byref(t)))
    return t.value


def quake_server_wait(server: int, ticket: int, k: int, timeout_s: float = -1.0):
    """(ids int64 [k], dist f32 [k], nscanned, status) of a finished ticket (host numpy)."""
    ids = np.full(k, -1, dtype=np.int64)
    dist = np.full(k, np.inf, dtype=np.float32)
    ns, st = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().quake_server_wait(server, ticket, timeout_s, ids.ctypes.data, dist.ctypes.data,
                                            ctypes.byref(ns), ctypes.byref(st)))
    return ids, dist, ns.value, st.value


def quake_server_stats(server: int, reset: bool = False) -> dict:
    r = ServerReport()
    _check(load_library().quake_server_stats(server, ctypes.byref(r), int(reset)))
    return {name: getattr(r, name) for name, _ in ServerReport._fields_}


def quake_server_destroy(server: int):
    if server:
        load_library().quake_server_destroy(server)


class Server:
    """Owning wrapper around a quake_server handle (continuous batching over an Index)."""

    def __init__(self, index: "Index", **kw):
        self.k = kw.get("k", 10)
        self.index = index
        self.handle = quake_server_create(index.handle, **kw)

    def search(self, q) -> list:
        q = _host(q, np.float32, 2)
        first = quake_server_search(self.handle, q)
        return list(range(first, first + q.shape[0]))

    def insert(self, x, ids) -> int:
        return quake_server_insert(self.handle, x, ids)

    def delete(self, ids) -> int:
        return quake_server_delete(self.handle, ids)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        return quake_server_wait(self.handle, ticket, self.k, timeout_s)

    def stats(self, reset=False):
        return quake_server_stats(self.handle, reset)

    def close(self):
        quake_server_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.close()
        except Exception:
            pass


class Index:
    """Owning wrapper around a quake_index handle."""

    def __init__(self, x, ids=None, **build_kw):
        self.d = x.shape[1]
        self.metric = build_kw.get("metric", "l2")
        self.handle = quake_build(x, ids, **build_kw)

    @classmethod
    def load(cls, path, **load_kw) -> "Index":
        """The index saved at `path` (quake_load)."""
        self = cls.__new__(cls)
        self.handle = quake_load(path, **load_kw)
        info = quake_describe(self.handle)
        self.d, self.metric = info["d"], info["metric"]
        return self

    def save(self, path):
        quake_save(self.handle, path)

    def level_sizes(self):
        return quake_level_sizes(self.handle)

    def export_level(self, level):
        return quake_export_level(self.handle, level, self.d)

    def add_level(self, nlist_top, kmeans_iters=10, seed=0):
        quake_add_level(self.handle, nlist_top, kmeans_iters, seed)

    def remove_level(self):
        quake_remove_level(self.handle)

    def adjust_levels(self, **kw):
        return quake_adjust_levels(self.handle, **kw)

    def describe(self):
        return quake_describe(self.handle)

    def search(self, q, **kw):
        return quake_search(self.handle, q, **kw)

    def insert(self, x, ids, attrs=None):
        if attrs is None:
            quake_insert(self.handle, x, ids)
        else:
            quake_insert_attrs(self.handle, x, ids, attrs)

    def delete(self, ids):
        quake_delete(self.handle, ids)

    def stats(self):
        return quake_stats(self.handle)

    def export(self):
        return quake_export(self.handle, self.d)

    def export_pq(self):
        return quake_export_pq(self.handle, self.d)

    def candidates(self, q, f_M=0.05, **upper_kw):
        return quake_candidates(self.handle, q, f_M, **upper_kw)

    def set_tuning(self, **kw):
        quake_set_tuning(self.handle, **kw)

    def autotune(self, q, reps=3, **search_kw):
        return quake_autotune(self.handle, q, reps, **search_kw)

    def profile(self, enable=True, reset=False):
        return quake_profile(self.handle, enable, reset)

    def access_stats(self, reset=False):
        return quake_access_stats(self.handle, 0, reset)

    def profile_latency(self, sizes, nq=1024, reps=3, **search_kw):
        return quake_profile_latency(self.handle, sizes, nq, reps, **search_kw)

    def maintain(self, lambda_size, lambda_cost, **kw):
        return quake_maintain(self.handle, lambda_size, lambda_cost, **kw)

    def free(self):
        quake_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.free()
        except Exception:
            pass
