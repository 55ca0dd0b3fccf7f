"""Sample-based classic closeness centrality on AMD Instinct MI355X (gfx950).

Python binding of the C-ABI library ``libccgpu.so`` (declared in
``include/ccgpu.h``).  The functions below carry the C names and only marshal
arguments: every step of the estimate runs in the library's HIP kernels.
PyTorch is used only to hold device buffers and to name HIP streams.

Importing this package does not need a GPU; the library is loaded on first
use and its absence is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccgpu.so")

CC_OK, CC_EINVAL, CC_EDISCONNECTED, CC_ENOMEM, CC_EOVERFLOW = 0, 1, 2, 3, 4
CC_EDEVICE, CC_EBUSY, CC_ECANCELLED, CC_ENOTREADY = 5, 6, 7, 8
CC_DIRECTED, CC_VALIDATE = 1, 2
CC_BATCHED, CC_PLAIN = 0, 1
CC_GRAPH = 0x100  # or-ed into CC_BATCHED: capture the estimate as a HIP graph and replay it

EXPORTED = [
    "cc_context_create", "cc_context_destroy", "cc_graph_upload", "cc_graph_borrow_device", "cc_graph_release",
    "cc_graph_info",
    "cc_draw_samples", "cc_estimate", "cc_estimate_device", "cc_estimate_device_noalloc", "cc_last_timing",
    "cc_submit", "cc_poll",
    "cc_wait", "cc_cancel", "cc_job_times", "cc_job_release", "cc_status_str", "cc_last_error",
    "cc_graph_get_tuning", "cc_graph_set_tuning", "cc_autotune", "cc_estimate_batch", "cc_reach_estimate",
    "cc_draw_weighted", "cc_estimate_weighted", "cc_reach_weighted",
]


class cc_reach_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("inbound", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("order", ctypes.c_void_p)]


REACH_FIELDS = {"count": np.int32, "distsum": np.int64, "T": np.int64, "B": np.float64, "R": np.float64}


class cc_reach_result(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in REACH_FIELDS]


class cc_weighted_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("mode", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("eps_num", ctypes.c_int32), ("eps_den", ctypes.c_int32), ("beta", ctypes.c_void_p)]


class cc_weighted_result(ctypes.Structure):
    _fields_ = [("S_beta", ctypes.c_void_p), ("S_beta_var", ctypes.c_void_p), ("samples", ctypes.c_void_p),
                ("adjusted", ctypes.c_void_p), ("tau", ctypes.c_void_p), ("sample_size", ctypes.c_void_p),
                ("S_beta_err", ctypes.c_void_p)]


class cc_reach_weighted_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("inbound", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("beta", ctypes.c_void_p)]


class cc_reach_weighted_result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_void_p), ("kth", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("R", ctypes.c_void_p)]


class cc_config(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class cc_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("mode", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("samples", ctypes.c_void_p), ("eps_num", ctypes.c_int32), ("eps_den", ctypes.c_int32)]


_RESULT_FIELDS = ["S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum", "samples",
                  "dmat", "D", "S_err", "S_ad", "S_ad_err", "S_sweep", "S_sweep_err"]


class cc_result(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in _RESULT_FIELDS]


class cc_timing(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("traverse_ms", ctypes.c_double),
                ("epilogue_ms", ctypes.c_double), ("levels", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
                ("nodes_visited", ctypes.c_int64), ("launches", ctypes.c_int64), ("dist_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_int64),
                ("arcs_matched", ctypes.c_int64), ("scatter_ms", ctypes.c_double),
                ("scatter_launches", ctypes.c_int64), ("scatter_arcs", ctypes.c_int64), ("hub_arcs", ctypes.c_int64),
                ("pull_scatter_ms", ctypes.c_double), ("pull_levels", ctypes.c_int64)]


class cc_tuning(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("level_blocks", ctypes.c_int32), ("scatter_blocks", ctypes.c_int32),
                ("delta", ctypes.c_int32), ("round_blocks", ctypes.c_int32), ("local_passes", ctypes.c_int32)]


TUNING_FIELDS = tuple(f for f, _ in cc_tuning._fields_)


# per-field element type and whether the length is n, k or k*k / n*k
_FIELD_SPEC = {
    "S_hyb": (np.float64, "n"), "S_samp": (np.float64, "n"), "S_piv": (np.int64, "n"), "S_pub": (np.int64, "n"),
    "pivot": (np.int32, "n"), "delta": (np.int32, "n"), "sampsum": (np.int64, "n"), "src_sum": (np.int64, "k"),
    "samples": (np.int32, "k"), "dmat": (np.int32, "kk"), "D": (np.int32, "nk"),
    "S_err": (np.float64, "n"), "S_ad": (np.float64, "n"), "S_ad_err": (np.float64, "n"),
    "S_sweep": (np.float64, "n"), "S_sweep_err": (np.float64, "n"),
}

_lib = None


class CCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{cc_status_str(status)} ({status}): {message}")
        self.status = status
        self.message = message


def load_library():
    """Load libccgpu.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1409_0035_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    # PyTorch ships its own HIP runtime under the same soname as ROCm's; load
    # it first so that the library and torch's device memory and streams share
    # one runtime in this process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "cc_context_create": (i32, [ctypes.c_int, ctypes.POINTER(cc_config), PP]),
        "cc_context_destroy": (None, [P]),
        "cc_graph_upload": (i32, [P, i64, i64, P, P, P, u32, PP]),
        "cc_graph_borrow_device": (i32, [P, i64, i64, P, P, P, u32, PP]),
        "cc_graph_release": (None, [P]),
        "cc_graph_info": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(u32)]),
        "cc_draw_samples": (i32, [i64, i32, u64, P]),
        "cc_estimate": (i32, [P, P, ctypes.POINTER(cc_params), ctypes.POINTER(cc_result)]),
        "cc_estimate_device": (i32, [P, P, ctypes.POINTER(cc_params), ctypes.POINTER(cc_result), P]),
        "cc_estimate_device_noalloc": (i32, [P, P, ctypes.POINTER(cc_params), ctypes.POINTER(cc_result), P]),
        "cc_last_timing": (i32, [P, ctypes.POINTER(cc_timing)]),
        "cc_submit": (i32, [P, P, ctypes.POINTER(cc_params), ctypes.POINTER(cc_result), PP]),
        "cc_poll": (i32, [P]),
        "cc_wait": (i32, [P]),
        "cc_cancel": (i32, [P]),
        "cc_job_times": (i32, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "cc_job_release": (None, [P]),
        "cc_estimate_batch": (i32, [P, i32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(cc_params),
                                    ctypes.POINTER(cc_result), ctypes.POINTER(i32)]),
        "cc_graph_get_tuning": (i32, [P, ctypes.POINTER(cc_tuning)]),
        "cc_graph_set_tuning": (i32, [P, ctypes.POINTER(cc_tuning)]),
        "cc_autotune": (i32, [P, P, i32, u64, i32, ctypes.POINTER(cc_tuning), ctypes.POINTER(ctypes.c_double)]),
        "cc_reach_estimate": (i32, [P, P, ctypes.POINTER(cc_reach_params), ctypes.POINTER(cc_reach_result)]),
        "cc_draw_weighted": (i32, [i64, P, i32, u64, P, P, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]),
        "cc_estimate_weighted": (i32, [P, P, ctypes.POINTER(cc_weighted_params), ctypes.POINTER(cc_weighted_result)]),
        "cc_reach_weighted": (i32, [P, P, ctypes.POINTER(cc_reach_weighted_params),
                                    ctypes.POINTER(cc_reach_weighted_result)]),
        "cc_status_str": (ctypes.c_char_p, [i32]),
        "cc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != CC_OK:
        raise CCError(status, cc_last_error())


def cc_status_str(status: int) -> str:
    return load_library().cc_status_str(int(status)).decode()


def cc_last_error() -> str:
    return load_library().cc_last_error().decode()


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- context / graphs

def cc_context_create(device: int = 0, mem_budget_bytes: int = 0, max_inflight: int = 0) -> ctypes.c_void_p:
    lib = load_library()
    cfg = cc_config(mem_budget_bytes, max_inflight, 0)
    out = ctypes.c_void_p()
    _check(lib.cc_context_create(int(device), ctypes.byref(cfg), ctypes.byref(out)))
    return out


def cc_context_destroy(ctx) -> None:
    load_library().cc_context_destroy(ctx)


def cc_graph_upload(ctx, n: int, arcs: int, row_ptr, col_idx, w=None, flags: int = 0) -> ctypes.c_void_p:
    lib = load_library()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col_idx, dtype=np.int32)
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib.cc_graph_upload(ctx, int(n), int(arcs), _ptr(rp), _ptr(col), _ptr(wa), int(flags),
                               ctypes.byref(out)))
    return out


def cc_graph_borrow_device(ctx, n: int, arcs: int, row_ptr, col_idx, w=None, flags: int = 0) -> ctypes.c_void_p:
    """A graph over a CSR already in device memory (torch tensors on the
    context's device: int64 row_ptr, int32 col_idx, int32 w or None).  The
    library reads the tensors in place; keep them alive and unchanged until
    the graph is released and its jobs have ended."""
    import torch
    for name, t, dt in (("row_ptr", row_ptr, torch.int64), ("col_idx", col_idx, torch.int32), ("w", w, torch.int32)):
        if t is None:
            continue
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dt:
            raise ValueError(f"{name}: need a contiguous {dt} device tensor")
    torch.cuda.synchronize()  # the library reads them on its own stream
    out = ctypes.c_void_p()
    _check(load_library().cc_graph_borrow_device(ctx, int(n), int(arcs), ctypes.c_void_p(row_ptr.data_ptr()),
                                                 ctypes.c_void_p(col_idx.data_ptr()),
                                                 None if w is None else ctypes.c_void_p(w.data_ptr()), int(flags),
                                                 ctypes.byref(out)))
    return out


def cc_graph_release(g) -> None:
    load_library().cc_graph_release(g)


def cc_graph_info(g):
    n, arcs, fl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint32()
    _check(load_library().cc_graph_info(g, ctypes.byref(n), ctypes.byref(arcs), ctypes.byref(fl)))
    return n.value, arcs.value, fl.value


def cc_graph_get_tuning(g) -> dict:
    t = cc_tuning()
    _check(load_library().cc_graph_get_tuning(g, ctypes.byref(t)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def cc_graph_set_tuning(g, **fields) -> dict:
    """Changes the named knobs of the graph's tuning; returns the new setting."""
    cur = cc_graph_get_tuning(g)
    unknown = set(fields) - set(TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    cur.update(fields)
    t = cc_tuning(**{f: int(cur[f]) for f in TUNING_FIELDS})
    _check(load_library().cc_graph_set_tuning(g, ctypes.byref(t)))
    return cur


def cc_autotune(ctx, g, k: int, seed: int = 0, reps: int = 3):
    """Runs the library's autotuner on a resident graph; returns (tuning dict, ms)."""
    t, ms = cc_tuning(), ctypes.c_double()
    _check(load_library().cc_autotune(ctx, g, int(k), int(seed), int(reps), ctypes.byref(t), ctypes.byref(ms)))
    return {f: getattr(t, f) for f in TUNING_FIELDS}, ms.value


def cc_draw_samples(n: int, k: int, seed: int) -> np.ndarray:
    out = np.empty(k, dtype=np.int32)
    _check(load_library().cc_draw_samples(int(n), int(k), int(seed), _ptr(out)))
    return out


def _params(k, mode, seed, samples, eps):
    s = None if samples is None else np.ascontiguousarray(samples, dtype=np.int32)
    en, ed = (0, 0) if eps is None else eps
    p = cc_params(int(k), int(mode), int(seed), None if s is None else s.ctypes.data, int(en), int(ed))
    return p, s


def _sizes(n, k):
    return {"n": n, "k": k, "kk": k * k, "nk": n * k}


def cc_estimate(ctx, g, k: int, mode: int = CC_BATCHED, seed: int = 0, samples=None, eps=None,
                outputs=("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum",
                         "samples", "dmat")) -> dict:
    """Synchronous estimate into host numpy arrays (one per requested field)."""
    n, _, _ = cc_graph_info(g)
    p, keep = _params(k, mode, seed, samples, eps)
    sz = _sizes(n, k)
    res = cc_result()
    arrays = {}
    for f in outputs:
        dt, which = _FIELD_SPEC[f]
        arrays[f] = np.empty(sz[which], dtype=dt)
        setattr(res, f, arrays[f].ctypes.data)
    _check(load_library().cc_estimate(ctx, g, ctypes.byref(p), ctypes.byref(res)))
    if "dmat" in arrays:
        arrays["dmat"] = arrays["dmat"].reshape(k, k)
    if "D" in arrays:
        arrays["D"] = arrays["D"].reshape(n, k)
    del keep
    return arrays


def cc_draw_weighted(beta, k: int, seed: int):
    """The node-weighted sample of Sec. 5: (ids in increasing order, light
    flags, R, m) with tau = R/m."""
    beta = np.ascontiguousarray(beta, dtype=np.uint32)
    ids = np.empty(k, dtype=np.int32)
    light = np.empty(k, dtype=np.uint8)
    R, m, c = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().cc_draw_weighted(int(beta.shape[0]), _ptr(beta), int(k), int(seed), _ptr(ids), _ptr(light),
                                           ctypes.byref(R), ctypes.byref(m), ctypes.byref(c)))
    return ids[:c.value].copy(), light[:c.value].astype(bool), int(R.value), int(m.value)


def cc_estimate_weighted(ctx, g, beta, k: int, seed: int = 0, mode: int = CC_BATCHED, eps=None) -> dict:
    """Node-weighted hybrid estimate (Sec. 5 / Algorithm 3) for every node,
    with its variance estimate, the sample, adjusted weights and tau."""
    n, _, _ = cc_graph_info(g)
    beta = np.ascontiguousarray(beta, dtype=np.uint32)
    if beta.shape[0] != n:
        raise ValueError("one weight per node")
    en, ed = (0, 0) if eps is None else (int(eps[0]), int(eps[1]))
    p = cc_weighted_params(int(k), int(mode), int(seed), en, ed, beta.ctypes.data)
    out = dict(S_beta=np.empty(n, np.float64), S_beta_var=np.empty(n, np.float64),
               samples=np.empty(k, np.int32), adjusted=np.empty(k, np.float64), tau=np.zeros(1, np.float64),
               sample_size=np.zeros(1, np.int32), S_beta_err=np.empty(n, np.float64))
    res = cc_weighted_result(*(out[f].ctypes.data for f in ("S_beta", "S_beta_var", "samples", "adjusted", "tau",
                                                            "sample_size", "S_beta_err")))
    _check(load_library().cc_estimate_weighted(ctx, g, ctypes.byref(p), ctypes.byref(res)))
    c = int(out["sample_size"][0])
    out["samples"] = out["samples"][:c]
    out["adjusted"] = out["adjusted"][:c]
    out["tau"] = float(out["tau"][0])
    out["sample_size"] = c
    return out


def cc_reach_weighted(ctx, g, beta, k: int, inbound: bool = False, seed: int = 0) -> dict:
    """Node-weighted reachability sampling of Sec. 6.2 / Algorithm 5 for
    every node: count, the k-th member, and the estimates S and R."""
    n, _, _ = cc_graph_info(g)
    beta = np.ascontiguousarray(beta, dtype=np.uint32)
    if beta.shape[0] != n:
        raise ValueError("one weight per node")
    p = cc_reach_weighted_params(int(k), 1 if inbound else 0, int(seed), beta.ctypes.data)
    out = dict(count=np.empty(n, np.int32), kth=np.empty(n, np.int32), S=np.empty(n, np.float64),
               R=np.empty(n, np.float64))
    res = cc_reach_weighted_result(*(out[f].ctypes.data for f in ("count", "kth", "S", "R")))
    _check(load_library().cc_reach_weighted(ctx, g, ctypes.byref(p), ctypes.byref(res)))
    return out


def cc_reach_estimate(ctx, g, k: int, inbound: bool = False, seed: int = 0, order=None,
                      outputs=tuple(REACH_FIELDS)) -> dict:
    """Outbound (or inbound) reachability sampling of Sec. 6.2 / Algorithm 4
    for every node, into host numpy arrays (one per requested field)."""
    n, _, _ = cc_graph_info(g)
    keep = None
    if order is not None:
        keep = np.ascontiguousarray(order, dtype=np.int32)
        if keep.shape[0] != n:
            raise ValueError("order must list every node once")
    p = cc_reach_params(int(k), 1 if inbound else 0, int(seed), None if keep is None else keep.ctypes.data)
    res = cc_reach_result()
    arrays = {}
    for f in outputs:
        arrays[f] = np.empty(n, dtype=REACH_FIELDS[f])
        setattr(res, f, arrays[f].ctypes.data)
    _check(load_library().cc_reach_estimate(ctx, g, ctypes.byref(p), ctypes.byref(res)))
    del keep
    return arrays


def cc_estimate_batch(ctx, jobs, outputs=("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum")):
    """Several estimates in one call.  `jobs` is a list of (graph handle, k,
    seed) or (graph handle, k, seed, eps).  Returns (list of output dicts,
    list of statuses); a job whose status is not CC_OK has unspecified
    outputs."""
    lib = load_library()
    count = len(jobs)
    graphs = (ctypes.c_void_p * count)()
    params = (cc_params * count)()
    results = (cc_result * count)()
    statuses = (ctypes.c_int32 * count)()
    arrays, keep = [], []
    for j, job in enumerate(jobs):
        g, k, seed = job[0], int(job[1]), int(job[2])
        eps = job[3] if len(job) > 3 else None
        graphs[j] = g.value if isinstance(g, ctypes.c_void_p) else g
        p, kp = _params(k, CC_BATCHED, seed, None, eps)
        params[j] = p
        keep.append(kp)
        n, _, _ = cc_graph_info(g)
        sz = _sizes(n, k)
        arr = {}
        for f in outputs:
            dt, which = _FIELD_SPEC[f]
            arr[f] = np.empty(sz[which], dtype=dt)
            setattr(results[j], f, arr[f].ctypes.data)
        arrays.append((arr, n, k))
    lib.cc_estimate_batch(ctx, count, graphs, params, results, statuses)
    out = []
    for arr, n, k in arrays:
        if "dmat" in arr:
            arr["dmat"] = arr["dmat"].reshape(k, k)
        if "D" in arr:
            arr["D"] = arr["D"].reshape(n, k)
        out.append(arr)
    del keep
    return out, [int(x) for x in statuses]


def cc_estimate_device(ctx, g, k: int, out: dict, mode: int = CC_BATCHED, seed: int = 0, samples=None,
                       eps=None, stream=None, noalloc: bool = False) -> None:
    """Estimate into device tensors.  `out` maps result field names to torch
    tensors on the context's device (contiguous, of the field's dtype and
    length); `stream` is a torch.cuda.Stream (default: torch's current).
    noalloc=True calls cc_estimate_device_noalloc (no device allocation)."""
    import torch
    p, keep = _params(k, mode, seed, samples, eps)
    res = cc_result()
    for f, t in out.items():
        dt, _ = _FIELD_SPEC[f]
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{f}: need a contiguous device tensor")
        if t.element_size() != np.dtype(dt).itemsize:
            raise ValueError(f"{f}: wrong element type")
        setattr(res, f, t.data_ptr())
    if stream is None:
        stream = torch.cuda.current_stream()
    fn = load_library().cc_estimate_device_noalloc if noalloc else load_library().cc_estimate_device
    _check(fn(ctx, g, ctypes.byref(p), ctypes.byref(res), ctypes.c_void_p(stream.cuda_stream)))
    del keep


def cc_last_timing(ctx) -> dict:
    t = cc_timing()
    _check(load_library().cc_last_timing(ctx, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in cc_timing._fields_ if f != "reserved"}


# ---------------------------------------------------------------- serving

@dataclass
class Job:
    handle: ctypes.c_void_p
    arrays: dict
    keep: object
    n: int = 0
    k: int = 0


def cc_submit(ctx, g, k: int, mode: int = CC_BATCHED, seed: int = 0, samples=None, eps=None,
              outputs=("S_hyb", "pivot", "delta")) -> Job:
    n, _, _ = cc_graph_info(g)
    p, keep = _params(k, mode, seed, samples, eps)
    sz = _sizes(n, k)
    res = cc_result()
    arrays = {}
    for f in outputs:
        dt, which = _FIELD_SPEC[f]
        arrays[f] = np.empty(sz[which], dtype=dt)
        setattr(res, f, arrays[f].ctypes.data)
    h = ctypes.c_void_p()
    _check(load_library().cc_submit(ctx, g, ctypes.byref(p), ctypes.byref(res), ctypes.byref(h)))
    return Job(h, arrays, keep, n, k)


def cc_poll(job: Job) -> int:
    return int(load_library().cc_poll(job.handle))


def cc_wait(job: Job) -> dict:
    """Block until the job ends; its output arrays (dmat as k x k, D as n x k)."""
    _check(load_library().cc_wait(job.handle))
    out = dict(job.arrays)
    if "dmat" in out:
        out["dmat"] = out["dmat"].reshape(job.k, job.k)
    if "D" in out:
        out["D"] = out["D"].reshape(job.n, job.k)
    return out


def cc_cancel(job: Job) -> int:
    return int(load_library().cc_cancel(job.handle))


def cc_job_times(job: Job):
    q, t = ctypes.c_double(), ctypes.c_double()
    st = load_library().cc_job_times(job.handle, ctypes.byref(q), ctypes.byref(t))
    if st == CC_ENOTREADY:
        return None
    _check(st)
    return q.value, t.value


def cc_job_release(job: Job) -> None:
    load_library().cc_job_release(job.handle)
    job.handle = None


# ---------------------------------------------------------------- convenience

class Context:
    """Owns a context handle; uploads graph objects with .n/.row_ptr/.col_idx/.w/.directed."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0, max_inflight: int = 0):
        self.handle = cc_context_create(device, mem_budget_bytes, max_inflight)
        self._graphs = []

    def upload(self, graph, validate: bool = False):
        flags = (CC_DIRECTED if graph.directed else 0) | (CC_VALIDATE if validate else 0)
        h = cc_graph_upload(self.handle, graph.n, graph.arcs, graph.row_ptr, graph.col_idx, graph.w, flags)
        self._graphs.append(h)
        return h

    def release(self, gh):
        cc_graph_release(gh)
        self._graphs = [x for x in self._graphs if x is not gh]

    def close(self):
        for h in self._graphs:
            cc_graph_release(h)
        self._graphs = []
        if self.handle is not None:
            cc_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
