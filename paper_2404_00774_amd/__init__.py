"""Python binding of the SOAR gfx950 library (libsoar.so, C ABI in include/soar.h).

Argument marshalling only: tensors are checked for dtype, device and contiguity, workspaces are
allocated as torch tensors, and every computation runs in the library's HIP kernels.  If the
library has not been built the import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsoar.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2404_00774_amd.build`"
                      " (hipcc, gfx950) before importing the binding")

_lib = ctypes.CDLL(LIB_PATH)

FP32, BF16, FP8_E4M3 = 0, 1, 2
_PREC = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3}
ASYNC = 1
SPILL_GROUPED, SPILL_DIRECT = 2, 4
NO_BOUND, BOUND_ALWAYS = 8, 16
_BOUND = {True: 0, "auto": 0, False: NO_BOUND, "off": NO_BOUND, "always": BOUND_ALWAYS}
_SPILL_FORM = {"auto": 0, "grouped": SPILL_GROUPED, "direct": SPILL_DIRECT}

_STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
           -4: "unsupported", -5: "non-finite input", -6: "timeout", -7: "shutdown"}


class SoarError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.soar_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class AssignOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("lambda_", ctypes.c_float),
                ("precision", ctypes.c_int32), ("topk", ctypes.c_int32),
                ("near_tie_rel", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device_ms", ctypes.c_float),
                ("assign_kernel_ms", ctypes.c_float), ("rows_full_scan", ctypes.c_int64), ("rows_fp64", ctypes.c_int64),
                ("mfma_flops", ctypes.c_double), ("phase_ms", ctypes.c_float * 6),
                ("rows_bounded", ctypes.c_int64)]

    PHASES = ("prep", "primary_sweep", "primary_rescore", "grouping", "spill_sweep",
              "spill_rescore")

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("struct_size", "phase_ms")}
        d["phase_ms"] = dict(zip(self.PHASES, [float(v) for v in self.phase_ms]))
        return d


_vp, _i64, _i32, _u64, _f32, _f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_uint64, ctypes.c_float, ctypes.c_double)
_sz = ctypes.c_size_t


def _sig(name, args, res=ctypes.c_int):
    fn = getattr(_lib, name, None)
    if fn is None:
        return None
    fn.argtypes, fn.restype = args, res
    return fn


_lib.soar_status_string.argtypes, _lib.soar_status_string.restype = [ctypes.c_int], ctypes.c_char_p
_sig("soar_assign_workspace_size", [_i64, _i32, _i32, ctypes.POINTER(AssignOpts),
                                    ctypes.POINTER(_sz)])
_sig("soar_assign", [_vp, _i64, _i32, _vp, _i32, ctypes.POINTER(AssignOpts), _vp, _vp, _vp, _vp,
                     _vp, _sz, _vp, ctypes.POINTER(Stats)])
_sig("soar_assign_noalloc", [_vp, _i64, _i32, _vp, _i32, ctypes.POINTER(AssignOpts), _vp, _vp, _vp,
                             _vp, _vp])
_sig("soar_assign_noalloc_limit", [], _sz)
_sig("soar_assign_candidates", [_i64, _i32, _i32, ctypes.POINTER(AssignOpts), ctypes.POINTER(_sz),
                                ctypes.POINTER(_sz), ctypes.POINTER(_i32), ctypes.POINTER(_sz)])
_sig("soar_spill_further_workspace_size", [_i64, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_sig("soar_spill_further", [_vp, _i64, _i32, _vp, _i32, _vp, _i32, _f32, _f32, _vp, _vp, _vp, _sz,
                            _vp, ctypes.POINTER(Stats)])
_sig("soar_pq_encode", [_vp, _i64, _i32, _vp, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _sz, _vp])
_sig("soar_lists_workspace_size", [_i64, _i32, ctypes.POINTER(_sz)])
_sig("soar_lists_build", [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _sz, _vp])
_sig("soar_search_workspace_size", [_i64, _i32, _i32, ctypes.POINTER(_sz)])
_sig("soar_search", [_vp, _i64, _i32, _vp, _i32, _vp, _i64, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp,
                     _sz, _vp])
_sig("soar_lists_codes", [_vp, _vp, _i32, _i64, _vp, _i32, _vp, _i32, _vp, ctypes.POINTER(_i64),
                          _vp, _sz, _vp])
_sig("soar_lists_probe_bound", [_vp, _i32, _i32, ctypes.POINTER(_i64), _vp])
_sig("soar_search_pq_workspace_size", [_i64, _i32, _i32, _i32, _i64, ctypes.POINTER(_sz)])
_sig("soar_search_pq", [_vp, _i64, _i32, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _i32, _i32,
                        _i32, _i32, _i64, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("soar_search_two_level_workspace_size", [_i64, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_sig("soar_search_two_level", [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _i64,
                               _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("soar_train_workspace_size", [_i64, _i32, _i32, ctypes.POINTER(_sz)])
_sig("soar_kmeanspp", [_vp, _i64, _i32, _i32, _u64, _vp, _vp, _vp, _sz, _vp])
_sig("soar_lloyd_update", [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("soar_train_codebook", [_vp, _i64, _i32, _i32, _i32, _u64, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("soar_index_arena_size", [_i32, _i32, _i32, _i32, _i64, ctypes.POINTER(_sz)])
_sig("soar_index_create", [_vp, _i32, _i32, _f32, _i32, _vp, _sz, _i32, ctypes.POINTER(_vp)])
_sig("soar_insert", [_vp, _vp, _i64, _i64, ctypes.POINTER(_u64)])
_sig("soar_wait", [_vp, _u64, _vp, _vp, _f64])
_sig("soar_index_list", [_vp, _i32, _vp, _i64, ctypes.POINTER(_i64)])
_sig("soar_index_destroy", [_vp], None)


class IndexStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("requests", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("max_steps_in_flight", ctypes.c_int64), ("chunks_used", ctypes.c_int64),
                ("chunks_total", ctypes.c_int64)]


_sig("soar_index_get_stats", [_vp, ctypes.POINTER(IndexStats)])
_sig("soar_index_chunk_bytes", [], _sz)

EXPORTED = [n for n in ("soar_assign_workspace_size", "soar_assign", "soar_assign_candidates",
                        "soar_assign_noalloc",
                        "soar_assign_noalloc_limit", "soar_train_workspace_size",
                        "soar_kmeanspp", "soar_lloyd_update", "soar_train_codebook",
                        "soar_index_arena_size", "soar_index_create", "soar_insert", "soar_wait",
                        "soar_index_list", "soar_index_get_stats", "soar_index_chunk_bytes",
                        "soar_lists_workspace_size", "soar_lists_build", "soar_search_workspace_size",
                        "soar_search", "soar_spill_further_workspace_size",
                        "soar_spill_further", "soar_pq_encode", "soar_lists_codes",
                        "soar_lists_probe_bound", "soar_search_pq_workspace_size",
                        "soar_search_pq",
                        "soar_search_two_level_workspace_size", "soar_search_two_level",
                        "soar_index_destroy", "soar_status_string") if hasattr(_lib, n)]


def _check(status, where):
    if status != 0:
        raise SoarError(status, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _f32_matrix(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must be on the GPU")
    return t.contiguous()


def _opts(lam, precision, topk, near_tie_rel, flags):
    o = AssignOpts()
    o.struct_size = ctypes.sizeof(AssignOpts)
    o.lambda_ = float(lam)
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.topk = int(topk)
    o.near_tie_rel = float(near_tie_rel)
    o.flags = int(flags)
    return o


def assign_workspace_size(n, d, K, lam=1.0, precision="fp32", topk=0, near_tie_rel=0.0):
    o = _opts(lam, precision, topk, near_tie_rel, 0)
    b = _sz()
    _check(_lib.soar_assign_workspace_size(n, d, K, ctypes.byref(o), ctypes.byref(b)),
           "soar_assign_workspace_size")
    return b.value


def assign(X, C, lam, precision="fp32", topk=0, near_tie_rel=0.0, stream=None, out=None,
           workspace=None, flags=0, stats=False, spill_form="auto", bound=True):
    """SOAR assignment of every row of X against codebook C (both float32 on the GPU).

    ``spill_form``: "auto", "grouped" or "direct" (the form of the spill sweep; same results).
    ``bound``: "auto" (or True; the library decides), False ("off": SOAR_NO_BOUND, every row's
    spill goes through the sweep) or "always" (SOAR_BOUND_ALWAYS).
    Returns (primary int32[n], spill int32[n], primary_dist float32[n], spill_loss float32[n])
    and, with ``stats=True``, a dict of call statistics as a fifth element."""
    flags = int(flags) | _SPILL_FORM[spill_form] | _BOUND[bound]
    X, C = _f32_matrix(X, "X"), _f32_matrix(C, "C")
    n, d = X.shape
    K = C.shape[0]
    if C.shape[1] != d:
        raise ValueError("X and C must have the same number of columns")
    dev = X.device
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=dev),
               torch.empty(n, dtype=torch.int32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev))
    o = _opts(lam, precision, topk, near_tie_rel, flags)
    need = assign_workspace_size(n, d, K, lam, precision, topk, near_tie_rel)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    status = _lib.soar_assign(_ptr(X), n, d, _ptr(C), K, ctypes.byref(o), _ptr(out[0]),
                              _ptr(out[1]), _ptr(out[2]), _ptr(out[3]), _ptr(workspace),
                              workspace.numel(), _stream(stream), ctypes.byref(st))
    _check(status, "soar_assign")
    return (*out, st.as_dict()) if stats else out


def assign_candidates(workspace, n, d, K, lam=1.0, precision="bf16", topk=0, near_tie_rel=0.0,
                      bound_key=False):
    """The re-scored candidates the last BF16/FP8 assign() left in ``workspace`` (same sizes and
    options): (primary int32[n, topk], spill int32[n, topk]) views of the workspace, -1 for an
    empty place.  With ``bound_key=True`` a third view, int32[n]: after a call that used the
    spill bound, -1 for the rows it decided (and rows without a primary), else the primary."""
    o = _opts(lam, precision, topk, near_tie_rel, 0)
    po, so, tk, bo = _sz(), _sz(), _i32(), _sz()
    _check(_lib.soar_assign_candidates(n, d, K, ctypes.byref(o), ctypes.byref(po),
                                       ctypes.byref(so), ctypes.byref(tk), ctypes.byref(bo)),
           "soar_assign_candidates")
    nb = n * tk.value * 4
    view = lambda off: workspace[off:off + nb].view(torch.int32).view(n, tk.value)  # noqa: E731
    if bound_key:
        return (view(po.value), view(so.value),
                workspace[bo.value:bo.value + n * 4].view(torch.int32))
    return view(po.value), view(so.value)


def assign_noalloc(X, C, lam, precision="fp32", topk=0, near_tie_rel=0.0, stream=None, out=None,
                   flags=0, spill_form="auto"):
    """soar_assign_noalloc: the same assignment with the library's fixed device workspace
    (nothing is allocated by the library; at most assign_noalloc_limit() bytes of workspace)."""
    flags = int(flags) | _SPILL_FORM[spill_form]
    X, C = _f32_matrix(X, "X"), _f32_matrix(C, "C")
    n, d = X.shape
    K = C.shape[0]
    if C.shape[1] != d:
        raise ValueError("X and C must have the same number of columns")
    dev = X.device
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=dev),
               torch.empty(n, dtype=torch.int32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev))
    o = _opts(lam, precision, topk, near_tie_rel, flags)
    _check(_lib.soar_assign_noalloc(_ptr(X), n, d, _ptr(C), K, ctypes.byref(o), _ptr(out[0]),
                                    _ptr(out[1]), _ptr(out[2]), _ptr(out[3]), _stream(stream)),
           "soar_assign_noalloc")
    return out


def assign_noalloc_limit():
    return int(_lib.soar_assign_noalloc_limit())


def spill_further(X, C, prior, lam, near_tie_rel=0.0, stream=None, stats=False):
    """soar_spill_further: the next assignment of every row given its earlier ones
    (prior int32[n, m] on the GPU, m = 1..3, distinct per row).  Returns (next int32[n],
    loss float32[n]) and, with ``stats=True``, a dict of call statistics."""
    X, C = _f32_matrix(X, "X"), _f32_matrix(C, "C")
    n, d = X.shape
    K = C.shape[0]
    if C.shape[1] != d:
        raise ValueError("X and C must have the same number of columns")
    if not isinstance(prior, torch.Tensor) or prior.dtype != torch.int32 or not prior.is_cuda:
        raise TypeError("prior must be an int32 tensor on the GPU")
    P = prior.reshape(n, -1).contiguous()
    m = P.shape[1]
    b = _sz()
    _check(_lib.soar_spill_further_workspace_size(n, d, K, m, ctypes.byref(b)),
           "soar_spill_further_workspace_size")
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=X.device)
    nxt = torch.empty(n, dtype=torch.int32, device=X.device)
    loss = torch.empty(n, dtype=torch.float32, device=X.device)
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    _check(_lib.soar_spill_further(_ptr(X), n, d, _ptr(C), K, _ptr(P), m, float(lam),
                                   float(near_tie_rel), _ptr(nxt), _ptr(loss), _ptr(ws),
                                   ws.numel(), _stream(stream), ctypes.byref(st)),
           "soar_spill_further")
    return (nxt, loss, st.as_dict()) if stats else (nxt, loss)


def assign_multi(X, C, lam, M, near_tie_rel=0.0, stream=None):
    """M assignments per row (M = 1..4): the FP32 primary and spill of soar_assign, then M - 2
    further assignments, each given all earlier ones.  Returns (int32[n, M], float32[n, M]):
    indices, and the primary distance followed by each spill's loss."""
    if not 1 <= M <= 4:
        raise ValueError("M must be in 1..4")
    p, s, dp, ls = assign(X, C, lam, near_tie_rel=near_tie_rel, stream=stream)
    A, V = [p, s], [dp, ls]
    for _ in range(2, M):
        j, v = spill_further(X, C, torch.stack(A, dim=1), lam, near_tie_rel, stream)
        A.append(j)
        V.append(v)
    return torch.stack(A[:M], dim=1), torch.stack(V[:M], dim=1)


def pq_encode(X, C, assign, P, stream=None):
    """soar_pq_encode: 4-bit PQ codes of every assignment's residual.  assign int32 [n, m] (or [n])
    and P float32 [M, 16, s] on the GPU; returns uint8 [n, m, M / 2] (two codes per byte, the
    even subspace in the low nibble)."""
    X, C = _f32_matrix(X, "X"), _f32_matrix(C, "C")
    n, d = X.shape
    if not isinstance(assign, torch.Tensor) or assign.dtype != torch.int32 or not assign.is_cuda:
        raise TypeError("assign must be an int32 tensor on the GPU")
    if not isinstance(P, torch.Tensor) or P.dtype != torch.float32 or P.dim() != 3 or not P.is_cuda:
        raise TypeError("P must be a float32 [M, 16, s] tensor on the GPU")
    A = assign.reshape(n, -1).contiguous()
    m = A.shape[1]
    M, h, s = P.shape
    if h != 16 or M * s != d:
        raise ValueError("P must be [d / s, 16, s]")
    codes = torch.empty((n, m, M // 2), dtype=torch.uint8, device=X.device)
    ws = torch.empty(256, dtype=torch.uint8, device=X.device)
    _check(_lib.soar_pq_encode(_ptr(X), n, d, _ptr(C), C.shape[0], _ptr(A), m,
                               _ptr(P.contiguous()), s, _ptr(codes), _ptr(ws), ws.numel(),
                               _stream(stream)), "soar_pq_encode")
    return codes


def pq_train(R, s, iters=10, seed=0, stream=None):
    """A PQ codebook [d / s, 16, s] for residual rows R (float32 [n, d] on the GPU): per subspace,
    k-means++ then `iters` Lloyd iterations (soar_train_codebook) on that subspace's columns."""
    R = _f32_matrix(R, "R")
    n, d = R.shape
    if d % s:
        raise ValueError("s must divide d")
    out = []
    for m in range(d // s):
        Rm = R[:, m * s:(m + 1) * s].contiguous()
        Cm, _, _ = train_codebook(Rm, 16, iters, seed=seed + m, stream=stream)
        out.append(Cm)
    return torch.stack(out)


def train_workspace_size(n, d, K):
    b = _sz()
    _check(_lib.soar_train_workspace_size(n, d, K, ctypes.byref(b)), "soar_train_workspace_size")
    return b.value


def _train_ws(n, d, K, dev):
    return torch.empty(max(train_workspace_size(n, d, K), 256), dtype=torch.uint8, device=dev)


def kmeanspp(X, K, seed, stream=None):
    """k-means++ seeding with Philox4x32-10 draws. Returns (C float32[K, d], rows int32[K])."""
    X = _f32_matrix(X, "X")
    n, d = X.shape
    C = torch.empty((K, d), dtype=torch.float32, device=X.device)
    rows = torch.empty(K, dtype=torch.int32, device=X.device)
    ws = _train_ws(n, d, K, X.device)
    _check(_lib.soar_kmeanspp(_ptr(X), n, d, K, int(seed), _ptr(C), _ptr(rows), _ptr(ws),
                              ws.numel(), _stream(stream)), "soar_kmeanspp")
    return C, rows


def lloyd_update(X, labels, C_prev, stream=None):
    """One Lloyd update. Returns (C float32[K, d], counts int32[K])."""
    X, C_prev = _f32_matrix(X, "X"), _f32_matrix(C_prev, "C_prev")
    n, d = X.shape
    K = C_prev.shape[0]
    if labels.dtype != torch.int32 or labels.numel() != n or not labels.is_cuda:
        raise TypeError("labels must be int32[n] on the GPU")
    labels = labels.contiguous()
    C = torch.empty_like(C_prev)
    counts = torch.empty(K, dtype=torch.int32, device=X.device)
    ws = _train_ws(n, d, K, X.device)
    _check(_lib.soar_lloyd_update(_ptr(X), n, d, _ptr(labels), K, _ptr(C_prev), _ptr(C),
                                  _ptr(counts), _ptr(ws), ws.numel(), _stream(stream)),
           "soar_lloyd_update")
    return C, counts


def train_codebook(X, K, iters, seed=0, C_init=None, stream=None):
    """k-means++ (unless C_init) then ``iters`` Lloyd iterations.

    Returns (C float32[K, d], labels int32[n], inertia list of iters + 1 floats)."""
    X = _f32_matrix(X, "X")
    n, d = X.shape
    C = torch.empty((K, d), dtype=torch.float32, device=X.device)
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    inertia = (ctypes.c_double * (iters + 1))()
    ws = _train_ws(n, d, K, X.device)
    ci = None if C_init is None else _f32_matrix(C_init, "C_init")
    _check(_lib.soar_train_codebook(_ptr(X), n, d, K, iters, int(seed), _ptr(ci), _ptr(C),
                                    _ptr(labels), inertia, _ptr(ws), ws.numel(), _stream(stream)),
           "soar_train_codebook")
    return C, labels, list(inertia)


def build_lists(primary, spill, K, stream=None):
    """CSR inverted lists (offsets int64[K + 1], ids int32[n or 2 n]) of the assignments."""
    if primary.dtype != torch.int32 or not primary.is_cuda:
        raise TypeError("primary must be int32 on the GPU")
    n = primary.numel()
    dev = primary.device
    offsets = torch.empty(K + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(n * (2 if spill is not None else 1), dtype=torch.int32, device=dev)
    b = _sz()
    _check(_lib.soar_lists_workspace_size(n, K, ctypes.byref(b)), "soar_lists_workspace_size")
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    _check(_lib.soar_lists_build(_ptr(primary.contiguous()),
                                 None if spill is None else _ptr(spill.contiguous()), n, K,
                                 _ptr(offsets), _ptr(ids), _ptr(ws), ws.numel(), _stream(stream)),
           "soar_lists_build")
    return offsets, ids


def search(Q, C, X, offsets, ids, t, k=10, stream=None, workspace=None):
    """Probe the t best partitions per query and return the k best distinct points:
    (ids int32[nq, k], scores float64[nq, k], searched int64[nq])."""
    Q, C, X = _f32_matrix(Q, "Q"), _f32_matrix(C, "C"), _f32_matrix(X, "X")
    nq, d = Q.shape
    K, n = C.shape[0], X.shape[0]
    dev = Q.device
    out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    out_sc = torch.empty((nq, k), dtype=torch.float64, device=dev)
    searched = torch.empty(nq, dtype=torch.int64, device=dev)
    b = _sz()
    _check(_lib.soar_search_workspace_size(nq, d, K, ctypes.byref(b)), "soar_search_workspace_size")
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    _check(_lib.soar_search(_ptr(Q), nq, d, _ptr(C), K, _ptr(X), n, _ptr(offsets), _ptr(ids),
                            int(t), int(k), _ptr(out_ids), _ptr(out_sc), _ptr(searched),
                            _ptr(workspace), workspace.numel(), _stream(stream)), "soar_search")
    return out_ids, out_sc, searched


def search_two_level(Q, U, upper_offsets, upper_ids, t2, C, X, offsets, ids, t, k=10,
                     stream=None, workspace=None):
    """soar_search_two_level: probe the t2 best upper centroids of U, then the t best of the
    partitions listed under them (upper_offsets / upper_ids: lists of partitions, e.g. from
    build_lists over the partitions' upper assignment), then search their lists as search():
    (ids int32[nq, k], scores float64[nq, k], searched int64[nq])."""
    Q, U, C, X = (_f32_matrix(a, nm) for a, nm in ((Q, "Q"), (U, "U"), (C, "C"), (X, "X")))
    nq, d = Q.shape
    K, K2, n = C.shape[0], U.shape[0], X.shape[0]
    dev = Q.device
    out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    out_sc = torch.empty((nq, k), dtype=torch.float64, device=dev)
    searched = torch.empty(nq, dtype=torch.int64, device=dev)
    b = _sz()
    _check(_lib.soar_search_two_level_workspace_size(nq, d, K, K2, ctypes.byref(b)),
           "soar_search_two_level_workspace_size")
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    _check(_lib.soar_search_two_level(_ptr(Q), nq, d, _ptr(U), K2, _ptr(upper_offsets),
                                      _ptr(upper_ids), int(t2), _ptr(C), K, _ptr(X), n,
                                      _ptr(offsets), _ptr(ids), int(t), int(k), _ptr(out_ids),
                                      _ptr(out_sc), _ptr(searched), _ptr(workspace),
                                      workspace.numel(), _stream(stream)),
           "soar_search_two_level")
    return out_ids, out_sc, searched


def list_codes(offsets, ids, assign, codes, stream=None):
    """soar_lists_codes: the PQ codes of the list entries in list order.  assign int32 [n, m] and
    codes uint8 [n, m, M / 2] (soar_pq_encode) on the GPU.  Returns (list_codes uint8
    [offsets[K], M / 2], max_list: the longest list's length)."""
    if not isinstance(codes, torch.Tensor) or codes.dtype != torch.uint8 or codes.dim() != 3:
        raise TypeError("codes must be a uint8 [n, m, M / 2] tensor")
    n, m, nb = codes.shape
    A = assign.reshape(n, m).contiguous()
    if A.dtype != torch.int32:
        raise TypeError("assign must be int32")
    K = offsets.numel() - 1
    out = torch.empty((ids.numel(), nb), dtype=torch.uint8, device=codes.device)
    ws = torch.empty(256, dtype=torch.uint8, device=codes.device)
    mx = ctypes.c_int64(0)
    _check(_lib.soar_lists_codes(_ptr(offsets), _ptr(ids), K, n, _ptr(A), m,
                                 _ptr(codes.contiguous()), nb, _ptr(out), ctypes.byref(mx),
                                 _ptr(ws), ws.numel(), _stream(stream)), "soar_lists_codes")
    return out, mx.value


def lists_probe_bound(offsets, t, stream=None):
    """soar_lists_probe_bound: the most entries any t of the lists hold."""
    b = ctypes.c_int64(0)
    _check(_lib.soar_lists_probe_bound(_ptr(offsets), offsets.numel() - 1, int(t), ctypes.byref(b),
                                       _stream(stream)), "soar_lists_probe_bound")
    return b.value


def search_pq(Q, C, X, offsets, ids, list_codes_, P, max_probed, t, R, k=10, stream=None,
              workspace=None):
    """soar_search_pq: probe t partitions, estimate every listed copy from its PQ code, re-score
    the R best points exactly and return the k best: (ids int32[nq, k], scores float64[nq, k],
    scored int64[nq]: copies estimated).  P float32 [d / s, 16, s] on the GPU; max_probed bounds
    the entries of any t lists (None: lists_probe_bound)."""
    if max_probed is None:
        max_probed = lists_probe_bound(offsets, min(int(t), offsets.numel() - 1), stream)
    Q, C, X = _f32_matrix(Q, "Q"), _f32_matrix(C, "C"), _f32_matrix(X, "X")
    nq, d = Q.shape
    K, n = C.shape[0], X.shape[0]
    if not isinstance(P, torch.Tensor) or P.dtype != torch.float32 or P.dim() != 3:
        raise TypeError("P must be a float32 [M, 16, s] tensor")
    s = P.shape[2]
    dev = Q.device
    out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    out_sc = torch.empty((nq, k), dtype=torch.float64, device=dev)
    scored = torch.empty(nq, dtype=torch.int64, device=dev)
    b = _sz()
    _check(_lib.soar_search_pq_workspace_size(nq, d, K, int(t), int(max_probed), ctypes.byref(b)),
           "soar_search_pq_workspace_size")
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    _check(_lib.soar_search_pq(_ptr(Q), nq, d, _ptr(C), K, _ptr(X), n, _ptr(offsets), _ptr(ids),
                               _ptr(list_codes_), _ptr(P.contiguous()), s, int(t), int(R), int(k),
                               int(max_probed), _ptr(out_ids), _ptr(out_sc), _ptr(scored),
                               _ptr(workspace), workspace.numel(), _stream(stream)),
           "soar_search_pq")
    return out_ids, out_sc, scored


class SoarIndex:
    """Serving index: resident codebook and inverted lists in a device arena owned by this object.

    insert() queues host rows and returns a ticket at once; wait() returns their (primary, spill)
    indices; list(p) returns the ids in partition p.  All work runs in the library's scheduler
    thread and HIP kernels."""

    def __init__(self, C, lam, precision="bf16", max_step_rows=4096, list_capacity=1 << 20,
                 arena_bytes=None):
        C = _f32_matrix(C, "C")
        self.K, self.d = C.shape
        self.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
        need = _sz()
        _check(_lib.soar_index_arena_size(self.K, self.d, self.precision, int(max_step_rows),
                                          int(list_capacity), ctypes.byref(need)),
               "soar_index_arena_size")
        nbytes = need.value if arena_bytes is None else int(arena_bytes)
        self.arena = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=C.device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(_lib.soar_index_create(_ptr(C), self.K, self.d, float(lam), self.precision,
                                      _ptr(self.arena), self.arena.numel(), int(max_step_rows),
                                      ctypes.byref(h)), "soar_index_create")
        self._h = h
        self._n = {}

    def insert(self, X, first_id):
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float32)
        if X.ndim != 2 or X.shape[1] != self.d:
            raise ValueError("X must be (n, d) float32")
        t = _u64()
        _check(_lib.soar_insert(self._h, X.ctypes.data_as(_vp), X.shape[0], int(first_id),
                                ctypes.byref(t)), "soar_insert")
        self._n[t.value] = X.shape[0]
        return t.value

    def wait(self, ticket, timeout=-1.0):
        import numpy as np
        n = self._n[ticket]
        p = np.empty(n, dtype=np.int32)
        s = np.empty(n, dtype=np.int32)
        st = _lib.soar_wait(self._h, ticket, p.ctypes.data_as(_vp), s.ctypes.data_as(_vp),
                            float(timeout))
        if st != -6:
            self._n.pop(ticket, None)
        _check(st, "soar_wait")
        return p, s

    CHUNK_BYTES = property(lambda self: int(_lib.soar_index_chunk_bytes()))

    def stats(self):
        st = IndexStats()
        st.struct_size = ctypes.sizeof(IndexStats)
        _check(_lib.soar_index_get_stats(self._h, ctypes.byref(st)), "soar_index_get_stats")
        return {f: getattr(st, f) for f, _ in IndexStats._fields_ if f != "struct_size"}

    def list_len(self, part):
        ln = _i64()
        _check(_lib.soar_index_list(self._h, int(part), None, 0, ctypes.byref(ln)),
               "soar_index_list")
        return ln.value

    def list(self, part):
        import numpy as np
        ln = _i64()
        _check(_lib.soar_index_list(self._h, int(part), None, 0, ctypes.byref(ln)),
               "soar_index_list")
        out = np.empty(ln.value, dtype=np.int64)
        if ln.value:
            _check(_lib.soar_index_list(self._h, int(part), out.ctypes.data_as(_vp), ln.value,
                                        ctypes.byref(ln)), "soar_index_list")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.soar_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
