"""ctypes marshalling for libnsga3.so.  No computation happens here."""
from __future__ import annotations

import ctypes
import os
import re
import threading
from dataclasses import dataclass
from typing import Dict, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "nsga3.h")


def lib_path() -> str:
    return os.environ.get("NSGA3_LIB", os.path.join(HERE, "libnsga3.so"))


STATUS = {0: "NSGA3_OK", -1: "NSGA3_E_INVALID", -2: "NSGA3_E_NONFINITE", -3: "NSGA3_E_NOMEM",
          -4: "NSGA3_E_HIP", -5: "NSGA3_E_UNSUPPORTED"}
OK, E_INVALID, E_NONFINITE, E_NOMEM, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
NUM_PHASES = 6
PHASES = ("prep_sort", "dominance_count", "peel", "normalize", "associate", "niching")
ASSOC_FP32 = 0
ASSOC_BF16 = 1
NICHING_EXACT = 0
NICHING_ONESHOT = 1


class NativeError(RuntimeError):
    def __init__(self, what: str, code: int, lib=None):
        msg = STATUS.get(code, str(code))
        if lib is not None:
            try:
                msg += ": " + lib.nsga3_status_string(code).decode()
            except Exception:  # pragma: no cover - best effort
                pass
        super().__init__(f"{what} failed ({msg})")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("assoc", ctypes.c_int), ("autotune", ctypes.c_int32),
                ("max_workspace_bytes", ctypes.c_size_t), ("niching", ctypes.c_int)]


PLAN_STAGES = ("keys_refs", "radix_hist", "radix_scatter", "records", "dominance",
               "split_count", "split_write", "peel_decrements", "orig_order", "extremes",
               "association", "bucket_scatter", "niche_picks", "compact_count", "compact_write",
               "split_one", "peel_tail", "rank_2d", "front_tables", "done")


class _Problem(ctypes.Structure):
    _fields_ = [("objs", ctypes.c_void_p), ("N", ctypes.c_int64), ("M", ctypes.c_int32),
                ("refs", ctypes.c_void_p), ("H", ctypes.c_int32), ("K", ctypes.c_int64),
                ("selected", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("niche", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("dom_in", ctypes.c_void_p), ("dom_out", ctypes.c_void_p),
                ("info", ctypes.c_void_p)]


INFO_FIELDS = ("status", "last_front", "num_fronts", "last_front_size", "num_from_last",
               "intercept_fallback", "near_ties", "reserved")

_lib = None
_lock = threading.Lock()


def load():
    """Load libnsga3.so (built by paper_2503_20286_amd.build); raise if absent."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = lib_path()
        if not os.path.exists(path):
            raise ImportError(f"libnsga3.so not found at {path}: build it first "
                              "(python -m paper_2503_20286_amd.build or __graft_entry__.build())")
        L = ctypes.CDLL(path)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.nsga3_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(_Options)]
        L.nsga3_create.restype = ctypes.c_int
        L.nsga3_destroy.argtypes = [P]
        L.nsga3_destroy.restype = None
        L.nsga3_reserve.argtypes = [P, i64, i32, i32]
        L.nsga3_reserve.restype = ctypes.c_int
        L.nsga3_workspace_size.argtypes = [i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.nsga3_workspace_size.restype = ctypes.c_int
        L.nsga3_select.argtypes = [P, P, i64, i32, P, i32, i64, P, P, P, P, P, P, P, P]
        L.nsga3_select.restype = ctypes.c_int
        L.nsga3_select_noalloc.argtypes = [P, i64, i32, P, i32, i64, P, P, P, P, P, P, P, P]
        L.nsga3_select_noalloc.restype = ctypes.c_int
        L.nsga3_rvea_select.argtypes = [P, P, i64, i32, P, i32, i64, i64, ctypes.c_double, P, P, P,
                                        P, P]
        L.nsga3_hype_select.argtypes = [P, P, i64, i32, P, P, i64, i64, P, P, P, P, P]
        L.nsga3_hype_select.restype = ctypes.c_int
        L.nsga3_sbx_pm.argtypes = [P, i64, i32, P, P, ctypes.c_double, ctypes.c_double, P, P, P, P, P]
        L.nsga3_sbx_pm.restype = ctypes.c_int
        L.nsga3_gather_rows.argtypes = [P, i64, i32, P, i64, P, P, P]
        L.nsga3_gather_rows.restype = ctypes.c_int
        L.nsga3_rvea_select.restype = ctypes.c_int
        L.nsga3_status_string.argtypes = [ctypes.c_int]
        L.nsga3_status_string.restype = ctypes.c_char_p
        L.nsga3_profile.argtypes = [P, ctypes.c_int]
        L.nsga3_profile.restype = ctypes.c_int
        L.nsga3_phase_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.nsga3_phase_times.restype = ctypes.c_int
        L.nsga3_plan_create.argtypes = [P, ctypes.POINTER(_Problem), i32, ctypes.POINTER(P)]
        L.nsga3_plan_create.restype = ctypes.c_int
        L.nsga3_plan_launch.argtypes = [P, P]
        L.nsga3_plan_launch.restype = ctypes.c_int
        L.nsga3_plan_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.nsga3_plan_info.restype = ctypes.c_int
        L.nsga3_plan_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]
        L.nsga3_plan_stage_times.restype = ctypes.c_int
        L.nsga3_tuned_shapes.argtypes = [P, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
        L.nsga3_tuned_shapes.restype = ctypes.c_int
        L.nsga3_tuned_save.argtypes = [P, ctypes.c_char_p]
        L.nsga3_tuned_save.restype = ctypes.c_int
        L.nsga3_tuned_load.argtypes = [P, ctypes.c_char_p]
        L.nsga3_tuned_load.restype = ctypes.c_int
        L.nsga3_plan_destroy.argtypes = [P]
        L.nsga3_plan_destroy.restype = None
        L.nsga3_version.argtypes = []
        L.nsga3_version.restype = ctypes.c_int32
        _lib = L
        return L


def version() -> int:
    return int(load().nsga3_version())


def workspace_size(N: int, M: int, H: int) -> int:
    """Bytes of context workspace a single selection of this size needs."""
    L = load()
    b = ctypes.c_size_t()
    rc = L.nsga3_workspace_size(int(N), int(M), int(H), ctypes.byref(b))
    if rc != 0:
        raise NativeError("nsga3_workspace_size", rc, L)
    return int(b.value)


def header_symbols():
    """Function names declared by include/nsga3.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsga3_[a-z_]+)\s*\(", text)))


def exported_symbols():
    """Which header-declared functions the shared library exports (name -> bool)."""
    L = load()
    out = {}
    for name in header_symbols():
        try:
            getattr(L, name)
            out[name] = True
        except AttributeError:
            out[name] = False
    return out


class Context:
    """Owns an nsga3_ctx (device workspace) on one HIP device."""

    def __init__(self, device: int = 0, assoc: int = ASSOC_FP32, max_workspace_bytes: int = 0,
                 autotune: bool = False, niching: int = NICHING_EXACT):
        self._lib = load()
        opt = _Options(assoc, 1 if autotune else 0, max_workspace_bytes, niching)
        h = ctypes.c_void_p()
        rc = self._lib.nsga3_create(ctypes.byref(h), int(device), ctypes.byref(opt))
        if rc != 0:
            raise NativeError("nsga3_create", rc, self._lib)
        self._h = h
        self.device = int(device)
        self.assoc = assoc
        self.niching = niching

    @property
    def handle(self):
        return self._h

    def reserve(self, N: int, M: int, H: int) -> None:
        rc = self._lib.nsga3_reserve(self._h, int(N), int(M), int(H))
        if rc != 0:
            raise NativeError("nsga3_reserve", rc, self._lib)

    def profile(self, enable: bool) -> None:
        rc = self._lib.nsga3_profile(self._h, 1 if enable else 0)
        if rc != 0:
            raise NativeError("nsga3_profile", rc, self._lib)

    def tuned_shapes(self):
        """Autotuned engine shapes: list of dicts (M, n_range, pa_items, tail_max, tail_front)."""
        cnt = ctypes.c_int32()
        rc = self._lib.nsga3_tuned_shapes(self._h, None, 0, ctypes.byref(cnt))
        if rc != 0:
            raise NativeError("nsga3_tuned_shapes", rc, self._lib)
        buf = (ctypes.c_int32 * (5 * max(cnt.value, 1)))()
        rc = self._lib.nsga3_tuned_shapes(self._h, buf, cnt.value, ctypes.byref(cnt))
        if rc != 0:
            raise NativeError("nsga3_tuned_shapes", rc, self._lib)
        keys = ("M", "n_range", "pa_items", "tail_max", "tail_front")
        return [dict(zip(keys, buf[5 * q:5 * q + 5])) for q in range(cnt.value)]

    def save_tuned(self, path):
        """Write the tuned shapes to a text file (nsga3_tuned_save)."""
        rc = self._lib.nsga3_tuned_save(self._h, os.fsencode(path))
        if rc != 0:
            raise NativeError("nsga3_tuned_save", rc, self._lib)

    def load_tuned(self, path):
        """Merge tuned shapes from a file written by save_tuned (nsga3_tuned_load)."""
        rc = self._lib.nsga3_tuned_load(self._h, os.fsencode(path))
        if rc != 0:
            raise NativeError("nsga3_tuned_load", rc, self._lib)

    def phase_times(self):
        """(per-phase summed milliseconds, number of calls) since profiling was enabled."""
        ms = (ctypes.c_double * NUM_PHASES)()
        calls = ctypes.c_int64()
        rc = self._lib.nsga3_phase_times(self._h, ms, ctypes.byref(calls))
        if rc != 0:
            raise NativeError("nsga3_phase_times", rc, self._lib)
        return [float(x) for x in ms], int(calls.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.nsga3_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Dict[tuple, Context] = {}


def default_context(device: int, assoc: int = ASSOC_FP32, niching: int = NICHING_EXACT) -> Context:
    key = (device, assoc, niching)
    if key not in _default_ctx:
        _default_ctx[key] = Context(device, assoc, niching=niching)
    return _default_ctx[key]


@dataclass
class Info:
    status: int
    last_front: int
    num_fronts: int
    last_front_size: int
    num_from_last: int
    intercept_fallback: int
    near_ties: int
    device_err_bits: int


@dataclass
class Selection:
    selected: "object"
    rank: "object"
    niche: "object"
    dist: "object"
    dom_in: "object"
    dom_out: "object"
    info_raw: "object"

    def info(self) -> Info:
        """Copies the device-side nsga3_info to the host (synchronises)."""
        v = [int(x) for x in self.info_raw.cpu().tolist()]
        return Info(*v)


def _check_tensor(t, name, ndim):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a HIP device")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != ndim or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {ndim}-D tensor")


def select(objs, refs, K: int, *, ctx: Optional[Context] = None, assoc: int = ASSOC_FP32,
           niching: int = NICHING_EXACT, want_counts: bool = True, want_dist: bool = True,
           out: Optional[Selection] = None, stream=None) -> Selection:
    """Environmental selection of K of the N rows of ``objs`` (N x M float32,
    minimised) with reference directions ``refs`` (H x M float32).  Returns
    device tensors; the call is asynchronous on the current (or given) stream."""
    import torch
    _check_tensor(objs, "objs", 2)
    _check_tensor(refs, "refs", 2)
    if objs.device != refs.device:
        raise ValueError("objs and refs must be on the same device")
    N, M = objs.shape
    H = refs.shape[0]
    if refs.shape[1] != M:
        raise ValueError("refs must have M columns")
    dev = objs.device
    if ctx is None:
        ctx = default_context(dev.index if dev.index is not None else torch.cuda.current_device(),
                              assoc, niching)
    if out is None:
        i32 = dict(dtype=torch.int32, device=dev)
        out = Selection(
            selected=torch.empty(int(K), **i32) if K >= 1 else torch.empty(1, **i32),
            rank=torch.empty(N, **i32),
            niche=torch.empty(N, **i32),
            dist=torch.empty(N, dtype=torch.float32, device=dev) if want_dist else None,
            dom_in=torch.empty(N, **i32) if want_counts else None,
            dom_out=torch.empty(N, **i32) if want_counts else None,
            info_raw=torch.zeros(8, **i32),
        )
    s = stream if stream is not None else torch.cuda.current_stream(dev)

    def p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    rc = ctx._lib.nsga3_select(ctx.handle, p(objs), int(N), int(M), p(refs), int(H), int(K),
                               p(out.selected), p(out.rank), p(out.niche), p(out.dist),
                               p(out.dom_in), p(out.dom_out), p(out.info_raw),
                               ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_select", rc, ctx._lib)
    return out


def select_noalloc(objs, refs, K: int, *, out: Selection, stream=None) -> Selection:
    """The allocation-free entry point (nsga3_select_noalloc): same results as
    select() with float32 screening, into the caller's ``out`` buffers (see
    ``alloc_outputs``), on the current device; the library allocates nothing.
    Raises NativeError (code NSGA3_E_NOMEM) when the problem's workspace is
    larger than the library's fixed scratch array."""
    import torch
    _check_tensor(objs, "objs", 2)
    _check_tensor(refs, "refs", 2)
    N, M = objs.shape
    H = refs.shape[0]
    if refs.shape[1] != M:
        raise ValueError("refs must have M columns")
    s = stream if stream is not None else torch.cuda.current_stream(objs.device)
    L = load()

    def p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    rc = L.nsga3_select_noalloc(p(objs), int(N), int(M), p(refs), int(H), int(K),
                                p(out.selected), p(out.rank), p(out.niche), p(out.dist),
                                p(out.dom_in), p(out.dom_out), p(out.info_raw),
                                ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_select_noalloc", rc, L)
    return out


@dataclass
class RveaSelection:
    elite: "object"      # int32[H]
    assign: "object"     # int32[N]
    apd: "object"        # float64[N]
    info_raw: "object"

    def info(self) -> Info:
        v = [int(x) for x in self.info_raw.cpu().tolist()]
        return Info(*v)


def rvea_select(objs, refs, t: int, t_max: int, alpha: float = 2.0, *,
                ctx: Optional[Context] = None, stream=None) -> RveaSelection:
    """TensorRVEA environmental selection (nsga3_rvea_select): the elite of
    every reference vector's partition by angle-penalized distance."""
    import torch
    _check_tensor(objs, "objs", 2)
    _check_tensor(refs, "refs", 2)
    N, M = objs.shape
    H = refs.shape[0]
    if refs.shape[1] != M:
        raise ValueError("refs must have M columns")
    dev = objs.device
    if ctx is None:
        ctx = default_context(dev.index if dev.index is not None else torch.cuda.current_device())
    out = RveaSelection(elite=torch.empty(H, dtype=torch.int32, device=dev),
                        assign=torch.empty(N, dtype=torch.int32, device=dev),
                        apd=torch.empty(N, dtype=torch.float64, device=dev),
                        info_raw=torch.zeros(8, dtype=torch.int32, device=dev))
    s = stream if stream is not None else torch.cuda.current_stream(dev)

    def p(t_):
        return ctypes.c_void_p(t_.data_ptr())

    rc = ctx._lib.nsga3_rvea_select(ctx.handle, p(objs), int(N), int(M), p(refs), int(H), int(t),
                                    int(t_max), float(alpha), p(out.elite), p(out.assign),
                                    p(out.apd), p(out.info_raw), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_rvea_select", rc, ctx._lib)
    return out


@dataclass
class HypeSelection:
    selected: "object"   # int32[n], ascending
    d: "object"          # float64[N]: HV estimate for rank <= l, -inf elsewhere
    rank: "object"       # int32[N]
    info_raw: "object"

    def info(self) -> Info:
        v = [int(x) for x in self.info_raw.cpu().tolist()]
        return Info(*v)


def hype_select(objs, vref, U, n: int, *, ctx: Optional[Context] = None,
                stream=None) -> HypeSelection:
    """TensorHypE environmental selection (nsga3_hype_select): keep n of the
    N rows of ``objs``, the last front by Monte Carlo hypervolume estimates
    from the caller's uniform draws ``U`` (s x M) and reference point ``vref``."""
    import torch
    _check_tensor(objs, "objs", 2)
    _check_tensor(U, "U", 2)
    _check_tensor(vref, "vref", 1)
    N, M = objs.shape
    if U.shape[1] != M or vref.shape[0] != M:
        raise ValueError("U must have M columns and vref M entries")
    dev = objs.device
    if ctx is None:
        ctx = default_context(dev.index if dev.index is not None else torch.cuda.current_device())
    out = HypeSelection(selected=torch.empty(int(n), dtype=torch.int32, device=dev),
                        d=torch.empty(N, dtype=torch.float64, device=dev),
                        rank=torch.empty(N, dtype=torch.int32, device=dev),
                        info_raw=torch.zeros(8, dtype=torch.int32, device=dev))
    s = stream if stream is not None else torch.cuda.current_stream(dev)

    def p(t_):
        return ctypes.c_void_p(t_.data_ptr())

    rc = ctx._lib.nsga3_hype_select(ctx.handle, p(objs), int(N), int(M), p(vref), p(U),
                                    int(U.shape[0]), int(n), p(out.selected), p(out.d), p(out.rank),
                                    p(out.info_raw), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_hype_select", rc, ctx._lib)
    return out


def sbx_pm(X, lower, upper, eta_c: float, eta_m: float, r_sbx, r_pm, *, out=None, status=None,
           stream=None):
    """Simulated binary crossover and polynomial mutation (nsga3_sbx_pm):
    offspring of the n x d population X from the caller's uniform draws
    (r_sbx: h x d, r_pm: 2h x d, h = n // 2).  Returns (offspring, status)."""
    import torch
    for t_, nm in ((X, "X"), (r_sbx, "r_sbx"), (r_pm, "r_pm")):
        _check_tensor(t_, nm, 2)
    _check_tensor(lower, "lower", 1)
    _check_tensor(upper, "upper", 1)
    n, d = X.shape
    h = n // 2
    if tuple(r_sbx.shape) != (h, d) or tuple(r_pm.shape) != (2 * h, d):
        raise ValueError("r_sbx must be (n//2, d) and r_pm (2*(n//2), d)")
    if lower.shape[0] != d or upper.shape[0] != d:
        raise ValueError("bounds must have d entries")
    dev = X.device
    if out is None:
        out = torch.empty((2 * h, d), dtype=torch.float32, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    L = load()
    rc = L.nsga3_sbx_pm(ctypes.c_void_p(X.data_ptr()), int(n), int(d), ctypes.c_void_p(lower.data_ptr()),
                        ctypes.c_void_p(upper.data_ptr()), float(eta_c), float(eta_m),
                        ctypes.c_void_p(r_sbx.data_ptr()), ctypes.c_void_p(r_pm.data_ptr()),
                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                        ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_sbx_pm", rc, L)
    return out, status


def gather_rows(X, idx, *, out=None, status=None, stream=None):
    """Rows idx of X (nsga3_gather_rows, Eq. (13)).  Returns (rows, status)."""
    import torch
    _check_tensor(X, "X", 2)
    if idx.dtype != torch.int32 or idx.device != X.device or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous int32 tensor on X's device")
    N, d = X.shape
    K = idx.shape[0]
    if out is None:
        out = torch.empty((K, d), dtype=torch.float32, device=X.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    s = stream if stream is not None else torch.cuda.current_stream(X.device)
    L = load()
    rc = L.nsga3_gather_rows(ctypes.c_void_p(X.data_ptr()), int(N), int(d),
                             ctypes.c_void_p(idx.data_ptr()), int(K), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise NativeError("nsga3_gather_rows", rc, L)
    return out, status


def alloc_outputs(N: int, K: int, device, want_counts: bool = True,
                  want_dist: bool = True) -> Selection:
    """Output tensors for one selection of K of N points on ``device``."""
    return _alloc_outputs(N, K, device, want_counts, want_dist)


def _alloc_outputs(N, K, dev, want_counts=True, want_dist=True):
    import torch
    i32 = dict(dtype=torch.int32, device=dev)
    return Selection(
        selected=torch.empty(int(K), **i32),
        rank=torch.empty(N, **i32),
        niche=torch.empty(N, **i32),
        dist=torch.empty(N, dtype=torch.float32, device=dev) if want_dist else None,
        dom_in=torch.empty(N, **i32) if want_counts else None,
        dom_out=torch.empty(N, **i32) if want_counts else None,
        info_raw=torch.zeros(8, **i32),
    )


class Plan:
    """A batched plan: many independent selections captured into one HIP graph.

    ``problems`` is a list of (objs, refs, K) with device float32 tensors; the
    plan allocates one output Selection per problem (``results``) and keeps
    every buffer alive.  ``launch()`` replays the graph; rewrite the input
    tensors in place to select on new data."""

    def __init__(self, problems, ctx: Optional[Context] = None, want_counts: bool = True,
                 want_dist: bool = True):
        import torch
        if not problems:
            raise ValueError("empty batch")
        dev = problems[0][0].device
        self.ctx = ctx if ctx is not None else default_context(
            dev.index if dev.index is not None else torch.cuda.current_device())
        self._lib = self.ctx._lib
        self.inputs = []
        self.results = []
        descs = (_Problem * len(problems))()
        for b, (objs, refs, K) in enumerate(problems):
            _check_tensor(objs, "objs", 2)
            _check_tensor(refs, "refs", 2)
            N, M = objs.shape
            out = _alloc_outputs(N, K, dev, want_counts, want_dist)
            self.inputs.append((objs, refs))
            self.results.append(out)

            def ptr(t):
                return None if t is None else t.data_ptr()
            descs[b] = _Problem(ptr(objs), int(N), int(M), ptr(refs), int(refs.shape[0]), int(K),
                                ptr(out.selected), ptr(out.rank), ptr(out.niche), ptr(out.dist),
                                ptr(out.dom_in), ptr(out.dom_out), ptr(out.info_raw))
        h = ctypes.c_void_p()
        rc = self._lib.nsga3_plan_create(self.ctx.handle, descs, len(problems), ctypes.byref(h))
        if rc != 0:
            raise NativeError("nsga3_plan_create", rc, self._lib)
        self._h = h

    def info(self):
        b = ctypes.c_int32()
        n = ctypes.c_int64()
        rc = self._lib.nsga3_plan_info(self._h, ctypes.byref(b), ctypes.byref(n))
        if rc != 0:
            raise NativeError("nsga3_plan_info", rc, self._lib)
        return {"branches": b.value, "nodes": n.value}

    def stage_times(self):
        """Engine diagnostics (plan created while ctx profiling was on): per
        stage block-ms in items and epilogues, item counts; probe / idle block-ms."""
        n = len(PLAN_STAGES)
        it = (ctypes.c_double * n)()
        ep = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        pr = ctypes.c_double()
        idl = ctypes.c_double()
        rc = self._lib.nsga3_plan_stage_times(self._h, it, ep, cnt, ctypes.byref(pr), ctypes.byref(idl))
        if rc != 0:
            raise NativeError("nsga3_plan_stage_times", rc, self._lib)
        return {"stages": {PLAN_STAGES[q]: {"item_ms": it[q], "epilogue_ms": ep[q], "items": cnt[q]}
                           for q in range(n) if cnt[q] or ep[q]},
                "probe_ms": pr.value, "idle_ms": idl.value}

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = self._lib.nsga3_plan_launch(self._h, ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise NativeError("nsga3_plan_launch", rc, self._lib)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nsga3_plan_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
