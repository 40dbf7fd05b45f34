"""CPU oracle for NSGA-III environmental selection -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``oracle.c`` (plain float64 C, OpenMP over host
cores).  Only the tests, the smoke check and the benchmark's CPU-baseline leg
use it; the GPU library never imports, links or calls anything here, and this
package imports nothing from the GPU library.

Every function mirrors one stage of the selection and cites the paper passage
it follows in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from .build import build as _build, LIB_PATH

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int
    L.oracle_dominates.argtypes = [P, i32, i64, i64]
    L.oracle_dominance.argtypes = [P, i64, i32, P, P]
    L.oracle_dominance_one.argtypes = [P, i64, i32, i64, P, P]
    L.oracle_ranks.argtypes = [P, i64, i32, P, P]
    L.oracle_last_front.argtypes = [P, i64, i64, P, P, P]
    L.oracle_normalize.argtypes = [P, i64, i32, P, ctypes.c_int32, P, P, P, P]
    L.oracle_associate.argtypes = [P, i64, i32, P, ctypes.c_int32, P, P, P, i32, P, P, P]
    L.oracle_niche_count.argtypes = [P, P, i64, ctypes.c_int32, i32, P]
    L.oracle_niching.argtypes = [P, P, P, i64, ctypes.c_int32, i32, i64, P, P]
    L.oracle_niching_oneshot.argtypes = [P, P, P, i64, ctypes.c_int32, i32, i64, P, P, P]
    L.oracle_select.argtypes = [P, i64, i32, P, i32, i64, P, P, P, P, P, P, P]
    L.oracle_select_mode.argtypes = [P, i64, i32, P, i32, i64, i32, P, P, P, P, P, P, P]
    L.oracle_num_threads.argtypes = []
    L.oracle_sbx_pm.argtypes = [P, i64, i32, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    L.oracle_sbx_pm.restype = ctypes.c_int
    L.oracle_gather_rows.argtypes = [P, i64, i32, P, i64, P]
    L.oracle_gather_rows.restype = ctypes.c_int
    L.oracle_hype_alpha.argtypes = [i64, i64, P]
    L.oracle_hype_alpha.restype = ctypes.c_int
    L.oracle_hype_hv.argtypes = [P, i64, i32, P, P, i64, i64, P, P]
    L.oracle_hype_hv.restype = ctypes.c_int
    L.oracle_hype_select.argtypes = [P, i64, i32, P, P, i64, i64, P, P, P, P]
    L.oracle_hype_select.restype = ctypes.c_int
    L.oracle_rvea_gamma.argtypes = [P, i32, i32, P]
    L.oracle_rvea_gamma.restype = ctypes.c_int
    L.oracle_rvea_select.argtypes = [P, i64, i32, P, i32, i64, i64, ctypes.c_double, P, P, P, P, P]
    L.oracle_rvea_select.restype = ctypes.c_int
    L.oracle_set_num_threads.argtypes = [i32]
    L.oracle_set_num_threads.restype = None
    for name in ("oracle_dominates", "oracle_dominance", "oracle_dominance_one", "oracle_ranks",
                 "oracle_last_front", "oracle_normalize", "oracle_associate",
                 "oracle_niche_count", "oracle_niching", "oracle_niching_oneshot",
                 "oracle_select", "oracle_select_mode", "oracle_num_threads"):
        getattr(L, name).restype = ctypes.c_int


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc} ({'invalid argument' if rc == -1 else 'non-finite input'})")


def _objs(objs):
    a = np.ascontiguousarray(objs, dtype=np.float32)
    if a.ndim != 2:
        raise ValueError("objs must be (N, M)")
    return a


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for later oracle calls from this thread (n < 1: one per core)."""
    lib().oracle_set_num_threads(int(n))


def dominance(objs):
    """(dom_in, dom_out): number of dominators of / points dominated by each point."""
    f = _objs(objs)
    N, M = f.shape
    din = np.zeros(N, np.int32)
    dout = np.zeros(N, np.int32)
    _check(lib().oracle_dominance(_ptr(f), N, M, _ptr(din), _ptr(dout)), "oracle_dominance")
    return din, dout


def dominance_one(objs, j):
    f = _objs(objs)
    N, M = f.shape
    a = ctypes.c_int32()
    b = ctypes.c_int32()
    _check(lib().oracle_dominance_one(_ptr(f), N, M, int(j), ctypes.byref(a), ctypes.byref(b)),
           "oracle_dominance_one")
    return a.value, b.value


def dominates(objs, i, j) -> bool:
    f = _objs(objs)
    return bool(lib().oracle_dominates(_ptr(f), f.shape[1], int(i), int(j)))


def ranks(objs):
    """(rank int32[N], number of fronts): rank = longest dominance chain ending at the point."""
    f = _objs(objs)
    N, M = f.shape
    r = np.zeros(N, np.int32)
    L = ctypes.c_int32()
    _check(lib().oracle_ranks(_ptr(f), N, M, _ptr(r), ctypes.byref(L)), "oracle_ranks")
    return r, L.value


def last_front(rank, K):
    r = np.ascontiguousarray(rank, dtype=np.int32)
    l = ctypes.c_int32()
    nb = ctypes.c_int64()
    nl = ctypes.c_int64()
    _check(lib().oracle_last_front(_ptr(r), r.size, int(K), ctypes.byref(l), ctypes.byref(nb),
                                   ctypes.byref(nl)), "oracle_last_front")
    return l.value, nb.value, nl.value


@dataclass
class Normalization:
    z: np.ndarray
    a: np.ndarray
    extreme: np.ndarray
    fallback: int


def normalize(objs, rank, l):
    f = _objs(objs)
    N, M = f.shape
    r = np.ascontiguousarray(rank, dtype=np.int32)
    z = np.zeros(M, np.float64)
    a = np.zeros(M, np.float64)
    e = np.zeros(M, np.int32)
    fb = ctypes.c_int32()
    _check(lib().oracle_normalize(_ptr(f), N, M, _ptr(r), int(l), _ptr(z), _ptr(a), _ptr(e),
                                  ctypes.byref(fb)), "oracle_normalize")
    return Normalization(z, a, e, fb.value)


def associate(objs, rank, l, z, a, refs):
    """(niche int32[N], dist float64[N], gap float64[N]); -1 outside S."""
    f = _objs(objs)
    N, M = f.shape
    R = np.ascontiguousarray(refs, dtype=np.float32)
    r = np.ascontiguousarray(rank, dtype=np.int32)
    z = np.ascontiguousarray(z, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    niche = np.zeros(N, np.int32)
    dist = np.zeros(N, np.float64)
    gap = np.zeros(N, np.float64)
    _check(lib().oracle_associate(_ptr(f), N, M, _ptr(r), int(l), _ptr(z), _ptr(a), _ptr(R),
                                  R.shape[0], _ptr(niche), _ptr(dist), _ptr(gap)),
           "oracle_associate")
    return niche, dist, gap


def niche_count(rank, niche, l, H):
    r = np.ascontiguousarray(rank, dtype=np.int32)
    n = np.ascontiguousarray(niche, dtype=np.int32)
    rho = np.zeros(H, np.int32)
    _check(lib().oracle_niche_count(_ptr(r), _ptr(n), r.size, int(l), int(H), _ptr(rho)),
           "oracle_niche_count")
    return rho


def niching(rank, niche, dist, l, H, R, rho):
    """bool[N]: last-front members picked by the niche-preserving loop."""
    r = np.ascontiguousarray(rank, dtype=np.int32)
    n = np.ascontiguousarray(niche, dtype=np.int32)
    d = np.ascontiguousarray(dist, dtype=np.float64)
    rh = np.ascontiguousarray(rho, dtype=np.int32)
    chosen = np.zeros(r.size, np.uint8)
    _check(lib().oracle_niching(_ptr(r), _ptr(n), _ptr(d), r.size, int(l), int(H), int(R),
                                _ptr(rh), _ptr(chosen)), "oracle_niching")
    return chosen.astype(bool)


def niching_oneshot(rank, niche, dist, l, H, R, rho):
    """(bool[N] admitted last-front members, |E|) of the one-shot niche selection."""
    r = np.ascontiguousarray(rank, dtype=np.int32)
    n = np.ascontiguousarray(niche, dtype=np.int32)
    d = np.ascontiguousarray(dist, dtype=np.float64)
    rh = np.ascontiguousarray(rho, dtype=np.int32)
    chosen = np.zeros(r.size, np.uint8)
    ne = ctypes.c_int64()
    _check(lib().oracle_niching_oneshot(_ptr(r), _ptr(n), _ptr(d), r.size, int(l), int(H), int(R),
                                        _ptr(rh), _ptr(chosen), ctypes.byref(ne)),
           "oracle_niching_oneshot")
    return chosen.astype(bool), ne.value


NICHING = {"exact": 0, "oneshot": 1}


@dataclass
class Selection:
    selected: np.ndarray
    rank: np.ndarray
    niche: np.ndarray
    dist: np.ndarray
    dom_in: np.ndarray | None
    dom_out: np.ndarray | None
    last_front: int
    num_fronts: int
    last_front_size: int
    num_from_last: int
    intercept_fallback: int
    near_ties: int


def select(objs, refs, K, with_counts=True, niching="exact"):
    """Whole environmental selection on the CPU (float64).  niching: "exact"
    (the loop of Alg. S.1) or "oneshot" (the one-shot form of Alg. S.4)."""
    f = _objs(objs)
    N, M = f.shape
    R = np.ascontiguousarray(refs, dtype=np.float32)
    sel = np.zeros(K, np.int32)
    rank = np.zeros(N, np.int32)
    niche = np.zeros(N, np.int32)
    dist = np.zeros(N, np.float64)
    din = np.zeros(N, np.int32) if with_counts else None
    dout = np.zeros(N, np.int32) if with_counts else None
    info = np.zeros(6, np.int64)
    _check(lib().oracle_select_mode(_ptr(f), N, M, _ptr(R), R.shape[0], int(K), NICHING[niching],
                                    _ptr(sel), _ptr(rank), _ptr(niche), _ptr(dist), _ptr(din),
                                    _ptr(dout), _ptr(info)),
           "oracle_select_mode")
    return Selection(sel, rank, niche, dist, din, dout, *[int(v) for v in info])


# ---------------------------------------------------------------------------
# TensorRVEA environmental selection (Supplementary Sec. S.V, Alg. S.12)
# ---------------------------------------------------------------------------
def rvea_gamma(refs):
    """gamma[H]: smallest angle between each reference vector and any other."""
    R = np.ascontiguousarray(refs, dtype=np.float32)
    g = np.zeros(R.shape[0], np.float64)
    _check(lib().oracle_rvea_gamma(_ptr(R), R.shape[0], R.shape[1], _ptr(g)), "oracle_rvea_gamma")
    return g


@dataclass
class RveaSelection:
    elite: np.ndarray    # int32[H]: the partition's smallest-APD point, -1 if empty
    assign: np.ndarray   # int32[N]: partition (reference with the smallest angle)
    apd: np.ndarray      # float64[N]: angle-penalized distance
    theta: np.ndarray    # float64[N]: angle to the own reference
    gap: np.ndarray      # float64[H]: relative gap between the two smallest APDs


def rvea_select(objs, refs, t, t_max, alpha=2.0):
    f = _objs(objs)
    N, M = f.shape
    R = np.ascontiguousarray(refs, dtype=np.float32)
    H = R.shape[0]
    elite = np.zeros(H, np.int32)
    assign = np.zeros(N, np.int32)
    apd = np.zeros(N, np.float64)
    theta = np.zeros(N, np.float64)
    gap = np.zeros(H, np.float64)
    _check(lib().oracle_rvea_select(_ptr(f), N, M, _ptr(R), H, int(t), int(t_max), float(alpha),
                                    _ptr(elite), _ptr(assign), _ptr(apd), _ptr(theta), _ptr(gap)),
           "oracle_rvea_select")
    return RveaSelection(elite, assign, apd, theta, gap)


# ---------------------------------------------------------------------------
# TensorHypE environmental selection (Sec. IV-C; Supplementary Alg. S.10/S.11)
# ---------------------------------------------------------------------------
def hype_alpha(k, N):
    """alpha_c for c = 1..k (float64[k])."""
    a = np.zeros(max(int(k), 1), np.float64)
    _check(lib().oracle_hype_alpha(int(k), int(N), _ptr(a)), "oracle_hype_alpha")
    return a[:int(k)]


def hype_hv(objs, vref, U, k):
    """(HV estimate float64[N], sample dominance counts int32[s]) for a given k."""
    f = _objs(objs)
    N, M = f.shape
    v = np.ascontiguousarray(vref, dtype=np.float32)
    u = np.ascontiguousarray(U, dtype=np.float32)
    hv = np.zeros(N, np.float64)
    cnt = np.zeros(u.shape[0], np.int32)
    _check(lib().oracle_hype_hv(_ptr(f), N, M, _ptr(v), _ptr(u), u.shape[0], int(k), _ptr(hv),
                                _ptr(cnt)), "oracle_hype_hv")
    return hv, cnt


@dataclass
class HypeSelection:
    selected: np.ndarray   # int32[n], ascending
    d: np.ndarray          # float64[N]: HV estimate for rank <= l, -inf elsewhere
    rank: np.ndarray
    last_front: int
    num_fronts: int
    k: int
    last_front_size: int


def hype_select(objs, vref, U, n):
    f = _objs(objs)
    N, M = f.shape
    v = np.ascontiguousarray(vref, dtype=np.float32)
    u = np.ascontiguousarray(U, dtype=np.float32)
    sel = np.zeros(int(n), np.int32)
    d = np.zeros(N, np.float64)
    rank = np.zeros(N, np.int32)
    info = np.zeros(4, np.int64)
    _check(lib().oracle_hype_select(_ptr(f), N, M, _ptr(v), _ptr(u), u.shape[0], int(n), _ptr(sel),
                                    _ptr(d), _ptr(rank), _ptr(info)), "oracle_hype_select")
    return HypeSelection(sel, d, rank, *[int(x) for x in info])


# ---------------------------------------------------------------------------
# Variation (Supplementary Sec. S.I: SBX and polynomial mutation) and the
# gather of the selected rows (Eq. (13))
# ---------------------------------------------------------------------------
def sbx_pm(X, lower, upper, eta_c, eta_m, r_sbx, r_pm):
    """float64[2h, d] offspring: SBX children of rows r and h + r, clipped,
    then polynomially mutated (every variable)."""
    x = np.ascontiguousarray(X, dtype=np.float32)
    n, d = x.shape
    h = n // 2
    lo = np.ascontiguousarray(lower, dtype=np.float32)
    hi = np.ascontiguousarray(upper, dtype=np.float32)
    rs = np.ascontiguousarray(r_sbx, dtype=np.float32)
    rp = np.ascontiguousarray(r_pm, dtype=np.float32)
    out = np.zeros((2 * h, d), np.float64)
    _check(lib().oracle_sbx_pm(_ptr(x), n, d, _ptr(lo), _ptr(hi), float(eta_c), float(eta_m),
                               _ptr(rs), _ptr(rp), _ptr(out)), "oracle_sbx_pm")
    return out


def gather_rows(X, idx):
    x = np.ascontiguousarray(X, dtype=np.float32)
    i = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.zeros((i.size, x.shape[1]), np.float32)
    _check(lib().oracle_gather_rows(_ptr(x), x.shape[0], x.shape[1], _ptr(i), i.size, _ptr(out)),
           "oracle_gather_rows")
    return out
