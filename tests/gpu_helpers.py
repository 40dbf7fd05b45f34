"""Shared helpers for the GPU parity tests (run the library, compare with the oracle)."""
from __future__ import annotations

import numpy as np

import oracle


def gpu_select(objs: np.ndarray, refs: np.ndarray, K: int, **kw):
    import torch
    import paper_2503_20286_amd as nsga3
    # pass assoc=... (and any other select() keyword) straight through
    o = torch.from_numpy(np.ascontiguousarray(objs, np.float32)).cuda()
    r = torch.from_numpy(np.ascontiguousarray(refs, np.float32)).cuda()
    res = nsga3.select(o, r, K, **kw)
    torch.cuda.synchronize()
    out = dict(
        selected=res.selected.cpu().numpy(),
        rank=res.rank.cpu().numpy(),
        niche=res.niche.cpu().numpy(),
        dist=None if res.dist is None else res.dist.cpu().numpy(),
        dom_in=None if res.dom_in is None else res.dom_in.cpu().numpy(),
        dom_out=None if res.dom_out is None else res.dom_out.cpu().numpy(),
        info=res.info(),
    )
    return out


def dist_close(d_gpu: np.ndarray, d_ref: np.ndarray, fp_norm: np.ndarray) -> np.ndarray:
    """Normalised distances agree within 1e-5 * max(1, ||f'||)."""
    return np.abs(d_gpu.astype(np.float64) - d_ref) <= 1e-5 * np.maximum(1.0, fp_norm)


def line_distance64(objs, z, a, refs, ref_idx):
    """Float64 residual distance ||f' - (f'.r) r|| of each row to reference
    ref_idx[row], summed left to right as the library and the oracle do."""
    f = (objs.astype(np.float64) - z) / a
    R = refs.astype(np.float64)[ref_idx]
    nn = np.zeros(len(f))
    for k in range(R.shape[1]):
        nn = nn + R[:, k] * R[:, k]
    r = R / np.sqrt(nn)[:, None]
    s = np.zeros(len(f))
    for k in range(R.shape[1]):
        s = s + f[:, k] * r[:, k]
    q = np.zeros(len(f))
    for k in range(R.shape[1]):
        e = f[:, k] - s * r[:, k]
        q = q + e * e
    return np.sqrt(q)


def compare_full(objs, refs, K, g, with_counts=True, s=None, niching="exact"):
    """Element-by-element comparison with the oracle's whole selection ``s``
    (computed here when not given) under the niching rule ``niching``
    ("exact": the loop of Alg. S.1, "oneshot": the one-shot form).  Returns a
    dict of mismatch counts (all must be zero) and the number of near-tie
    points."""
    if s is None:
        s = oracle.select(objs, refs, K, with_counts=with_counts, niching=niching)
    pick = oracle.niching if niching == "exact" else (
        lambda *a: oracle.niching_oneshot(*a)[0])
    rep = {}
    rep["rank"] = int(np.sum(g["rank"] != s.rank))
    if with_counts:
        rep["dom_in"] = int(np.sum(g["dom_in"] != s.dom_in))
        rep["dom_out"] = int(np.sum(g["dom_out"] != s.dom_out))
    info = g["info"]
    rep["info"] = int((info.status, info.last_front, info.num_fronts, info.last_front_size,
                       info.num_from_last, info.intercept_fallback) !=
                      (0, s.last_front, s.num_fronts, s.last_front_size, s.num_from_last,
                       s.intercept_fallback))
    # association: exact outside near-ties (oracle gap < 1e-6)
    l = s.last_front
    nz = oracle.normalize(objs, s.rank, l)
    niche, dist, gap = oracle.associate(objs, s.rank, l, nz.z, nz.a, refs)
    S = s.rank <= l
    tie = S & (gap < 1e-6)
    rep["niche"] = int(np.sum((g["niche"] != niche) & ~tie))
    fp = (objs.astype(np.float64) - nz.z) / nz.a
    fpn = np.linalg.norm(fp, axis=1)
    if g["dist"] is not None:
        ok = np.where(S, dist_close(g["dist"], dist, fpn), g["dist"] == -1.0)
        rep["dist"] = int(np.sum(~ok & ~tie))
    if not np.any(tie):
        rep["selected"] = _sel_mismatch(g["selected"], s.selected)
    else:
        # stage-wise: oracle niching on the GPU's association, with the float64
        # distance of each near-tie point to the reference the GPU chose
        rho = oracle.niche_count(g["rank"], g["niche"], l, refs.shape[0])
        d64 = np.where(S, dist, -1.0)
        moved = tie & (g["niche"] != niche)
        if np.any(moved):
            d64[moved] = line_distance64(objs[moved], nz.z, nz.a, refs, g["niche"][moved])
        chosen = pick(g["rank"], g["niche"], d64, l, refs.shape[0], s.num_from_last, rho)
        want = np.nonzero((g["rank"] < l) | chosen)[0]
        rep["selected"] = _sel_mismatch(g["selected"], want)
    rep["near_ties"] = int(np.sum(tie))
    return rep


def _sel_mismatch(got, want):
    """Number of indices in one selection and not the other (0 iff equal)."""
    if got.shape == want.shape and np.array_equal(got, want):
        return 0
    return int(np.setxor1d(got, want).size) or 1
