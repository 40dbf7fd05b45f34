"""Independent brute-force references used to pin the CPU oracle.

Written directly from the definitions, in NumPy / plain Python, for tiny inputs
only.  Nothing here is shared with the oracle or with the GPU library.
"""
from __future__ import annotations

import functools

import numpy as np


def dominance_matrix(F: np.ndarray) -> np.ndarray:
    """D[i, j] = F_i dominates F_j: broadcast form of Listing 1 / Eq. (6)."""
    F = np.asarray(F, dtype=np.float64)
    P1 = F[:, None, :]
    P2 = F[None, :, :]
    return np.all(P1 <= P2, axis=2) & np.any(P1 < P2, axis=2)


def deb_fronts(F: np.ndarray) -> np.ndarray:
    """Fast nondominated sort with dominated sets and counters (Alg. S.2),
    written as plain loops.  Returns 0-based ranks."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]

    def dom(a, b):
        return bool(np.all(F[a] <= F[b]) and np.any(F[a] < F[b]))

    S = [[] for _ in range(n)]
    cnt = [0] * n
    rank = [-1] * n
    front = []
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            if dom(i, j):
                S[i].append(j)
            elif dom(j, i):
                cnt[i] += 1
        if cnt[i] == 0:
            rank[i] = 0
            front.append(i)
    k = 0
    while front:
        nxt = []
        for i in front:
            for j in S[i]:
                cnt[j] -= 1
                if cnt[j] == 0:
                    rank[j] = k + 1
                    nxt.append(j)
        k += 1
        front = nxt
    return np.asarray(rank, dtype=np.int32)


def longest_chain_ranks(F: np.ndarray) -> np.ndarray:
    """rank[j] = length of the longest dominance chain ending in j (memoised
    recursion over the dominance matrix)."""
    D = dominance_matrix(F)
    n = D.shape[0]

    @functools.lru_cache(maxsize=None)
    def r(j):
        doms = np.nonzero(D[:, j])[0]
        return 0 if doms.size == 0 else 1 + max(r(int(i)) for i in doms)

    return np.asarray([r(j) for j in range(n)], dtype=np.int32)


def ranks_2d_sweep(F: np.ndarray) -> np.ndarray:
    """Textbook two-objective sort: visit points in lexicographic (f1, f2)
    order; a point joins the first front whose most recently added member
    does not dominate it (that member has the front's smallest f2)."""
    F = np.asarray(F, dtype=np.float64)
    assert F.shape[1] == 2
    order = np.lexsort((F[:, 1], F[:, 0]))
    tails = []  # last member of each front
    rank = np.empty(F.shape[0], np.int32)

    def dom(a, b):
        return (F[a, 0] <= F[b, 0] and F[a, 1] <= F[b, 1]) and (F[a, 0] < F[b, 0] or F[a, 1] < F[b, 1])

    for q in order:
        k = 0
        while k < len(tails) and dom(tails[k], q):
            k += 1
        if k == len(tails):
            tails.append(q)
        else:
            tails[k] = q
        rank[q] = k
    return rank


def paper_distance(fp: np.ndarray, refs: np.ndarray) -> np.ndarray:
    """Eq. (10) as printed: ||F'|| * sqrt(1 - (F' R^T / (||F'|| ||R||))^2), float64."""
    fp = np.asarray(fp, dtype=np.float64)
    R = np.asarray(refs, dtype=np.float64)
    nf = np.linalg.norm(fp, axis=1, keepdims=True)
    nr = np.linalg.norm(R, axis=1)[None, :]
    cos = (fp @ R.T) / (nf * nr)
    return nf * np.sqrt(np.clip(1.0 - cos * cos, 0.0, None))


def keysort_niching(rank, niche, dist, l, rho, R):
    """Parallel form of the niching loop: last-front member i gets the key
    (rho[niche_i] + t_i, niche_i), t_i its position among the same reference's
    last-front members ordered by (distance, index); the R smallest keys win."""
    idx = np.nonzero(np.asarray(rank) == l)[0]
    keys = []
    by_ref = {}
    for i in idx:
        by_ref.setdefault(int(niche[i]), []).append(int(i))
    for j, members in by_ref.items():
        members.sort(key=lambda i: (float(dist[i]), i))
        for t, i in enumerate(members):
            keys.append(((int(rho[j]) + t, j), i))
    keys.sort()
    chosen = np.zeros(len(rank), bool)
    for _, i in keys[:R]:
        chosen[i] = True
    return chosen
