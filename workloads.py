"""Seeded synthetic inputs for NSGA-III environmental selection.

This module only *creates inputs*: merged-population objective matrices and
reference-direction sets.  It holds none of the selection arithmetic, so both
the CPU oracle's tests and the GPU path's tests and benchmark can draw from it
without sharing any method code.

The paper evaluates on DTLZ1 merged populations (merged size 2n, Sec. IV-A.1;
Sec. VI-A; Table S.II settings) whose problem definitions are not part of the
paper.  The generators below stand in for them with DTLZ-shaped "mid-run"
populations: points f = r * u with u a direction in the positive orthant
(sphere-shaped like DTLZ2, or simplex-shaped like DTLZ1) and a radius r >= 1,
a share of the points sitting exactly on the r = 1 front.

Every array is generated in float64 with numpy's PCG64 and cast to float32
once (round-to-nearest-even); that float32 array is what both sides consume.
Reference directions come from the Das-Dennis simplex lattice; the paper treats
them as an input (the reference tensor R with n_r rows, Sec. IV-A.3 and
Algorithm S.4), so how they are built does not affect parity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

__all__ = [
    "Workload", "das_dennis", "two_layer_das_dennis", "sphere_shell",
    "simplex_shell", "make", "make_batch", "CONFIG_NAMES", "batch_instance_specs",
]


# --------------------------------------------------------------------------
# Reference directions
# --------------------------------------------------------------------------
def das_dennis(M: int, p: int) -> np.ndarray:
    """All points of the simplex lattice {i/p : i in N^M, sum i = p}, float64.

    Enumeration order: the first part ascends slowest-varying first
    (i_0 = 0, 1, ..., p), then i_1, ..., the last part is the remainder.
    The count is C(p + M - 1, M - 1).
    """
    out: List[List[int]] = []

    def rec(prefix: List[int], left: int, depth: int) -> None:
        if depth == M - 1:
            out.append(prefix + [left])
            return
        for i in range(left + 1):
            rec(prefix + [i], left - i, depth + 1)

    rec([], p, 0)
    a = np.asarray(out, dtype=np.float64) / float(p)
    assert a.shape[0] == math.comb(p + M - 1, M - 1)
    return a


def two_layer_das_dennis(M: int, p_outer: int, p_inner: int,
                         shrink: float = 0.5) -> np.ndarray:
    """Outer lattice followed by an inner lattice pulled toward the centroid:
    w' = shrink * w + (1 - shrink) / M (a common many-objective construction;
    the 0.5 is this project's choice)."""
    outer = das_dennis(M, p_outer)
    inner = das_dennis(M, p_inner) * shrink + (1.0 - shrink) / M
    return np.concatenate([outer, inner], axis=0)


# --------------------------------------------------------------------------
# Objective matrices
# --------------------------------------------------------------------------
def _front_radius(rng: np.random.Generator, N: int, draw, exact_share: float) -> np.ndarray:
    r = 1.0 + draw(rng, N)
    if exact_share > 0.0:
        k = int(round(exact_share * N))
        idx = rng.permutation(N)[:k]
        r[idx] = 1.0
    return r


def sphere_shell(rng: np.random.Generator, N: int, M: int, radius_draw,
                 exact_share: float = 0.2) -> np.ndarray:
    """f = r * u, u = |g| / ||g||, g ~ N(0, I_M): directions uniform on the
    positive part of the unit sphere (DTLZ2-shaped)."""
    g = np.abs(rng.standard_normal((N, M)))
    u = g / np.linalg.norm(g, axis=1, keepdims=True)
    r = _front_radius(rng, N, radius_draw, exact_share)
    return r[:, None] * u


def simplex_shell(rng: np.random.Generator, N: int, M: int, radius_draw,
                  exact_share: float = 0.0) -> np.ndarray:
    """f = r * u, u = e / sum(e), e ~ Exp(1)^M: directions uniform on the unit
    simplex (DTLZ1-shaped linear front)."""
    e = rng.exponential(1.0, size=(N, M))
    u = e / e.sum(axis=1, keepdims=True)
    r = _front_radius(rng, N, radius_draw, exact_share)
    return r[:, None] * u


def _quantize_256(f: np.ndarray) -> np.ndarray:
    """Round to multiples of 1/256 (half-to-even); exact in float32 for the
    value ranges used here.  Creates duplicate rows and weak dominance."""
    return np.round(f * 256.0) / 256.0


@dataclass
class Workload:
    name: str
    objs: np.ndarray  # (N, M) float32, C-contiguous, minimise
    refs: np.ndarray  # (H, M) float32, C-contiguous, non-negative, nonzero rows
    K: int

    @property
    def N(self) -> int:
        return int(self.objs.shape[0])

    @property
    def M(self) -> int:
        return int(self.objs.shape[1])

    @property
    def H(self) -> int:
        return int(self.refs.shape[0])


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a.astype(np.float32))


_U05 = lambda rng, n: rng.uniform(0.0, 0.5, n)  # noqa: E731
_U03 = lambda rng, n: rng.uniform(0.0, 0.3, n)  # noqa: E731
_EXP4 = lambda rng, n: rng.exponential(1.0 / 4.0, n)  # noqa: E731  rate 4, mean 0.25

_REFS_P = {2: 99, 3: 12, 5: 6}

CONFIG_NAMES = ("small", "ties", "large", "batched", "many")


def make(name: str, N: int | None = None, seed: int | None = None) -> Workload:
    """Build one of the named workloads.

    small : N=200,    M=3,  sphere shell, r = 1 + U(0, 0.5), 20% at r = 1; H=91 (p=12); K=N/2
    ties  : N=20000,  M=3,  as small, quantised to 1/256;                  H=91;        K=N/2
    large : N=200000, M=5,  sphere shell, r = 1 + Exp(rate 4), 20% at r=1; H=210 (p=6); K=N/2
    many  : N=100000, M=10, simplex shell, r = 1 + U(0, 0.3);              H=275 two-layer (3, 2); K=N/2

    ``N`` overrides the size (same recipe, same seed) for scaled-down cases.
    """
    if name == "small":
        s = 1 if seed is None else seed
        n = 200 if N is None else N
        rng = np.random.Generator(np.random.PCG64(s))
        f = sphere_shell(rng, n, 3, _U05, 0.2)
        refs = das_dennis(3, 12)
    elif name == "ties":
        s = 2 if seed is None else seed
        n = 20000 if N is None else N
        rng = np.random.Generator(np.random.PCG64(s))
        f = _quantize_256(sphere_shell(rng, n, 3, _U05, 0.2))
        refs = das_dennis(3, 12)
    elif name == "large":
        s = 3 if seed is None else seed
        n = 200000 if N is None else N
        rng = np.random.Generator(np.random.PCG64(s))
        f = sphere_shell(rng, n, 5, _EXP4, 0.2)
        refs = das_dennis(5, 6)
    elif name == "many":
        s = 5 if seed is None else seed
        n = 100000 if N is None else N
        rng = np.random.Generator(np.random.PCG64(s))
        f = simplex_shell(rng, n, 10, _U03, 0.0)
        refs = two_layer_das_dennis(10, 3, 2)
    else:
        raise ValueError(f"unknown workload {name!r}")
    return Workload(name, _f32(f), _f32(refs), n // 2)


def batch_instance_specs(B: int = 512, n_lo: int = 200, n_hi: int = 20000,
                         base_seed: int = 4000) -> List[tuple]:
    """(seed, N, M) for each instance of the batched workload: N ~ U{n_lo..n_hi},
    M uniform in {2, 3, 5}, both drawn from the instance's own seed."""
    specs = []
    for b in range(B):
        rng = np.random.Generator(np.random.PCG64(base_seed + b))
        n = int(rng.integers(n_lo, n_hi + 1))
        m = int(rng.choice([2, 3, 5]))
        specs.append((base_seed + b, n, m))
    return specs


def make_instance(seed: int, N: int, M: int) -> Workload:
    """One batched instance: quantised sphere shell as in ``ties``, per-instance
    seed; H = 100 (p=99) for M=2, 91 (p=12) for M=3, 210 (p=6) for M=5."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_000))
    f = _quantize_256(sphere_shell(rng, N, M, _U05, 0.2))
    refs = das_dennis(M, _REFS_P[M])
    return Workload(f"inst{seed}", _f32(f), _f32(refs), N // 2)


def make_batch(B: int = 512, n_lo: int = 200, n_hi: int = 20000,
               base_seed: int = 4000) -> List[Workload]:
    return [make_instance(s, n, m) for (s, n, m) in batch_instance_specs(B, n_lo, n_hi, base_seed)]
