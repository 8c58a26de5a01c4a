"""Seeded synthetic inputs for all-pairs Pearson correlation.

This module only draws random numbers.  It holds none of the correlation
method's arithmetic (no centring, no scaling, no dot products), so that both
the FP64 oracle and the HIP path can consume the very same arrays without
sharing any code that computes a result.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``) and
produces data in FP64 first; the device dtype is reached by one cast.

Workload recipes (the paper's own data are artificial uniform matrices and a
microarray compendium that is not available here; these shapes stand in for
them, see the evaluation section of the paper):

* ``planted``: entries i.i.d. N(0,1); ``n_planted`` disjoint row pairs
  (u, v) are drawn with ``rng.choice(n, 2*n_planted, replace=False)``, and the
  v row is overwritten by ``a*u + b + 0.1*eps`` with ``a = +-U[0.5, 2]``
  (sign equiprobable), ``b ~ U[-1, 1]`` and ``eps ~ N(0, 1)``.
* ``expression``: latent ``w ~ N(0,1)``; ``n_modules`` disjoint modules of
  ``module_size`` genes share a factor ``f_m ~ N(0,1)``:
  ``w_g = lam_g*f_m + sqrt(1-lam_g^2)*eps_g`` with ``lam_g ~ U[0.6, 0.95]``;
  value ``log2(1 + exp(2 + 1.5*w))`` (log-normal counts, log2 scale).
* ``uniform_matrix``: entries i.i.d. U[0, 1], the paper's artificial data
  (its Table I runs n = 16,000, 32,000 and 64,000 profiles of l = 5,000);
  ``table3_shape``: an expression-shaped stand-in with the shape of the
  paper's real compendium (17,555 x 5,072), whose values are not available.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

# Seeds of the five standard workloads.
SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5}


@dataclasses.dataclass
class Planted:
    u: np.ndarray      # int64 row index of the source row of each planted pair
    v: np.ndarray      # int64 row index of the dependent row
    a: np.ndarray      # slope of each planted pair


def planted(n: int, l: int, seed: int, n_planted: int = 20,
            dtype=np.float64, rng: Optional[np.random.Generator] = None,
            chunk_rows: int = 4096) -> Tuple[np.ndarray, Planted]:
    """N(0,1) matrix (n x l, row-major) with ``n_planted`` planted pairs."""
    if rng is None:
        rng = np.random.default_rng(seed)
    X = np.empty((n, l), dtype=dtype)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        X[r0:r1] = rng.standard_normal((r1 - r0, l))
    k = min(n_planted, n // 2)
    sel = rng.choice(n, 2 * k, replace=False).astype(np.int64)
    u, v = sel[0::2].copy(), sel[1::2].copy()
    sign = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    a = sign * rng.uniform(0.5, 2.0, k)
    b = rng.uniform(-1.0, 1.0, k)
    for t in range(k):
        eps = rng.standard_normal(l)
        row = a[t] * X[u[t]].astype(np.float64) + b[t] + 0.1 * eps
        X[v[t]] = row.astype(dtype)
    return X, Planted(u=u, v=v, a=a)


def expression(n: int, l: int, seed: int, n_modules: int = 50,
               module_size: int = 40, dtype=np.float32,
               chunk_rows: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    """Expression-shaped matrix; returns (X, modules[n_modules, module_size])."""
    rng = np.random.default_rng(seed)
    W = np.empty((n, l), dtype=np.float64)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        W[r0:r1] = rng.standard_normal((r1 - r0, l))
    mods = rng.choice(n, n_modules * module_size, replace=False).astype(np.int64)
    mods = mods.reshape(n_modules, module_size)
    for m in range(n_modules):
        f = rng.standard_normal(l)
        lam = rng.uniform(0.6, 0.95, module_size)
        for g in range(module_size):
            eps = rng.standard_normal(l)
            W[mods[m, g]] = lam[g] * f + np.sqrt(1.0 - lam[g] ** 2) * eps
    X = np.empty((n, l), dtype=dtype)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        X[r0:r1] = np.log2(1.0 + np.exp(2.0 + 1.5 * W[r0:r1]))
    return X, mods


def permutations(P: int, l: int, seed: int) -> np.ndarray:
    """P seeded permutations of range(l), int32, shape (P, l)."""
    rng = np.random.default_rng(seed)
    out = np.empty((P, l), dtype=np.int32)
    for p in range(P):
        out[p] = rng.permutation(l)
    return out


def check_blocks(n: int, nblocks: int = 256, bs: int = 128,
                 seed: int = 0) -> np.ndarray:
    """``nblocks`` seeded bs x bs blocks drawn uniformly from the inclusive
    upper block triangle of an n x n pair matrix; rows of (block_y, block_x)."""
    rng = np.random.default_rng(seed)
    mb = (n + bs - 1) // bs
    total = mb * (mb + 1) // 2
    picks = rng.choice(total, min(nblocks, total), replace=False)
    # enumerate the inclusive block triangle row by row (plain loops)
    coords = np.empty((total, 2), dtype=np.int64)
    t = 0
    for by in range(mb):
        for bx in range(by, mb):
            coords[t] = (by, bx)
            t += 1
    return coords[np.sort(picks)]


def block_pairs(n: int, blocks: np.ndarray, bs: int = 128) -> Tuple[np.ndarray, np.ndarray]:
    """All (i, j) with i < j < n inside the given blocks."""
    I_all, J_all = [], []
    for by, bx in blocks:
        ii = np.arange(by * bs, min(n, (by + 1) * bs), dtype=np.int64)
        jj = np.arange(bx * bs, min(n, (bx + 1) * bs), dtype=np.int64)
        I, J = np.meshgrid(ii, jj, indexing="ij")
        keep = I < J
        I_all.append(I[keep])
        J_all.append(J[keep])
    return np.concatenate(I_all), np.concatenate(J_all)


def random_pairs(n: int, count: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """``count`` seeded distinct-pair samples (i < j), not necessarily unique."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, count)
    j = rng.integers(0, n - 1, count)
    j = np.where(j >= i, j + 1, j)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    return lo.astype(np.int64), hi.astype(np.int64)


# --------------------------------------------------------------------------
# The five standard workloads.

def config1() -> Tuple[np.ndarray, Planted]:
    """n=2000 x l=256, FP64, N(0,1) with 20 planted pairs."""
    return planted(2000, 256, SEEDS[1], dtype=np.float64)


def config2() -> Tuple[np.ndarray, np.ndarray]:
    """n=16384 x l=1024 FP32 expression-shaped with 50 modules of 40 genes."""
    return expression(16384, 1024, SEEDS[2], dtype=np.float32)


def config3(n: int = 32768, l: int = 4096) -> Tuple[np.ndarray, Planted]:
    """n=32768 x l=4096 FP32, the config-1 distribution."""
    return planted(n, l, SEEDS[3], dtype=np.float32)


def config4(n: int = 8192, l: int = 512, P: int = 1000):
    """n=8192 x l=512 FP32 (config-1 distribution) and P permutations."""
    X, pl = planted(n, l, SEEDS[4], dtype=np.float32)
    perms = permutations(P, l, SEEDS[4] + 1000)
    return X, pl, perms


def config5_shapes(D: int = 64) -> List[Tuple[int, int]]:
    rng = np.random.default_rng(SEEDS[5])
    ns = rng.integers(500, 8001, D)
    ls = rng.integers(50, 2001, D)
    return [(int(a), int(b)) for a, b in zip(ns, ls)]


def config5_batch(D: int = 64):
    """64 datasets of uneven (n, l), each in the config-1 distribution."""
    out = []
    for d, (n, l) in enumerate(config5_shapes(D)):
        X, pl = planted(n, l, SEEDS[5] * 1000 + d, dtype=np.float32)
        out.append((X, pl))
    return out


def config5_big(n: int = 65536, l: int = 2048) -> Tuple[np.ndarray, Planted]:
    """One n=65536 x l=2048 FP32 matrix in the config-1 distribution."""
    return planted(n, l, SEEDS[5] + 100, dtype=np.float32)


# Table I of the paper: n profiles of 5,000 samples drawn uniformly from [0, 1].
TABLE1_SIZES = (16000, 32000, 64000)
TABLE1_L = 5000


def uniform_matrix(n: int, l: int, seed: int) -> np.ndarray:
    """n x l FP64 entries i.i.d. U[0, 1]."""
    return np.random.default_rng(seed).random((n, l))


def table1(n: int) -> np.ndarray:
    """The paper's Table I workload with n profiles (FP64, seeded by n)."""
    return uniform_matrix(n, TABLE1_L, 6000 + n // 1000)


# Table III of the paper runs a 17,555 x 5,072 microarray compendium, which is
# not available; an expression-shaped matrix of that shape stands in for it.
TABLE3_SHAPE = (17555, 5072)


def table3_shape() -> np.ndarray:
    """Expression-shaped FP64 matrix with the shape of the paper's real data."""
    return expression(TABLE3_SHAPE[0], TABLE3_SHAPE[1], 7000, dtype=np.float64)[0]
