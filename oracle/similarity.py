"""Similarity, tie-break noise, median preference and net similarity in FP64 (test infrastructure).

* Similarity (Section 2): s_ij = -||x_i - x_j||^2, the negative squared Euclidean
  distance, computed here from the direct differences in FP64.
* Tie-break noise (a reading: the paper breaks no ties): for i != j,
      s_ij <- s_ij + (rel * |s_ij|) * u_ij,
  u_ij = (splitmix64(seed XOR (i*N + j)) >> 11) * 2^-53, where splitmix64(x) is
  the first output of a SplitMix64 generator started at state x (Steele, Lea and
  Flood, OOPSLA 2014): z = x + 0x9E3779B97F4A7C15, then
  z = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z = (z ^ z>>27) * 0x94D049BB133111EB,
  z ^ z>>31, all modulo 2^64.
* Preference (Section 2 discusses data-driven constant preferences; a reading):
  the median of the N(N-1) off-diagonal entries, i.e. the mean of the two middle
  order statistics v[M/2-1] and v[M/2] (M even), formed in FP64 and rounded to
  the working precision.
* Net similarity (the AP objective; not defined in the paper): NS^l = sum_i s^l_{i,e_i},
  where s^l_ii is the preference p^l_i.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """First output of SplitMix64 started at state x (Python integers, exact)."""
    z = (x + _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64_np(x: np.ndarray) -> np.ndarray:
    """Vectorised splitmix64 over a uint64 array (wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def noise_uniform(seed: int, n: int, rows=None) -> np.ndarray:
    """u_ij in [0, 1) for the given rows (all rows by default), shape (len(rows), n)."""
    rows = np.arange(n) if rows is None else np.asarray(rows)
    ctr = rows.astype(np.uint64)[:, None] * np.uint64(n) + np.arange(n, dtype=np.uint64)[None, :]
    z = splitmix64_np(ctr ^ np.uint64(seed & _MASK))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def similarity(X: np.ndarray, squared: bool = True) -> np.ndarray:
    """s_ij = -sum_k (x_ik - x_jk)^2 in FP64 (diagonal 0); squared=False gives the negative
    Euclidean distance -sqrt(sum_k (x_ik - x_jk)^2) the paper uses for images (Section 4)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    S = np.zeros((n, n))
    for k in range(d):
        diff = X[:, k][:, None] - X[:, k][None, :]
        S = S + diff * diff
    return -S if squared else -np.sqrt(S)


def similarity_rows(X: np.ndarray, rows, squared: bool = True) -> np.ndarray:
    """Rows `rows` of similarity(X), with the same arithmetic (FP64, coordinates in order),
    for problems too large to hold the whole matrix."""
    X = np.asarray(X, dtype=np.float64)
    rows = np.asarray(rows)
    S = np.zeros((rows.size, X.shape[0]))
    for k in range(X.shape[1]):
        diff = X[rows, k][:, None] - X[:, k][None, :]
        S = S + diff * diff
    return -S if squared else -np.sqrt(S)


def add_noise(S: np.ndarray, rel: float, seed: int) -> np.ndarray:
    """Off-diagonal tie-break noise: s_ij + (rel * |s_ij|) * u_ij (FP64)."""
    S = np.array(S, dtype=np.float64, copy=True)
    n = S.shape[0]
    u = noise_uniform(seed, n)
    t = rel * np.abs(S)
    t = t * u
    off = ~np.eye(n, dtype=bool)
    S[off] = S[off] + t[off]
    return S


def median_offdiag(S: np.ndarray, dtype=np.float64):
    """Median of the off-diagonal entries of S, as stored in `dtype`.

    The order statistics are taken on the values in `dtype`; their mean is formed
    in FP64 and rounded once to `dtype`.
    """
    S = np.asarray(S).astype(dtype)
    n = S.shape[0]
    v = np.sort(S[~np.eye(n, dtype=bool)].astype(np.float64))
    M = v.size
    lo, hi = v[M // 2 - 1], v[M // 2]
    return dtype((lo + hi) / 2.0)


def net_similarity(S: np.ndarray, pref_l, labels_l: np.ndarray) -> float:
    """NS = sum_i s_{i, e_i} with s_ii = p_i, accumulated in FP64."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    p = np.broadcast_to(np.asarray(pref_l, dtype=np.float64), (n,))
    e = np.asarray(labels_l)
    vals = S[np.arange(n), e]
    self_ = e == np.arange(n)
    vals = np.where(self_, p, vals)
    return float(np.sum(vals))
