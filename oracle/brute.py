"""Exhaustive exemplar-set search for tiny inputs (test infrastructure).

Affinity Propagation maximises the net similarity of an exemplar set X:
    E(X) = sum_{k in X} p_k + sum_{i not in X} max_{k in X} s_ik,
every exemplar being its own exemplar and every other point joining the most
similar exemplar.  For N <= 14 all 2^N - 1 non-empty sets are enumerated.
"""
from __future__ import annotations

import itertools

import numpy as np


def best_exemplar_set(S, pref):
    """Return (labels, value) of the optimal set; labels[i] = exemplar of point i."""
    s = np.array(S, dtype=np.float64, copy=True)
    n = s.shape[0]
    if n > 14:
        raise ValueError("brute force is for N <= 14")
    p = np.broadcast_to(np.asarray(pref, dtype=np.float64), (n,))
    best_val, best_set = -np.inf, None
    for size in range(1, n + 1):
        for X in itertools.combinations(range(n), size):
            Xa = np.array(X)
            val = p[Xa].sum()
            others = np.setdiff1d(np.arange(n), Xa)
            if others.size:
                val += s[np.ix_(others, Xa)].max(axis=1).sum()
            if val > best_val:
                best_val, best_set = val, Xa
    labels = np.empty(n, dtype=np.int64)
    for i in range(n):
        if i in best_set:
            labels[i] = i
        else:
            labels[i] = best_set[np.argmax(s[i, best_set])]
    return labels, best_val
