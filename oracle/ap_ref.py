"""Plain Affinity Propagation (Frey and Dueck, Science 2007) in FP64 (test infrastructure).

Written on its own, in the AP paper's notation, so that the HAP oracle can be
checked against it: the paper presents HAP as AP extended with tiered levels
(Section 2), and with one level HAP must reduce to this.

  r(i,k) <- s(i,k) - max_{k' != k} [a(i,k') + s(i,k')]
  a(i,k) <- min{0, r(k,k) + sum_{i' not in {i,k}} max{0, r(i',k)}}   (i != k)
  a(k,k) <- sum_{i' != k} max{0, r(i',k)}
Both messages are damped: m <- lam * m_old + (1 - lam) * m_new, and a is
computed from the damped r.  The exemplar of i is argmax_k [a(i,k) + r(i,k)]
(lowest index on ties).
"""
from __future__ import annotations

import numpy as np


def affinity_propagation(S, pref, damping, iters):
    """S: (N, N) similarity (diagonal replaced by pref); returns (labels, r, a)."""
    s = np.array(S, dtype=np.float64, copy=True)
    n = s.shape[0]
    s[np.diag_indices(n)] = pref
    r = np.zeros((n, n))
    a = np.zeros((n, n))
    for _ in range(iters):
        # responsibilities: the best competitor of column k is the row maximum unless
        # k itself is the maximiser, in which case it is the runner-up.
        r_new = np.empty((n, n))
        for i in range(n):
            row = a[i] + s[i]
            order = np.argsort(-row, kind="stable")
            best, second = row[order[0]], row[order[1]]
            r_new[i] = s[i] - best
            r_new[i, order[0]] = s[i, order[0]] - second
        r = damping * r + (1.0 - damping) * r_new
        # availabilities, column by column
        a_new = np.empty((n, n))
        for k in range(n):
            col = r[:, k]
            pos = np.where(col > 0.0, col, 0.0)
            pos_sum_others = pos.sum() - pos[k]          # sum over i' != k of max(0, r(i',k))
            for i in range(n):
                if i == k:
                    a_new[k, k] = pos_sum_others
                else:
                    a_new[i, k] = min(0.0, r[k, k] + pos_sum_others - pos[i])
        a = damping * a + (1.0 - damping) * a_new
    labels = np.argmax(a + r, axis=1)
    return labels, r, a
