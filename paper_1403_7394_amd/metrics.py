"""Clustering diagnostics on the host (evaluation only; not part of the method's path).

purity (the extrinsic quality measure the paper reports, Section 4): the fraction of points
whose cluster's most frequent generating class is their own class,
    purity = (1/N) * sum over clusters k of max over classes c of |cluster_k intersect class_c|.
adjusted_rand_index: agreement of two partitions corrected for chance (Hubert and Arabie,
1985), in pair-counting form.
"""
from __future__ import annotations

import numpy as np


def _contingency(a, b) -> np.ndarray:
    _, ia = np.unique(np.asarray(a), return_inverse=True)
    _, ib = np.unique(np.asarray(b), return_inverse=True)
    cont = np.zeros((ia.max() + 1, ib.max() + 1), dtype=np.int64)
    np.add.at(cont, (ia, ib), 1)
    return cont


def purity(labels, truth) -> float:
    labels = np.asarray(labels)
    if labels.size == 0:
        raise ValueError("purity of an empty labelling")
    return float(_contingency(labels, truth).max(axis=1).sum() / labels.size)


def adjusted_rand_index(a, b) -> float:
    cont = _contingency(a, b)
    comb = lambda x: x * (x - 1) / 2.0
    s_ij = comb(cont).sum()
    s_a = comb(cont.sum(axis=1)).sum()
    s_b = comb(cont.sum(axis=0)).sum()
    tot = comb(float(np.asarray(a).size))
    expected = s_a * s_b / tot
    top = 0.5 * (s_a + s_b)
    return float((s_ij - expected) / (top - expected)) if top != expected else 1.0
