"""The 8192-point 2-D workload over its whole run on the GPU, against the oracle's labels.

The run is the benchmark's: FP32, L = 3, damping 0.9, median preference, points mode, the
default launch, 500 iterations (this workload does not meet the stop rule).  The expected
labels at checkpoint iterations come from `tests/golden/full_run_plain8192_oracle_*.npz`,
written by `tests/golden/full_run_plain8192.py` from the oracle alone, once evaluated in FP64
and once with every operation rounded to FP32 (same steps, same order).

Bars, taken from how far the two oracle evaluations themselves lie apart:
- up to iteration 100 the messages are still contracting: at every level the GPU labels agree
  with the FP64 oracle's on at least as many points as the FP32 evaluation's do, less 0.1% of
  the points, and on at least 99% of them;
- later the L = 3 run oscillates without settling (the exemplar counts rise and fall by tens
  of percent between checkpoints in every evaluation), and runs that differ only in rounding
  order drift apart in phase: the FP32 and FP64 oracle evaluations part at the top level, and
  GPU runs that differ only in rows per workgroup (the order of the column sums) part from
  each other as much as from the oracle.  There the test checks what holds for any run in the
  same regime: labels are column indices, and every level's exemplar count lies within a
  factor of two of the range the oracle runs visit over their late checkpoints.
"""
from pathlib import Path

import numpy as np
import pytest
import torch

from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLD = Path(__file__).resolve().parent / "golden"


def _oracle(dtype):
    with np.load(GOLD / f"full_run_plain8192_oracle_{dtype}.npz") as z:
        return {k: z[k] for k in z.files}


def _agree(x, y):
    return np.array([float(np.mean(x[l] == y[l])) for l in range(x.shape[0])])


def test_full_run_against_oracle_labels(hap_gpu):
    o64, o32 = _oracle("float64"), _oracle("float32")
    ts = [int(t) for t in o64["checkpoints"]]
    assert ts == [int(t) for t in o32["checkpoints"]]
    b, rp = synth.workload_plain_f32()
    n, L = b.X.shape[0], rp.levels
    X = torch.from_numpy(b.X).to(DEV)
    S = torch.empty((n, n), dtype=torch.float32, device=DEV)
    hap_gpu.build_similarity(X, S)
    h = hap_gpu.Hap(S, L, rp.damping)
    h.set_points(X)
    assert h.preference() == [float(o64["pref"])] * L
    got = {}
    prev = 0
    for t in ts:
        h.iterate(t - prev, 0)
        prev = t
        got[t] = (h.labels().cpu().numpy(), [h.net_similarity(l) for l in range(L)])
    h.close()

    late = [k for k, t in enumerate(ts) if t > 100]
    counts = np.array([[len(np.unique(o["labels"][k][l])) for l in range(L)] for o in (o64, o32) for k in late])
    lo, hi = counts.min(axis=0), counts.max(axis=0)
    for k, t in enumerate(ts):
        g, ns = got[t]
        assert g.shape == (L, n) and g.min() >= 0 and g.max() < n
        ref64, ref32 = o64["labels"][k], o32["labels"][k]
        a_gpu, a_32 = _agree(g, ref64), _agree(ref32, ref64)
        print(f"t={t}: agreement with FP64 oracle {np.round(a_gpu, 4)} (FP32 oracle {np.round(a_32, 4)}), "
              f"exemplars {[len(np.unique(g[l])) for l in range(L)]}, NS {np.round(ns, 1)} "
              f"(oracle {np.round(o64['net_similarity'][k], 1)})")
        if t <= 100:
            assert np.all(a_gpu >= np.minimum(a_32, 1.0) - 1e-3), (t, a_gpu, a_32)
            assert np.all(a_gpu >= 0.99), (t, a_gpu)
        else:
            cnt = np.array([len(np.unique(g[l])) for l in range(L)])
            assert np.all(cnt >= lo / 2) and np.all(cnt <= hi * 2), (t, cnt, lo, hi)


def test_full_run_row_ordered_launch_is_the_fp32_oracle(hap_gpu):
    """The benchmark's run (points mode, 500 iterations) with one row per workgroup, which sums
    every column in row order as the FP32 evaluation of the oracle does: labels identical to
    the stored FP32 oracle labels at every checkpoint, net similarity within 1e-12."""
    o32 = _oracle("float32")
    ts = [int(t) for t in o32["checkpoints"]]
    b, rp = synth.workload_plain_f32()
    n, L = b.X.shape[0], rp.levels
    X = torch.from_numpy(b.X).to(DEV)
    S = torch.empty((n, n), dtype=torch.float32, device=DEV)
    hap_gpu.build_similarity(X, S)
    h = hap_gpu.Hap(S, L, rp.damping)
    h.set_points(X)
    h.set_launch(rows_per_block=1)
    assert h.get_launch()[2] == 1
    assert h.preference() == [float(o32["pref"])] * L
    prev = 0
    for k, t in enumerate(ts):
        h.iterate(t - prev, 0)
        prev = t
        g = h.labels().cpu().numpy()
        ns = np.array([h.net_similarity(l) for l in range(L)])
        ref = o32["labels"][k]
        print(f"t={t}: exemplars {[len(np.unique(g[l])) for l in range(L)]}, "
              f"equal to the FP32 oracle: {[bool(np.array_equal(g[l], ref[l])) for l in range(L)]}", flush=True)
        assert np.array_equal(g, ref), (t, _agree(g, ref))
        assert np.all(np.abs(ns - o32["net_similarity"][k]) <= 1e-12 * np.abs(o32["net_similarity"][k])), t
    h.close()
