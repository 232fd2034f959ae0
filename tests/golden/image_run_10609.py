"""Writes image_run_10609_oracle_float32.npz: the oracle's run of the image-style workload at the
size of the paper's first image (103 x 103 = 10,609 RGB pixels from 16 colour blobs, negative
Euclidean distance, preferences U[-1e6, 0] per point, L = 3, damping 0.5, 30 iterations;
Section 4), evaluated with every operation rounded to FP32, with the labels and the FP64 net
similarity of every level at a few checkpoint iterations.

Calls only the oracle and the seeded input generators.  About ten minutes on one core.
Usage: python tests/golden/image_run_10609.py
"""
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import hap_ref  # noqa: E402
from oracle import similarity as sim  # noqa: E402
from paper_1403_7394_amd import synth  # noqa: E402

CHECKPOINTS = (5, 10, 20, 30)


def main() -> int:
    b, prefs, rp = synth.workload_image("mandrill")
    n, L = b.X.shape[0], rp.levels
    S32 = sim.similarity(b.X, squared=False).astype(np.float32)
    p32 = prefs.astype(np.float32)
    S64 = S32.astype(np.float64)
    snaps = {}
    t0 = time.perf_counter()

    def record(t, l, st):
        if l == L - 1 and t in CHECKPOINTS:
            snaps[t] = hap_ref.labels_of(st).astype(np.int32)
            print(f"t={t} exemplars per level {[len(np.unique(e)) for e in snaps[t]]} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)

    res = hap_ref.hap(S32, p32, L, rp.damping, rp.max_iters, record=record, dtype=np.float32)
    ts = np.array(sorted(snaps), dtype=np.int32)
    lab = np.stack([snaps[t] for t in ts])
    ns = np.array([[sim.net_similarity(S64, p32.astype(np.float64), lab[k, l]) for l in range(L)]
                   for k in range(ts.size)])
    out = Path(__file__).with_name("image_run_10609_oracle_float32.npz")
    np.savez_compressed(out, checkpoints=ts, labels=lab, net_similarity=ns, n=np.int32(n),
                        iters=np.int32(res.iters), seconds=np.float64(time.perf_counter() - t0))
    print(f"wrote {out.name}: {res.iters} iterations", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
