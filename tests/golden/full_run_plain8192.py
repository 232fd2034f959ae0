"""Writes full_run_plain8192_oracle_<dtype>.npz: the oracle's labels over a whole run of the
8192-point 2-D workload (64 blobs, FP32 points, L = 3, damping 0.9, median preference, up to
500 iterations or 50 stable), at a few checkpoint iterations.

Calls only the oracle and the seeded point generator.  About 20 minutes on one core (FP64).
Usage: python tests/golden/full_run_plain8192.py [float64|float32]
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

CHECKPOINTS = (3, 10, 50, 100, 200, 300, 500)


def main() -> int:
    dt = np.dtype(sys.argv[1] if len(sys.argv) > 1 else "float64")
    b, rp = synth.workload_plain_f32()
    S32 = sim.similarity(b.X).astype(np.float32)
    p = np.float32(sim.median_offdiag(S32, np.float32))
    S = S32.astype(dt)
    L = rp.levels
    snaps = {}

    out = Path(__file__).with_name(f"full_run_plain8192_oracle_{dt.name}.npz")
    S64 = S32.astype(np.float64)
    t0 = time.perf_counter()

    def save(final=None):
        # written after every checkpoint, so that a long run leaves its prefix behind
        ts = np.array(sorted(snaps), dtype=np.int32)
        lab = np.stack([snaps[t] for t in ts])
        ns = np.array([[sim.net_similarity(S64, np.float64(p), lab[k, l]) for l in range(L)]
                       for k in range(ts.size)])
        extra = {} if final is None else dict(iters=np.int32(final.iters), converged=np.bool_(final.converged),
                                               final_labels=final.labels.astype(np.int32))
        np.savez_compressed(out, checkpoints=ts, labels=lab, net_similarity=ns, pref=np.float32(p),
                            seconds=np.float64(time.perf_counter() - t0), **extra)

    def record(t, l, st):
        if l == L - 1 and t in CHECKPOINTS:
            snaps[t] = hap_ref.labels_of(st).astype(np.int32)
            save()
            print(f"t={t} exemplars per level {[len(np.unique(e)) for e in snaps[t]]} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)

    res = hap_ref.hap(S, p, L, rp.damping, rp.max_iters, rp.stable_iters, record=record, dtype=dt)
    save(res)
    print(f"wrote {out.name}: iters {res.iters}, converged {res.converged}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
