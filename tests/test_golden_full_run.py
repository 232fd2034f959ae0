"""The stored full-run oracle labels of the 8192-point workload are the oracle's own: the first
checkpoint (iteration 3) is recomputed here and must match exactly, and so must the preference."""
from pathlib import Path

import numpy as np

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth

GOLD = Path(__file__).resolve().parent / "golden"


def test_stored_full_run_starts_like_the_oracle():
    b, rp = synth.workload_plain_f32()
    S32 = sim.similarity(b.X).astype(np.float32)
    p = np.float32(sim.median_offdiag(S32, np.float32))
    for dtype in ("float32", "float64"):
        with np.load(GOLD / f"full_run_plain8192_oracle_{dtype}.npz") as z:
            ts, labels, pref = z["checkpoints"], z["labels"], z["pref"]
        assert pref == p
        assert int(ts[0]) == 3 and list(ts) == sorted(ts)
        assert labels.shape == (len(ts), rp.levels, b.X.shape[0])
        if dtype == "float32":
            r = hap_ref.hap(S32, p, rp.levels, rp.damping, int(ts[0]), dtype=np.float32)
            assert np.array_equal(r.labels, labels[0])
