"""The oracle's row-block option (one block of a run split by rows): the whole matrix as one
block reproduces the plain run exactly, rows outside the block keep their initial state, and
the block's column sums are the sums over its own rows."""
import numpy as np
import pytest

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_block_of_all_rows_equals_the_plain_run(dtype):
    b = synth.small_blobs(71, 60, k=4)
    S = sim.similarity(b.X).astype(dtype)
    p = sim.median_offdiag(S, dtype)
    full = hap_ref.hap(S, p, 3, 0.7, 25, dtype=dtype)
    blk = hap_ref.hap(S, p, 3, 0.7, 25, dtype=dtype, rows=60)
    assert np.array_equal(full.labels, blk.labels)
    for name in ("rho", "alpha", "c", "phi", "tau"):
        assert np.array_equal(getattr(full.state, name), getattr(blk.state, name)), name


def test_rows_outside_the_block_keep_their_initial_state():
    b = synth.small_blobs(72, 50, k=3)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, 3, 0.5, 12, rows=17)
    st = r.state
    assert np.all(st.rho[:, 17:] == 0) and np.all(st.alpha[:, 17:] == 0)
    assert np.all(st.c[:, 17:] == 0) and np.all(st.phi[:, 17:] == 0)
    # the column sums of the last level are those of the block's rows alone
    rho = st.rho[2][:17]
    want = np.maximum(rho, 0).sum(axis=0)
    idx = np.arange(17)
    want[idx] += rho[idx, idx] - np.maximum(rho[idx, idx], 0)
    assert np.allclose(r.Q[2], want, rtol=0, atol=1e-9 * np.abs(want).max())


def test_block_rejects_other_schedules_and_bad_sizes():
    S = sim.similarity(synth.small_blobs(73, 10, k=2).X)
    with pytest.raises(ValueError):
        hap_ref.hap(S, -5.0, 2, 0.5, 3, rows=5, schedule="mrhap")
    with pytest.raises(ValueError):
        hap_ref.hap(S, -5.0, 2, 0.5, 3, rows=5, kappa=0.5)
    with pytest.raises(ValueError):
        hap_ref.hap(S, -5.0, 2, 0.5, 3, rows=0)
