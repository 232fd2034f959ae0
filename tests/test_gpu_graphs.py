"""Sweep chunks replayed from captured graphs give the same results as launches issued one
by one, across chunk boundaries and the stop rule; per-launch timing (which launches one
kernel at a time) is unaffected by the graph setting."""
import numpy as np
import pytest
import torch

from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(hap, S, L, lam, T, K, eager, profile, schedule):
    h = hap.Hap(S, L, lam, schedule=schedule)
    h.set_launch(eager=eager)
    assert bool(h.launch_flags() & hap.LAUNCH_EAGER) == eager
    if profile:
        h.profile(True)
    res = h.iterate(T, K)
    prof = h.profile_read() if profile else None
    out = (res.iters, res.converged, h.labels().cpu().numpy(), h.messages(L - 1)["rho"].cpu().numpy(), prof)
    h.close()
    return out


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("profile", [False, True])
def test_graph_replay_equals_eager_launches(hap_gpu, schedule, profile):
    b = synth.small_blobs(1500, 1200, d=2, k=7, dtype=np.float32)
    S = torch.from_numpy(sim.similarity(b.X).astype(np.float32)).to(DEV)
    L, lam = 3, 0.9
    # 37 sweeps: two full chunks of 16 and a chunk of 5
    g = _run(hap_gpu, S, L, lam, 37, 0, False, profile, schedule)
    e = _run(hap_gpu, S, L, lam, 37, 0, True, profile, schedule)
    assert g[0] == e[0] == 37
    assert np.array_equal(g[2], e[2]) and np.array_equal(g[3], e[3])
    if profile:
        # row-pass launches: one per level, or one per sweep for the MapReduce schedule's fused
        # pass (this FP32 problem reads S with four chunks per thread); column sums one per level
        rows = 37 if schedule == 1 else 37 * L
        assert g[4][1] == e[4][1] == rows and g[4][3] == e[4][3] == 37 * L
        assert g[4][0] > 0 and g[4][2] > 0


def test_graph_replay_stops_where_eager_stops(hap_gpu):
    b = synth.small_blobs(1501, 500, d=2, k=4, dtype=np.float32)
    S = torch.from_numpy(sim.similarity(b.X).astype(np.float32)).to(DEV)
    g = _run(hap_gpu, S, 1, 0.9, 800, 20, False, False, 0)
    e = _run(hap_gpu, S, 1, 0.9, 800, 20, True, False, 0)
    assert g[1] and e[1] and g[0] == e[0]
    assert np.array_equal(g[2], e[2])
