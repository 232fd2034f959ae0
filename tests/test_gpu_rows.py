"""One block of a run split by rows (hap_set_row_count) against the oracle's row-block option.

Bars: with column sums in row order (one row per workgroup) the block run is bit-identical
to the oracle's (FP64, and FP32 against the FP32-evaluated oracle, for the resident,
streaming and points-mode row passes); rho and tau (levels above the first) are compared on
every row (the rows outside the block keep their initial rho on both sides), and alpha, c,
phi and the labels, which the library reports from alpha finished on the fly, on the
block's rows.  With the default launch the block run stays within 1e-4 of the FP64
oracle.  Setting the whole row count back reproduces the plain run.
"""
import numpy as np
import pytest
import torch

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _device_S(S):
    n = S.shape[0]
    vw = 4 if S.dtype == np.float32 else 2
    buf = torch.zeros((n, n + (-n) % vw), dtype=torch.float32 if S.dtype == np.float32 else torch.float64, device=DEV)
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(S))
    return buf[:, :n]


def _run(hap, S, L, lam, T, rows, launch=None, streaming=None, X=None):
    h = hap.Hap(_device_S(S), L, lam)
    h.set_row_count(rows)
    assert h.get_row_count() == rows
    if launch is not None or streaming is not None:
        lc = launch or (0, 0, 0)
        h.set_launch(*lc, streaming=streaming)
    if X is not None:
        h.set_points(torch.from_numpy(X).to(DEV))
    h.iterate(T)
    out = dict(labels=h.labels().cpu().numpy(),
               msgs=[{k: v.cpu().numpy() for k, v in h.messages(l).items()} for l in range(L)])
    h.close()
    return out


def _same(g, r, L, rows):
    st = r.state
    assert np.array_equal(g["labels"][:, :rows], r.labels[:, :rows])
    for l in range(L):
        m = g["msgs"][l]
        assert np.array_equal(m["rho"], st.rho[l]), ("rho", l)
        assert np.array_equal(m["alpha"][:rows], st.alpha[l][:rows]), ("alpha", l)
        if l > 0:
            assert np.array_equal(m["tau"], st.tau[l]), ("tau", l)
        if l < L - 1:
            assert np.array_equal(m["c"][:rows], st.c[l][:rows]), ("c", l)
            assert np.array_equal(m["phi"][:rows], st.phi[l][:rows]), ("phi", l)


@pytest.mark.parametrize("rows", [1, 97, 299, 300])
def test_block_f64_bit_identical(hap_gpu, rows):
    b, rp = synth.workload_small_f64()
    S = sim.add_noise(sim.similarity(b.X), rp.noise_rel, rp.noise_seed)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, rp.levels, rp.damping, 60, rows=rows)
    g = _run(hap_gpu, S, rp.levels, rp.damping, 60, rows, launch=(0, 0, 1))
    _same(g, r, rp.levels, rows)


@pytest.mark.parametrize("n,rows,mode", [(1000, 333, "resident"), (1000, 333, "points"), (1500, 700, "streaming"),
                                         (257, 64, "resident")])
def test_block_f32_bit_identical_to_fp32_oracle(hap_gpu, n, rows, mode):
    b, _ = synth.workload_plain_f32(n=n)
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    r = hap_ref.hap(S32, p, 3, 0.9, 40, dtype=np.float32, rows=rows)
    if mode == "streaming":
        g = _run(hap_gpu, S32, 3, 0.9, 40, rows, launch=(1024, 2, 1), streaming=True)
    elif mode == "points":
        g = _run(hap_gpu, S32, 3, 0.9, 40, rows, launch=(0, 0, 1), X=b.X)
    else:
        g = _run(hap_gpu, S32, 3, 0.9, 40, rows, launch=(0, 0, 1))
    _same(g, r, 3, rows)


def test_block_default_launch_near_fp64_oracle(hap_gpu):
    b, _ = synth.workload_plain_f32(n=2048)
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    rows = 512
    r = hap_ref.hap(S32.astype(np.float64), float(p), 3, 0.9, 3, rows=rows)
    g = _run(hap_gpu, S32, 3, 0.9, 3, rows, X=b.X)
    for l in range(3):
        for name, ref in (("rho", r.state.rho[l]), ("alpha", r.state.alpha[l][:rows])):
            got = g["msgs"][l][name] if name == "rho" else g["msgs"][l][name][:rows]
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert err <= 1e-4, (name, l, err)


def test_whole_row_count_is_the_plain_run_and_bad_counts_fail(hap_gpu):
    b, _ = synth.workload_plain_f32(n=300)
    S32 = sim.similarity(b.X).astype(np.float32)
    plain = _run(hap_gpu, S32, 3, 0.5, 30, 300)
    h = hap_gpu.Hap(_device_S(S32), 3, 0.5)
    h.set_row_count(100)
    h.set_row_count(300)
    h.iterate(30)
    assert np.array_equal(h.labels().cpu().numpy(), plain["labels"])
    for bad in (0, 301):
        with pytest.raises(hap_gpu.HapError):
            h.set_row_count(bad)
    h.close()
    for kw in (dict(schedule=hap_gpu.SCHEDULE_MRHAP), dict(kappa=0.5)):
        h = hap_gpu.Hap(_device_S(S32), 3, 0.5, **kw)
        with pytest.raises(hap_gpu.HapError):
            h.set_row_count(100)
        h.close()


def test_block_stop_rule_at_the_cap_and_exemplar_count(hap_gpu):
    """The stop rule and the exemplar count take the block's rows only: a block run that meets
    the stop rule exactly at the cap reports it (the rows outside the block, whose labels
    the finished availabilities would change, do not count), one iteration less does not,
    and the counts are those of the block's labels."""
    b = synth.separated_blobs(96, k=3, m=4)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 96)
    p = sim.median_offdiag(S)
    n = S.shape[0]
    rows, L, K = n - 1, 2, 10
    r = hap_ref.hap(S, p, L, 0.5, 400, stable_iters=K, rows=rows)
    assert r.converged
    for cap, want in ((r.iters, True), (r.iters - 1, False)):
        h = hap_gpu.Hap(_device_S(S), L, 0.5)
        h.set_launch(rows_per_block=1)
        h.set_row_count(rows)
        res = h.iterate(cap, K)
        assert bool(res.converged) == want and res.iters == cap, (cap, res)
        if want:
            lab = h.labels().cpu().numpy()
            assert np.array_equal(lab[:, :rows], r.labels[:, :rows])
            assert [h.exemplars(l)[1] for l in range(L)] == [len(np.unique(r.labels[l][:rows])) for l in range(L)]
        h.close()
