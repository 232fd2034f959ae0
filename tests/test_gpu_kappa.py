"""The optional level-wise similarity update (Eq. 2.7) on the GPU against the oracle,
through the C ABI.

With one row per workgroup the column sums run in row order, so FP64 and FP32 runs are
bit-identical to the oracle evaluated in the same precision: messages, c, phi, tau, the row
offsets delta, labels and the stop iteration, for the register-resident and the streaming
row pass and in points mode.  The default launch (row blocks, partials summed per block) is
held to the FP64 tolerance of the plain path, and at full size to the FP32 one.
"""
import numpy as np
import pytest
import torch

from oracle import hap_ref
from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def to_device(S):
    n = S.shape[0]
    vw = 4 if S.dtype == np.float32 else 2
    ld = n + (-n) % vw
    buf = torch.zeros((n, ld), dtype=torch.float32 if S.dtype == np.float32 else torch.float64, device=DEV)
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(S))
    return buf[:, :n]


def run(hap, S, L, lam, T, kappa, K=0, launch=(0, 0, 1), streaming=None, X=None, eager=None):
    h = hap.Hap(to_device(S), L, lam, kappa=kappa)
    h.set_launch(*launch, streaming=streaming, eager=eager)
    if X is not None:
        h.set_points(torch.from_numpy(X).to(DEV))
    res = h.iterate(T, K)
    out = dict(iters=res.iters, converged=res.converged, labels=h.labels().cpu().numpy(),
               msgs=[{k: v.cpu().numpy() for k, v in h.messages(l).items()} for l in range(L)],
               delta=[h.offsets(l).cpu().numpy() for l in range(L)])
    h.close()
    return out


def same_as_oracle(g, r, L):
    st = r.state
    for l in range(L):
        m = g["msgs"][l]
        assert np.array_equal(m["rho"], st.rho[l]), ("rho", l)
        assert np.array_equal(m["alpha"], st.alpha[l]), ("alpha", l)
        if l < L - 1:
            assert np.array_equal(m["c"], st.c[l]), ("c", l)
            assert np.array_equal(m["phi"], st.phi[l]), ("phi", l)
        if l > 0:
            assert np.array_equal(m["tau"], st.tau[l]), ("tau", l)
        assert np.array_equal(g["delta"][l], st.delta[l]), ("delta", l)
    assert np.array_equal(g["labels"], r.labels)


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def test_fp64_bit_identical(hap_gpu):
    b, rp = synth.workload_small_f64()
    S = sim.add_noise(sim.similarity(b.X), rp.noise_rel, rp.noise_seed)
    p = sim.median_offdiag(S)
    g = run(hap_gpu, S, 3, 0.5, 60, 0.5)
    r = hap_ref.hap(S, p, 3, 0.5, 60, kappa=0.5)
    assert np.any(r.state.delta[1] != 0) and np.any(r.state.delta[2] != r.state.delta[1])
    same_as_oracle(g, r, 3)


@pytest.mark.parametrize("n,lam,kappa,T", [(300, 0.9, 0.5, 80), (130, 0.5, 0.25, 100), (1000, 0.7, 1.0, 40),
                                           (67, 0.9, 0.75, 60)])
def test_fp32_bit_identical(hap_gpu, n, lam, kappa, T):
    b, _ = synth.workload_plain_f32(n=n)
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    g = run(hap_gpu, S32, 3, lam, T, kappa)
    same_as_oracle(g, hap_ref.hap(S32, p, 3, lam, T, dtype=np.float32, kappa=kappa), 3)


@pytest.mark.parametrize("launch", [(1024, 3, 1), (512, 16, 1)])
def test_fp32_streaming_bit_identical(hap_gpu, launch):
    """The streaming and the held-row passes, forced, with the Eq. 2.7 offsets."""
    b, _ = synth.workload_plain_f32(n=1500)
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    g = run(hap_gpu, S32, 3, 0.7, 30, 0.5, launch=launch, streaming=True)
    same_as_oracle(g, hap_ref.hap(S32, p, 3, 0.7, 30, dtype=np.float32, kappa=0.5), 3)


@pytest.mark.parametrize("launch,streaming", [((0, 0, 7), None), ((1024, 1, 3), True)])
def test_several_rows_per_workgroup_both_orders(hap_gpu, launch, streaming):
    """With several rows per workgroup the column sums run in another order than the oracle's
    (interleaved rows, the default, or contiguous blocks): FP64 messages and offsets within
    1e-10 of the oracle (rounding of reordered sums over 40 sweeps, as in the plain parity
    tests) and the labels equal, for the register-resident and the streaming pass."""
    b, rp = synth.workload_small_f64()
    S = sim.add_noise(sim.similarity(b.X), rp.noise_rel, rp.noise_seed)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, 3, 0.5, 40, kappa=0.5)
    for blocks in (False, True):
        h = hap_gpu.Hap(to_device(S), 3, 0.5, kappa=0.5)
        h.set_launch(*launch, streaming=streaming, blocks=blocks)
        h.iterate(40)
        labels = h.labels().cpu().numpy()
        for l in range(3):
            m = h.messages(l)
            assert normwise(m["rho"].cpu().numpy(), r.state.rho[l]) <= 1e-10, (blocks, l)
            assert normwise(m["alpha"].cpu().numpy(), r.state.alpha[l]) <= 1e-10, (blocks, l)
            if l > 0:
                assert normwise(h.offsets(l).cpu().numpy(), r.state.delta[l]) <= 1e-10, (blocks, l)
        h.close()
        assert np.array_equal(labels, r.labels), blocks


def test_fp32_points_mode_bit_identical(hap_gpu):
    b, _ = synth.workload_plain_f32(n=700)
    X = b.X.astype(np.float32)
    S32 = sim.similarity(X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    g = run(hap_gpu, S32, 3, 0.9, 40, 0.5, X=X)
    same_as_oracle(g, hap_ref.hap(S32, p, 3, 0.9, 40, dtype=np.float32, kappa=0.5), 3)


def test_stop_rule_and_eager_launches(hap_gpu):
    """The stop iteration and its labels match the oracle's.  The row pass that detects the
    stop has already run one more iteration, so the messages and offsets left in the state
    are those of iteration stop + 1 (the oracle run for that many iterations)."""
    b, rp = synth.workload_small_f64()
    S = sim.add_noise(sim.similarity(b.X), rp.noise_rel, rp.noise_seed)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, 2, 0.9, 600, stable_iters=20, kappa=0.5)
    assert r.converged
    r_next = hap_ref.hap(S, p, 2, 0.9, r.iters + 1, kappa=0.5)
    for eager in (False, True):
        g = run(hap_gpu, S, 2, 0.9, 600, 0.5, K=20, eager=eager)
        assert g["converged"] and g["iters"] == r.iters
        assert np.array_equal(g["labels"], r.labels)
        g["labels"] = r_next.labels
        same_as_oracle(g, r_next, 2)


def test_fp32_default_launch_within_tolerance(hap_gpu):
    """FP32 in the default launch (several rows per workgroup, partials summed per block)
    against the FP64 oracle on the same FP32 similarity, over a horizon where the FP32 and
    FP64 trajectories have not separated."""
    b, _ = synth.workload_plain_f32(n=1000)
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    r = hap_ref.hap(S32.astype(np.float64), float(p), 3, 0.9, 40, kappa=0.5)
    h = hap_gpu.Hap(to_device(S32), 3, 0.9, kappa=0.5)
    assert h.get_launch()[2] > 1
    h.iterate(40)
    for l in range(3):
        m = h.messages(l)
        assert normwise(m["rho"].cpu().numpy(), r.state.rho[l]) <= 1e-4, ("rho", l)
        assert normwise(m["alpha"].cpu().numpy(), r.state.alpha[l]) <= 1e-4, ("alpha", l)
        assert normwise(h.offsets(l).cpu().numpy(), r.state.delta[l]) <= 1e-4, ("delta", l)
    h.close()


def test_full_size_first_sweeps(hap_gpu):
    """8192 points, 64 blobs, FP32 in the default launch: three sweeps against the FP64 oracle."""
    b, rp = synth.workload_plain_f32()
    S32 = sim.similarity(b.X).astype(np.float32)
    p = sim.median_offdiag(S32, np.float32)
    r = hap_ref.hap(S32.astype(np.float64), float(p), rp.levels, rp.damping, 3, kappa=0.5)
    St = to_device(S32)
    h = hap_gpu.Hap(St, rp.levels, rp.damping, kappa=0.5)
    h.iterate(3)
    for l in range(rp.levels):
        m = h.messages(l)
        assert normwise(m["rho"].cpu().numpy(), r.state.rho[l]) <= 1e-4, ("rho", l)
        assert normwise(m["alpha"].cpu().numpy(), r.state.alpha[l]) <= 1e-4, ("alpha", l)
        assert normwise(h.offsets(l).cpu().numpy(), r.state.delta[l]) <= 1e-4, ("delta", l)
        if l < rp.levels - 1:
            assert normwise(m["phi"].cpu().numpy(), r.state.phi[l]) <= 1e-4, ("phi", l)
    h.close()


def test_kappa_zero_matches_the_plain_path(hap_gpu):
    b, _ = synth.workload_plain_f32(n=400)
    S32 = sim.similarity(b.X).astype(np.float32)
    a = run(hap_gpu, S32, 3, 0.9, 30, 0.0)
    h = hap_gpu.Hap(to_device(S32), 3, 0.9)
    h.set_launch(0, 0, 1)
    h.iterate(30)
    for l in range(3):
        m = h.messages(l)
        assert np.array_equal(m["rho"].cpu().numpy(), a["msgs"][l]["rho"])
        assert not np.any(a["delta"][l])
    h.close()
