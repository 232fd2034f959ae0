"""Pins of the warm-start oracle (oracle/warm.py) against hand derivations, closed forms,
finite differences and properties that do not depend on the oracle's own code."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import hap_ref, warm
from oracle import similarity as sim
from paper_1403_7394_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(None, 1)
            rows = [[float(Fraction(x)) for x in r.split()] for r in rest.split(";")]
            out[key] = np.array(rows if len(rows) > 1 else rows[0])
    return out


def test_features_match_hand_derivation():
    g = _golden_rows("warm_features_n4.txt")
    F = warm.row_features(g["S"], float(g["p"].item()))
    want = np.stack([g[f"F{i}"] for i in range(4)])
    assert F.shape == (4, warm.NFEAT)
    np.testing.assert_allclose(F, want, rtol=1e-15, atol=1e-16)


def test_features_are_scale_free_and_permutation_equivariant():
    b = synth.small_blobs(71, 40, d=2, k=3)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    F = warm.row_features(S, p)
    # scaling S and p by a power of two changes no feature (every step is scale-free)
    np.testing.assert_allclose(warm.row_features(8.0 * S, 8.0 * p), F, rtol=1e-12, atol=1e-14)
    perm = np.random.default_rng(5).permutation(40)
    Fp = warm.row_features(S[np.ix_(perm, perm)], p)
    np.testing.assert_allclose(Fp, F[perm], rtol=1e-12, atol=1e-14)
    assert np.all(np.diff(F[:, :16], axis=1) <= 0)        # descending top-16
    assert np.all((F[:, 26:] >= -1) & (F[:, 26:] <= 1))


def test_neighbourhood_is_the_sixteen_most_similar_lower_index_first():
    """Point 0 sees every other point at the same similarity, so its neighbourhood is points
    1..16 (lower index first); point 19 alone has a much larger soft count and is outside it."""
    n = 20
    S = np.full((n, n), -10.0)
    S[0, 1:] = -1.0
    S[19, :19] = -0.01            # point 19 is close to everyone (its own row only)
    for i in range(1, 19):
        S[i, (i % 18) + 1] = -0.5  # a little structure among 1..18
    np.fill_diagonal(S, 0.0)
    p = -4.0
    F = warm.row_features(S, p)
    D0 = np.array([np.sum(np.maximum(0.0, np.delete(S[i], i) + 4.0)) / 4.0 for i in range(n)])
    assert D0[19] > D0[1:17].max()
    want = (D0[0] - D0[1:17].max()) / max(D0[0], D0[1:17].max())
    assert F[0, 26] == pytest.approx(want, rel=1e-14)


def test_transform_closed_forms():
    assert warm.g_fwd(3.0) == 1.0 and warm.g_fwd(-8.0) == -2.0 and warm.g_fwd(0.0) == 0.0
    assert warm.g_inv(1.0) == 3.0 and warm.g_inv(-2.0) == -8.0 and warm.g_inv(0.0) == 0.0
    v = np.array([-1e6, -3.5, -1e-9, 0.0, 2e-7, 0.75, 12.0, 4e5])
    np.testing.assert_allclose(warm.g_inv(warm.g_fwd(v)), v, rtol=1e-12, atol=1e-18)
    assert np.all(np.diff(warm.g_fwd(v)) > 0)


def test_warm_alpha_hand_example_and_eq22_23_at_zero_rho():
    A = warm.warm_alpha0(np.array([[2.0, -3.0]]), 2)
    np.testing.assert_array_equal(A[0], [[2.0, -3.0], [0.0, -3.0]])
    B = np.array([1.5, -0.25, 0.0, -7.0, 3.0])
    # availabilities of Eq. 2.2-2.3 evaluated at rho = 0 with base B
    np.testing.assert_array_equal(warm.warm_alpha0(B[None], 5)[0], hap_ref.availability(np.zeros((5, 5)), B))


def test_bases_invert_targets_of_a_finished_run():
    b = synth.small_blobs(72, 60, d=2, k=3)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, 2, 0.9, 80)
    T = warm.targets(r, p)
    B = warm.warm_bases(T, p)
    idx = np.arange(60)
    for l in range(2):
        np.testing.assert_allclose(B[l], r.state.alpha[l][idx, idx] + r.state.rho[l][idx, idx], rtol=1e-12, atol=1e-9)


def test_zero_outputs_give_the_cold_start_exactly():
    b = synth.small_blobs(73, 50, d=2, k=4)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    cold = hap_ref.hap(S, p, 3, 0.8, 40)
    warm_r = hap_ref.hap(S, p, 3, 0.8, 40, alpha0=warm.warm_alpha0(warm.warm_bases(np.zeros((50, 3)), p), 50))
    for l in range(3):
        np.testing.assert_array_equal(warm_r.state.rho[l], cold.state.rho[l])
        np.testing.assert_array_equal(warm_r.state.alpha[l], cold.state.alpha[l])


def test_fixed_point_bases_restart_at_the_fixed_point():
    """At L = 1 a converged run's bases alpha_jj + rho_jj reproduce its exemplars from the warm
    start, and the warm run stops no later than the cold one."""
    b = synth.separated_blobs(74, k=4, m=10, sep=30.0)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    cold = hap_ref.hap(S, p, 1, 0.9, 1000, stable_iters=30)
    assert cold.converged
    r, fell = warm.warm_run(S, p, 1, 0.9, 1000, 30, warm.targets(cold, p))
    assert not fell and r.converged
    np.testing.assert_array_equal(r.labels, cold.labels)
    assert r.iters <= cold.iters


def test_fallback_runs_the_cold_start():
    b = synth.small_blobs(75, 40, d=2, k=3)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    cold = hap_ref.hap(S, p, 1, 0.9, 12, stable_iters=50)      # too short to converge
    assert not cold.converged
    Y = np.random.default_rng(3).standard_normal((40, 1))
    r, fell = warm.warm_run(S, p, 1, 0.9, 12, 50, Y)
    assert fell
    np.testing.assert_array_equal(r.labels, cold.labels)
    np.testing.assert_array_equal(r.state.alpha, cold.state.alpha)
    r2, fell2 = warm.warm_run(S, p, 1, 0.9, 12, 50, None)
    assert not fell2
    np.testing.assert_array_equal(r2.state.rho, cold.state.rho)


def _small_net(seed=11, n_in=5, hidden=7, n_out=3, rows=13):
    rng = np.random.default_rng(seed)
    flat = synth.mlp_init(seed, n_in, hidden, n_out).astype(np.float64)
    flat[n_in * hidden:n_in * hidden + hidden] = 0.1 * rng.standard_normal(hidden)   # nonzero biases
    X = rng.standard_normal((rows, n_in))
    T = rng.standard_normal((rows, n_out))
    return warm.unpack(flat, n_in, hidden, n_out), X, T


def test_backprop_matches_central_differences():
    P, X, T = _small_net()
    _, G = warm.loss_and_grads(P, X, T)
    h = 1e-6
    for k in P:
        fd = np.zeros_like(P[k])
        for idx in np.ndindex(P[k].shape):
            Pp = {q: v.copy() for q, v in P.items()}
            Pm = {q: v.copy() for q, v in P.items()}
            Pp[k][idx] += h
            Pm[k][idx] -= h
            fd[idx] = (warm.loss_and_grads(Pp, X, T)[0] - warm.loss_and_grads(Pm, X, T)[0]) / (2 * h)
        np.testing.assert_allclose(G[k], fd, rtol=1e-6, atol=1e-9, err_msg=k)


def test_pack_unpack_layout():
    n_in, hidden, n_out = 3, 4, 2
    flat = np.arange(warm.param_count(n_in, hidden, n_out), dtype=np.float64)
    P = warm.unpack(flat, n_in, hidden, n_out)
    assert P["W1"][1, 2] == 1 * hidden + 2            # row-major, W1 first
    assert P["b1"][0] == n_in * hidden
    assert P["W3"][0, 1] == n_in * hidden + hidden + hidden * hidden + hidden + 1
    np.testing.assert_array_equal(warm.pack(P), flat)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr * g / (|g| + eps)."""
    P, X, T = _small_net()
    _, G = warm.loss_and_grads(P, X, T)
    M = {k: np.zeros_like(v) for k, v in P.items()}
    V = {k: np.zeros_like(v) for k, v in P.items()}
    P0 = {k: v.copy() for k, v in P.items()}
    warm.adam_step(P, G, M, V, 1, 1e-2)
    for k in P:
        np.testing.assert_allclose(P[k], P0[k] - 1e-2 * G[k] / (np.abs(G[k]) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_fits_a_realisable_teacher():
    rng = np.random.default_rng(12)
    n_in, hidden, n_out = 6, 16, 2
    teacher = warm.unpack(synth.mlp_init(100, n_in, hidden, n_out).astype(np.float64), n_in, hidden, n_out)
    X = rng.standard_normal((512, n_in))
    T, _ = warm.forward(teacher, X)
    P = warm.unpack(synth.mlp_init(101, n_in, hidden, n_out).astype(np.float64), n_in, hidden, n_out)
    idx = synth.minibatch_order(7, 512, 64, 600)
    losses, _, _ = warm.train(P, X, T, idx, 64, 600, 3e-3)
    assert losses[-20:].mean() < 0.05 * losses[:5].mean()


def test_sampled_features_equal_full_features():
    b = synth.small_blobs(76, 90, d=3, k=5)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    F = warm.row_features(S, p)
    rows = [0, 13, 44, 89]
    G = warm.row_features_sampled(lambda i: S[i], 90, p, rows)
    assert np.array_equal(G, F[rows])
