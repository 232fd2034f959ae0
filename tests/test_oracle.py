"""Pins for the CPU oracle, checked against things other than the oracle itself.

Runs on the CPU only.  Each test names the property of the paper or of the
mathematics it pins.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import ap_ref, brute, hap_ref, literal
from oracle import similarity as sim
from paper_1403_7394_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(None, 1)
            rows = [[float(x) for x in r.split()] for r in rest.split(";")]
            out[key] = np.array(rows if len(rows) > 1 else rows[0])
    return out


def _normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


# --------------------------------------------------------------------------
# Hand-derived first iteration (Eq. 2.1-2.6 with the Algorithm 1 initial values)
# --------------------------------------------------------------------------

def test_first_sweep_matches_hand_derivation():
    g = _read_golden("first_sweep_n3_l2.txt")
    S = g["S"]
    seen = {}

    def rec(t, l, st):
        seen[(t, l)] = st.copy()

    r = hap_ref.hap(S, -2.0, levels=2, damping=0.5, max_iters=1, record=rec)
    st1 = seen[(1, 0)]
    assert np.array_equal(st1.rho[0], g["rho1"])
    assert np.array_equal(st1.alpha[0], g["alpha1"])
    assert np.array_equal(st1.tau[1], g["tau2"])
    assert np.array_equal(st1.c[0], g["c1"])
    st = r.state
    assert np.array_equal(r.Q[0], g["Q1"])
    assert np.array_equal(st.rho[1], g["rho2"])
    assert np.array_equal(r.Q[1], g["Q2"])
    assert np.array_equal(st.alpha[1], g["alpha2"])
    assert np.array_equal(st.phi[0], g["phi1"])
    assert np.array_equal(r.labels[0], g["e1"].astype(int))
    assert np.array_equal(r.labels[1], g["e2"].astype(int))
    # the pure-Python evaluator reproduces the same hand-derived numbers exactly
    lab, rho, alpha, c, phi, tau = literal.hap_literal(S.tolist(), [[-2] * 3] * 2, 2, Fraction(1, 2), 1)
    assert np.array_equal(np.array(rho[1], dtype=float), g["rho2"])
    assert np.array_equal(np.array(alpha[1], dtype=float), g["alpha2"])
    assert lab == [list(g["e1"].astype(int)), list(g["e2"].astype(int))]


# --------------------------------------------------------------------------
# Exact rationals: the FP64 oracle against the literal evaluator over Fractions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,L,lam,T,seed", [
    (4, 1, Fraction(1, 2), 6, 11), (4, 2, Fraction(1, 2), 6, 12), (5, 3, Fraction(1, 2), 5, 13),
    (5, 3, Fraction(9, 10), 6, 14), (3, 3, Fraction(9, 10), 8, 15), (5, 2, Fraction(1, 2), 8, 16),
])
def test_fp64_oracle_matches_exact_rationals(n, L, lam, T, seed):
    S = synth.integer_matrix(seed, n)
    pref = np.stack([synth.integer_vector(seed + l, n) for l in range(L)])
    lab, rho, alpha, c, phi, tau = literal.hap_literal(S.astype(int).tolist(), pref.astype(int).tolist(), L, lam, T)
    r = hap_ref.hap(S, pref, L, float(lam), T)
    for l in range(L):
        rho_x = np.array([[float(v) for v in row] for row in rho[l]])
        alpha_x = np.array([[float(v) for v in row] for row in alpha[l]])
        assert _normwise(r.state.rho[l], rho_x) <= 1e-14
        assert _normwise(r.state.alpha[l], alpha_x) <= 1e-14
        if l < L - 1:
            assert _normwise(r.state.c[l], np.array([float(v) for v in c[l]])) <= 1e-14
        if l > 0:
            assert _normwise(r.state.tau[l], np.array([float(v) for v in tau[l]])) <= 1e-14
            assert _normwise(r.state.phi[l - 1], np.array([float(v) for v in phi[l - 1]])) <= 1e-14
    # labels are decided on exact values: identical unless an exact tie is broken differently
    assert r.labels.tolist() == lab


@pytest.mark.parametrize("seed", [21, 22])
def test_fp64_oracle_matches_literal_floats(seed):
    b = synth.small_blobs(seed, 8, k=3)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    lab, rho, alpha, *_ = literal.hap_literal(S.tolist(), [[p] * 8] * 3, 3, 0.5, 12, num=float)
    r = hap_ref.hap(S, p, 3, 0.5, 12)
    for l in range(3):
        assert _normwise(r.state.rho[l], np.array(rho[l])) <= 1e-12
        assert _normwise(r.state.alpha[l], np.array(alpha[l])) <= 1e-12
    assert r.labels.tolist() == lab


# --------------------------------------------------------------------------
# L = 1 is plain Affinity Propagation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,lam", [(31, 40, 0.5), (32, 64, 0.9), (33, 25, 0.7)])
def test_single_level_is_plain_ap(seed, n, lam):
    b = synth.small_blobs(seed, n, k=4)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, seed)
    p = sim.median_offdiag(S)
    lab_ap, r_ap, a_ap = ap_ref.affinity_propagation(S, p, lam, 60)
    r = hap_ref.hap(S, p, 1, lam, 60)
    assert _normwise(r.state.rho[0], r_ap) <= 1e-14
    assert _normwise(r.state.alpha[0], a_ap) <= 1e-14
    assert np.array_equal(r.labels[0], lab_ap)


@pytest.mark.parametrize("seed,k,m", [(41, 3, 4), (42, 2, 6), (43, 4, 3), (44, 3, 4), (46, 2, 5)])
def test_single_level_reaches_the_brute_force_optimum(seed, k, m):
    """AP is a heuristic: on well-separated blobs it must find the optimal partition into
    clusters, a self-consistent labelling, and a net similarity within 1e-4 of the optimum
    (the medoid it keeps inside a blob may be a near-tie runner-up)."""
    b = synth.separated_blobs(seed, k=k, m=m)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, seed)
    p = sim.median_offdiag(S)
    lab_opt, v_opt = brute.best_exemplar_set(S, p)
    r = hap_ref.hap(S, p, 1, 0.5, 1000, stable_iters=50)
    assert r.converged
    e = r.labels[0]
    n = k * m
    # one medoid per blob is the optimum here
    assert len(np.unique(lab_opt)) == k
    # every exemplar is its own exemplar
    assert np.all(e[e] == e)
    same = (e[:, None] == e[None, :])
    same_opt = (lab_opt[:, None] == lab_opt[None, :])
    assert np.array_equal(same, same_opt)
    v = sim.net_similarity(S, p, e)
    assert v <= v_opt + 1e-9 * abs(v_opt)
    assert (v_opt - v) <= 1e-4 * abs(v_opt)
    assert n == e.size


def test_single_level_fixed_point_residual():
    b = synth.small_blobs(51, 40, k=3)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 51)
    p = sim.median_offdiag(S)
    r = hap_ref.hap(S, p, 1, 0.5, 3000)
    s = hap_ref.level_similarity(S, p)
    rho, alpha = r.state.rho[0], r.state.alpha[0]
    # undamped updates evaluated at the final state reproduce it (Eq. 2.1-2.3 at L=1)
    rho_fp = hap_ref.responsibility(s, alpha, None)
    alpha_fp = hap_ref.availability(rho, hap_ref.column_sums(rho))
    scale = max(np.abs(rho).max(), np.abs(alpha).max())
    assert np.max(np.abs(rho_fp - rho)) <= 1e-9 * scale
    assert np.max(np.abs(alpha_fp - alpha)) <= 1e-9 * scale


# --------------------------------------------------------------------------
# Invariants of the update equations
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [-3, 5])
def test_positive_homogeneity_is_exact(k):
    b = synth.small_blobs(61, 30, k=3)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 61)
    p = sim.median_offdiag(S)
    r1 = hap_ref.hap(S, p, 3, 0.5, 25)
    r2 = hap_ref.hap(S * 2.0 ** k, p * 2.0 ** k, 3, 0.5, 25)
    assert np.array_equal(r1.labels, r2.labels)
    assert np.array_equal(r1.state.rho * 2.0 ** k, r2.state.rho)
    assert np.array_equal(r1.state.alpha * 2.0 ** k, r2.state.alpha)
    assert np.array_equal(r1.state.c * 2.0 ** k, r2.state.c)


def test_permutation_equivariance():
    b = synth.small_blobs(71, 36, k=3)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 71)
    p = sim.median_offdiag(S)
    perm = np.random.default_rng(7).permutation(36)
    inv = np.argsort(perm)
    r1 = hap_ref.hap(S, p, 3, 0.5, 40)
    r2 = hap_ref.hap(S[np.ix_(perm, perm)], p, 3, 0.5, 40)
    # point q of the permuted problem is point perm[q] of the original one
    for l in range(3):
        assert np.array_equal(perm[r2.labels[l]], r1.labels[l][perm])
        assert _normwise(r2.state.rho[l], r1.state.rho[l][np.ix_(perm, perm)]) <= 1e-12
    assert inv.shape == perm.shape


def test_single_level_row_shift_invariance():
    b = synth.small_blobs(81, 30, k=3)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 81)
    p = sim.median_offdiag(S)
    s = hap_ref.level_similarity(S, p)
    shift = np.random.default_rng(8).uniform(-50, 50, size=30)
    s2 = s + shift[:, None]
    r1 = hap_ref.hap(s, np.diag(s), 1, 0.5, 50)
    r2 = hap_ref.hap(s2, np.diag(s2), 1, 0.5, 50)
    assert np.array_equal(r1.labels, r2.labels)
    assert np.max(np.abs(r1.state.rho - r2.state.rho)) <= 1e-12 * np.abs(r1.state.rho).max() * 100
    assert np.max(np.abs(r1.state.alpha - r2.state.alpha)) <= 1e-12 * np.abs(r1.state.alpha).max() * 100


def test_offdiagonal_availability_never_positive():
    b = synth.small_blobs(91, 40, k=4)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 91)
    p = sim.median_offdiag(S)
    off = ~np.eye(40, dtype=bool)
    bad = []

    def rec(t, l, st):
        if np.any(st.alpha[l][off] > 0):
            bad.append((t, l))

    hap_ref.hap(S, p, 3, 0.9, 60, record=rec)
    assert not bad


def test_resume_from_state_is_identical():
    b = synth.small_blobs(95, 30, k=3)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 95)
    p = sim.median_offdiag(S)
    full = hap_ref.hap(S, p, 3, 0.5, 40)
    half = hap_ref.hap(S, p, 3, 0.5, 17)
    rest = hap_ref.hap(S, p, 3, 0.5, 23, state=half.state)
    assert rest.iters == 40
    assert np.array_equal(full.state.rho, rest.state.rho)
    assert np.array_equal(full.state.alpha, rest.state.alpha)
    assert np.array_equal(full.labels, rest.labels)


def test_stop_rule_counts_consecutive_stable_iterations():
    b = synth.separated_blobs(96, k=3, m=4)
    S = sim.add_noise(sim.similarity(b.X), 1e-12, 96)
    p = sim.median_offdiag(S)
    K = 10
    r = hap_ref.hap(S, p, 2, 0.5, 400, stable_iters=K)
    assert r.converged
    # replay without the stop rule and find the first t whose labels equal those of the K previous iterations
    hist = []

    def rec(t, l, st):
        if l == 1:
            hist.append(hap_ref.labels_of(st))

    hap_ref.hap(S, p, 2, 0.5, r.iters, record=rec)
    first = None
    for t in range(K + 1, len(hist) + 1):
        if all(np.array_equal(hist[t - 1], hist[t - 1 - q]) for q in range(1, K + 1)):
            first = t
            break
    assert first == r.iters
    assert np.array_equal(hist[-1], r.labels)


# --------------------------------------------------------------------------
# Similarity, noise, median, net similarity
# --------------------------------------------------------------------------

def test_similarity_matches_scipy_sqeuclidean():
    b = synth.small_blobs(101, 50, d=5, k=3)
    S = sim.similarity(b.X)
    ref = -cdist(b.X, b.X, "sqeuclidean")
    assert np.max(np.abs(S - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.all(np.diag(S) == 0)


def test_row_blocks_match_the_full_matrix():
    """similarity_rows and a row block of responsibility give the rows of the full-matrix
    results (the blocks serve sampled checks of problems too large for the oracle)."""
    b = synth.small_blobs(102, 60, d=3, k=4)
    rows = np.array([0, 7, 31, 59])
    ref = -cdist(b.X[rows], b.X, "sqeuclidean")
    blk = sim.similarity_rows(b.X, rows)
    assert np.max(np.abs(blk - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(blk, sim.similarity(b.X)[rows])
    assert np.array_equal(sim.similarity_rows(b.X, rows, squared=False), sim.similarity(b.X, squared=False)[rows])
    S = sim.similarity(b.X)
    np.fill_diagonal(S, -5.0)
    A = np.minimum(0.0, np.random.default_rng(3).standard_normal((60, 60)))
    tau = np.random.default_rng(4).standard_normal(60)
    for t in (None, tau):
        full = hap_ref.responsibility(S, A, t)
        part = hap_ref.responsibility(S[rows], A[rows], None if t is None else t[rows])
        assert np.array_equal(part, full[rows])


def test_splitmix64_published_outputs():
    gamma = 0x9E3779B97F4A7C15
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for state, idx, out in rows:
        x = (int(state) + int(idx) * gamma) % (1 << 64)
        assert sim.splitmix64(x) == int(out)
        assert int(sim.splitmix64_np(np.array([x], dtype=np.uint64))[0]) == int(out)


def test_noise_uniform_range_and_counter():
    u = sim.noise_uniform(1234, 17)
    assert u.shape == (17, 17)
    assert np.all((u >= 0) & (u < 1))
    # u_ij depends on (seed, i*N + j) only
    x = (1234 ^ (5 * 17 + 3))
    assert u[5, 3] == (sim.splitmix64(x) >> 11) * 2.0 ** -53


@pytest.mark.parametrize("n,dtype", [(7, np.float64), (10, np.float32), (33, np.float32)])
def test_median_matches_sorting(n, dtype):
    rng = np.random.default_rng(n)
    S = -rng.exponential(10, size=(n, n))
    got = sim.median_offdiag(S, dtype)
    v = S.astype(dtype)[~np.eye(n, dtype=bool)]
    assert got == dtype(np.median(v.astype(np.float64)))
    assert got.dtype == np.dtype(dtype)


def test_net_similarity_definition():
    S = np.array([[0., -1., -4.], [-1., 0., -9.], [-4., -9., 0.]])
    # exemplars {0, 2}: point 1 joins 0
    assert sim.net_similarity(S, -2.0, np.array([0, 0, 2])) == -2.0 - 1.0 - 2.0


def test_unsquared_similarity_matches_scipy_euclidean():
    from scipy.spatial.distance import cdist
    b = synth.rgb_pixels(61, 50)
    S = sim.similarity(b.X, squared=False)
    ref = -cdist(b.X.astype(np.float64), b.X.astype(np.float64), metric="euclidean")
    np.testing.assert_allclose(S, ref, rtol=1e-15, atol=1e-12)
    assert np.all(np.diag(S) == 0.0)
    # integer pixels: every squared distance is an integer, so the root of a perfect square is exact
    assert np.all(b.X == np.rint(b.X)) and b.X.min() >= 0 and b.X.max() <= 255
