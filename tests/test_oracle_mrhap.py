"""Pins of the MapReduce schedule (Section 3) in the oracle: a hand-derived first iteration,
exact rationals of the literal evaluator, and the single-level reduction."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import hap_ref, literal
from oracle import similarity as sim
from paper_1403_7394_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
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


def test_first_iteration_matches_hand_derivation():
    g = _read("mrhap_first_iteration_n3_l2.txt")
    r = hap_ref.hap(g["S"], -2.0, 2, 0.5, 1, schedule="mrhap")
    st = r.state
    assert np.array_equal(st.rho[0], g["rho"]) and np.array_equal(st.rho[1], g["rho"])
    assert np.array_equal(st.phi[0], g["phi1"])
    assert np.array_equal(st.alpha[0], g["alpha1"])
    assert np.array_equal(st.alpha[1], g["alpha2"])
    assert np.all(st.c == 0) and np.all(np.isinf(st.tau[1]))
    r2 = hap_ref.hap(g["S"], -2.0, 2, 0.5, 1, schedule="mrhap", state=st)
    assert np.array_equal(r2.state.c[0], g["c1_iter2"])
    assert np.array_equal(r2.state.tau[1], g["tau2_iter2"])
    lab, rho, alpha, c, phi, tau = literal.hap_literal(g["S"].tolist(), [[-2] * 3] * 2, 2, Fraction(1, 2), 1,
                                                       schedule="mrhap")
    assert np.array_equal(np.array(alpha[0], dtype=float), g["alpha1"])
    assert np.array_equal(np.array(phi[0], dtype=float), g["phi1"])


@pytest.mark.parametrize("n,L,lam,T,seed", [
    (4, 2, Fraction(1, 2), 6, 31), (5, 3, Fraction(1, 2), 5, 32), (5, 3, Fraction(9, 10), 6, 33),
    (3, 3, Fraction(9, 10), 8, 34), (5, 2, Fraction(1, 2), 8, 35),
])
def test_fp64_oracle_matches_exact_rationals(n, L, lam, T, seed):
    S = synth.integer_matrix(seed, n)
    pref = np.stack([synth.integer_vector(seed + l, n) for l in range(L)])
    lab, rho, alpha, c, phi, tau = literal.hap_literal(S.astype(int).tolist(), pref.astype(int).tolist(), L, lam, T,
                                                       schedule="mrhap")
    r = hap_ref.hap(S, pref, L, float(lam), T, schedule="mrhap")
    for l in range(L):
        assert _normwise(r.state.rho[l], np.array([[float(v) for v in row] for row in rho[l]])) <= 1e-14
        assert _normwise(r.state.alpha[l], np.array([[float(v) for v in row] for row in alpha[l]])) <= 1e-14
        if l < L - 1:
            assert _normwise(r.state.c[l], np.array([float(v) for v in c[l]])) <= 1e-14
            assert _normwise(r.state.phi[l], np.array([float(v) for v in phi[l]])) <= 1e-14
        if l > 0:
            assert _normwise(r.state.tau[l], np.array([float(v) for v in tau[l]])) <= 1e-14
    assert r.labels.tolist() == lab


def test_schedules_differ_above_one_level_and_agree_at_one():
    b = synth.small_blobs(36, 60, d=2, k=4)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    a = hap_ref.hap(S, p, 1, 0.7, 40)
    m = hap_ref.hap(S, p, 1, 0.7, 40, schedule="mrhap")
    assert np.array_equal(a.state.rho, m.state.rho) and np.array_equal(a.state.alpha, m.state.alpha)
    a3 = hap_ref.hap(S, p, 3, 0.7, 5)
    m3 = hap_ref.hap(S, p, 3, 0.7, 5, schedule="mrhap")
    assert not np.array_equal(a3.state.rho[1], m3.state.rho[1])


def test_unknown_schedule_is_rejected():
    with pytest.raises(ValueError):
        hap_ref.hap(np.zeros((3, 3)), -1.0, 1, 0.5, 1, schedule="jacobi")
