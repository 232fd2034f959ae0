"""Pins of the optional level-wise similarity update (Eq. 2.7) in the oracle: a two-iteration
example worked by hand with exact fractions, the exact rational evaluator on random integer
inputs, and the special cases kappa = 0 and L = 1."""
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
            rows = [[Fraction(x) for x in r.split()] for r in rest.split(";")]
            out[key] = rows if len(rows) > 1 else rows[0]
    return out


def _f(x):
    return np.array(x, dtype=float)


def test_hand_worked_two_iterations():
    g = _read("kappa_two_iterations_n3_l2.txt")
    S = _f(g["S"])
    r1 = hap_ref.hap(S, -2.0, 2, 0.5, 1, kappa=0.5)
    st = r1.state
    assert np.array_equal(st.delta[0], [0, 0, 0])
    assert np.array_equal(st.delta[1], _f(g["delta2_iter1"]))
    assert np.array_equal(st.rho[1], _f(g["rho2_iter1"]))
    assert np.array_equal(st.alpha[1], _f(g["alpha2_iter1"]))
    assert np.array_equal(st.phi[0], _f(g["phi1_iter1"]))
    assert np.array_equal(r1.labels[1], _f(g["labels2_iter1"]))
    r2 = hap_ref.hap(S, -2.0, 2, 0.5, 1, kappa=0.5, state=st)
    assert np.array_equal(r2.state.rho[0], _f(g["rho1_iter2"]))
    assert np.array_equal(r2.state.alpha[0], _f(g["alpha1_iter2"]))
    assert np.array_equal(r2.state.c[0], _f(g["c1_iter2"]))
    assert np.array_equal(r2.state.tau[1], _f(g["tau2_iter2"]))
    assert np.array_equal(r2.state.delta[1], _f(g["delta2_iter2"]))
    # the exact evaluator, from the defining sums
    Si = [[int(v) for v in row] for row in g["S"]]
    out1 = literal.hap_literal(Si, [[-2] * 3] * 2, 2, Fraction(1, 2), 1, kappa=Fraction(1, 2))
    assert out1[6][1] == g["delta2_iter1"]
    assert out1[1][1] == g["rho2_iter1"] and out1[2][1] == g["alpha2_iter1"] and out1[4][0] == g["phi1_iter1"]
    out2 = literal.hap_literal(Si, [[-2] * 3] * 2, 2, Fraction(1, 2), 2, kappa=Fraction(1, 2))
    assert out2[1][0] == g["rho1_iter2"] and out2[2][0] == g["alpha1_iter2"]
    assert out2[3][0] == g["c1_iter2"] and out2[5][1] == g["tau2_iter2"] and out2[6][1] == g["delta2_iter2"]


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("n,L,lam,kappa,T,seed", [
    (4, 2, Fraction(1, 2), Fraction(1, 2), 6, 41), (5, 3, Fraction(1, 2), Fraction(1, 4), 5, 42),
    (5, 3, Fraction(9, 10), Fraction(1), 6, 43), (3, 4, Fraction(9, 10), Fraction(3, 4), 7, 44),
])
def test_fp64_oracle_matches_exact_rationals(n, L, lam, kappa, T, seed):
    S = synth.integer_matrix(seed, n)
    pref = np.stack([synth.integer_vector(seed + l, n) for l in range(L)])
    lab, rho, alpha, c, phi, tau, delta = literal.hap_literal(S.astype(int).tolist(), pref.astype(int).tolist(), L,
                                                              lam, T, kappa=kappa)
    r = hap_ref.hap(S, pref, L, float(lam), T, kappa=float(kappa))
    for l in range(L):
        assert _normwise(r.state.rho[l], _f([[float(v) for v in row] for row in rho[l]])) <= 1e-13
        assert _normwise(r.state.alpha[l], _f([[float(v) for v in row] for row in alpha[l]])) <= 1e-13
        assert _normwise(r.state.delta[l], _f([float(v) for v in delta[l]])) <= 1e-13
        if l > 0:
            assert _normwise(r.state.tau[l], _f([float(v) for v in tau[l]])) <= 1e-13
    assert r.labels.tolist() == lab


def test_kappa_zero_is_the_plain_method_and_one_level_ignores_it():
    b = synth.small_blobs(45, 50, d=2, k=4)
    S = sim.similarity(b.X)
    p = sim.median_offdiag(S)
    plain = hap_ref.hap(S, p, 3, 0.8, 25)
    zero = hap_ref.hap(S, p, 3, 0.8, 25, kappa=0.0)
    assert np.array_equal(plain.state.rho, zero.state.rho) and np.array_equal(plain.state.alpha, zero.state.alpha)
    assert not np.any(zero.state.delta)
    one = hap_ref.hap(S, p, 1, 0.8, 25)
    one_k = hap_ref.hap(S, p, 1, 0.8, 25, kappa=0.7)
    assert np.array_equal(one.state.rho, one_k.state.rho) and np.array_equal(one.labels, one_k.labels)
    # the first iteration's bottom level runs before any offset exists
    a = hap_ref.hap(S, p, 3, 0.8, 1)
    k = hap_ref.hap(S, p, 3, 0.8, 1, kappa=0.7)
    assert np.array_equal(a.state.rho[0], k.state.rho[0]) and np.array_equal(a.state.alpha[0], k.state.alpha[0])
    assert not np.array_equal(a.state.rho[1], k.state.rho[1])


def test_kappa_arguments_are_checked():
    S = -np.ones((4, 4))
    with pytest.raises(ValueError):
        hap_ref.hap(S, -1.0, 2, 0.5, 1, kappa=1.5)
    with pytest.raises(ValueError):
        hap_ref.hap(S, -1.0, 2, 0.5, 1, kappa=-0.1)
    with pytest.raises(ValueError):
        hap_ref.hap(S, -1.0, 2, 0.5, 1, kappa=0.5, schedule="mrhap")
