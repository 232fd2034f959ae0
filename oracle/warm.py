"""Learned warm start in FP64 (test infrastructure; see the package header).

The paper starts every run from alpha = rho = 0 (Algorithm 1).  The warm start replaces only
the initial availabilities alpha^{l,0}; every other initial value stays as in Algorithm 1.

Availability base.  With rho = 0, Eq. 2.2 and Eq. 2.3 give alpha_jj = B_j and
alpha_ij = min(0, B_j) (i != j) for a column base B_j (c_j + phi_j + Q_j below the top level,
Q_j at the top).  At a fixed point alpha_jj + rho_jj = B_j (Eq. 2.3), so the warm start
predicts v^l_j = (alpha^l_jj + rho^l_jj) / |p_j| of a finished run and sets
alpha^{l,0}_jj = B and alpha^{l,0}_ij = min(0, B) with B = v |p_j|.

Features of point i (32 numbers, scale-free: similarities are divided by a = |p_i|):
  f[0:16]   the 16 largest off-diagonal s_ij of row i, descending, / a
            (a row with fewer than 16 off-diagonal entries repeats its smallest one)
  f[16]     p_i / a
  f[17]     #{j != i : s_ij > p_i} / (n - 1)
  f[18]     mean over j != i of s_ij, / a
  f[19]     log(1 + #{j != i : s_ij > p_i}) / 10
  f[20+m]   log(1 + D_m(i)) / 10,  D_m(i) = sum_{j != i} max(0, s_ij - q_m p_i) / a,
            q_m = 2^-m, m = 0..5 (soft neighbour counts at six radii)
  f[26+m]   (D_m(i) - M_m(i)) / max(D_m(i), M_m(i)) (0 when both are 0), where M_m(i) is
            the largest D_m(j) over the neighbourhood N(i) of i: the 16 largest off-diagonal
            s_ij (the lower index first among equal values), all j != i when n - 1 < 16

Targets and outputs go through g(v) = sign(v) (sqrt(1 + |v|) - 1), whose inverse is
g^-1(y) = sign(y) |y| (|y| + 2).

Perceptron (n_in -> hidden -> hidden -> n_out, ReLU after both hidden layers):
  h1 = relu(X W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3,
  loss = mean over rows and outputs of (y - t)^2.
Parameters are one flat vector: W1 (n_in x hidden, row-major), b1, W2 (hidden x hidden), b2,
W3 (hidden x n_out), b3.  Training is minibatch Adam (Kingma and Ba, 2015).
"""
from __future__ import annotations

import numpy as np

from . import hap_ref

NFEAT = 32
NTOP = 16
NSCALE = 6


# ---------------------------------------------------------------------------- features

def _top_order(row: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Positions of row sorted by value descending, the lower column index first on ties."""
    return np.lexsort((cols, -row))


def _point_part(row: np.ndarray, cols: np.ndarray, p_i: float):
    """Features 0..19 of one point, its soft counts D_m (m = 0..5) and its neighbourhood,
    from its off-diagonal similarities `row` at columns `cols`."""
    f = np.zeros(NFEAT)
    a = abs(p_i)
    order = _top_order(row, cols)[:NTOP]
    top = row[order]
    nbrs = cols[order]
    if top.size < NTOP:
        top = np.concatenate([top, np.full(NTOP - top.size, top[-1])])
    cnt = int(np.count_nonzero(row > p_i))
    f[:NTOP] = top / a
    f[16] = p_i / a
    f[17] = cnt / row.size
    f[18] = row.mean() / a
    f[19] = np.log1p(cnt) / 10.0
    D = np.zeros(NSCALE)
    for m in range(NSCALE):
        q = 2.0 ** -m
        D[m] = np.sum(np.maximum(0.0, row - q * p_i)) / a
    return f, D, nbrs


def _density_contrast(D_i: np.ndarray, D_nbrs: np.ndarray) -> np.ndarray:
    """Features 26..31: (D_m(i) - M_m(i)) / max(D_m(i), M_m(i)), M_m(i) the largest D_m over
    the neighbourhood (0 when both are 0)."""
    M = D_nbrs.max(axis=0)
    top = np.maximum(D_i, M)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(top > 0, (D_i - M) / np.where(top > 0, top, 1.0), 0.0)


def row_features(S: np.ndarray, pref) -> np.ndarray:
    """(n, 32) features of every point (see the module header); n >= 2."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    if n < 2:
        raise ValueError("features need at least two points")
    p = np.broadcast_to(np.asarray(pref, dtype=np.float64), (n,))
    F = np.zeros((n, NFEAT))
    D = np.zeros((n, NSCALE))
    nbrs = []
    for i in range(n):
        cols = np.delete(np.arange(n), i)
        F[i], D[i], nb = _point_part(S[i, cols], cols, p[i])
        nbrs.append(nb)
    F[:, 20:26] = np.log1p(D) / 10.0
    for i in range(n):
        F[i, 26:32] = _density_contrast(D[i], D[nbrs[i]])
    return F


def row_features_sampled(row_of, n: int, pref, rows) -> np.ndarray:
    """Features of the points `rows` only, for problems too large to hold S: row_of(i)
    returns row i of S (length n, FP64).  Reads the rows of the sampled points and of their
    neighbourhoods; the values equal the matching rows of row_features(S, pref)."""
    p = np.broadcast_to(np.asarray(pref, dtype=np.float64), (n,))
    parts = {}

    def part(i):
        if i not in parts:
            cols = np.delete(np.arange(n), i)
            parts[i] = _point_part(np.asarray(row_of(i), dtype=np.float64)[cols], cols, p[i])
        return parts[i]

    out = np.zeros((len(rows), NFEAT))
    for k, i in enumerate(rows):
        f, D_i, nb = part(int(i))
        out[k] = f
        out[k, 20:26] = np.log1p(D_i) / 10.0
        out[k, 26:32] = _density_contrast(D_i, np.stack([part(int(j))[1] for j in nb]))
    return out


def g_fwd(v):
    """sign(v) (sqrt(1 + |v|) - 1), evaluated as sign(v) |v| / (sqrt(1 + |v|) + 1), which has
    no cancellation near zero."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    return np.sign(v) * (a / (np.sqrt(1.0 + a) + 1.0))


def g_inv(y):
    """sign(y) |y| (|y| + 2), the inverse of g_fwd."""
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    return np.sign(y) * (a * (a + 2.0))


def targets(result: "hap_ref.HapResult", pref) -> np.ndarray:
    """(n, L) training targets g((alpha^l_jj + rho^l_jj) / |p_j|) of a finished oracle run."""
    st = result.state
    L, n = st.alpha.shape[0], st.alpha.shape[1]
    p = np.broadcast_to(np.asarray(pref, dtype=np.float64), (n,))
    idx = np.arange(n)
    v = np.stack([(st.alpha[l][idx, idx].astype(np.float64) + st.rho[l][idx, idx]) / np.abs(p) for l in range(L)], 1)
    return g_fwd(v)


def warm_bases(Y: np.ndarray, pref) -> np.ndarray:
    """(L, n) availability bases B^l_j = g^-1(y_jl) |p_j| from network outputs Y (n, L)."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    p = np.broadcast_to(np.asarray(pref, dtype=np.float64), (n,))
    return (g_inv(Y) * np.abs(p)[:, None]).T.copy()


def warm_alpha0(B0: np.ndarray, n: int, dtype=np.float64) -> np.ndarray:
    """(L, n, n) initial availabilities from bases B0 (L, n): Eq. 2.2-2.3 at rho = 0."""
    B0 = np.asarray(B0, dtype=np.float64).astype(dtype)
    L = B0.shape[0]
    A = np.empty((L, n, n), dtype=dtype)
    for l in range(L):
        A[l] = np.minimum(dtype(0), B0[l])[None, :]
        A[l][np.arange(n), np.arange(n)] = B0[l]
    return A


def warm_run(S, pref, levels, damping, max_iters, stable_iters, Y, dtype=np.float64):
    """Warm-started run with the cold start as fallback: start from the warm availabilities of
    Y (or cold when Y is None); when that run does not converge, run again from the cold
    start.  Returns (result, fell_back)."""
    n = np.asarray(S).shape[0]
    if Y is not None:
        a0 = warm_alpha0(warm_bases(Y, pref), n, dtype)
        r = hap_ref.hap(S, pref, levels, damping, max_iters, stable_iters, alpha0=a0, dtype=dtype)
        if r.converged:
            return r, False
    return hap_ref.hap(S, pref, levels, damping, max_iters, stable_iters, dtype=dtype), Y is not None


# ---------------------------------------------------------------------------- perceptron

def param_count(n_in: int, hidden: int, n_out: int) -> int:
    return n_in * hidden + hidden + hidden * hidden + hidden + hidden * n_out + n_out


def unpack(flat, n_in: int, hidden: int, n_out: int) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != param_count(n_in, hidden, n_out):
        raise ValueError("parameter vector has the wrong size")
    shapes = [("W1", (n_in, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
              ("W3", (hidden, n_out)), ("b3", (n_out,))]
    P, o = {}, 0
    for k, sh in shapes:
        size = int(np.prod(sh))
        P[k] = flat[o:o + size].reshape(sh).copy()
        o += size
    return P


def pack(P: dict) -> np.ndarray:
    return np.concatenate([P[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def forward(P: dict, X: np.ndarray):
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"] + P["b3"]
    return y, (z1, h1, z2, h2)


def loss_and_grads(P: dict, X: np.ndarray, T: np.ndarray):
    """Mean-squared-error loss and its gradient for every parameter (backpropagation)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(P, X)
    m = y.size
    loss = float(np.sum((y - T) ** 2) / m)
    dy = 2.0 * (y - T) / m
    g = {"W3": h2.T @ dy, "b3": dy.sum(axis=0)}
    dh2 = (dy @ P["W3"].T) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return loss, g


def adam_step(P: dict, G: dict, M: dict, V: dict, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> None:
    """One Adam update in place; step counts from 1."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] * G[k]
        mh = M[k] / (1 - b1 ** step)
        vh = V[k] / (1 - b2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def train(P: dict, X, T, idx, batch: int, steps: int, lr: float, step0: int = 0, M=None, V=None):
    """Minibatch Adam: step s (0-based) uses the rows idx[s*batch:(s+1)*batch].  Returns the
    per-step losses; P, M and V are updated in place (M and V start at zero when None)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    idx = np.asarray(idx)
    M = {k: np.zeros_like(v) for k, v in P.items()} if M is None else M
    V = {k: np.zeros_like(v) for k, v in P.items()} if V is None else V
    losses = []
    for s in range(steps):
        rows = idx[s * batch:(s + 1) * batch]
        loss, G = loss_and_grads(P, X[rows], T[rows])
        adam_step(P, G, M, V, step0 + s + 1, lr)
        losses.append(loss)
    return np.array(losses), M, V
