"""Plain FP64 HAP (test infrastructure; see the package header).

Follows Algorithm 1 of the paper (Section 2): for every iteration, for every
level l = 1..L in order, update the responsibilities (Eq. 2.1) and damp them,
update the availabilities (Eq. 2.2, 2.3) and damp them, then update the
inter-level messages tau, phi and the cluster preference c (Eq. 2.4-2.6).
After the last iteration the exemplar of every point at every level is the
argmax of alpha + rho (Eq. 2.8).

Readings of points the paper leaves open (each is listed in the design notes):
  * Levels run one after another inside an iteration (Algorithm 1), not all at
    once from the previous state.
  * Level l emits tau^{l+1} (up) and phi^{l-1} (down) after its own rho and
    alpha updates, and updates c^l last; tau^{l+1} therefore uses c^l from the
    previous iteration.  At iteration 1 that c is 0 (the initial value).
  * Eq. 2.1 carries the tau clip only for l > 1 (tau^1 is +inf from the
    initialisation); Eq. 2.2-2.3 carry c and phi only for l < L, so the top level
    uses the plain AP availability and L = 1 is exactly plain AP.
  * Damping: new = lambda*old + (1-lambda)*computed, for rho and alpha only;
    alpha is computed from the already damped rho.
  * max_{k != j} runs over every column k != j including k = i (whose
    similarity is the preference); a maximum attained twice gives M2 = M1.
  * argmax ties go to the lowest index.
  * The similarity is the same at every level unless kappa != 0 (the optional
    Eq. 2.7 update is off by default); the diagonal s^l_jj holds the level-l
    preference p^l_j.
  * Eq. 2.7 (kappa != 0, level-sequential schedule only): the maximum over j != i
    leaves one number per row, so the update adds a per-row offset to the
    off-diagonal of the next level's similarity, s^{l+1}_ij = s_ij + delta^{l+1}_i
    with delta^{l+1}_i = delta^l_i + kappa * max_{j != i}(alpha^l_ij + rho^l_ij) and
    delta^1 = 0.  It runs as the last step of level l in every iteration (after the
    c update, from that iteration's alpha^l and rho^l), so delta is recomputed in
    every iteration and not accumulated over iterations; the diagonal keeps the
    preference.
  * Stopping with K > 0: after each iteration t the labels of every level are
    compared with those of iteration t-1; the stable count goes up by one when
    none changed (t >= 2) and resets to 0 otherwise; the run stops at the end of
    the iteration where the count reaches K.

The column sum over k not in {i, j} of Eq. 2.2 is evaluated as the full column
sum minus the (i, j) term; the pure-Python evaluator in ``literal`` sums the
defining terms directly and pins this identity.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class HapState:
    """Everything that determines the continuation of a run (Algorithm 1 state)."""
    rho: np.ndarray      # (L, N, N) responsibilities
    alpha: np.ndarray    # (L, N, N) availabilities
    c: np.ndarray        # (L, N) cluster preference, Eq. 2.6
    phi: np.ndarray      # (L, N) downward message, Eq. 2.5 (phi^l is sent by level l+1)
    tau: np.ndarray      # (L, N) upward message, Eq. 2.4 (tau^1 = +inf)
    delta: np.ndarray | None = None    # (L, N) Eq. 2.7 row offsets of s^l (delta^1 = 0)
    t: int = 0           # completed iterations
    stable: int = 0      # consecutive iterations with unchanged labels
    labels: np.ndarray | None = None   # (L, N) labels of iteration t

    def copy(self) -> "HapState":
        return HapState(self.rho.copy(), self.alpha.copy(), self.c.copy(), self.phi.copy(),
                        self.tau.copy(), None if self.delta is None else self.delta.copy(), self.t,
                        self.stable, None if self.labels is None else self.labels.copy())


@dataclass
class HapResult:
    labels: np.ndarray           # (L, N) int64 exemplar index of every point at every level
    iters: int                   # iterations performed (the stop iteration when converged)
    converged: bool              # stable count reached K
    state: HapState
    Q: np.ndarray                # (L, N) last column sums rho_jj + sum_{k!=j} max(0, rho_kj)
    history: list = field(default_factory=list)


def level_similarity(S: np.ndarray, pref_l: np.ndarray, dtype=np.float64) -> np.ndarray:
    """s^l: the off-diagonal of S with the level-l preferences on the diagonal."""
    s = np.array(S, dtype=dtype, copy=True)
    np.fill_diagonal(s, pref_l)
    return s


def offset_similarity(S: np.ndarray, pref_l: np.ndarray, delta_l: np.ndarray, dtype=np.float64) -> np.ndarray:
    """s^l under Eq. 2.7: S_ij + delta^l_i off the diagonal, the level-l preferences on it."""
    S = np.asarray(S, dtype=dtype)
    s = S + np.asarray(delta_l, dtype=dtype)[:, None]
    np.fill_diagonal(s, pref_l)
    return s


def offdiag_max(v: np.ndarray) -> np.ndarray:
    """max_{j != i} v_ij of every row (-inf for a 1 x 1 matrix)."""
    w = np.array(v, copy=True)
    np.fill_diagonal(w, -np.inf)
    return np.max(w, axis=1)


def init_state(N: int, L: int, alpha0: np.ndarray | None = None, dtype=np.float64) -> HapState:
    """Algorithm 1 initialisation: alpha = rho = 0, tau = +inf, phi = c = 0."""
    alpha = np.zeros((L, N, N), dtype) if alpha0 is None else np.array(alpha0, dtype=dtype, copy=True)
    return HapState(rho=np.zeros((L, N, N), dtype), alpha=alpha, c=np.zeros((L, N), dtype),
                    phi=np.zeros((L, N), dtype), tau=np.full((L, N), np.inf, dtype),
                    delta=np.zeros((L, N), dtype))


def responsibility(s: np.ndarray, alpha: np.ndarray, tau: np.ndarray | None) -> np.ndarray:
    """Undamped Eq. 2.1 for one level: s_ij + min(tau_i, -max_{k!=j}(alpha_ik + s_ik)).

    tau=None is the l = 1 case (tau = +inf), giving s_ij - max_{k!=j}(...).
    s may also be a block of whole rows (r x N, each row's own diagonal entry holding its
    preference); tau then has r entries.
    """
    N = s.shape[1]
    rows = np.arange(s.shape[0])
    v = alpha + s
    k1 = np.argmax(v, axis=1)                 # first maximum (lowest index)
    M1 = v[rows, k1]
    v[rows, k1] = -np.inf
    M2 = np.max(v, axis=1)                    # maximum over k != k1
    m = np.repeat(M1[:, None], N, axis=1)     # max_{k != j}: M1 unless j is the argmax
    m[rows, k1] = M2
    if tau is None:
        return s - m
    return s + np.minimum(tau[:, None], -m)


def column_sums(rho: np.ndarray) -> np.ndarray:
    """Q_j = rho_jj + sum_{k != j} max(0, rho_kj) (the common part of Eq. 2.2-2.4)."""
    pos = np.maximum(rho, rho.dtype.type(0))
    idx = np.arange(rho.shape[0])
    pos[idx, idx] = rho[idx, idx]
    return pos.sum(axis=0)


def availability(rho: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Undamped Eq. 2.2 (i != j) and Eq. 2.3 (i == j) given B_j = [c_j + phi_j +] Q_j."""
    zero = rho.dtype.type(0)
    a = np.minimum(zero, B[None, :] - np.maximum(rho, zero))
    idx = np.arange(rho.shape[0])
    a[idx, idx] = B - rho[idx, idx]
    return a


def labels_of(state: HapState) -> np.ndarray:
    """Eq. 2.8 at every level: e^l_i = lowest argmax_j (alpha^l_ij + rho^l_ij)."""
    return np.argmax(state.alpha + state.rho, axis=2)


def _iteration_mrhap(st: HapState, s, L: int, lam, oml, Q, record, c_zero: bool) -> None:
    """One iteration of the MapReduce schedule (Section 3): every level is updated from the
    state the previous iteration left.  The first job updates tau and c (both skipped in the
    first iteration) and then rho at every level; the second updates phi (from the level
    above's availabilities as they were before this job) and then alpha at every level."""
    # job 1: tau and c from the previous state (not in the first iteration), then rho
    if st.t >= 2:
        c_new = st.c.copy()
        for l in range(L - 1):
            if not c_zero:
                c_new[l] = np.max(st.alpha[l] + st.rho[l], axis=1)          # Eq. 2.6
        for l in range(1, L):
            st.tau[l] = c_new[l - 1] + column_sums(st.rho[l - 1])          # Eq. 2.4
        st.c = c_new
    for l in range(L):
        rhat = responsibility(s[l], st.alpha[l], None if l == 0 else st.tau[l])   # Eq. 2.1
        st.rho[l] = lam * st.rho[l] + oml * rhat
    # job 2: phi from the level above's previous availabilities, then alpha
    phi_new = st.phi.copy()
    for l in range(L - 1):
        phi_new[l] = np.max(st.alpha[l + 1] + s[l + 1], axis=1)            # Eq. 2.5
    st.phi = phi_new
    for l in range(L):
        Q[l] = column_sums(st.rho[l])
        B = (st.c[l] + st.phi[l]) + Q[l] if l < L - 1 else Q[l].copy()
        st.alpha[l] = lam * st.alpha[l] + oml * availability(st.rho[l], B)  # Eq. 2.2 / 2.3
        if record is not None:
            record(st.t, l, st)


def _iteration_block(st: HapState, s, L: int, lam, oml, Q, R: int, record) -> None:
    """One level-sequential iteration that updates rows [0, R) only (see `hap`, `rows`)."""
    for l in range(L):
        rhat = responsibility(s[l][:R], st.alpha[l][:R], None if l == 0 else st.tau[l][:R])
        st.rho[l][:R] = lam * st.rho[l][:R] + oml * rhat
        Q[l] = column_sums(st.rho[l])          # rows >= R hold zeros and add nothing
        B = (st.c[l] + st.phi[l]) + Q[l] if l < L - 1 else Q[l].copy()
        st.alpha[l][:R] = lam * st.alpha[l][:R] + oml * availability(st.rho[l], B)[:R]
        if l < L - 1:
            st.tau[l + 1] = st.c[l] + Q[l]
        if l > 0:
            st.phi[l - 1][:R] = np.max(st.alpha[l][:R] + s[l][:R], axis=1)
        if l < L - 1:
            st.c[l][:R] = np.max(st.alpha[l][:R] + st.rho[l][:R], axis=1)
        if record is not None:
            record(st.t, l, st)


def hap(S, pref, levels: int, damping: float, max_iters: int, stable_iters: int = 0,
        alpha0=None, state: HapState | None = None, record=None, c_zero: bool = False,
        dtype=np.float64, schedule: str = "sequential", kappa: float = 0.0,
        rows: int | None = None) -> HapResult:
    """Run HAP (Algorithm 1), in FP64 unless `dtype` says otherwise.

    The paper fixes no precision.  dtype=np.float32 evaluates the same steps with every
    operation rounded to single precision (NumPy computes float32 arithmetic in float32,
    and its column sum over axis 0 adds the rows one after another), which is the
    arithmetic of an FP32 implementation that sums columns in row order.

    S      (N, N) similarity; its diagonal is ignored.
    pref   preferences: scalar, (N,) shared by all levels, or (L, N).
    alpha0 optional (L, N, N) initial availabilities (warm start); everything else starts
           at the Algorithm 1 initial values.
    state  optional state to continue from (checkpoint / resume).
    record optional callable(t, l, state) called after every level update.
    c_zero diagnosis switch: keep c = 0 (a constant cluster preference) instead of Eq. 2.6.
    schedule "sequential": the levels one after another inside an iteration (Algorithm 1);
           "mrhap": the MapReduce schedule of Section 3 (every level from the previous
           iteration's state; tau and c not updated in the first iteration).
    kappa  Eq. 2.7 weight in [0, 1]; 0 (the default) keeps s^l = s at every level.  Defined
           for the level-sequential schedule only.
    rows   one block of a run split by rows (sequential schedule, kappa = 0): only rows
           [0, rows) are updated; the others keep their initial messages, so they add nothing
           to the column sums and the sums hold this block's contribution alone.  Per-row
           quantities (c, phi) of the other rows stay at their initial values; tau is formed
           for every column as in the full run.  None updates every row.
    """
    if schedule not in ("sequential", "mrhap"):
        raise ValueError(schedule)
    if not 0.0 <= float(kappa) <= 1.0:
        raise ValueError("kappa must lie in [0, 1]")
    if float(kappa) != 0.0 and schedule != "sequential":
        raise ValueError("the level-wise similarity update is defined for the level-sequential schedule")
    if rows is not None and (schedule != "sequential" or float(kappa) != 0.0):
        raise ValueError("a row block is defined for the level-sequential schedule without kappa")
    dt = np.dtype(dtype).type
    S = np.asarray(S, dtype=dt)
    N = S.shape[0]
    L = int(levels)
    lam = dt(damping)
    oml = dt(1.0 - float(damping))
    p = np.asarray(pref, dtype=dt)
    if p.ndim == 0:
        p = np.full((L, N), p, dtype=dt)
    elif p.ndim == 1:
        p = np.repeat(p[None, :], L, axis=0)
    s = [level_similarity(S, p[l], dt) for l in range(L)]

    R = N if rows is None else int(rows)
    if not 1 <= R <= N:
        raise ValueError("rows must lie in [1, N]")
    st = init_state(N, L, alpha0, dt) if state is None else state.copy()
    if st.delta is None:
        st.delta = np.zeros((L, N), dt)
    kap = dt(kappa)
    use_kappa = float(kappa) != 0.0
    Q = np.zeros((L, N), dt)
    converged = False
    for _ in range(max_iters):
        st.t += 1
        if schedule == "mrhap":
            _iteration_mrhap(st, s, L, lam, oml, Q, record, c_zero)
        if rows is not None:
            _iteration_block(st, s, L, lam, oml, Q, R, record)
        for l in (range(L) if schedule == "sequential" and rows is None else ()):
            if use_kappa and l > 0:
                s[l] = offset_similarity(S, p[l], st.delta[l], dt)   # s^l of this iteration (Eq. 2.7)
            # Eq. 2.1, then damp
            rhat = responsibility(s[l], st.alpha[l], None if l == 0 else st.tau[l])
            st.rho[l] = lam * st.rho[l] + oml * rhat
            # Eq. 2.2 / 2.3 with the damped rho, then damp
            Q[l] = column_sums(st.rho[l])
            B = (st.c[l] + st.phi[l]) + Q[l] if l < L - 1 else Q[l].copy()
            st.alpha[l] = lam * st.alpha[l] + oml * availability(st.rho[l], B)
            # Eq. 2.4 (up, uses c^l before its update), Eq. 2.5 (down), Eq. 2.6
            if l < L - 1:
                st.tau[l + 1] = st.c[l] + Q[l]
            if l > 0:
                st.phi[l - 1] = np.max(st.alpha[l] + s[l], axis=1)
            if l < L - 1 and not c_zero:
                st.c[l] = np.max(st.alpha[l] + st.rho[l], axis=1)
            # Eq. 2.7 (optional): row offsets of the next level's similarity
            if use_kappa and l < L - 1:
                st.delta[l + 1] = st.delta[l] + kap * offdiag_max(st.alpha[l] + st.rho[l])
            if record is not None:
                record(st.t, l, st)
        if stable_iters > 0:
            e = labels_of(st)
            if st.labels is not None and st.t >= 2 and np.array_equal(e, st.labels):
                st.stable += 1
            else:
                st.stable = 0
            st.labels = e
            if st.stable >= stable_iters:
                converged = True
                break
    if st.labels is None or stable_iters == 0:
        st.labels = labels_of(st)
    return HapResult(labels=st.labels.copy(), iters=st.t, converged=converged, state=st, Q=Q)


def exemplar_set(labels_l: np.ndarray) -> np.ndarray:
    """Distinct exemplar indices at one level (sorted)."""
    return np.unique(labels_l)
