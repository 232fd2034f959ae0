"""Pure-Python HAP evaluated from the defining sums (test infrastructure).

Every message is computed straight from its equation in Section 2, with explicit
loops and no algebraic shortcut:
  Eq. 2.1  rho_ij = s_ij + min(tau_i, -max_{k != j}(alpha_ik + s_ik))      (l > 1)
           rho_ij = s_ij - max_{k != j}(alpha_ik + s_ik)                     (l = 1)
  Eq. 2.2  alpha_ij = min(0, c_j + phi_j + rho_jj + sum_{k not in {i,j}} max(0, rho_kj))   (i != j)
  Eq. 2.3  alpha_jj = c_j + phi_j + sum_{k != j} max(0, rho_kj)
           (c and phi are dropped at the top level l = L)
  Eq. 2.4  tau^{l+1}_j = c^l_j + rho^l_jj + sum_{k != j} max(0, rho^l_kj)
  Eq. 2.5  phi^{l-1}_i = max_k(alpha^l_ik + s^l_ik)
  Eq. 2.6  c^l_i = max_j(alpha^l_ij + rho^l_ij)
  Eq. 2.8  e^l_i = argmax_j(alpha^l_ij + rho^l_ij), lowest index on ties
  Eq. 2.7  (optional, kappa given) s^{l+1}_ij = s_ij + delta^{l+1}_i for j != i, with the row
           offset delta^{l+1}_i = delta^l_i + kappa * max_{j != i}(alpha^l_ij + rho^l_ij),
           delta^1 = 0, recomputed in every iteration after the level's c update
The schedule and readings are the same as in ``hap_ref`` (schedule="mrhap" gives the
MapReduce schedule of Section 3: every level from the previous iteration's state, tau and
c not updated in the first iteration).  The cost is O(L N^3) per iteration, so this is for
N <= 8 only.

The number type is a parameter.  With ``fractions.Fraction`` inputs (integer
similarities, a rational damping such as 1/2 or 9/10) every operation (+, *,
max, min) is exact, so the result is the exact rational trajectory; +inf is
represented by None.
"""
from __future__ import annotations

from fractions import Fraction


def _min_tau(tau, x):
    return x if tau is None else (tau if tau < x else x)


def _colsum_plus(rho_l, j, N, zero, c_j):
    """c_j + rho_jj + sum_{k != j} max(0, rho_kj) (the right-hand side of Eq. 2.4)."""
    acc = c_j + rho_l[j][j]
    for k in range(N):
        if k != j:
            acc = acc + max(zero, rho_l[k][j])
    return acc


def hap_literal(S, pref, levels, damping, iters, num=Fraction, schedule="sequential", kappa=None):
    """S: N x N nested lists/array (diagonal ignored); pref: L x N; damping: number.

    Returns (labels, rho, alpha, c, phi, tau) as nested lists of `num`, and when `kappa` is
    given (level-sequential schedule only) the row offsets delta (L x N) as a seventh item.
    """
    N = len(S)
    L = int(levels)
    lam = num(damping) if not isinstance(damping, num) else damping
    one = num(1)
    zero = num(0)
    s = [[[num(pref[l][j]) if i == j else num(S[i][j]) for j in range(N)] for i in range(N)]
         for l in range(L)]
    rho = [[[zero] * N for _ in range(N)] for _ in range(L)]
    alpha = [[[zero] * N for _ in range(N)] for _ in range(L)]
    c = [[zero] * N for _ in range(L)]
    phi = [[zero] * N for _ in range(L)]
    tau = [[None] * N for _ in range(L)]
    delta = [[zero] * N for _ in range(L)]
    kap = None if kappa is None else (num(kappa) if not isinstance(kappa, num) else kappa)
    if kap is not None and schedule != "sequential":
        raise ValueError("the level-wise similarity update is defined for the level-sequential schedule")

    def rho_update(l):
        # Eq. 2.1 with damping
        new_rho = [[None] * N for _ in range(N)]
        for i in range(N):
            for j in range(N):
                mx = None
                for k in range(N):
                    if k == j:
                        continue
                    v = alpha[l][i][k] + s[l][i][k]
                    if mx is None or v > mx:
                        mx = v
                r = s[l][i][j] - mx if l == 0 else s[l][i][j] + _min_tau(tau[l][i], -mx)
                new_rho[i][j] = lam * rho[l][i][j] + (one - lam) * r
        rho[l] = new_rho

    def alpha_update(l):
        # Eq. 2.2 / 2.3 with damping
        top = (l == L - 1)
        new_alpha = [[None] * N for _ in range(N)]
        for j in range(N):
            base = zero if top else c[l][j] + phi[l][j]
            for i in range(N):
                if i == j:
                    acc = base
                    for k in range(N):
                        if k != j:
                            acc = acc + max(zero, rho[l][k][j])
                    a = acc
                else:
                    acc = base + rho[l][j][j]
                    for k in range(N):
                        if k != i and k != j:
                            acc = acc + max(zero, rho[l][k][j])
                    a = min(zero, acc)
                new_alpha[i][j] = lam * alpha[l][i][j] + (one - lam) * a
        alpha[l] = new_alpha

    def c_of(l):
        return [max(alpha[l][i][j] + rho[l][i][j] for j in range(N)) for i in range(N)]

    for t in range(1, iters + 1):
        if schedule == "mrhap":
            # first job: tau and c from the previous state (not at t = 1), then rho
            if t >= 2:
                new_c = [c_of(l) if l < L - 1 else c[l] for l in range(L)]
                for l in range(1, L):
                    tau[l] = [_colsum_plus(rho[l - 1], j, N, zero, new_c[l - 1][j]) for j in range(N)]
                for l in range(L):
                    c[l] = new_c[l]
            for l in range(L):
                rho_update(l)
            # second job: phi from the level above's previous alpha, then alpha
            new_phi = [[max(alpha[l + 1][i][k] + s[l + 1][i][k] for k in range(N)) for i in range(N)]
                       if l < L - 1 else phi[l] for l in range(L)]
            for l in range(L):
                phi[l] = new_phi[l]
            for l in range(L):
                alpha_update(l)
            continue
        for l in range(L):
            rho_update(l)
            alpha_update(l)
            # Eq. 2.4 (c^l from before its update), 2.5, 2.6
            if l < L - 1:
                tau[l + 1] = [_colsum_plus(rho[l], j, N, zero, c[l][j]) for j in range(N)]
            if l > 0:
                phi[l - 1] = [max(alpha[l][i][k] + s[l][i][k] for k in range(N)) for i in range(N)]
            if l < L - 1:
                c[l] = c_of(l)
            # Eq. 2.7: the next level's similarity, row offsets from this level's messages
            if kap is not None and l < L - 1:
                for i in range(N):
                    mx = None
                    for j in range(N):
                        if j != i:
                            v = alpha[l][i][j] + rho[l][i][j]
                            if mx is None or v > mx:
                                mx = v
                    delta[l + 1][i] = delta[l][i] + kap * mx
                    for j in range(N):
                        if j != i:
                            s[l + 1][i][j] = num(S[i][j]) + delta[l + 1][i]

    labels = []
    for l in range(L):
        row = []
        for i in range(N):
            best, arg = None, -1
            for j in range(N):
                v = alpha[l][i][j] + rho[l][i][j]
                if best is None or v > best:
                    best, arg = v, j
            row.append(arg)
        labels.append(row)
    if kap is not None:
        return labels, rho, alpha, c, phi, tau, delta
    return labels, rho, alpha, c, phi, tau
