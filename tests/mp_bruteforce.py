"""Arbitrary-precision brute force of the ground-state map q[n] on tiny systems.

Independent of the oracle: mpmath matrices throughout, Cholesky congruence
factor, dense symmetric eigensolver, bisection for mu, and the response taken
as a central finite difference with a step so small (1e-15 at 50 digits) that
truncation (~h^2) and rounding (~10^-50/h) errors are both below 1e-25.
"""

from __future__ import annotations

import mpmath as mp
import numpy as np


def _mat(a):
    return mp.matrix([[mp.mpf(float(x)) for x in row] for row in np.asarray(a)])


def q_of_n_mp(H0, S, gamma, W, offsets, n, n_electrons, kT, dps=50):
    with mp.workdps(dps):
        nb = len(H0)
        N = len(gamma)
        H0m, Sm, Gm = _mat(H0), _mat(S), _mat(gamma)
        n = [mp.mpf(x) if not isinstance(x, mp.mpf) else x for x in n]
        nq, nm = n[:N], n[N:]
        atom_of = []
        for a in range(N):
            atom_of += [a] * (offsets[a + 1] - offsets[a])
        L = mp.cholesky(Sm)
        Linv = mp.inverse(L)
        Z = Linv.T
        eps_all, vecs_all = [], []
        for s in (1, -1):
            u = [sum(Gm[a, b] * nq[b] for b in range(N)) + s * mp.mpf(float(W)) * nm[a] for a in range(N)]
            H = mp.matrix(nb, nb)
            for i in range(nb):
                for j in range(nb):
                    H[i, j] = H0m[i, j] + (u[atom_of[i]] + u[atom_of[j]]) * Sm[i, j] / 2
            Hp = Z.T * H * Z
            E, Q = mp.eigsy(Hp)
            eps_all.append([E[k] for k in range(nb)])
            vecs_all.append(Q)
        kT = mp.mpf(float(kT))

        def count(mu):
            return sum(1 / (1 + mp.exp((e - mu) / kT)) for es in eps_all for e in es)

        lo = min(min(es) for es in eps_all) - 60 * kT
        hi = max(max(es) for es in eps_all) + 60 * kT
        target = mp.mpf(float(n_electrons))
        for _ in range(int(dps * 3.5) + 20):
            mid = (lo + hi) / 2
            if count(mid) < target:
                lo = mid
            else:
                hi = mid
        mu = (lo + hi) / 2
        pops = []
        for es, Q in zip(eps_all, vecs_all):
            f = [1 / (1 + mp.exp((e - mu) / kT)) for e in es]
            Dp = mp.matrix(nb, nb)
            for i in range(nb):
                for j in range(nb):
                    Dp[i, j] = sum(Q[i, k] * f[k] * Q[j, k] for k in range(nb))
            D = Z * Dp * Z.T
            DS = D * Sm
            pops.append([sum(DS[i, i] for i in range(offsets[a], offsets[a + 1])) for a in range(N)])
        return [pops[0][a] + pops[1][a] for a in range(N)] + [pops[0][a] - pops[1][a] for a in range(N)]


def response_mp(H0, S, gamma, W, offsets, n_ref, v, n_electrons, kT, dps=50, h="1e-15"):
    with mp.workdps(dps):
        h = mp.mpf(h)
        nref = [mp.mpf(float(x)) for x in n_ref]
        vv = [mp.mpf(float(x)) for x in v]
        plus = q_of_n_mp(H0, S, gamma, W, offsets, [a + h * b for a, b in zip(nref, vv)], n_electrons, kT, dps)
        minus = q_of_n_mp(H0, S, gamma, W, offsets, [a - h * b for a, b in zip(nref, vv)], n_electrons, kT, dps)
        return np.array([float((p - m) / (2 * h)) for p, m in zip(plus, minus)])
