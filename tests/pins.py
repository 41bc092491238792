"""Independent mathematical references used to pin the oracle (tests only).

Nothing here calls the oracle or the HIP library.  Each function computes the
quantity from a different route than Algorithm 2 / Algorithm 1 do:

* even_vertices(d)          the vertex set P_d of PP_d (eq. spcConst / def.parPoly)
* min_norm_point(P)         Wolfe's finite min-norm-point algorithm (1976) -> the
                            Euclidean projection onto conv(vertices), by brute force
* in_parity_polytope(z)     membership of z in PP_d as an LP feasibility problem
                            over vertex weights (HiGHS)
* vi_gap(v, z)              max over vertices e of <v - z, e - z>; z is the
                            projection of v iff z in PP_d and this is <= 0
* feldman_lp / yannakakis_lp  the LP decoding problem (eq. feldmanLP) solved by
                            a generic simplex in two formulations (Sec. 2)
* ml_decode                 exhaustive ML decoding over all codewords (Sec. 2)
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog, minimize_scalar


def even_vertices(d: int) -> np.ndarray:
    out = [e for e in itertools.product((0, 1), repeat=d) if sum(e) % 2 == 0]
    return np.array(out, dtype=np.float64)


def min_norm_point(P: np.ndarray, tol: float = 1e-13, max_iter: int = 10000) -> np.ndarray:
    """Point of minimum Euclidean norm in conv(rows of P) (Wolfe's algorithm)."""
    P = np.asarray(P, dtype=np.float64)
    scale = max(1.0, float(np.max(np.sum(P * P, axis=1))))
    S = [int(np.argmin(np.sum(P * P, axis=1)))]
    lam = np.array([1.0])
    x = P[S[0]].copy()
    for _ in range(max_iter):
        j = int(np.argmin(P @ x))
        if x @ x - P[j] @ x <= tol * scale or j in S:
            break
        S.append(j)
        lam = np.append(lam, 0.0)
        while True:
            Q = P[S]
            k = len(S)
            A = np.zeros((k + 1, k + 1))
            A[:k, :k] = Q @ Q.T
            A[:k, k] = 1.0
            A[k, :k] = 1.0
            rhs = np.zeros(k + 1)
            rhs[k] = 1.0
            sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
            a = sol[:k]
            if np.all(a > 1e-15):
                lam = a
                x = Q.T @ lam
                break
            neg = a <= 1e-15
            theta = np.min(lam[neg] / (lam[neg] - a[neg]))
            lam = lam + theta * (a - lam)
            keep = lam > 1e-15
            S = [s for s, kf in zip(S, keep) if kf]
            lam = lam[keep]
            lam = lam / lam.sum()
            x = P[S].T @ lam
    return x


def project_brute(v: np.ndarray) -> np.ndarray:
    """Pi_PPd(v) as the min-norm point of {e - v : e in P_d}, shifted back."""
    v = np.asarray(v, dtype=np.float64)
    V = even_vertices(v.size)
    return min_norm_point(V - v) + v


def in_parity_polytope(z: np.ndarray, tol: float = 1e-9) -> bool:
    """Is z a convex combination of even-weight binary vectors?  Solved as an LP that
    minimises the L1 infeasibility sum |V^T a - z| over the simplex of vertex weights a."""
    z = np.asarray(z, dtype=np.float64)
    V = even_vertices(z.size)
    k, d = V.shape
    # variables: a (k), s_plus (d), s_minus (d)
    c = np.concatenate([np.zeros(k), np.ones(2 * d)])
    A_eq = np.zeros((d + 1, k + 2 * d))
    A_eq[:d, :k] = V.T
    A_eq[:d, k:k + d] = -np.eye(d)
    A_eq[:d, k + d:] = np.eye(d)
    A_eq[d, :k] = 1.0
    b_eq = np.concatenate([z, [1.0]])
    res = linprog(c, A_eq=A_eq, b_eq=b_eq, bounds=[(0, None)] * (k + 2 * d), method="highs",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        return False
    return float(res.fun) <= tol


def vi_gap(v: np.ndarray, z: np.ndarray) -> float:
    """max_e <v - z, e - z> over the vertices e of PP_d (<= 0 at the projection)."""
    V = even_vertices(len(z))
    return float(np.max((V - z) @ (np.asarray(v) - z)))


def _check_rows(row_ptr, col_idx):
    return [col_idx[row_ptr[j]:row_ptr[j + 1]] for j in range(len(row_ptr) - 1)]


def feldman_lp(row_ptr, col_idx, n: int, gamma: np.ndarray):
    """min gamma^T x s.t. P_j x in PP_d for all j, with PP_d written as the convex
    hull of its even-weight vertices (one weight per vertex per check)."""
    rows = _check_rows(row_ptr, col_idx)
    nv = n
    blocks = []
    for nb in rows:
        d = len(nb)
        blocks.append((nb, even_vertices(d)))
    nw = sum(V.shape[0] for _, V in blocks)
    nvar = nv + nw
    A, b = [], []
    off = nv
    for nb, V in blocks:
        k = V.shape[0]
        row = np.zeros(nvar)
        row[off:off + k] = 1.0
        A.append(row)
        b.append(1.0)
        for t, i in enumerate(nb):
            row = np.zeros(nvar)
            row[i] = 1.0
            row[off:off + k] = -V[:, t]
            A.append(row)
            b.append(0.0)
        off += k
    c = np.concatenate([np.asarray(gamma, np.float64), np.zeros(nw)])
    bounds = [(0.0, 1.0)] * nv + [(0.0, None)] * nw
    res = linprog(c, A_eq=np.array(A), b_eq=np.array(b), bounds=bounds, method="highs-ds")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun), res.x[:nv]


def yannakakis_lp(row_ptr, col_idx, n: int, gamma: np.ndarray):
    """The same LP with Yannakakis' lifted description of PP_d (Sec. 2): per check,
    weights mu_s over even s <= d and z_{i,s} in [0, mu_s] with
    sum_s mu_s = 1, x_i = sum_s z_{i,s}, sum_i z_{i,s} = s mu_s."""
    rows = _check_rows(row_ptr, col_idx)
    idx = n
    layout = []
    for nb in rows:
        d = len(nb)
        ss = list(range(0, d + 1, 2))
        mu_idx = {s: idx + t for t, s in enumerate(ss)}
        idx += len(ss)
        z_idx = {}
        for i in nb:
            for s in ss:
                z_idx[(i, s)] = idx
                idx += 1
        layout.append((nb, ss, mu_idx, z_idx))
    nvar = idx
    Aeq, beq, Aub, bub = [], [], [], []
    for nb, ss, mu_idx, z_idx in layout:
        row = np.zeros(nvar)
        for s in ss:
            row[mu_idx[s]] = 1.0
        Aeq.append(row); beq.append(1.0)
        for i in nb:
            row = np.zeros(nvar)
            row[i] = 1.0
            for s in ss:
                row[z_idx[(i, s)]] = -1.0
            Aeq.append(row); beq.append(0.0)
        for s in ss:
            row = np.zeros(nvar)
            for i in nb:
                row[z_idx[(i, s)]] = 1.0
            row[mu_idx[s]] = -float(s)
            Aeq.append(row); beq.append(0.0)
            for i in nb:
                row = np.zeros(nvar)
                row[z_idx[(i, s)]] = 1.0
                row[mu_idx[s]] = -1.0
                Aub.append(row); bub.append(0.0)
    c = np.zeros(nvar)
    c[:n] = gamma
    bounds = [(0.0, 1.0)] * n + [(0.0, None)] * (nvar - n)
    res = linprog(c, A_ub=np.array(Aub), b_ub=np.array(bub), A_eq=np.array(Aeq), b_eq=np.array(beq),
                  bounds=bounds, method="highs-ds")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun), res.x[:n]


def codewords(H_dense: np.ndarray) -> np.ndarray:
    """All codewords of the binary code with parity-check matrix H (small n only)."""
    H = (np.asarray(H_dense) % 2).astype(np.uint8)
    m, n = H.shape
    A = H.copy()
    pivots = []
    r = 0
    for c in range(n):
        p = next((i for i in range(r, m) if A[i, c]), None)
        if p is None:
            continue
        A[[r, p]] = A[[p, r]]
        for i in range(m):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        pivots.append(c)
        r += 1
        if r == m:
            break
    free = [c for c in range(n) if c not in pivots]
    words = []
    for bits in itertools.product((0, 1), repeat=len(free)):
        x = np.zeros(n, np.uint8)
        x[free] = bits
        for row, c in zip(range(len(pivots)), pivots):
            x[c] = (A[row, free] @ np.array(bits, np.uint8)) % 2 if free else 0
        words.append(x)
    W = np.array(words, dtype=np.uint8)
    assert not np.any((H.astype(np.int64) @ W.T.astype(np.int64)) % 2)
    return W


def ml_decode(H_dense: np.ndarray, gamma: np.ndarray):
    """argmin_{x in C} gamma^T x by enumeration; returns (codeword, cost, unique?)."""
    W = codewords(H_dense)
    cost = W.astype(np.float64) @ np.asarray(gamma, np.float64)
    order = np.argsort(cost)
    unique = len(cost) == 1 or cost[order[1]] - cost[order[0]] > 1e-9
    return W[order[0]], float(cost[order[0]]), unique


def lagrangian_x_argmin(gamma_i: float, z_i: np.ndarray, lam_i: np.ndarray, mu: float) -> float:
    """argmin over x in [0,1] of gamma_i x + sum_j lam_j (x - z_j) + mu/2 sum_j (x - z_j)^2,
    the i-th coordinate of the x-update's objective (eq. augLag), by a bounded
    scalar minimiser (no closed form used)."""
    def f(x):
        return gamma_i * x + float(np.sum(lam_i * (x - z_i))) + 0.5 * mu * float(np.sum((x - z_i) ** 2))
    res = minimize_scalar(f, bounds=(0.0, 1.0), method="bounded", options={"xatol": 1e-12})
    cands = [0.0, 1.0, float(res.x)]
    return min(cands, key=f)
