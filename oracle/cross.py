"""Cross-oracles that pin the Brandes oracle from outside.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each routine here
reaches BC by a route that shares nothing with brandes.c:

  brute_force       enumerate every simple path from the definitions of
                    Sec. 1.1: d(s,t), lambda_st, lambda_st(v),
                    delta_st(v) = lambda_st(v) / lambda_st and
                    BC(v) = sum over ordered s != v != t of delta_st(v),
                    in exact rationals.  Tiny graphs only.
  allpairs_counts   all-pairs distances and shortest-path counts by
                    Floyd-Warshall with counting (a shortest path meets an
                    intermediate vertex k at most once because every weight is
                    positive, so paths through k number lambda_ik * lambda_kj).
  algorithm2        Algorithm 2 of Sec. 4.2.1: BC(v) is the sum, over pairs
                    (s,t) with d(s,t) = d(s,v) + d(v,t) and v not in {s,t}, of
                    lambda_sv * lambda_vt / lambda_st.
  algebraic         the dense algebraic method of Sec. 3.1 in exact integer and
                    rational arithmetic: path counts as the first non-zero
                    power of A (Compute Path Count, with the mask taken over
                    every earlier level, as its correctness argument states),
                    then Compute Dependency with
                    Delta_{l-1} = Mask(((D_l + Delta_l) div Lambda) . A, l-1)
                    mult Lambda, and BC as column sums of Delta without the
                    diagonal.  Unit weights only.
  algebraic_weighted
                    the algebraic method for integer weights 1..M (Sec. 3.2),
                    read as per-weight-class products: with A_c the 0/1 matrix
                    of the edges of weight c and levels taken as distances,
                    F_L = Mask_unreached(sum_c F_{L-c} . A_c) gives d and
                    lambda; the backward takes, for j at distance L from i,
                    Delta[i][j] = Lambda[i][j] * sum_c (X_{L+c} . A_c)[i][j]
                    with X_L = (1 + Delta) div Lambda on level L: a weighted
                    edge (j, k) of weight c leads to a successor exactly when
                    d(i,k) = d(i,j) + c.  Exact integers and rationals.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _adjacency(g):
    """Dict-of-lists adjacency with weights (1 when unweighted)."""
    adj = [[] for _ in range(g.n)]
    for v in range(g.n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            w = 1 if g.weight is None else int(g.weight[e])
            adj[v].append((int(g.col[e]), w))
    return adj


def brute_force(g):
    """(dist, count, bc): dist[s][t] (None = unreachable), count[s][t]
    (= lambda_st) and bc[v] as Fractions, by enumerating all simple paths."""
    n = g.n
    adj = _adjacency(g)
    dist = [[None] * n for _ in range(n)]
    count = [[0] * n for _ in range(n)]
    through = [[None] * n for _ in range(n)]  # through[s][t][v] = lambda_st(v)
    for s in range(n):
        best = [None] * n
        cnt = [0] * n
        thr = [dict() for _ in range(n)]
        # iterative DFS over simple paths starting at s
        stack = [(s, 1 << s, 0, ())]
        while stack:
            v, seen, length, inner = stack.pop()
            if best[v] is None or length < best[v]:
                best[v] = length
                cnt[v] = 1
                thr[v] = {x: 1 for x in inner}
            elif length == best[v]:
                cnt[v] += 1
                for x in inner:
                    thr[v][x] = thr[v].get(x, 0) + 1
            for x, w in adj[v]:
                if not (seen >> x) & 1:
                    stack.append((x, seen | (1 << x), length + w, inner + ((v,) if v != s else ())))
        for t in range(n):
            dist[s][t] = best[t]
            count[s][t] = cnt[t]
            through[s][t] = thr[t]
    bc = [Fraction(0)] * n
    for s in range(n):
        for t in range(n):
            if s == t or count[s][t] == 0:
                continue
            for v, c in through[s][t].items():
                bc[v] += Fraction(c, count[s][t])
    return dist, count, bc


def brute_force_edges(g):
    """Edge betweenness from the definition: for every ordered pair (s,t) the
    fraction of shortest s-t paths (all simple paths enumerated) that use each
    edge, summed.  Returns {(min(u,x), max(u,x)): Fraction}."""
    n = g.n
    adj = _adjacency(g)
    eb = {}
    for s in range(n):
        best = [None] * n
        cnt = [0] * n
        thr = [dict() for _ in range(n)]  # thr[t][edge] = shortest s-t paths through edge
        stack = [(s, 1 << s, 0, ())]
        while stack:
            v, seen, length, edges = stack.pop()
            if best[v] is None or length < best[v]:
                best[v] = length
                cnt[v] = 1
                thr[v] = {e: 1 for e in edges}
            elif length == best[v]:
                cnt[v] += 1
                for e in edges:
                    thr[v][e] = thr[v].get(e, 0) + 1
            for x, w in adj[v]:
                if not (seen >> x) & 1:
                    stack.append((x, seen | (1 << x), length + w, edges + ((min(v, x), max(v, x)),)))
        for t in range(n):
            if t == s or cnt[t] == 0:
                continue
            for e, c in thr[t].items():
                eb[e] = eb.get(e, Fraction(0)) + Fraction(c, cnt[t])
    return eb


INF = np.int64(1) << np.int64(50)


def allpairs_counts(g, exact: bool = False):
    """(D, L): int64 distances (INF = unreachable) and shortest-path counts
    (int64, or Python ints when ``exact``) by Floyd-Warshall with counting."""
    n = g.n
    D = np.full((n, n), INF, dtype=np.int64)
    L = np.zeros((n, n), dtype=object if exact else np.int64)
    np.fill_diagonal(D, 0)
    for i in range(n):
        L[i, i] = 1
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    w = np.ones(g.nnz, np.int64) if g.weight is None else g.weight.astype(np.int64)
    D[rows, g.col] = w
    for r, c in zip(rows, g.col):
        L[r, c] = 1
    idx = np.arange(n)
    for k in range(n):
        cand = D[:, k, None] + D[None, k, :]
        via = L[:, k, None] * L[None, k, :]
        shorter = cand < D
        equal = (cand == D) & (cand < INF)
        equal[k, :] = False
        equal[:, k] = False
        D = np.where(shorter, cand, D)
        L = np.where(shorter, via, np.where(equal, L + via, L))
        if not exact and np.any(L < 0):
            raise OverflowError("path count overflowed int64; use exact=True")
    del idx
    return D, L


def algorithm2(D, L, exact: bool = False):
    """BC(v) = sum over ordered (s,t), v not in {s,t}, d(s,t) = d(s,v) + d(v,t)
    of lambda_sv * lambda_vt / lambda_st  (Algorithm 2, Sec. 4.2.1)."""
    n = D.shape[0]
    out = [Fraction(0)] * n if exact else np.zeros(n, dtype=np.float64)
    for v in range(n):
        through = (D[:, v, None] + D[None, v, :] == D) & (D[:, v, None] < INF) & (D[None, v, :] < INF)
        through[v, :] = False
        through[:, v] = False
        if exact:
            ss, tt = np.nonzero(through)
            acc = Fraction(0)
            for s, t in zip(ss, tt):
                acc += Fraction(int(L[s, v]) * int(L[v, t]), int(L[s, t]))
            out[v] = acc
        else:
            num = L[:, v, None].astype(np.float64) * L[None, v, :].astype(np.float64)
            out[v] = float(np.sum(np.where(through, num / np.where(through, L, 1).astype(np.float64), 0.0)))
    return out


def algebraic(g):
    """(D, Lambda, Delta, bc) by the dense algebraic method of Sec. 3.1, in
    exact arithmetic (Python ints and Fractions).  D uses -1 for unreachable
    pairs; Delta[i][j] = delta_i*(j) including the diagonal delta_i*(i)."""
    if g.weight is not None:
        raise ValueError("the unweighted algebraic method needs unit weights")
    n = g.n
    A = np.zeros((n, n), dtype=object)
    A[:, :] = 0
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    for r, c in zip(rows, g.col):
        A[r, c] = 1
    # Compute Path Count: Z = A^l; the first non-zero (A^l)_ij is lambda_ij and
    # that l is d(i,j).
    D = np.full((n, n), -1, dtype=np.int64)
    Lam = np.zeros((n, n), dtype=object)
    Lam[:, :] = 0
    for i in range(n):
        D[i, i] = 0
        Lam[i, i] = 1
    Z = np.zeros((n, n), dtype=object)
    Z[:, :] = 0
    for i in range(n):
        Z[i, i] = 1
    level = 0
    while True:
        level += 1
        Z = Z.dot(A)
        first = (D < 0) & (Z != 0)
        if not first.any():
            break
        D[first] = level
        Lam[first] = Z[first]
    diam = int(D.max()) if n else 0
    # Compute Dependency, from the deepest level down to 1.
    Delta = np.zeros((n, n), dtype=object)
    Delta[:, :] = Fraction(0)
    Delta_l = np.zeros((n, n), dtype=object)
    Delta_l[:, :] = Fraction(0)
    for l in range(diam, 0, -1):
        Dl = (D == l)
        X = np.zeros((n, n), dtype=object)
        X[:, :] = Fraction(0)
        for i, j in zip(*np.nonzero(Dl)):
            X[i, j] = (1 + Delta_l[i, j]) / Fraction(int(Lam[i, j]))
        Y = X.dot(A)
        nxt = np.zeros((n, n), dtype=object)
        nxt[:, :] = Fraction(0)
        for i, j in zip(*np.nonzero(D == l - 1)):
            nxt[i, j] = Y[i, j] * int(Lam[i, j])
        Delta = Delta + nxt
        Delta_l = nxt
    bc = [sum((Delta[i, j] for i in range(n) if i != j), Fraction(0)) for j in range(n)]
    return D, Lam, Delta, bc


def algebraic_weighted(g):
    """(D, Lambda, Delta, bc) by per-weight-class products (Sec. 3.2, as read
    in the module docstring), in exact arithmetic.  Integer weights >= 1;
    unit weights give the method of Sec. 3.1 with M = 1."""
    n = g.n
    w = np.ones(g.col.size, dtype=np.int64) if g.weight is None else np.asarray(g.weight, dtype=np.int64)
    M = int(w.max()) if w.size else 1
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    A = []
    for c in range(1, M + 1):
        Ac = np.zeros((n, n), dtype=object)
        Ac[:, :] = 0
        for r, col, wc in zip(rows, g.col, w):
            if wc == c:
                Ac[r, col] = 1
        A.append(Ac)
    zero = np.zeros((n, n), dtype=object)
    zero[:, :] = 0
    # Forward: levels are distances.  F[L][i][j] = lambda_ij where d(i,j) = L.
    D = np.full((n, n), -1, dtype=np.int64)
    Lam = zero.copy()
    F = [zero.copy()]
    for i in range(n):
        D[i, i] = 0
        Lam[i, i] = 1
        F[0][i, i] = 1
    L, empty_run = 0, 0
    while empty_run < M:
        L += 1
        P = zero.copy()
        for c in range(1, M + 1):
            if L - c >= 0:
                P = P + F[L - c].dot(A[c - 1])
        first = (D < 0) & (P != 0)
        Fl = zero.copy()
        Fl[first] = P[first]
        D[first] = L
        Lam[first] = P[first]
        F.append(Fl)
        empty_run = 0 if first.any() else empty_run + 1
    top = int(D.max()) if n else 0
    # Backward, from the deepest level down to 0 (level 0 gives the diagonal).
    X = {}
    Delta = zero.copy()
    Delta[:, :] = Fraction(0)
    for l in range(top, -1, -1):
        Y = zero.copy()
        Y[:, :] = Fraction(0)
        for c in range(1, M + 1):
            if l + c in X:
                Y = Y + X[l + c].dot(A[c - 1])
        Xl = zero.copy()
        Xl[:, :] = Fraction(0)
        for i, j in zip(*np.nonzero(D == l)):
            Delta[i, j] = Y[i, j] * int(Lam[i, j])
            Xl[i, j] = (1 + Delta[i, j]) / Fraction(int(Lam[i, j]))
        X[l] = Xl
    bc = [sum((Delta[i, j] for i in range(n) if i != j), Fraction(0)) for j in range(n)]
    return D, Lam, Delta, bc
