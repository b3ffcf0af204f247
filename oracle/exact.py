"""Exact rational-arithmetic (fractions.Fraction) versions of Alg. 1-4.

TEST INFRASTRUCTURE ONLY (same rules as the FP64 oracle).  Written
independently of the FP64 oracle, with plain nested lists, for tiny inputs.
The paper states that the s-step variants reproduce the classical iterates in
exact arithmetic (Section 1, Section 3.1 derivation of eq. (recur) and
Section 3.2); with Fractions that identity can be checked for equality.

The b x b systems are solved by Gaussian elimination over the rationals, which
gives the exact solution of the same linear system the Cholesky-based solvers
approximate.
"""

from fractions import Fraction


def _F(v):
    return Fraction(v)


def _mat(rows, cols):
    return [[Fraction(0)] * cols for _ in range(rows)]


def _solve(M, rhs):
    """Exact solution of M x = rhs (M nonsingular) by Gaussian elimination."""
    k = len(rhs)
    A = [list(M[i]) + [rhs[i]] for i in range(k)]
    for c in range(k):
        p = next(r for r in range(c, k) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        for r in range(k):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [A[r][q] - f * A[c][q] for q in range(k + 1)]
    return [A[i][k] / A[i][i] for i in range(k)]


def _dot(a, b):
    return sum((x * y for x, y in zip(a, b)), Fraction(0))


def primal_bcd_exact(X, y, lam, blocks, s, w0=None):
    """Alg. 1 when s == 1, Alg. 2 otherwise; `blocks` lists the index blocks of
    iterations 1..H.  X is a d x n list of lists of Fractions."""
    d, n = len(X), len(X[0])
    lam = _F(lam)
    w = [Fraction(0)] * d if w0 is None else [_F(v) for v in w0]
    z = [_dot([X[i][c] for i in range(d)], w) for c in range(n)]
    Xy = [_dot(X[i], y) for i in range(d)]
    H = len(blocks)
    if s == 1:
        for Ih in blocks:
            b = len(Ih)
            Gam = [[_dot(X[Ih[u]], X[Ih[v]]) / n + (lam if Ih[u] == Ih[v] else 0)
                    for v in range(b)] for u in range(b)]
            rhs = [-lam * w[Ih[u]] - _dot(X[Ih[u]], z) / n + Xy[Ih[u]] / n
                   for u in range(b)]
            dw = _solve(Gam, rhs)
            for u in range(b):
                w[Ih[u]] += dw[u]
            for c in range(n):
                z[c] += sum((X[Ih[u]][c] * dw[u] for u in range(b)), Fraction(0))
        return w, z
    h = 0
    while h < H:
        blk = blocks[h:h + s]
        I = [i for bb in blk for i in bb]
        m = len(I)
        G = [[_dot(X[I[p]], X[I[q]]) / n + (lam if p == q else 0) for q in range(m)]
             for p in range(m)]
        deltas = []
        off = 0
        for j, Ij in enumerate(blk):
            b = len(Ij)
            Gam = [[G[off + u][off + v] for v in range(b)] for u in range(b)]
            rhs = []
            for u in range(b):
                val = -lam * w[Ij[u]] - _dot(X[Ij[u]], z) / n + Xy[Ij[u]] / n
                toff = 0
                for t in range(j):
                    It = blk[t]
                    for v in range(len(It)):
                        if Ij[u] == It[v]:
                            val -= lam * deltas[t][v]
                        val -= G[off + u][toff + v] * deltas[t][v]
                    toff += len(It)
                rhs.append(val)
            deltas.append(_solve(Gam, rhs))
            off += b
        for t, It in enumerate(blk):
            for u, i in enumerate(It):
                w[i] += deltas[t][u]
                for c in range(n):
                    z[c] += X[i][c] * deltas[t][u]
        h += len(blk)
    return w, z


def dual_bcd_exact(X, y, lam, blocks, s, alpha0=None):
    """Alg. 3 when s == 1, Alg. 4 otherwise.  Returns (alpha, w)."""
    d, n = len(X), len(X[0])
    lam = _F(lam)
    col = [[X[i][c] for i in range(d)] for c in range(n)]
    alpha = [Fraction(0)] * n if alpha0 is None else [_F(v) for v in alpha0]
    w = [-_dot(X[i], alpha) / (lam * n) for i in range(d)]
    H = len(blocks)
    if s == 1:
        for Ih in blocks:
            b = len(Ih)
            Th = [[_dot(col[Ih[u]], col[Ih[v]]) / (lam * n * n)
                   + (Fraction(1, n) if Ih[u] == Ih[v] else 0)
                   for v in range(b)] for u in range(b)]
            rhs = [-_dot(col[Ih[u]], w) + alpha[Ih[u]] + y[Ih[u]] for u in range(b)]
            da = [-v / n for v in _solve(Th, rhs)]
            for u in range(b):
                alpha[Ih[u]] += da[u]
                for i in range(d):
                    w[i] -= col[Ih[u]][i] * da[u] / (lam * n)
        return alpha, w
    h = 0
    while h < H:
        blk = blocks[h:h + s]
        I = [i for bb in blk for i in bb]
        m = len(I)
        Gp = [[_dot(col[I[p]], col[I[q]]) / (lam * n * n)
               + (Fraction(1, n) if p == q else 0) for q in range(m)] for p in range(m)]
        deltas = []
        off = 0
        for j, Ij in enumerate(blk):
            b = len(Ij)
            Th = [[Gp[off + u][off + v] for v in range(b)] for u in range(b)]
            rhs = []
            for u in range(b):
                val = -_dot(col[Ij[u]], w) + alpha[Ij[u]] + y[Ij[u]]
                for t in range(j):
                    It = blk[t]
                    for v in range(len(It)):
                        val += _dot(col[Ij[u]], col[It[v]]) * deltas[t][v] / (lam * n)
                        if Ij[u] == It[v]:
                            val += deltas[t][v]
                rhs.append(val)
            deltas.append([-v / n for v in _solve(Th, rhs)])
            off += b
        for t, It in enumerate(blk):
            for u, i in enumerate(It):
                alpha[i] += deltas[t][u]
                for r in range(d):
                    w[r] -= col[i][r] * deltas[t][u] / (lam * n)
        h += len(blk)
    return alpha, w


def primal_objective_exact(X, y, lam, w):
    d, n = len(X), len(X[0])
    r = [_dot([X[i][c] for i in range(d)], w) - y[c] for c in range(n)]
    return _dot(r, r) / (2 * n) + _F(lam) * _dot(w, w) / 2


def dual_objective_exact(X, y, lam, alpha):
    d, n = len(X), len(X[0])
    lam = _F(lam)
    v = [_dot(X[i], alpha) / (lam * n) for i in range(d)]
    a = [alpha[c] + y[c] for c in range(n)]
    return lam * _dot(v, v) / 2 + _dot(a, a) / (2 * n)
