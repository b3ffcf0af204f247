"""Plain FP64 CPU oracle of (CA-)BCD and (CA-)BDCD for ridge regression.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path never
does.  It shares no code with the HIP library.

Notation is the paper's: X is d x n (rows = features, columns = data points),
y in R^n, lambda > 0.
  primal (eq. primal):  f(w) = lambda/2 ||w||^2 + 1/(2n) ||X^T w - y||^2
  dual   (eq. 6):       D(a) = lambda/2 ||X a / (lambda n)||^2 + 1/(2n) ||a + y||^2
  primal-dual map (eq. 3): w = -X a / (lambda n)

Every step is the paper's, in the paper's order; library calls (a matrix
product, a Cholesky factorisation) are used only as whole steps.  Readings of
points the paper leaves open:
  * H counts inner iterations; the outer loop runs ceil(H/s) times and the last
    outer step has H - s*(ceil(H/s)-1) inner iterations (Alg. 2/4 print the
    loop bound as H/s).
  * z_0 = X^T w_0 for the primal (Alg. 1/2 use z without initialising it).
  * The b x b systems are solved by an unpivoted Cholesky factorisation; a
    non-positive pivot is an error (the paper does not name the solver).
  * Deferred updates add the s block steps (duplicates across blocks add up).

X may be a dense ndarray or any scipy.sparse matrix; sparse data is only ever
sliced and multiplied, never densified as a whole.
"""

import numpy as np
import scipy.linalg
import scipy.sparse

from .sampler import sample_block


class NotSPDError(ArithmeticError):
    pass


def _is_sparse(X):
    return scipy.sparse.issparse(X)


def _rows(X, idx):
    """I^T X for the selection matrix I = [e_i1 ... e_ik] (rows of X), dense."""
    if _is_sparse(X):
        return np.asarray(X[idx, :].todense(), dtype=np.float64)
    return np.asarray(X[idx, :], dtype=np.float64)


def _cols(X, idx):
    """X I (columns of X), as a sparse or dense matrix."""
    if _is_sparse(X):
        return X[:, idx]
    return np.asarray(X[:, idx], dtype=np.float64)


def _chol_solve(M, rhs):
    """Solve M x = rhs with an unpivoted Cholesky factorisation of SPD M."""
    try:
        c = scipy.linalg.cho_factor(M, lower=True, check_finite=True)
    except (np.linalg.LinAlgError, ValueError) as e:
        raise NotSPDError(str(e)) from e
    return scipy.linalg.cho_solve(c, rhs, check_finite=False)


def _block_list(seed, h0, count, b, m, explicit):
    if explicit is not None:
        return [list(map(int, explicit[h0 + i])) for i in range(count)]
    return [sample_block(seed, h0 + i, b, m) for i in range(count)]


def _overlap(Ij, It):
    """I_j^T I_t: entry (u, v) is 1 where the u-th index of block j equals the
    v-th index of block t."""
    return (np.asarray(Ij)[:, None] == np.asarray(It)[None, :]).astype(np.float64)


# ----------------------------------------------------------------------------
# objectives and closed forms
# ----------------------------------------------------------------------------

def primal_objective(X, y, lam, w):
    """f(w) of eq. (primal), recomputed from scratch."""
    n = X.shape[1]
    r = X.T @ w - y
    return 0.5 * float(r @ r) / n + 0.5 * lam * float(w @ w)


def dual_objective(X, y, lam, alpha):
    """D(alpha) of eq. (6), recomputed from scratch."""
    n = X.shape[1]
    v = (X @ alpha) / (lam * n)
    a = alpha + y
    return 0.5 * lam * float(v @ v) + 0.5 * float(a @ a) / n


def ridge_closed_form(X, y, lam):
    """Unique minimiser of eq. (primal): (X X^T / n + lam I) w = X y / n."""
    d, n = X.shape
    if _is_sparse(X):
        XXt = np.asarray((X @ X.T).todense())
    else:
        XXt = X @ X.T
    M = XXt / n + lam * np.eye(d)
    return _chol_solve(M, (X @ y) / n)


def gram(A, idx, scale, shift, u=None):
    """scale * Y Y^T + shift * I and Y u, where Y holds the rows idx of A.

    This is the s-step Gram of Alg. 2 (A = X, scale 1/n, shift lambda) and of
    Alg. 4 (A = X^T, scale 1/(lambda n^2), shift 1/n).
    """
    if _is_sparse(A):
        A = A.tocsr()
    Y = _rows(A, list(idx))
    G = scale * (Y @ Y.T) + shift * np.eye(len(idx))
    Yu = None if u is None else Y @ np.asarray(u, dtype=np.float64)
    return G, Yu


# ----------------------------------------------------------------------------
# primal: Alg. 1 (s = 1) and Alg. 2 (CA-BCD)
# ----------------------------------------------------------------------------

def _primal_steps(X, y, lam, b, s, H, seed, w0, explicit_idx, h0):
    """The outer steps of Alg. 2; yields (h, w, z) after each one."""
    d, n = X.shape
    if not (lam > 0 and 1 <= b <= d and s >= 1 and H >= 0):
        raise ValueError("invalid arguments")
    if _is_sparse(X):
        X = X.tocsr()
    w = np.zeros(d) if w0 is None else np.array(w0, dtype=np.float64)
    z = X.T @ w                      # z_0 = X^T w_0
    Xy = X @ y                       # 1/n I^T X y is read off this vector
    h = 0
    while h < H:
        sk = min(s, H - h)
        blocks = _block_list(seed, h0 + h, sk, b, d, explicit_idx)
        I = [i for blk in blocks for i in blk]
        Y = _rows(X, I)                                  # Y = [I_1 .. I_s]^T X
        G = (Y @ Y.T) / n + lam * np.eye(sk * b)         # G = 1/n Y Y^T + lam I
        Yz = Y @ z
        deltas = []
        for j in range(sk):
            J = slice(j * b, (j + 1) * b)
            Gamma = G[J, J]                              # diagonal block of G
            rhs = -lam * w[blocks[j]] - Yz[J] / n + Xy[blocks[j]] / n
            for t in range(j):
                T = slice(t * b, (t + 1) * b)
                rhs -= lam * (_overlap(blocks[j], blocks[t]) @ deltas[t])
                rhs -= G[J, T] @ deltas[t]               # 1/n I_j^T X X^T I_t dw_t
            deltas.append(_chol_solve(Gamma, rhs))
        v = np.zeros(d)                                  # sum_t I_t dw_t
        for t in range(sk):
            for u, i in enumerate(blocks[t]):
                v[i] += deltas[t][u]
        w = w + v
        z = z + X.T @ v
        h += sk
        yield h, w, z
    if H == 0:
        yield 0, w, z


def primal_bcd(X, y, lam, b, s, H, seed, w0=None, explicit_idx=None, h0=0,
               monitor=None):
    """CA-BCD (Alg. 2); with s = 1 it is BCD (Alg. 1).

    Returns (w_H, z_H) with z_H = X^T w_H maintained by the recurrence.
    `explicit_idx`, if given, is indexable by global iteration and replaces the
    sampler.  `monitor(h, w, z)` is called after every outer step.
    """
    for h, w, z in _primal_steps(X, y, lam, b, s, H, seed, w0, explicit_idx, h0):
        if monitor is not None and h > 0:
            monitor(h, w, z)
    return w, z


def primal_residual(X, y, lam, w, z):
    """The full primal residual of Section 5.1.5 (stopping criterion),
    -lam w - 1/n X z + 1/n X y, with z = X^T w as maintained by the iteration
    (the b-row subsample of this vector is the right-hand side of every block
    solve).  With the exact z it is -grad f(w)."""
    n = X.shape[1]
    return -lam * np.asarray(w, dtype=np.float64) - np.asarray(X @ (z - y)).ravel() / n


def primal_bcd_tol(X, y, lam, b, s, H, seed, tol, check_every=1, w0=None,
                   explicit_idx=None, h0=0):
    """Alg. 2 stopped by the residual test of Section 5.1.5: after every
    `check_every`-th outer step the full primal residual (with the maintained
    z) is formed, and the run stops at the first check where its 2-norm is
    <= tol, else after H inner iterations.

    Returns (w, z, h, norm): the iterate, its maintained z, the inner
    iterations performed and the norm at the last check (nan if none)."""
    if not (check_every >= 1 and tol >= 0):
        raise ValueError("invalid arguments")
    k, norm = 0, float("nan")
    for h, w, z in _primal_steps(X, y, lam, b, s, H, seed, w0, explicit_idx, h0):
        if h == 0:
            break
        k += 1
        if k % check_every == 0:
            norm = float(np.linalg.norm(primal_residual(X, y, lam, w, z)))
            if norm <= tol:
                break
    return w, z, h, norm


# ----------------------------------------------------------------------------
# dual: Alg. 3 (s = 1) and Alg. 4 (CA-BDCD)
# ----------------------------------------------------------------------------

def _dual_steps(X, y, lam, b, s, H, seed, alpha0, explicit_idx, h0):
    """The outer steps of Alg. 4; yields (h, alpha, w) after each one."""
    d, n = X.shape
    if not (lam > 0 and 1 <= b <= n and s >= 1 and H >= 0):
        raise ValueError("invalid arguments")
    if _is_sparse(X):
        X = X.tocsc()
    alpha = np.zeros(n) if alpha0 is None else np.array(alpha0, dtype=np.float64)
    w = -(X @ alpha) / (lam * n)                         # w_0 = -X a_0 / (lam n)
    h = 0
    while h < H:
        sk = min(s, H - h)
        blocks = _block_list(seed, h0 + h, sk, b, n, explicit_idx)
        I = [i for blk in blocks for i in blk]
        Y = _cols(X, I)                                  # Y = X [I_1 .. I_s]
        YtY = Y.T @ Y
        if _is_sparse(YtY):
            YtY = np.asarray(YtY.todense())
        Gp = YtY / (lam * n * n) + np.eye(sk * b) / n    # G' of Alg. 4
        Ytw = np.asarray(Y.T @ w).ravel()
        deltas = []
        for j in range(sk):
            J = slice(j * b, (j + 1) * b)
            Theta = Gp[J, J]
            rhs = -Ytw[J] + alpha[blocks[j]] + y[blocks[j]]
            for t in range(j):
                T = slice(t * b, (t + 1) * b)
                rhs += (YtY[J, T] @ deltas[t]) / (lam * n)
                rhs += _overlap(blocks[j], blocks[t]) @ deltas[t]
            deltas.append(-_chol_solve(Theta, rhs) / n)
        v = np.zeros(n)                                  # sum_t I_t da_t
        for t in range(sk):
            for u, i in enumerate(blocks[t]):
                v[i] += deltas[t][u]
        alpha = alpha + v
        w = w - np.asarray(X @ v).ravel() / (lam * n)
        h += sk
        yield h, alpha, w
    if H == 0:
        yield 0, alpha, w


def dual_bcd(X, y, lam, b, s, H, seed, alpha0=None, explicit_idx=None, h0=0,
             monitor=None):
    """CA-BDCD (Alg. 4); with s = 1 it is BDCD (Alg. 3).

    Returns (alpha_H, w_H), w_H maintained by the recurrence.
    """
    for h, alpha, w in _dual_steps(X, y, lam, b, s, H, seed, alpha0, explicit_idx, h0):
        if monitor is not None and h > 0:
            monitor(h, alpha, w)
    return alpha, w


def dual_residual(X, y, alpha, w):
    """The full dual residual of Section 5.1.5, -X^T w + alpha + y, with w as
    maintained by the iteration (its b-entry subsample is the vector each
    block solve of Alg. 3/4 is applied to).  With w = -X alpha/(lam n) it is
    n grad D(alpha)."""
    return (-np.asarray(X.T @ w).ravel() + np.asarray(alpha, dtype=np.float64)
            + np.asarray(y, dtype=np.float64))


def dual_bcd_tol(X, y, lam, b, s, H, seed, tol, check_every=1, alpha0=None,
                 explicit_idx=None, h0=0):
    """Alg. 4 stopped by the dual residual test of Section 5.1.5 (2-norm of
    the full dual residual <= tol at every `check_every`-th outer step).
    Returns (alpha, w, h, norm) as primal_bcd_tol."""
    if not (check_every >= 1 and tol >= 0):
        raise ValueError("invalid arguments")
    k, norm = 0, float("nan")
    for h, alpha, w in _dual_steps(X, y, lam, b, s, H, seed, alpha0, explicit_idx, h0):
        if h == 0:
            break
        k += 1
        if k % check_every == 0:
            norm = float(np.linalg.norm(dual_residual(X, y, alpha, w)))
            if norm <= tol:
                break
    return alpha, w, h, norm
