"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against one of: published generator outputs, the
exact-arithmetic identity between the s-step and classical methods (Section 3),
the closed-form ridge minimiser (eq. primal is strictly convex for lambda > 0),
the primal-dual map (eq. 3) and duality identity, exact block minimisation
(the block step is the minimiser of the objective over the block, Section 3.1
and 3.2), decoupled coordinates on orthogonal designs, integer-exact Grams,
and distributional properties of the sampler.
"""

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse
import scipy.stats

from oracle import bcd, exact, sampler
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- sampler (P1)

def test_splitmix64_reference_outputs():
    vals = [l.strip() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [format(sampler.splitmix64_output(0, t), "016x") for t in range(len(vals))]
    assert got == vals


def test_lemire_power_of_two_is_top_bits():
    # For m = 2^k the rejection threshold (2^32 - m) mod m is 0, so the result is
    # the top k bits of the first word.
    for k in (1, 5, 11, 20, 31):
        for h in range(20):
            key = sampler.iteration_key(77, h)
            st = sampler._WordStream(key)
            x = sampler.splitmix64_output(key, 0) >> 32
            assert sampler.bounded(st, 1 << k) == x >> (32 - k)
            assert st.t == 1


def test_lemire_rejection_removes_bias():
    # For m = 3 * 2^30 the plain multiply-shift maps 4 words onto 3 results, so
    # without rejection results = 0 (mod 3) would have probability 1/2.  The
    # rejection threshold (2^32 - m) mod m = 2^30 removes exactly the extra word.
    m = 3 << 30
    assert ((1 << 32) - m) % m == 1 << 30
    cnt = np.zeros(3)
    for h in range(6000):
        st = sampler._WordStream(sampler.iteration_key(99, h))
        cnt[sampler.bounded(st, m) % 3] += 1
    p = scipy.stats.chisquare(cnt).pvalue
    assert p > 1e-3, (cnt, p)
    # and a word whose low product part is below the threshold is skipped
    class Fixed:
        def __init__(self, words):
            self.words, self.t = list(words), 0

        def next32(self):
            self.t += 1
            return self.words[self.t - 1]
    st = Fixed([4 * 12345, 4 * 12345 + 1])
    assert sampler.bounded(st, m) == ((4 * 12345 + 1) * m) >> 32 and st.t == 2


@pytest.mark.parametrize("m,b", [(64, 4), (2048, 8), (20000, 16), (7, 7), (5, 1)])
def test_blocks_distinct_and_in_range(m, b):
    for h in range(200):
        blk = sampler.sample_block(2000, h, b, m)
        assert len(blk) == b and len(set(blk)) == b
        assert all(0 <= v < m for v in blk)
    full = sampler.sample_block(3, 9, m, m)
    assert sorted(full) == list(range(m))


def test_blocks_depend_only_on_seed_and_h():
    a = sampler.sample_blocks(11, 0, 40, 4, 64)
    b = sampler.sample_blocks(11, 17, 10, 4, 64)
    assert a[17:27] == b
    assert sampler.sample_block(12, 3, 4, 64) != sampler.sample_block(11, 3, 4, 64)


def test_subsets_uniform_chi2():
    # Floyd's algorithm draws every b-subset with equal probability.
    m, b, N = 6, 3, 12000
    subsets = {frozenset(c): 0 for c in itertools.combinations(range(m), b)}
    for h in range(N):
        subsets[frozenset(sampler.sample_block(5, h, b, m))] += 1
    obs = np.array(list(subsets.values()), dtype=float)
    p = scipy.stats.chisquare(obs).pvalue
    assert p > 1e-3, p


def test_marginals_uniform_chi2():
    m, b, N = 50, 8, 6000
    cnt = np.zeros(m)
    for h in range(N):
        for v in sampler.sample_block(123, h, b, m):
            cnt[v] += 1
    p = scipy.stats.chisquare(cnt).pvalue
    assert p > 1e-3, p


# ---------------------------------------------------------------- Gram (P2)

def test_gram_integer_exact_and_orientation():
    rng = np.random.default_rng(0)
    A = rng.integers(-50, 50, size=(9, 13)).astype(np.float64)
    idx = [3, 0, 8, 3 - 3 + 5, 7]
    u = rng.integers(-9, 9, size=13).astype(np.float64)
    G, Yu = bcd.gram(A, idx, 1.0, 0.0, u)
    for p, i in enumerate(idx):
        assert Yu[p] == sum(int(A[i, c]) * int(u[c]) for c in range(13))
        for q, j in enumerate(idx):
            assert G[p, q] == sum(int(A[i, c]) * int(A[j, c]) for c in range(13))
    G2, _ = bcd.gram(A, idx, 0.25, 3.0)
    assert np.array_equal(G2, 0.25 * G + 3.0 * np.eye(len(idx)))


def test_gram_sparse_equals_dense():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 40)) * (rng.random((30, 40)) < 0.2)
    idx = [4, 29, 0, 17]
    Gd, Yd = bcd.gram(A, idx, 0.5, 0.1, np.arange(40.0))
    Gs, Ys = bcd.gram(scipy.sparse.csr_matrix(A), idx, 0.5, 0.1, np.arange(40.0))
    np.testing.assert_allclose(Gs, Gd, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(Ys, Yd, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------- exact recurrence (P3)

def _rational_problem(d, n, seed):
    rng = np.random.default_rng(seed)
    X = [[Fraction(int(v), 4) for v in rng.integers(-6, 7, size=n)] for _ in range(d)]
    y = [Fraction(int(v), 3) for v in rng.integers(-5, 6, size=n)]
    return X, y


# Blocks with deliberate overlaps across the s blocks of an outer step.
_BLOCKS_P = [[0, 1], [1, 2], [2, 0], [4, 3], [3, 1], [4, 2], [0, 4], [2, 3],
             [1, 0], [3, 4], [4, 1], [0, 2]]
_BLOCKS_D = [[0, 1], [1, 2], [6, 0], [4, 3], [3, 5], [4, 6], [0, 4], [2, 3],
             [5, 0], [1, 6], [4, 5], [0, 2]]


@pytest.mark.parametrize("s", [2, 3, 4, 5])
def test_exact_cabcd_equals_bcd(s):
    X, y = _rational_problem(5, 7, 3)
    lam = Fraction(3, 10)
    w1, z1 = exact.primal_bcd_exact(X, y, lam, _BLOCKS_P, 1)
    ws, zs = exact.primal_bcd_exact(X, y, lam, _BLOCKS_P, s)
    assert w1 == ws and z1 == zs


@pytest.mark.parametrize("s", [2, 3, 5])
def test_exact_cabdcd_equals_bdcd(s):
    X, y = _rational_problem(5, 7, 4)
    lam = Fraction(1, 7)
    a1, w1 = exact.dual_bcd_exact(X, y, lam, _BLOCKS_D, 1)
    a_s, w_s = exact.dual_bcd_exact(X, y, lam, _BLOCKS_D, s)
    assert a1 == a_s and w1 == w_s


def _to_np(X, y):
    return (np.array([[float(v) for v in row] for row in X]),
            np.array([float(v) for v in y]))


@pytest.mark.parametrize("s", [1, 3, 4])
def test_fp64_oracle_matches_exact_primal(s):
    X, y = _rational_problem(5, 7, 3)
    lam = Fraction(3, 10)
    wE, zE = exact.primal_bcd_exact(X, y, lam, _BLOCKS_P, 1)
    Xn, yn = _to_np(X, y)
    w, z = bcd.primal_bcd(Xn, yn, 0.3, 2, s, len(_BLOCKS_P), 0, explicit_idx=_BLOCKS_P)
    wE = np.array([float(v) for v in wE])
    zE = np.array([float(v) for v in zE])
    assert np.linalg.norm(w - wE) <= 1e-13 * np.linalg.norm(wE)
    assert np.linalg.norm(z - zE) <= 1e-13 * np.linalg.norm(zE)


@pytest.mark.parametrize("s", [1, 3, 5])
def test_fp64_oracle_matches_exact_dual(s):
    X, y = _rational_problem(5, 7, 4)
    aE, wE = exact.dual_bcd_exact(X, y, Fraction(1, 7), _BLOCKS_D, 1)
    Xn, yn = _to_np(X, y)
    a, w = bcd.dual_bcd(Xn, yn, 1.0 / 7.0, 2, s, len(_BLOCKS_D), 0, explicit_idx=_BLOCKS_D)
    aE = np.array([float(v) for v in aE])
    wE = np.array([float(v) for v in wE])
    assert np.linalg.norm(a - aE) <= 1e-13 * np.linalg.norm(aE)
    assert np.linalg.norm(w - wE) <= 1e-13 * np.linalg.norm(wE)


def test_fp64_oracle_sparse_matches_dense():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((40, 30)) * (rng.random((40, 30)) < 0.3)
    y = rng.standard_normal(30)
    Xs = scipy.sparse.csr_matrix(X)
    wd, zd = bcd.primal_bcd(X, y, 0.05, 4, 3, 50, 8)
    ws, zs = bcd.primal_bcd(Xs, y, 0.05, 4, 3, 50, 8)
    np.testing.assert_allclose(ws, wd, rtol=1e-12, atol=1e-13)
    ad, vd = bcd.dual_bcd(X, y, 0.05, 4, 3, 50, 8)
    as_, vs = bcd.dual_bcd(Xs, y, 0.05, 4, 3, 50, 8)
    np.testing.assert_allclose(as_, ad, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(vs, vd, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------- whole method (P4, P5)

@pytest.fixture(scope="module")
def cfg0():
    X, y, _ = synth.gaussian_ridge(64, 1024, 1000)
    return X.numpy(), y.numpy(), 1e-3


def test_cfg0_s_equivalence_at_outer_boundaries(cfg0):
    X, y, lam = cfg0
    rec1, rec8 = {}, {}
    bcd.primal_bcd(X, y, lam, 4, 1, 400, 2000, monitor=lambda h, w, z: rec1.__setitem__(h, w))
    bcd.primal_bcd(X, y, lam, 4, 8, 400, 2000, monitor=lambda h, w, z: rec8.__setitem__(h, w))
    for h, w8 in rec8.items():
        w1 = rec1[h]
        assert np.linalg.norm(w8 - w1) <= 1e-12 * np.linalg.norm(w1), h


@pytest.mark.parametrize("s", [1, 8])
def test_cfg0_converges_to_closed_form(cfg0, s):
    X, y, lam = cfg0
    wstar = bcd.ridge_closed_form(X, y, lam)
    fs = []
    w, z = bcd.primal_bcd(X, y, lam, 4, s, 2000, 2000,
                          monitor=lambda h, w, z: fs.append(bcd.primal_objective(X, y, lam, w)))
    assert np.linalg.norm(w - wstar) <= 1e-10 * np.linalg.norm(wstar)
    # maintained z stays X^T w
    assert np.linalg.norm(z - X.T @ w) <= 1e-10 * np.linalg.norm(z)
    # exact block minimisation never increases f (s = 1 checks every iteration)
    f0 = bcd.primal_objective(X, y, lam, np.zeros(64))
    seq = [f0] + fs
    assert all(b <= a * (1 + 1e-14) for a, b in zip(seq, seq[1:]))


def _grad_f(X, y, lam, w):
    n = X.shape[1]
    return lam * w + X @ (X.T @ w - y) / n


def test_block_step_is_block_minimiser():
    X, y, _ = synth.gaussian_ridge(12, 40, 5)
    X, y = X.numpy(), y.numpy()
    lam = 0.07
    w0 = np.linspace(-1, 1, 12)
    blk = sampler.sample_block(9, 0, 5, 12)
    w, _ = bcd.primal_bcd(X, y, lam, 5, 1, 1, 9, w0=w0)
    # the gradient restricted to the updated block vanishes
    g = _grad_f(X, y, lam, w)
    assert np.abs(g[blk]).max() <= 1e-13 * np.abs(_grad_f(X, y, lam, w0)).max()
    # coordinate-wise line minimisation of f finds no further decrease
    for i in blk:
        e = np.zeros(12)
        e[i] = 1.0
        res = scipy.optimize.minimize_scalar(
            lambda t: bcd.primal_objective(X, y, lam, w + t * e), bracket=(-1, 1), tol=1e-12)
        assert abs(res.x) < 1e-6


def test_dual_block_step_is_block_minimiser():
    X, y, _ = synth.gaussian_ridge(9, 30, 6)
    X, y = X.numpy(), y.numpy()
    lam = 0.2
    a0 = np.linspace(-0.5, 0.5, 30)
    blk = sampler.sample_block(4, 0, 6, 30)
    a, w = bcd.dual_bcd(X, y, lam, 6, 1, 1, 4, alpha0=a0)
    n = 30
    gD = (X.T @ (X @ a)) / (lam * n * n) + (a + y) / n     # gradient of eq. (6)
    gD0 = (X.T @ (X @ a0)) / (lam * n * n) + (a0 + y) / n
    assert np.abs(gD[blk]).max() <= 1e-13 * np.abs(gD0).max()
    for i in blk:
        e = np.zeros(n)
        e[i] = 1.0
        res = scipy.optimize.minimize_scalar(
            lambda t: bcd.dual_objective(X, y, lam, a + t * e), bracket=(-1, 1), tol=1e-12)
        assert abs(res.x) < 1e-6


def test_full_block_is_one_newton_step():
    X, y, _ = synth.gaussian_ridge(16, 100, 7)
    X, y = X.numpy(), y.numpy()
    wstar = bcd.ridge_closed_form(X, y, 0.01)
    w, _ = bcd.primal_bcd(X, y, 0.01, 16, 1, 1, 1)
    assert np.linalg.norm(w - wstar) <= 1e-12 * np.linalg.norm(wstar)
    X2, y2, _ = synth.gaussian_ridge(40, 12, 8)
    X2, y2 = X2.numpy(), y2.numpy()
    lam = 0.03
    wstar2 = bcd.ridge_closed_form(X2, y2, lam)
    a, w2 = bcd.dual_bcd(X2, y2, lam, 12, 1, 1, 1)
    assert np.linalg.norm(w2 - wstar2) <= 1e-11 * np.linalg.norm(wstar2)
    assert np.linalg.norm(a - (X2.T @ wstar2 - y2)) <= 1e-11 * np.linalg.norm(a)


def test_orthogonal_design_decouples():
    # Rows of a Sylvester-Hadamard matrix: X X^T = n I, so every coordinate
    # minimises independently, w*_i = (X y)_i / (n (1 + lam)).
    Hm = np.array([[1.0]])
    while Hm.shape[0] < 32:
        Hm = np.block([[Hm, Hm], [Hm, -Hm]])
    X = Hm[:8, :]
    y = np.random.default_rng(2).standard_normal(32)
    lam = 0.5
    wstar = (X @ y) / (32 * (1 + lam))
    seen = set()
    H = 0
    while len(seen) < 8:
        seen.update(sampler.sample_block(31, H, 3, 8))
        H += 1
    for s in (1, 4):
        w, _ = bcd.primal_bcd(X, y, lam, 3, s, H, 31)
        np.testing.assert_allclose(w, wstar, rtol=1e-14, atol=1e-15)


@pytest.fixture(scope="module")
def dual_small():
    X, y, _ = synth.gaussian_ridge(30, 200, 21)
    return X.numpy(), y.numpy(), 0.05


def test_duality_identity_and_dual_optimum(dual_small):
    X, y, lam = dual_small
    n = X.shape[1]
    wstar = bcd.ridge_closed_form(X, y, lam)
    astar = X.T @ wstar - y
    # eq. (3) at the optimum
    assert np.linalg.norm(wstar + X @ astar / (lam * n)) <= 1e-12 * np.linalg.norm(wstar)
    total = bcd.primal_objective(X, y, lam, wstar) + bcd.dual_objective(X, y, lam, astar)
    assert abs(total - (y @ y) / (2 * n)) <= 1e-12 * (y @ y) / (2 * n)


@pytest.mark.parametrize("s", [1, 6])
def test_dual_converges_keeps_link_and_decreases(dual_small, s):
    X, y, lam = dual_small
    n = X.shape[1]
    wstar = bcd.ridge_closed_form(X, y, lam)
    Ds, drift = [], []

    def mon(h, a, w):
        Ds.append(bcd.dual_objective(X, y, lam, a))
        drift.append(np.linalg.norm(w + X @ a / (lam * n)) / max(np.linalg.norm(w), 1e-300))

    a, w = bcd.dual_bcd(X, y, lam, 8, s, 3000, 77, monitor=mon)
    assert np.linalg.norm(w - wstar) <= 1e-10 * np.linalg.norm(wstar)
    assert max(drift) <= 1e-10
    D0 = bcd.dual_objective(X, y, lam, np.zeros(n))
    seq = [D0] + Ds
    assert all(b <= a_ + 1e-14 * abs(a_) for a_, b in zip(seq, seq[1:]))


def test_dual_s_equivalence(dual_small):
    X, y, lam = dual_small
    r1, r6 = {}, {}
    bcd.dual_bcd(X, y, lam, 8, 1, 300, 5, monitor=lambda h, a, w: r1.__setitem__(h, (a, w)))
    bcd.dual_bcd(X, y, lam, 8, 6, 300, 5, monitor=lambda h, a, w: r6.__setitem__(h, (a, w)))
    for h, (a6, w6) in r6.items():
        a1, w1 = r1[h]
        assert np.linalg.norm(a6 - a1) <= 1e-12 * np.linalg.norm(a1)
        assert np.linalg.norm(w6 - w1) <= 1e-12 * np.linalg.norm(w1)


def test_last_outer_step_is_partial():
    X, y, _ = synth.gaussian_ridge(20, 60, 3)
    X, y = X.numpy(), y.numpy()
    hs = []
    bcd.primal_bcd(X, y, 0.1, 3, 4, 10, 1, monitor=lambda h, w, z: hs.append(h))
    assert hs == [4, 8, 10]


def test_not_spd_is_an_error():
    # With a zero row and lambda tiny but positive the system stays SPD; a
    # negative lambda-like shift is rejected up front.
    X = np.ones((3, 4))
    with pytest.raises(ValueError):
        bcd.primal_bcd(X, np.ones(4), 0.0, 2, 1, 1, 0)
    with pytest.raises(bcd.NotSPDError):
        bcd._chol_solve(np.array([[1.0, 2.0], [2.0, 1.0]]), np.ones(2))
