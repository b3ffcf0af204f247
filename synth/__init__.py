"""Seeded synthetic ridge-regression workloads.

Shared by the tests, the benchmark and the oracle comparisons.  Holds no part of
the block coordinate descent method: it only draws inputs X, y (and the block
sizes / lambdas of a batch) with the shapes, spectra, sparsity and value
distributions of the paper's workloads.  The paper's LIBSVM datasets are not
available, so these stand in for them:

* dense n >> d primal problems (the shape of mnist8m / covtype, Table
  tbl:perfdsets) - `gaussian_ridge`, `spectral_ridge`, `colscaled_ridge`;
* sparse d >> n dual problems with power-law feature popularity (the shape of
  news20 / e2006 / rcv1) - `zipf_csr_ridge`;
* batches of uneven dense problems - `ridge_batch`.

Dense generators use torch on the requested device (CPU for tests, the GPU for
full-size runs) with a seeded torch.Generator; the sparse generator uses numpy
PCG64.  Draw order within a recipe is fixed: X, then w_true, then noise.
"""

import math

import numpy as np
import torch


def _gen(device, seed):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _orthonormal_columns(rows, cols, g, device):
    """Q factor of a Gaussian rows x cols matrix with the sign of diag(R) folded
    in (Haar-distributed when rows == cols; Mezzadri 2007)."""
    G = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(G, mode="reduced")
    sgn = torch.sign(torch.diagonal(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn


def gaussian_ridge(d, n, seed, noise=0.1, device="cpu"):
    """X ~ N(0,1)^{d x n}; w_true ~ N(0,1)^d; y = X^T w_true + noise N(0,1)."""
    g = _gen(device, seed)
    X = torch.randn(d, n, generator=g, device=device, dtype=torch.float64)
    w_true = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    e = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    y = X.t() @ w_true + noise * e
    return X, y, w_true


def spectral_ridge(d, n, seed, sigma_max=1e3, noise=0.1, device="cpu"):
    """X = U diag(sigma) V^T with U Haar-orthogonal (d x d), V orthonormal
    columns (n x d) and sigma_i = sigma_max^(i/(d-1)) log-spaced from 1;
    y = X^T w_true + noise N(0,1).  Requires n >= d."""
    g = _gen(device, seed)
    U = _orthonormal_columns(d, d, g, device)
    V = _orthonormal_columns(n, d, g, device)
    expo = torch.arange(d, device=device, dtype=torch.float64) / max(d - 1, 1)
    sigma = sigma_max ** expo
    X = (U * sigma) @ V.t()
    del V
    w_true = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    e = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    y = X.t() @ w_true + noise * e
    return X.contiguous(), y, w_true


def colscaled_ridge(d, n, seed, log_sigma=2.0, noise=0.1, device="cpu", chunk=64):
    """X_ij = c_i g_ij with g ~ N(0,1) and one scale per feature row
    c_i ~ lognormal(0, log_sigma); generated in `chunk`-row slabs with per-slab
    seeds so that large instances can be produced slab by slab.
    y = X^T w_true + noise N(0,1), accumulated in FP64."""
    g = _gen(device, seed)
    c = torch.exp(log_sigma * torch.randn(d, generator=g, device=device,
                                          dtype=torch.float64))
    w_true = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    e = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    X = torch.empty(d, n, device=device, dtype=torch.float64)
    y = noise * e
    for r0 in range(0, d, chunk):
        r1 = min(d, r0 + chunk)
        gs = _gen(device, seed * 1_000_003 + r0 + 1)
        slab = torch.randn(r1 - r0, n, generator=gs, device=device,
                           dtype=torch.float64) * c[r0:r1, None]
        X[r0:r1] = slab
        y += slab.t() @ w_true[r0:r1]
    return X, y, w_true, c


def zipf_csr_ridge(n, d, nnz_per_row, seed, zipf_a=1.1):
    """Sparse problem stored as A = X^T in CSR (n rows = data points, d columns
    = features).  Each row draws Zipf(zipf_a) ranks over 1..d until
    `nnz_per_row` distinct features are seen; ranks map to feature ids by a
    fixed seeded permutation; values lognormal(0,1); rows L2-normalised;
    columns sorted.  y = sign(X^T w_true) with sign(0) = +1.

    Returns numpy (rowptr int64, colidx int32, vals float64, y, w_true)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ranks = np.arange(1, d + 1, dtype=np.float64)
    pmf = ranks ** (-zipf_a)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    perm = rng.permutation(d).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols_all = []
    vals_all = []
    for p in range(n):
        seen = []
        seen_set = set()
        while len(seen) < nnz_per_row:
            draws = np.searchsorted(cdf, rng.random(4 * nnz_per_row), side="right")
            for r in draws:
                r = int(min(r, d - 1))
                if r not in seen_set:
                    seen_set.add(r)
                    seen.append(r)
                    if len(seen) == nnz_per_row:
                        break
        cols = np.sort(perm[np.asarray(seen, dtype=np.int64)])
        vals = rng.lognormal(0.0, 1.0, size=nnz_per_row)
        vals /= math.sqrt(float(vals @ vals))
        cols_all.append(cols.astype(np.int32))
        vals_all.append(vals)
        rowptr[p + 1] = rowptr[p] + nnz_per_row
    colidx = np.concatenate(cols_all)
    vals = np.concatenate(vals_all)
    w_true = rng.standard_normal(d)
    margins = np.zeros(n)
    for p in range(n):
        sl = slice(rowptr[p], rowptr[p + 1])
        margins[p] = vals[sl] @ w_true[colidx[sl]]
    y = np.where(margins >= 0.0, 1.0, -1.0)
    return rowptr, colidx, vals, y, w_true


def ridge_batch(P, seed, d_range=(32, 1024), n_range=(4096, 131072),
                lam_range=(1e-6, 1e-1)):
    """Shapes and lambdas of a batch of independent dense ridge problems:
    d, n and lambda log-uniform in the given ranges.  Returns lists
    (d_list, n_list, lam_list); the data of problem p is then
    `gaussian_ridge(d_p, n_p, seed + 1 + p)`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ds = np.rint(np.exp(rng.uniform(math.log(d_range[0]), math.log(d_range[1]), P)))
    ns = np.rint(np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), P)))
    lams = np.exp(rng.uniform(math.log(lam_range[0]), math.log(lam_range[1]), P))
    return [int(v) for v in ds], [int(v) for v in ns], [float(v) for v in lams]
