"""Seeded synthetic least-squares problems shaped like the paper's workloads.

This module holds no arithmetic of the method itself (no sketch, no QR of the
sketch, no LSQR): it only builds inputs A, b (and the true x used to build
them).  Both the HIP path and the CPU oracle consume the very same arrays.

Recipes (Sec. 4.1 describes the paper's synthetic matrices: dense with
prescribed condition number and Haar-like left singular vectors, the first n
columns of the identity as a hard case, and a +-1 sparse matrix with density
0.01; its real data sets are not available here, so these stand in for them):

  * ``svd``: A = U diag(sigma) V^T, U and V orthonormal factors of seeded
    Gaussians, sigma log-spaced from 1 down to 1/cond.  Optional row scaling of
    the Gaussian by lognormal(0,1) before orthonormalising gives uneven
    leverage scores (Table 1's coherence column).
  * ``colscale``: A_ij = g_ij * cond^(-j/(n-1)) with g ~ N(0,1).
  * ``identity``: the first n columns of the m x m identity.
  * ``sparse_sign``: each entry nonzero with probability density, value +-1.
  * ``integer``: small integers in [-2^10, 2^10] (exact sums in fp32 and fp64).

b = A x_true + noise * N(0,1) with x_true ~ N(0,1), unless stated otherwise.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BASE_SEED = 250603070


def config_seed(k: int) -> int:
    return BASE_SEED + 1000 * k


@dataclass
class Problem:
    A: np.ndarray            # (m, n), row-major (C order)
    b: np.ndarray            # (m,) float64
    x_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)


def _orthonormal(rng, rows, cols, row_scale=False):
    G = rng.standard_normal((rows, cols))
    if row_scale:
        G *= np.exp(rng.standard_normal(rows))[:, None]
    Q, _ = np.linalg.qr(G)
    return Q


def make_problem(m, n, kind="svd", cond=1e6, noise=1e-8, seed=BASE_SEED, row_scale=False,
                 density=0.01, dtype=np.float64) -> Problem:
    """Host (numpy) generator for problems small enough to build on the CPU."""
    rng = np.random.default_rng(seed)
    if kind == "svd":
        U = _orthonormal(rng, m, n, row_scale)
        V = _orthonormal(rng, n, n)
        sigma = np.logspace(0.0, -np.log10(cond), n)
        A = (U * sigma) @ V.T
    elif kind == "colscale":
        A = rng.standard_normal((m, n)) * np.logspace(0.0, -np.log10(cond), n)[None, :]
    elif kind == "identity":
        A = np.zeros((m, n))
        A[np.arange(n), np.arange(n)] = 1.0
    elif kind == "sparse_sign":
        mask = rng.random((m, n)) < density
        A = np.where(mask, np.where(rng.random((m, n)) < 0.5, -1.0, 1.0), 0.0)
    elif kind == "integer":
        A = rng.integers(-1024, 1025, size=(m, n)).astype(np.float64)
    else:
        raise ValueError(kind)
    A = np.ascontiguousarray(A.astype(dtype))
    x_true = rng.standard_normal(n)
    if kind == "integer":
        b = rng.integers(-1024, 1025, size=m).astype(np.float64)
    else:
        Ax = A.astype(np.float64) @ x_true
        scale = noise * (np.linalg.norm(Ax) / np.sqrt(m) if kind == "colscale" else 1.0)
        b = Ax + scale * rng.standard_normal(m)
    return Problem(A=A, b=np.ascontiguousarray(b, dtype=np.float64), x_true=x_true,
                   meta=dict(m=m, n=n, kind=kind, cond=cond, noise=noise, seed=seed,
                             row_scale=row_scale))


def make_sparse_problem(m, n, density=0.01, values="sign", noise=1e-8, seed=BASE_SEED):
    """Sparse A in CSR form (scipy.sparse.csr_matrix, columns sorted within
    rows, float64): each entry nonzero with probability `density`, value +-1
    (Sec. 4.1's sparse recipe) or N(0,1) (values="gauss").  b = A x_true +
    noise * N(0,1).  Returns (A, b, x_true)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    nnz = rng.binomial(m * n, density)
    flat = rng.choice(m * n, size=nnz, replace=False) if m * n <= (1 << 26) else np.unique(
        rng.integers(0, m * n, size=nnz))
    rows, cols = np.divmod(flat, n)
    if values == "sign":
        vals = np.where(rng.random(len(flat)) < 0.5, -1.0, 1.0)
    else:
        vals = rng.standard_normal(len(flat))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    x_true = rng.standard_normal(n)
    b = A @ x_true + noise * rng.standard_normal(m)
    return A, np.ascontiguousarray(b), x_true


def config0() -> Problem:
    """Plain FP64 workload: m=20000, n=100, sigma 1..1e-6, noise 1e-8."""
    p = make_problem(20000, 100, kind="svd", cond=1e6, noise=1e-8, seed=config_seed(0))
    p.meta.update(d=400, zeta=8, tol=1e-12, maxiter=200, sketch_seed=config_seed(0) + 1)
    return p


def make_problem_torch(m, n, kind="svd", cond=1e8, noise=1e-6, seed=BASE_SEED, row_scale=False,
                       device="cuda", dtype=None, chunk_rows=1 << 18):
    """Device-side generator for sizes too large to build on the host (the
    2^20 x 1000 FP64 and 2^22 x 4096 FP32 workloads).  Returns torch tensors
    (A, b, x_true) on ``device``.  Deterministic for a given seed and device
    type."""
    import torch
    dtype = dtype or torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x_true = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    if kind == "svd":
        G = torch.randn(m, n, generator=g, device=device, dtype=torch.float64)
        if row_scale:
            G *= torch.exp(torch.randn(m, 1, generator=g, device=device, dtype=torch.float64))
        U, _ = torch.linalg.qr(G)
        del G
        V, _ = torch.linalg.qr(torch.randn(n, n, generator=g, device=device, dtype=torch.float64))
        sigma = torch.logspace(0.0, -float(np.log10(cond)), n, device=device, dtype=torch.float64)
        W = (sigma[:, None] * V.T).contiguous()
        A = torch.empty(m, n, device=device, dtype=dtype)
        for r0 in range(0, m, chunk_rows):
            r1 = min(m, r0 + chunk_rows)
            A[r0:r1] = (U[r0:r1] @ W).to(dtype)
        del U
    elif kind == "colscale":
        scale = torch.logspace(0.0, -float(np.log10(cond)), n, device=device, dtype=torch.float64)
        A = torch.empty(m, n, device=device, dtype=dtype)
        for r0 in range(0, m, chunk_rows):
            r1 = min(m, r0 + chunk_rows)
            blk = torch.randn(r1 - r0, n, generator=g, device=device, dtype=torch.float64)
            A[r0:r1] = (blk * scale[None, :]).to(dtype)
    else:
        raise ValueError(kind)
    b = torch.empty(m, device=device, dtype=torch.float64)
    xt = x_true
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        b[r0:r1] = A[r0:r1].to(torch.float64) @ xt
    nrm = torch.linalg.vector_norm(b).item()
    scale = noise * (nrm / np.sqrt(m) if kind == "colscale" else 1.0)
    b += scale * torch.randn(m, generator=g, device=device, dtype=torch.float64)
    return A, b, x_true


def config1_torch(device="cuda", noise=1e-6):
    """m=2^20, n=1000, d=4000, zeta=8, FP64; U row-scaled by lognormal(0,1)
    for uneven leverage; sigma log-spaced 1..1e-8; b = A x_true + noise."""
    A, b, xt = make_problem_torch(1 << 20, 1000, kind="svd", cond=1e8, noise=noise,
                                  seed=config_seed(1), row_scale=True, device=device)
    meta = dict(m=1 << 20, n=1000, d=4000, zeta=8, tol=1e-12, maxiter=200,
                sketch_seed=config_seed(1) + 1, noise=noise)
    return A, b, xt, meta


def config2_torch(device="cuda", m=1 << 22, n=4096):
    """Mixed-precision workload: A_ij = g_ij * 10^(-6 j/(n-1)) stored FP32,
    d = 2n, zeta = 8."""
    import torch
    A, b, xt = make_problem_torch(m, n, kind="colscale", cond=1e6, noise=1e-8,
                                  seed=config_seed(2), device=device, dtype=torch.float32)
    meta = dict(m=m, n=n, d=2 * n, zeta=8, tol=1e-12, maxiter=300,
                sketch_seed=config_seed(2) + 1)
    return A, b, xt, meta


def batch_shapes(count=512, seed=None, m_lo=5000, m_hi=200000, n_lo=32, n_hi=256):
    """Shapes for the batched workload: m ~ U[5000, 200000], n ~ U{32..256},
    d = 4n, condition number log-uniform in [1e2, 1e8]."""
    rng = np.random.default_rng(config_seed(3) if seed is None else seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    conds = 10.0 ** rng.uniform(2.0, 8.0, size=count)
    return [dict(m=int(m), n=int(n), d=int(4 * n), zeta=8, cond=float(c), seed=int(config_seed(3) + 7 * k))
            for k, (m, n, c) in enumerate(zip(ms, ns, conds))]


def served_stream(rate=200.0, duration=60.0, seed=None, cap=1 << 21):
    """Poisson arrivals; m ~ lognormal(median 1e5, sigma 1) clamped to
    [8n, 2^21]; n uniform over {64,128,256,512}; d = 4n."""
    rng = np.random.default_rng(config_seed(4) if seed is None else seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(rng.choice([64, 128, 256, 512]))
        m = int(min(cap, max(8 * n, int(1e5 * np.exp(rng.standard_normal())))))
        out.append(dict(t=t, m=m, n=n, d=4 * n, zeta=8))
    return out
