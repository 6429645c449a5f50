"""ORACLE (test infrastructure) — solvers for the assembled system A phi = b.

The method of the paper (geometric multigrid V-cycles) is an iteration whose
fixed point is the solution of the finest-level system; the oracle computes
that solution directly and does not imitate the GPU multigrid:
  * dense LU (numpy) for tiny systems;
  * SuperLU (scipy) with FP64 iterative refinement;
  * GMRES (scipy) preconditioned by a plain aggregation multigrid built from
    A itself (2^D cells per aggregate and phase, Galerkin coarse matrices,
    damped Jacobi smoothing, SuperLU at the bottom), for systems too large
    for a direct factorisation. It is only a preconditioner: the answer is
    fixed by the GMRES residual.

The stopping rule of the paper's multigrid section (residual relative to the
residual at phi = 0) is ``rel_residual``.

Parity: dense vs SuperLU vs GMRES agree on overlapping sizes
(tests/test_oracle_solvers.py).
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def rel_residual(A, b, x):
    """||b - A x||_2 / ||b||_2 (the residual at x = 0 is b)."""
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(b - A @ x)) / nb if nb > 0 else float(np.linalg.norm(A @ x))


def solve_dense(A, b):
    return np.linalg.solve(A.toarray(), b)


def solve_splu(A, b, refine=2):
    lu = spla.splu(A.tocsc())
    x = lu.solve(b)
    for _ in range(refine):
        x = x + lu.solve(b - A @ x)
    return x


class AggregationMG:
    """Aggregation multigrid preconditioner on the assembled matrix."""

    def __init__(self, system, min_size=2000, nu=2, omega=0.6):
        A = system.A.tocsr()
        geo = system.geo
        self.levels = []
        shape = geo.shape
        # fine aggregation key: (coarse cell, phase)
        N, N2 = system.N, system.N2
        phase = np.zeros(N + N2, np.int64)
        phase[:N] = np.maximum(geo.primary.ravel(), 0)
        phase[N:] = 1
        cell = np.concatenate([np.arange(N), geo.sec_cells])
        self.nu = nu
        self.omega = omega
        while A.shape[0] > min_size and min(shape) >= 2:
            dims = len(shape)
            idx = np.unravel_index(cell, shape)
            cshape = tuple((m + 1) // 2 for m in shape)
            ccell = np.ravel_multi_index(tuple(q // 2 for q in idx), cshape)
            key = ccell * 2 + phase
            uk, agg = np.unique(key, return_inverse=True)
            P = sp.csr_matrix((np.ones(len(agg)), (np.arange(len(agg)), agg)), shape=(len(agg), len(uk)))
            Ac = (P.T @ A @ P).tocsr()
            self.levels.append((A, P, 1.0 / A.diagonal()))
            A = Ac
            shape = cshape
            cell = uk // 2
            phase = uk % 2
            if dims and A.shape[0] == P.shape[0]:
                break
        self.bottom = spla.splu(A.tocsc())
        self.nlev = len(self.levels)

    def vcycle(self, r, lev=0):
        if lev == self.nlev:
            return self.bottom.solve(r)
        A, P, dinv = self.levels[lev]
        x = self.omega * dinv * r
        for _ in range(self.nu - 1):
            x = x + self.omega * dinv * (r - A @ x)
        rc = P.T @ (r - A @ x)
        x = x + P @ self.vcycle(rc, lev + 1)
        for _ in range(self.nu):
            x = x + self.omega * dinv * (r - A @ x)
        return x

    def operator(self):
        n = self.levels[0][0].shape[0] if self.levels else self.bottom.shape[0]
        return spla.LinearOperator((n, n), matvec=self.vcycle, dtype=np.float64)


def solve_gmres(system, rtol=1e-13, restart=40, maxiter=400, info=None):
    t0 = time.perf_counter()
    mg = AggregationMG(system)
    M = mg.operator()
    A = system.A
    b = system.b
    count = [0]

    def cb(_):
        count[0] += 1
    x, rc = spla.gmres(A, b, M=M, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter,
                       callback=cb, callback_type="pr_norm")
    if info is not None:
        info["iterations"] = count[0]
        info["vcycles"] = count[0]
        info["seconds"] = time.perf_counter() - t0
        info["converged"] = rc == 0
    return x


def solve(system, method="auto", **kw):
    n = system.A.shape[0]
    if method == "auto":
        method = "dense" if n <= 600 else ("splu" if n <= 1_200_000 and system.geo.dim == 2 or n <= 300_000 else "gmres")
    if method == "dense":
        return solve_dense(system.A, system.b)
    if method == "splu":
        return solve_splu(system.A, system.b)
    return solve_gmres(system, **kw)
