"""Oracle rows of a full-size problem computed on windows (test helper).

Every row of the system depends only on level-set values, data and unknowns
within a few cells (ray stencils reach 2 cells, least-squares fits 3, face
interpolation 1 more). A window of the box, with the box's own boundary
conditions on the sides it shares with the box and any condition on the
other (artificial) sides, therefore reproduces exactly the full problem's rows
of cells at least ``MARGIN`` cells away from the artificial sides. This lets
the oracle check sampled rows of problems too large to assemble whole.
"""
import numpy as np

import workloads as W
from oracle.operator import assemble

MARGIN = 5


def window_problem(pr, lo, hi):
    """Sub-problem over cells [lo[d], hi[d]) (x, y, z order)."""
    dim = pr.dim
    sl_nodes = tuple(slice(lo[d], hi[d] + 1) for d in reversed(range(dim)))
    sl_cells = tuple(slice(lo[d], hi[d]) for d in reversed(range(dim)))
    objs = [W.Obj(o.kind, o.value, np.ascontiguousarray(o.sdf[sl_nodes])) for o in pr.objects]
    kind = list(pr.bc_kind)
    val = list(pr.bc_value)
    for d in range(dim):
        if lo[d] > 0:
            kind[2 * d] = W.BC_NEUMANN
            val[2 * d] = 0.0
        if hi[d] < pr.n[d]:
            kind[2 * d + 1] = W.BC_NEUMANN
            val[2 * d + 1] = 0.0
    n = tuple(hi[d] - lo[d] for d in range(dim))
    wlo = tuple(pr.lo[d] + lo[d] * pr.h for d in range(dim))
    rho = np.ascontiguousarray(pr.rho[sl_cells]) if pr.rho is not None else None
    sig = np.ascontiguousarray(pr.sigma[sl_cells]) if pr.sigma is not None else None
    return W.Problem(dim, n, pr.h, wlo, objs, kind, val, list(pr.robin_a1), list(pr.robin_a2),
                     alpha=pr.alpha, beta=pr.beta, a_gas=pr.a_gas, a_diel=pr.a_diel, b_gas=pr.b_gas,
                     rho=rho, sigma=sig)


def window_rows(pr, lo, hi):
    """Oracle system of the window and the mask of its exact rows.

    Returns (System, valid) where valid[q] marks window unknowns whose rows
    equal the full problem's rows."""
    wp = window_problem(pr, lo, hi)
    S = assemble(wp)
    g = S.geo
    ok = np.ones(g.shape, bool)
    idx = np.indices(g.shape)
    for d in range(pr.dim):
        ax = pr.dim - 1 - d
        if lo[d] > 0:
            ok &= idx[ax] >= MARGIN
        if hi[d] < pr.n[d]:
            ok &= idx[ax] < (hi[d] - lo[d]) - MARGIN
    okf = ok.ravel()
    valid = np.concatenate([okf & (g.primary.ravel() >= 0), okf[g.sec_cells]])
    return S, valid


def global_index(pr, lo, S, sec_cell_global):
    """Map window unknowns to the full problem's unknown indices. Second-phase
    unknowns are located in the full layout through ``sec_cell_global`` (the
    cells of the second-phase unknowns, in increasing cell order)."""
    g = S.geo
    dim = pr.dim
    widx = np.unravel_index(np.arange(g.N), g.shape)
    gidx = tuple(widx[a] + lo[dim - 1 - a] for a in range(dim))
    gcell = np.ravel_multi_index(gidx, pr.shape)
    Nfull = int(np.prod(pr.n))
    pos = {int(c): k for k, c in enumerate(sec_cell_global)}
    sec = np.array([Nfull + pos.get(int(gcell[c]), -10 ** 12) for c in g.sec_cells], dtype=np.int64)
    return np.concatenate([gcell, sec])
