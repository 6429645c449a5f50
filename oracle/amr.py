"""ORACLE (test infrastructure) — the composite operator of a nested AMR
hierarchy and its solution (Numerical methods: patch-based refinement;
Spatial discretization, Helmholtz equations: the refluxing paragraph and its
equation for the coarse divergence at coarse-fine faces).

A hierarchy (``workloads.AmrProblem``) is a tree of boxes: level 0 the whole
domain, every box of level l >= 1 inside one box of level l - 1 (its
parent), refinement ratio 2; boxes of one level lie apart, so their
coarse-fine stencils do not meet. The unknowns are those of every box's
cells that no finer box covers ("valid" cells). The composite operator is
written out from its definition, in this order:

  1. every level's own operator on its box (``operator.assemble``), the
     coarse-fine faces of a patch taken as homogeneous Dirichlet faces with
     the linear closure, i.e. a face flux (beta b / h^2)(0 - 2 phi_F);
  2. fine rows next to a coarse-fine face: the flux through that face is
     taken with a ghost value phi_G beyond it, so the row gains
     (beta b / h_f^2)(phi_G + phi_F), which turns the closure's -2 phi_F into
     phi_G - phi_F. The ghost is quadratic along the face normal through the
     coarse value one fine cell beyond the face and the two fine cells inside
     (positions -1, 1/2, 3/2 in fine cells from the face, evaluated at -1/2):
     phi_G = 8/15 phi_C + 2/3 phi_F - 1/5 phi_Fn. The coarse value phi_C is
     the coarse level's quadratic Taylor interpolant about the coarse cell C
     containing the ghost, taken at the ghost's position along the face: per
     tangential axis a first and a second difference (centred, or one-sided
     on the side where the cells exist), offsets +-1/4 coarse cells, and in
     3D the mixed difference (centred, or one-sided) times the product of the
     offsets;
  3. refluxing: in a valid coarse cell C next to the finer box, the flux
     through a face shared with a covered cell Cv, b (phi_Cv - phi_C) / h_c,
     is replaced by the mean of the fine fluxes through the 2^(D-1) fine
     faces on it, b (phi_F - phi_G) / h_f with the same ghosts as in 2.
     (The paper prints the correction as (1/dx)(sum F_f - F_c); the fine
     fluxes enter here area-weighted, 1/2^(D-1) each, which is what keeps the
     composite divergence telescoping: the tests check that the weighted sum
     of every row vanishes for any field with zero boundary flux.)
  4. covered cells are dropped (no row references them once 3 replaced the
     faces into them).

Cells used by the ghosts and the reflux (fine cells within two cells of a
coarse-fine face, coarse cells within two cells of the finer box and the
cells of the tangential stencils) must be regular gas cells; the setup
rejects a hierarchy otherwise.

Parity: pinned by tests/test_oracle_amr.py (every valid row exact for
quadratic fields in 2D and 3D, with two and three levels and boxes touching
the domain boundary; the area-weighted sum of the rows vanishes for fields
with zero boundary flux; second-order convergence of the composite solution
of a manufactured problem; a box covering the whole domain reproduces the
fine single-level system).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .operator import assemble

GHOST_W = (8.0 / 15.0, 2.0 / 3.0, -1.0 / 5.0)   # coarse, near fine, next fine


class AmrError(ValueError):
    pass


def _np(idx):
    """numpy index (reversed) of a cell index tuple (x first)."""
    return tuple(reversed(idx))


class Composite:
    """Composite system of an AMR hierarchy over the valid unknowns."""

    def __init__(self, amr, opts=None):
        self.amr = amr
        bx = amr.levels
        self.L = len(bx)
        self.dim = amr.dim
        self.children = [[j for j in range(self.L) if bx[j].parent == i] for i in range(self.L)]
        self.sys = [assemble(b.prob, opts) for b in bx]
        self.off = np.cumsum([0] + [s.N + s.N2 for s in self.sys])
        self.covered = [np.zeros(s.N + s.N2, bool) for s in self.sys]
        for i in range(1, self.L):
            self._cover(i)
        rows, cols, vals = [], [], []
        for i, s in enumerate(self.sys):
            A = s.A.tocoo()
            rows.append(A.row + self.off[i])
            cols.append(A.col + self.off[i])
            vals.append(A.data)
        extra = {}
        for i in range(1, self.L):
            self._couple(i, extra)
        if extra:
            k = np.array(list(extra.keys()), dtype=np.int64)
            rows.append(k[:, 0])
            cols.append(k[:, 1])
            vals.append(np.array(list(extra.values())))
        ntot = int(self.off[-1])
        A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ntot, ntot))
        A.sum_duplicates()
        cov = np.concatenate(self.covered)
        self.valid = ~cov
        # rows of valid unknowns must not reach covered ones (the reflux
        # replaced the faces into them; a residue is rounding)
        Avc = A[self.valid][:, cov]
        scale = abs(A).max()
        if Avc.nnz and abs(Avc).max() > 1e-12 * scale:
            raise AmrError("a valid row references a covered unknown beyond the coarse-fine faces")
        self.A_full = A
        self.A = A[self.valid][:, self.valid].tocsr()
        self.b = np.concatenate([s.b for s in self.sys])[self.valid]

    # -- geometry of the hierarchy ------------------------------------------
    def _box(self, i):
        b = self.amr.levels[i]
        return b.lo, b.prob.n

    def _inside(self, i, g):
        lo, n = self._box(i)
        return all(lo[d] <= g[d] < lo[d] + n[d] for d in range(self.dim))

    def _footprint(self, i, gc):
        """Coarse global cell gc (the parent's level) under box i."""
        lo, n = self._box(i)
        return all(2 * gc[d] >= lo[d] and 2 * gc[d] + 1 < lo[d] + n[d] for d in range(self.dim))

    def _local(self, i, g):
        lo, _ = self._box(i)
        return tuple(g[d] - lo[d] for d in range(self.dim))

    def _regular_gas(self, i, g):
        """Global cell g of box i's level is in box i, under none of its
        children and a regular gas cell (kappa 1, one unknown)."""
        if not self._inside(i, g):
            return False
        if any(self._footprint(c, g) for c in self.children[i]):
            return False
        geo = self.sys[i].geo
        ix = _np(self._local(i, g))
        if geo.primary[ix] != 0 or geo.has[1][ix]:
            return False
        return abs(geo.kappa(0, ix) - 1.0) < 1e-14

    def _dof(self, i, g, p=0):
        return self.sys[i].geo.dof(_np(self._local(i, g)), p)

    def _cover(self, i):
        pa = self.amr.levels[i].parent
        s = self.sys[pa]
        geo = s.geo
        lo, n = self._box(pa)
        for loc in itertools.product(*[range(m) for m in n]):
            g = tuple(lo[d] + loc[d] for d in range(self.dim))
            if self._footprint(i, g):
                for p in (0, 1):
                    k = geo.dof(_np(loc), p)
                    if k >= 0:
                        self.covered[pa][k] = True
                self.covered[pa][int(np.ravel_multi_index(_np(loc), geo.shape))] = True

    # -- ghosts -------------------------------------------------------------
    def coarse_interp(self, i, C, G, d):
        """{coarse dof: weight} of the interpolant of box i's parent at ghost
        G's position along the face (normal axis d), about coarse cell C."""
        pa = self.amr.levels[i].parent
        ok = lambda c: self._regular_gas(pa, c)
        sh = lambda c, e, k: tuple(c[q] + (k if q == e else 0) for q in range(self.dim))
        w = {C: 1.0}

        def add(stencil, f):
            for c, v in stencil.items():
                w[c] = w.get(c, 0.0) + f * v
        if not ok(C):
            raise AmrError(f"coarse cell {C} of a ghost is not a regular valid gas cell")
        tang = [e for e in range(self.dim) if e != d]
        delta = {e: (G[e] + 0.5) / 2.0 - (C[e] + 0.5) for e in tang}
        for e in tang:
            p1, m1, p2, m2 = sh(C, e, 1), sh(C, e, -1), sh(C, e, 2), sh(C, e, -2)
            if ok(p1) and ok(m1):
                d1 = {p1: 0.5, m1: -0.5}
                d2 = {p1: 1.0, C: -2.0, m1: 1.0}
            elif ok(p1) and ok(p2):
                d1 = {C: -1.5, p1: 2.0, p2: -0.5}
                d2 = {C: 1.0, p1: -2.0, p2: 1.0}
            elif ok(m1) and ok(m2):
                d1 = {C: 1.5, m1: -2.0, m2: 0.5}
                d2 = {C: 1.0, m1: -2.0, m2: 1.0}
            else:
                raise AmrError(f"no tangential stencil about coarse cell {C}")
            add(d1, delta[e])
            add(d2, 0.5 * delta[e] ** 2)
        if self.dim == 3:
            e1, e2 = tang
            corners = {(s1, s2): sh(sh(C, e1, s1), e2, s2) for s1 in (1, -1) for s2 in (1, -1)}
            if all(ok(c) for c in corners.values()):
                d12 = {corners[(1, 1)]: 0.25, corners[(1, -1)]: -0.25, corners[(-1, 1)]: -0.25,
                       corners[(-1, -1)]: 0.25}
            else:
                d12 = None
                for s1, s2 in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                    a, b_, c = sh(C, e1, s1), sh(C, e2, s2), corners[(s1, s2)]
                    if ok(a) and ok(b_) and ok(c):
                        d12 = {c: s1 * s2, a: -s1 * s2, b_: -s1 * s2}
                        d12[C] = d12.get(C, 0.0) + s1 * s2
                        break
                if d12 is None:
                    raise AmrError(f"no mixed stencil about coarse cell {C}")
            add(d12, delta[e1] * delta[e2])
        return {self._dof(pa, c): v for c, v in w.items()}

    def ghost(self, i, F, d, side):
        """Ghost of fine cell F (global, box i's level) across its face
        (d, side): ({parent dof: w}, {box i dof: w})."""
        sgn = 1 if side else -1
        G = tuple(F[q] + (sgn if q == d else 0) for q in range(self.dim))
        Fn = tuple(F[q] - (sgn if q == d else 0) for q in range(self.dim))
        for c in (F, Fn):
            if not self._regular_gas(i, c):
                raise AmrError(f"fine cell {c} next to a coarse-fine face is not a regular gas cell")
        C = tuple(G[q] // 2 for q in range(self.dim))
        wc = {k: GHOST_W[0] * v for k, v in self.coarse_interp(i, C, G, d).items()}
        wf = {self._dof(i, F): GHOST_W[1], self._dof(i, Fn): GHOST_W[2]}
        return wc, wf

    def _couple(self, i, extra):
        """Add the ghost terms of box i's rows and the reflux of its parent."""
        bx = self.amr.levels[i]
        pa = bx.parent
        pf = bx.prob
        pc = self.amr.levels[pa].prob
        hf, hc = pf.h, pc.h
        of, oc = self.off[i], self.off[pa]

        def put(r, c, v):
            extra[(r, c)] = extra.get((r, c), 0.0) + v
        lo, n = self._box(i)
        cf_face = lambda d, side: bx.cf[2 * d + side]
        # 2. fine rows
        kf = pf.beta * pf.b_gas / (hf * hf)
        for loc in itertools.product(*[range(m) for m in n]):
            F = tuple(lo[q] + loc[q] for q in range(self.dim))
            for d in range(self.dim):
                for side in (0, 1):
                    at = loc[d] == (n[d] - 1 if side else 0)
                    if not (at and cf_face(d, side)):
                        continue
                    wc, wf = self.ghost(i, F, d, side)
                    r = of + self._dof(i, F)
                    for k, v in wc.items():
                        put(r, oc + k, kf * v)
                    for k, v in wf.items():
                        put(r, of + k, kf * v)
                    put(r, r, kf)
        # 3. reflux of coarse cells next to the box
        kc = pc.beta * pc.b_gas / (hc * hc)
        kr = pc.beta * pc.b_gas / (hc * hf * 2 ** (self.dim - 1))
        clo, cn = self._box(pa)
        for loc in itertools.product(*[range(m) for m in cn]):
            C = tuple(clo[q] + loc[q] for q in range(self.dim))
            if self._footprint(i, C):
                continue
            for d in range(self.dim):
                for sgn in (1, -1):
                    Cv = tuple(C[q] + (sgn if q == d else 0) for q in range(self.dim))
                    if not self._inside(pa, Cv) or not self._footprint(i, Cv):
                        continue
                    if not self._regular_gas(pa, C):
                        raise AmrError(f"coarse cell {C} next to the finer box is not a regular gas cell")
                    r = oc + self._dof(pa, C)
                    put(r, oc + self._dof(pa, Cv), -kc)
                    put(r, r, kc)
                    tang = [e for e in range(self.dim) if e != d]
                    for offs in itertools.product((0, 1), repeat=self.dim - 1):
                        F = [0] * self.dim
                        F[d] = 2 * Cv[d] + (0 if sgn > 0 else 1)
                        for e, o in zip(tang, offs):
                            F[e] = 2 * Cv[e] + o
                        F = tuple(F)
                        wc, wf = self.ghost(i, F, d, 0 if sgn > 0 else 1)
                        put(r, of + self._dof(i, F), kr)
                        for k, v in wc.items():
                            put(r, oc + k, -kr * v)
                        for k, v in wf.items():
                            put(r, of + k, -kr * v)

    # -- vectors ------------------------------------------------------------
    def scatter(self, xv):
        """Per-box full vectors (covered entries 0) from a valid vector."""
        full = np.zeros(int(self.off[-1]))
        full[self.valid] = xv
        return [full[self.off[i]:self.off[i + 1]] for i in range(self.L)]

    def gather(self, xs):
        return np.concatenate(xs)[self.valid]

    def solve(self):
        """Composite solution (valid unknowns) by SuperLU with two steps of
        iterative refinement."""
        lu = spl.splu(self.A.tocsc())
        x = lu.solve(self.b)
        for _ in range(2):
            x = x + lu.solve(self.b - self.A @ x)
        return x
