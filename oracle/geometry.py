"""ORACLE (test infrastructure) — cut-cell geometry.

Follows the spatial-discretisation section of the paper: cells are cut by the
zero set of a level-set function s(x); inside each cut cell the boundary is
linearised (a segment in 2D, a planar-faceted patch in 3D). The moments kept
per phase are the volume fraction kappa, the face apertures alpha and face
centroids, and for cut cells the embedded-boundary (EB) area fraction, EB
centroid and outward normal, plus the volume centroid.

Readings (the paper defers the formulas to the EBChombo documentation):
  * phase p occupies s_p > 0 strictly; s = 0 is outside every phase;
  * the level set is sampled at nodes; along a grid edge whose ends are on
    different sides the crossing is at t = s_a / (s_a - s_b), measured from
    the lower-index node a;
  * 2D: the wet region of a cell is the polygon of inside corners and edge
    crossings; kappa and the volume centroid are its exact area and centroid;
    the EB is the segment joining the two crossings;
  * 3D: each face is treated by the 2D rule; the EB is the fan of triangles
    from the mean of the crossing loop; kappa and the volume centroid are
    those of the closed polyhedron (face polygons + fan), by cones from the
    cell centre;
  * the EB area vector (area fraction times outward normal) is taken from
    closure: alpha_EB n_EB = sum_d (alpha_{d,lo} - alpha_{d,hi}) e_d;
  * kappa < 1e-12 counts as covered, alpha < 1e-12 as closed;
  * a face with four crossings (saddle), a cell whose crossings form more than
    one loop, and a cell cut by two different objects are rejected; an object
    cuts a cell unless its level set has one strict sign at every corner (a
    node exactly on a surface belongs to neither side);
  * phase 0 (gas) is outside every object: s_gas = min_k d_k; phase 1
    (dielectric) is inside the dielectric object and outside electrodes:
    s_diel = min(min_electrodes d_k, -d_diel); a cell cut by the dielectric
    object carries one unknown per phase and both share the gas-side facet
    (same centroid and area, opposite normal).

Pins: exact areas/volumes of planar cuts, O(h^2) convergence of disk and
sphere areas/perimeters, per-cell closure, kappa_gas + kappa_diel +
kappa_electrode = 1, and the quadratic-exactness pins of the operator
(tests/test_oracle_geometry.py, tests/test_oracle_operator.py).
"""
from __future__ import annotations

import math

import numpy as np

import workloads as W

TINY = 1e-12


class GeometryError(ValueError):
    pass


# ---------------------------------------------------------------------------
# one square (a 2D cell, or a face of a 3D cell), unit coordinates (u, v)
# corners: c00=(0,0) c10=(1,0) c11=(1,1) c01=(0,1)
# ---------------------------------------------------------------------------

def _t(sa, sb):
    """Crossing parameter from the lower node a on an edge with a sign change."""
    return sa / (sa - sb)


def square_polygon(c00, c10, c11, c01):
    """Wet polygon {s > 0} of the unit square with linear edge crossings.

    Returns (vertices CCW as list of (u, v), crossings list in walk order,
    crossing edge ids). Edge ids: 0 bottom (v=0), 1 right (u=1), 2 top (v=1),
    3 left (u=0). Raises GeometryError on a saddle (four crossings)."""
    ins = (c00 > 0, c10 > 0, c11 > 0, c01 > 0)
    verts = []
    cross = []
    eids = []
    # corner (0,0)
    if ins[0]:
        verts.append((0.0, 0.0))
    if ins[0] != ins[1]:
        p = (_t(c00, c10), 0.0)
        verts.append(p); cross.append(p); eids.append(0)
    if ins[1]:
        verts.append((1.0, 0.0))
    if ins[1] != ins[2]:
        p = (1.0, _t(c10, c11))
        verts.append(p); cross.append(p); eids.append(1)
    if ins[2]:
        verts.append((1.0, 1.0))
    if ins[2] != ins[3]:
        p = (_t(c01, c11), 1.0)
        verts.append(p); cross.append(p); eids.append(2)
    if ins[3]:
        verts.append((0.0, 1.0))
    if ins[3] != ins[0]:
        p = (0.0, _t(c00, c01))
        verts.append(p); cross.append(p); eids.append(3)
    if len(cross) == 4:
        raise GeometryError("saddle (ambiguous) square")
    return verts, cross, eids


def polygon_area_centroid(verts):
    """Shoelace area and centroid of a simple CCW polygon."""
    n = len(verts)
    if n < 3:
        return 0.0, (0.5, 0.5)
    a = 0.0
    cx = 0.0
    cy = 0.0
    for k in range(n):
        x0, y0 = verts[k]
        x1, y1 = verts[(k + 1) % n]
        cr = x0 * y1 - x1 * y0
        a += cr
        cx += (x0 + x1) * cr
        cy += (y0 + y1) * cr
    a *= 0.5
    if a <= 0.0:
        return 0.0, (0.5, 0.5)
    return a, (cx / (6.0 * a), cy / (6.0 * a))


def square_moments(c00, c10, c11, c01):
    """(area fraction, centroid (u, v)) of the wet part of a unit square."""
    if c00 > 0 and c10 > 0 and c11 > 0 and c01 > 0:
        return 1.0, (0.5, 0.5)
    if not (c00 > 0 or c10 > 0 or c11 > 0 or c01 > 0):
        return 0.0, (0.5, 0.5)
    verts, _, _ = square_polygon(c00, c10, c11, c01)
    return polygon_area_centroid(verts)


def edge_moments(sa, sb):
    """(length fraction, centroid parameter) of the wet part of a unit edge."""
    ia, ib = sa > 0, sb > 0
    if ia and ib:
        return 1.0, 0.5
    if not ia and not ib:
        return 0.0, 0.5
    t = _t(sa, sb)
    if ia:
        return t, 0.5 * t
    return 1.0 - t, 0.5 * (1.0 + t)


# ---------------------------------------------------------------------------
# per-phase geometry on one box
# ---------------------------------------------------------------------------

class CutCell:
    __slots__ = ("kappa", "vcent", "eb_area", "eb_cent", "eb_normal", "cutter")

    def __init__(self):
        self.kappa = 0.0
        self.vcent = None
        self.eb_area = 0.0
        self.eb_cent = None
        self.eb_normal = None
        self.cutter = -1


class PhaseGeom:
    """Moments of one phase. Arrays use numpy order (z, y, x)."""

    def __init__(self, geo, s):
        self.geo = geo
        self.s = s
        dim, n = geo.dim, geo.n
        shp = geo.shape
        inside = s > 0
        # corner classification per cell
        corners = []
        for off in np.ndindex(*(2,) * dim):
            sl = tuple(slice(o, o + m) for o, m in zip(off, shp))
            corners.append(inside[sl])
        allin = np.logical_and.reduce(corners)
        anyin = np.logical_or.reduce(corners)
        self.kappa = np.where(allin, 1.0, 0.0)
        self.cutmask = anyin & ~allin
        # face apertures and centroid offsets (units of h; 0 for full faces)
        self.alpha = []
        self.foff = []    # dict (face numpy index) -> tuple of transverse offsets
        for d in range(dim):
            ax = dim - 1 - d
            fshp = list(shp)
            fshp[ax] += 1
            tr = [e for e in range(dim) if e != d]
            fc = []
            for off in np.ndindex(*(2,) * (dim - 1)):
                sl = [slice(None)] * dim
                for k, e in enumerate(tr):
                    sl[dim - 1 - e] = slice(off[k], off[k] + shp[dim - 1 - e])
                fc.append(inside[tuple(sl)])
            fall = np.logical_and.reduce(fc)
            fany = np.logical_or.reduce(fc)
            alpha = np.where(fall, 1.0, 0.0)
            offs = {}
            for idx in zip(*np.nonzero(fany & ~fall)):
                a, c = self._face_moments(d, idx)
                if a < TINY:
                    a = 0.0
                alpha[idx] = a
                offs[idx] = c
            self.alpha.append(alpha)
            self.foff.append(offs)
        self.cut = {}
        for idx in zip(*np.nonzero(self.cutmask)):
            cc = self._cell_moments(idx)
            if cc.kappa < TINY:
                self.kappa[idx] = 0.0
                continue
            self.kappa[idx] = cc.kappa
            self.cut[idx] = cc

    # -- faces ---------------------------------------------------------------
    def _face_corner_values(self, d, idx):
        """Corner values of face (d, idx) in (u, v) order: u, v = transverse
        axes in increasing order. idx is the numpy index of the face."""
        dim = self.geo.dim
        s = self.s
        if dim == 2:
            # face normal to d is an edge along the other axis e
            if d == 0:   # x-face at node column idx[1], cells row idx[0]
                j, i = idx
                return s[j, i], s[j + 1, i]
            j, i = idx
            return s[j, i], s[j, i + 1]
        k, j, i = idx
        if d == 0:   # u = y, v = z
            return s[k, j, i], s[k, j + 1, i], s[k + 1, j + 1, i], s[k + 1, j, i]
        if d == 1:   # u = x, v = z
            return s[k, j, i], s[k, j, i + 1], s[k + 1, j, i + 1], s[k + 1, j, i]
        return s[k, j, i], s[k, j, i + 1], s[k, j + 1, i + 1], s[k, j + 1, i]

    def _face_moments(self, d, idx):
        vals = self._face_corner_values(d, idx)
        if self.geo.dim == 2:
            a, c = edge_moments(*vals)
            return a, (c - 0.5,)
        a, (cu, cv) = square_moments(*vals)
        return a, (cu - 0.5, cv - 0.5)

    def face_offsets(self, d, idx):
        return self.foff[d].get(idx, (0.0,) * (self.geo.dim - 1))

    # -- cells ---------------------------------------------------------------
    def _cell_moments(self, idx):
        if self.geo.dim == 2:
            return self._cell2(idx)
        return self._cell3(idx)

    def _cell2(self, idx):
        geo = self.geo
        h = geo.h
        j, i = idx
        s = self.s
        verts, cross, _ = square_polygon(s[j, i], s[j, i + 1], s[j + 1, i + 1], s[j + 1, i])
        area, (cu, cv) = polygon_area_centroid(verts)
        cc = CutCell()
        cc.kappa = area
        x0 = geo.lo[0] + i * h
        y0 = geo.lo[1] + j * h
        cc.vcent = np.array([x0 + cu * h, y0 + cv * h])
        if len(cross) == 2:
            (u0, v0), (u1, v1) = cross
            cc.eb_cent = np.array([x0 + 0.5 * (u0 + u1) * h, y0 + 0.5 * (v0 + v1) * h])
            ax_lo = self.alpha[0][j, i]
            ax_hi = self.alpha[0][j, i + 1]
            ay_lo = self.alpha[1][j, i]
            ay_hi = self.alpha[1][j + 1, i]
            vec = np.array([ax_lo - ax_hi, ay_lo - ay_hi])
            nrm = math.hypot(vec[0], vec[1])
            cc.eb_area = nrm
            cc.eb_normal = vec / nrm if nrm > 0 else np.zeros(2)
        return cc

    def _cell3(self, idx):
        geo = self.geo
        h = geo.h
        k, j, i = idx
        s = self.s
        x0 = np.array([geo.lo[0] + i * h, geo.lo[1] + j * h, geo.lo[2] + k * h])
        xc = x0 + 0.5 * h
        # crossing points on the 12 cell edges, keyed (axis, a, b) with a, b the
        # offsets of the two transverse axes (increasing axis order)
        pts = {}
        for ax in range(3):
            tr = [e for e in range(3) if e != ax]
            for a in (0, 1):
                for b in (0, 1):
                    o = [0, 0, 0]
                    o[tr[0]] = a
                    o[tr[1]] = b
                    o2 = list(o)
                    o2[ax] = 1
                    sa = s[k + o[2], j + o[1], i + o[0]]
                    sb = s[k + o2[2], j + o2[1], i + o2[0]]
                    if (sa > 0) != (sb > 0):
                        p = x0 + np.array(o, dtype=float) * h
                        p[ax] += _t(sa, sb) * h
                        pts[(ax, a, b)] = p
        # faces: polygons (for volume) and segments (for the facet loop)
        vol = 0.0
        mom = np.zeros(3)
        seg_adj = {}
        alo = np.zeros(3)
        ahi = np.zeros(3)
        for d in range(3):
            tr = [e for e in range(3) if e != d]
            for side in (0, 1):
                fidx = [k, j, i]
                fidx[2 - d] += side
                fidx = tuple(fidx)
                a = self.alpha[d][fidx]
                if side == 0:
                    alo[d] = a
                else:
                    ahi[d] = a
                if a > 0:
                    off = self.face_offsets(d, fidx)
                    fc = x0.copy()
                    fc[d] += side * h
                    fc[tr[0]] += (0.5 + off[0]) * h
                    fc[tr[1]] += (0.5 + off[1]) * h
                    area = a * h * h
                    cone = area * (0.5 * h) / 3.0
                    vol += cone
                    mom += cone * (xc + 0.75 * (fc - xc))
                # facet segment on this face: crossings on its 4 edges
                ends = []
                for (ax, aa, bb), p in pts.items():
                    if ax == d:
                        continue
                    o = [None, None, None]
                    trax = [e for e in range(3) if e != ax]
                    o[trax[0]] = aa
                    o[trax[1]] = bb
                    if o[d] == side:
                        ends.append((ax, aa, bb))
                if len(ends) == 4:
                    raise GeometryError("saddle face in cell %s" % (idx,))
                if len(ends) == 2:
                    e0, e1 = ends
                    seg_adj.setdefault(e0, []).append(e1)
                    seg_adj.setdefault(e1, []).append(e0)
        cc = CutCell()
        if pts:
            # chain the crossing loop
            keys = sorted(pts.keys())
            start = keys[0]
            loop = [start]
            prev = None
            cur = start
            while True:
                nb = seg_adj.get(cur, [])
                if len(nb) != 2:
                    raise GeometryError("open crossing loop in cell %s" % (idx,))
                nxt = nb[0] if nb[0] != prev else nb[1]
                if nxt == start:
                    break
                loop.append(nxt)
                prev, cur = cur, nxt
                if len(loop) > 12:
                    raise GeometryError("bad crossing loop in cell %s" % (idx,))
            if len(loop) != len(pts):
                raise GeometryError("multi-valued cell %s" % (idx,))
            P = [pts[q] for q in loop]
            closure = (alo - ahi)
            m = sum(P) / len(P)
            tri = []
            tot = np.zeros(3)
            for q in range(len(P)):
                a = P[q]
                b = P[(q + 1) % len(P)]
                av = 0.5 * np.cross(a - m, b - m)
                tri.append((av, (m + a + b) / 3.0))
                tot += av
            sgn = 1.0 if float(np.dot(tot, closure)) >= 0.0 else -1.0
            nrm = float(np.linalg.norm(closure))
            cc.eb_area = nrm
            cc.eb_normal = closure / nrm if nrm > 0 else np.zeros(3)
            wsum = 0.0
            cent = np.zeros(3)
            for av, c in tri:
                av = sgn * av
                w = float(np.linalg.norm(av))
                wsum += w
                cent += w * c
                cone = float(np.dot(c - xc, av)) / 3.0
                vol += cone
                mom += cone * (xc + 0.75 * (c - xc))
            cc.eb_cent = cent / wsum if wsum > 0 else m
        cc.kappa = vol / h ** 3
        cc.vcent = mom / vol if vol > 0 else xc
        return cc


class Geometry:
    """All moments of one problem (both phases), plus unknown bookkeeping."""

    def __init__(self, prob):
        self.prob = prob
        self.dim = prob.dim
        self.n = prob.n
        self.h = prob.h
        self.lo = prob.lo
        self.shape = prob.shape
        objs = prob.objects
        diel = [k for k, o in enumerate(objs) if o.kind == W.OBJ_DIELECTRIC]
        if len(diel) > 1:
            raise GeometryError("at most one dielectric object")
        nshape = tuple(m + 1 for m in self.shape)
        for o in objs:
            if o.sdf.shape != nshape:
                raise GeometryError("level set shape")
        if objs:
            s_gas = np.minimum.reduce([o.sdf for o in objs]) if len(objs) > 1 else objs[0].sdf.copy()
        else:
            s_gas = np.ones(nshape)
        self.s = [s_gas]
        if diel:
            cov = [o.sdf for o in objs if o.kind != W.OBJ_DIELECTRIC]
            s_d = -objs[diel[0]].sdf
            if cov:
                s_d = np.minimum(np.minimum.reduce(cov), s_d)
            self.s.append(s_d)
        self.nphase = len(self.s)
        self.diel_obj = diel[0] if diel else -1
        # objects cutting each cell (G7 rejection, cutter lookup)
        self._cutters = self._object_cuts()
        self.ph = [PhaseGeom(self, s) for s in self.s]
        for p, pg in enumerate(self.ph):
            for idx, cc in pg.cut.items():
                cs = self._cutters.get(idx, [])
                if len(cs) != 1:
                    raise GeometryError("cell %s cut by %d objects" % (idx, len(cs)))
                cc.cutter = cs[0]
        # a gas/dielectric interface cell: dielectric shares the gas facet
        if self.nphase == 2:
            for idx, cd in self.ph[1].cut.items():
                cg = self.ph[0].cut.get(idx)
                if cg is not None and cd.cutter == self.diel_obj and cg.cutter == self.diel_obj:
                    cd.eb_cent = cg.eb_cent
                    cd.eb_area = cg.eb_area
                    cd.eb_normal = -cg.eb_normal
        self._number_dofs()

    def _object_cuts(self):
        out = {}
        dim = self.dim
        shp = self.shape
        for k, o in enumerate(self.prob.objects):
            # cut unless the level set has one strict sign at every corner
            # (a corner exactly on the surface belongs to neither side)
            pos, neg = o.sdf > 0, o.sdf < 0
            cp, cn = [], []
            for off in np.ndindex(*(2,) * dim):
                sl = tuple(slice(q, q + m) for q, m in zip(off, shp))
                cp.append(pos[sl])
                cn.append(neg[sl])
            mixed = ~np.logical_and.reduce(cp) & ~np.logical_and.reduce(cn)
            for idx in zip(*np.nonzero(mixed)):
                out.setdefault(idx, []).append(k)
        return out

    def _number_dofs(self):
        k0 = self.ph[0].kappa
        has0 = k0 > 0
        if self.nphase == 2:
            has1 = self.ph[1].kappa > 0
        else:
            has1 = np.zeros(self.shape, bool)
        self.has = [has0, has1]
        self.primary = np.where(has0, 0, np.where(has1, 1, -1)).astype(np.int8)
        two = has0 & has1
        self.N = int(np.prod(self.shape))
        lin = np.nonzero(two.ravel())[0]
        self.sec_cells = lin               # secondary DOF k lives in cell lin[k]
        self.N2 = len(lin)
        self.sec_index = np.full(self.N, -1, dtype=np.int64)
        self.sec_index[lin] = np.arange(self.N2)

    # -- helpers ---------------------------------------------------------------
    def lin(self, idx):
        return int(np.ravel_multi_index(idx, self.shape))

    def dof(self, idx, p):
        """Unknown index of phase p in cell idx, or -1."""
        if any(q < 0 or q >= m for q, m in zip(idx, self.shape)):
            return -1
        if not self.has[p][idx]:
            return -1
        c = self.lin(idx)
        if self.primary[idx] == p:
            return c
        return self.N + int(self.sec_index[c])

    def centre(self, idx):
        """Cell centre (x, y[, z]) of numpy index idx."""
        return np.array([self.lo[d] + (idx[self.dim - 1 - d] + 0.5) * self.h for d in range(self.dim)])

    def kappa(self, p, idx):
        return float(self.ph[p].kappa[idx])
