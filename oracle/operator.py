"""ORACLE (test infrastructure) — the finite-volume system A phi = b.

Written from the Helmholtz-equations section of the paper (the Helmholtz form,
its integral form over a cut cell, face-centred fluxes, centroid
interpolation of fluxes, domain and embedded-boundary conditions, the
multifluid matching condition with elimination of the boundary state).

Row of unknown (cell i, phase p), in the volume-weighted integral form:
    L_i(phi) = kappa_i alpha a_p phi_i
               + (beta/h) [ sum_faces alpha_f Fbar_f + alpha_EB F_EB ],
with every flux taken outward from the cell; b_i = kappa_i rho_i - L_i(0),
A = the linear part of L. All boundary data (domain values, electrode
potentials, wall fluxes, surface charge) therefore live in b.

Readings where the text is silent, garbled or ambiguous:
  * the Helmholtz form is alpha a phi + beta div(b grad phi) = rho;
  * face-centred flux F = b_p (phi_R - phi_L)/h between same-phase unknowns;
  * centroid interpolation (2D, as printed): Fbar = (1-|s|) F_f + |s| F_f',
    f' the parallel face one cell over toward the centroid, used only if f'
    is open and both its cells carry unknowns of the phase, else Fbar = F_f;
    3D: bilinear over 4 faces; if a neighbour face is missing, linear along
    the available axis with the larger |s|, else face-centred; |s| < 1e-12
    counts as 0;
  * domain faces (outward flux, phi_n = first cell, phi_nn = second):
      Neumann            F = b g
      Dirichlet linear   F = 2 b (phi_B - phi_n)/h              (default)
      Dirichlet quadratic F = -(b/h)(3 phi_n - phi_nn/3 - 8 phi_B/3)
        (the printed formula has its two cell indices swapped; as read here
        it is exact for quadratics)
      Robin a1 phi + a2 dphi/dn = a3, linear extrapolation to the face
        phi_b = (phi_n + (h/2) a3/a2)/(1 + (h/2) a1/a2), F = b (a3 - a1 phi_b)/a2
      Robin Taylor       phi_b = (3 phi_n - phi_nn)/2
    (quadratic / Taylor fall back to linear where phi_nn is missing);
  * EB Dirichlet normal derivative, second order: m = -n_EB (into the phase),
    d* = argmax |m_d| (ties within 1e-12 -> lowest d), rays to the planes of
    cell centres one and two cells away along d*, quadratic interpolation
    across the 3 (3x3) cells centred on the containing cell, and
    dphi/dm = [t2^2 (phi1 - phiB) - t1^2 (phi2 - phiB)] / (t1 t2 (t2 - t1));
    the cut cell itself is never used; first-order option: one plane,
    linear interpolation, (phi1 - phiB)/t1;
  * least-squares fallback when a ray stencil leaves the box or meets a
    cell without an unknown of the phase: unknowns within 2 cells that lie
    in front of the facet ((x_j - x_EB).m > 0, the side the phase occupies),
    plus the centres of Dirichlet domain faces of those cells and of the cut
    cell itself (known values; the cut cell's unknown is never used),
    weights 1/|x_j - x_EB|^2, fit phi_j - phiB = g.(x_j - x_EB); the fit is
    accepted when it has rank D and a negative weight on phiB (a one-sided
    derivative); otherwise the radius grows to 3 cells; as a last resort
    (slivers against box walls with no unknown in front of the facet), the
    derivative toward the Dirichlet domain face that m faces most,
    (m.n_w)(phi_wall - phiB)/d_w (d_w >= h/20); else the cell is rejected;
  * multifluid facet: eps_g dphi/dm_g + eps_s dphi/dm_s = -sigma (the sign that
    makes a thin layer of charge sigma/delta converge to it), phi_B eliminated;
  * EB wall (insulator without a phase): F_EB = b g.

Parity, per function (each pin is fixed by mathematics, not by this code):
  * face fluxes, centroid interpolation, regular template: cubic exactness of
    regular rows, quadratic exactness of 2D cut rows and 3D planar cut rows,
    symmetry and definiteness of the regular operator, the closed-form
    discrete sine solution (tests/test_oracle_operator.py);
  * domain closures: exactness per closure and degree, the Robin linear and
    Taylor closures for linear phi (test_oracle_operator.py,
    test_oracle_fallbacks.py);
  * _ray (order 2): quadratic exactness of cut rows; _ray (order 1): exact
    for linear p, directly and in assembled rows (test_oracle_fallbacks.py);
  * _lsq: exact derivative for linear p without and with Dirichlet wall
    values on both sides of the box, and zero flux divergence of linear p in
    every cut row with the ray switched off (test_oracle_fallbacks.py);
  * _wall: exact for a field linear along the chosen face's normal, face
    choice at all four corners (test_oracle_fallbacks.py);
  * multifluid elimination and the sign of sigma: planar piecewise-linear
    exactness, the coaxial closed form with and without surface charge;
  * the whole EB operator at scale: second-order Richardson convergence on
    the two-disk and pin-plane classes (test_oracle_richardson.py) and the
    coaxial test; flux balance.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

import workloads as W
from .geometry import Geometry, GeometryError, TINY

DIRICHLET_LINEAR, DIRICHLET_QUADRATIC = 0, 1
ROBIN_LINEAR, ROBIN_TAYLOR = 0, 1


class Options:
    def __init__(self, dirichlet_closure=DIRICHLET_LINEAR, robin_closure=ROBIN_LINEAR, eb_order=2):
        self.dirichlet_closure = dirichlet_closure
        self.robin_closure = robin_closure
        self.eb_order = eb_order


class Form:
    """Linear form: sum_j c[j] phi_j + sum_k d[k] * datum_k."""
    __slots__ = ("c", "d")

    def __init__(self, c=None, d=None):
        self.c = dict(c) if c else {}
        self.d = dict(d) if d else {}

    def axpy(self, w, other):
        if w == 0.0:
            return self
        for k, v in other.c.items():
            self.c[k] = self.c.get(k, 0.0) + w * v
        for k, v in other.d.items():
            self.d[k] = self.d.get(k, 0.0) + w * v
        return self

    def scaled(self, w):
        return Form().axpy(w, self)


def _cell_ix(geo, idx):
    """numpy index -> (i_x, i_y[, i_z])."""
    return tuple(reversed(idx))


def _np_ix(ic):
    return tuple(reversed(ic))


def _inbox(geo, ic):
    return all(0 <= ic[d] < geo.n[d] for d in range(geo.dim))


class Builder:
    def __init__(self, prob, opts=None):
        self.prob = prob
        self.geo = Geometry(prob)
        self.opts = opts or Options()
        g = self.geo
        self.bphase = [prob.b_gas]
        self.aphase = [prob.a_gas]
        if g.nphase == 2:
            self.bphase.append(prob.objects[g.diel_obj].value)
            self.aphase.append(prob.a_diel)

    # -- unknown lookup ------------------------------------------------------
    def dof(self, ic, p):
        g = self.geo
        if not _inbox(g, ic):
            return -1
        return g.dof(_np_ix(ic), p)

    # -- faces ---------------------------------------------------------------
    def _alpha(self, p, d, ic, side):
        """Aperture of face (d, side) of cell ic for phase p."""
        fi = list(ic)
        fi[d] += side
        return float(self.geo.ph[p].alpha[d][_np_ix(fi)]), _np_ix(fi)

    def _centred_out(self, ic, p, d, side):
        """Face-centred outward flux form of face (d, side) of cell ic, or None."""
        g = self.geo
        b = self.bphase[p]
        h = g.h
        me = self.dof(ic, p)
        if me < 0:
            return None
        nb = list(ic)
        nb[d] += 1 if side else -1
        if 0 <= nb[d] < g.n[d]:
            j = self.dof(nb, p)
            if j < 0:
                return None
            f = Form()
            f.c[j] = b / h
            f.c[me] = f.c.get(me, 0.0) - b / h
            return f
        # domain face
        fid = 2 * d + side
        kind = self.prob.bc_kind[fid]
        nn = list(ic)
        nn[d] += -1 if side else 1
        jn = self.dof(nn, p) if 0 <= nn[d] < g.n[d] else -1
        f = Form()
        if kind == W.BC_NEUMANN:
            f.d[("face", fid)] = b
        elif kind == W.BC_DIRICHLET:
            if self.opts.dirichlet_closure == DIRICHLET_QUADRATIC and jn >= 0:
                f.c[me] = -3.0 * b / h
                f.c[jn] = (1.0 / 3.0) * b / h
                f.d[("face", fid)] = (8.0 / 3.0) * b / h
            else:
                f.c[me] = -2.0 * b / h
                f.d[("face", fid)] = 2.0 * b / h
        elif kind == W.BC_ROBIN:
            a1 = self.prob.robin_a1[fid]
            a2 = self.prob.robin_a2[fid]
            if self.opts.robin_closure == ROBIN_TAYLOR and jn >= 0:
                f.c[me] = -(b / a2) * a1 * 1.5
                f.c[jn] = (b / a2) * a1 * 0.5
                f.d[("face", fid)] = b / a2
            else:
                cc = 1.0 / (1.0 + 0.5 * h * a1 / a2)
                f.c[me] = -(b * a1 / a2) * cc
                f.d[("face", fid)] = (b / a2) * (1.0 - a1 * cc * 0.5 * h / a2)
        else:
            raise ValueError("bad boundary kind")
        return f

    def _shifted(self, ic, p, d, side, shifts):
        """Centred flux of the parallel face shifted by `shifts` (dict axis->+-1)."""
        sc = list(ic)
        for e, s in shifts.items():
            sc[e] += s
        if not _inbox(self.geo, sc):
            return None
        a, _ = self._alpha(p, d, sc, side)
        if a <= 0.0:
            return None
        return self._centred_out(sc, p, d, side)

    def face_out(self, ic, p, d, side):
        """Centroid-interpolated outward flux form of a face, with its aperture."""
        g = self.geo
        a, fidx = self._alpha(p, d, ic, side)
        if a <= 0.0:
            return 0.0, None
        base = self._centred_out(ic, p, d, side)
        if base is None:
            return 0.0, None
        offs = g.ph[p].face_offsets(d, fidx)
        tr = [e for e in range(g.dim) if e != d]
        axes = [(tr[k], offs[k]) for k in range(len(tr)) if abs(offs[k]) >= TINY]
        if not axes:
            return a, base
        if len(axes) == 1:
            e, s = axes[0]
            f1 = self._shifted(ic, p, d, side, {e: 1 if s > 0 else -1})
            if f1 is None:
                return a, base
            return a, Form().axpy(1.0 - abs(s), base).axpy(abs(s), f1)
        (e1, s1), (e2, s2) = axes
        d1 = 1 if s1 > 0 else -1
        d2 = 1 if s2 > 0 else -1
        f1 = self._shifted(ic, p, d, side, {e1: d1})
        f2 = self._shifted(ic, p, d, side, {e2: d2})
        f12 = self._shifted(ic, p, d, side, {e1: d1, e2: d2})
        u1, u2 = abs(s1), abs(s2)
        if f1 is not None and f2 is not None and f12 is not None:
            out = Form()
            out.axpy((1 - u1) * (1 - u2), base).axpy(u1 * (1 - u2), f1)
            out.axpy((1 - u1) * u2, f2).axpy(u1 * u2, f12)
            return a, out
        # linear along the available axis with the larger |s| (ties: lower axis)
        cand = []
        if f1 is not None:
            cand.append((u1, e1, f1))
        if f2 is not None:
            cand.append((u2, e2, f2))
        if not cand:
            return a, base
        cand.sort(key=lambda t: (-t[0], t[1]))
        u, _, fx = cand[0]
        return a, Form().axpy(1.0 - u, base).axpy(u, fx)

    # -- embedded boundary ---------------------------------------------------
    def _ray(self, ic, p, xb, m, order):
        g = self.geo
        h = g.h
        dim = g.dim
        am = [abs(v) for v in m]
        mx = max(am)
        ds = min(d for d in range(dim) if am[d] >= mx - 1e-12)
        sr = 1 if m[ds] > 0 else -1
        ks = (1, 2) if order == 2 else (1,)
        ts = []
        vals = []
        for k in ks:
            plane = ic[ds] + k * sr
            if not (0 <= plane < g.n[ds]):
                return None
            xp = g.lo[ds] + (plane + 0.5) * h
            t = (xp - xb[ds]) / m[ds]
            pt = [xb[d] + t * m[d] for d in range(dim)]
            # tensor-product interpolation over the transverse axes
            terms = [({}, 1.0)]
            for e in range(dim):
                if e == ds:
                    continue
                q = (pt[e] - g.lo[e]) / h
                if order == 2:
                    c = math.floor(q)
                    xi = q - (c + 0.5)
                    ws = [(c - 1, 0.5 * xi * (xi - 1.0)), (c, 1.0 - xi * xi), (c + 1, 0.5 * xi * (xi + 1.0))]
                else:
                    c = math.floor(q - 0.5)
                    th = q - (c + 0.5)
                    ws = [(c, 1.0 - th), (c + 1, th)]
                new = []
                for sub, w in terms:
                    for cc, wc in ws:
                        s2 = dict(sub)
                        s2[e] = cc
                        new.append((s2, w * wc))
                terms = new
            form = Form()
            for sub, w in terms:
                cell = list(ic)
                cell[ds] = plane
                for e, cc in sub.items():
                    cell[e] = cc
                j = self.dof(cell, p)
                if j < 0:
                    return None
                form.c[j] = form.c.get(j, 0.0) + w
            ts.append(t)
            vals.append(form)
        if order == 2:
            t1, t2 = ts
            w1 = t2 / (t1 * (t2 - t1))
            w2 = -t1 / (t2 * (t2 - t1))
            out = Form().axpy(w1, vals[0]).axpy(w2, vals[1])
            return -(w1 + w2), out
        t1 = ts[0]
        return -1.0 / t1, Form().axpy(1.0 / t1, vals[0])

    def _lsq(self, ic, p, xb, m):
        g = self.geo
        dim = g.dim
        h = g.h
        mv = np.asarray(m, dtype=float)
        for R in (2, 3):
            rows = []   # (key, dx, weight); key = unknown index or ("face", f)
            for off in np.ndindex(*(2 * R + 1,) * dim):
                o = [q - R for q in off]
                own = max(abs(q) for q in o) < 1
                cell = [ic[d] + o[d] for d in range(dim)]
                j = self.dof(cell, p)
                if j < 0:
                    continue
                xj = np.array([g.lo[d] + (cell[d] + 0.5) * h for d in range(dim)])
                dx = xj - xb
                if not own and float(dx @ mv) > 1e-9 * h:
                    rows.append((j, dx, 1.0 / float(dx @ dx)))
                # Dirichlet domain faces of this cell: known values
                for d in range(dim):
                    for side in (0, 1):
                        if cell[d] != (g.n[d] - 1 if side else 0):
                            continue
                        f = 2 * d + side
                        if self.prob.bc_kind[f] != W.BC_DIRICHLET:
                            continue
                        dw = dx.copy()
                        dw[d] += 0.5 * h if side else -0.5 * h
                        if float(dw @ mv) > 1e-9 * h:
                            rows.append((("face", f), dw, 1.0 / float(dw @ dw)))
            if len(rows) < dim:
                continue
            M = np.zeros((dim, dim))
            for _, dx, w in rows:
                M += w * np.outer(dx, dx)
            tr = np.trace(M)
            if np.linalg.det(M) <= 1e-10 * (tr / dim) ** dim:
                continue
            Mi = np.linalg.inv(M)
            form = Form()
            wsum = 0.0
            for key, dx, w in rows:
                cj = w * float((Mi @ dx) @ mv)
                if isinstance(key, tuple):
                    form.d[key] = form.d.get(key, 0.0) + cj
                else:
                    form.c[key] = form.c.get(key, 0.0) + cj
                wsum += cj
            if wsum <= 0.0:
                continue
            return -wsum, form
        raise GeometryError("no least-squares stencil at cell %s phase %d" % (ic, p))

    def _wall(self, ic, p, xb, m):
        """Last resort: derivative toward the Dirichlet domain face of the cut
        cell that the direction m faces most, (m.n_w)(phi_wall - phiB)/d_w,
        with d_w the distance from xb to that face (at least h/20)."""
        g = self.geo
        h = g.h
        best = None
        for d in range(g.dim):
            for side in (0, 1):
                if ic[d] != (g.n[d] - 1 if side else 0):
                    continue
                f = 2 * d + side
                if self.prob.bc_kind[f] != W.BC_DIRICHLET:
                    continue
                mn = m[d] if side else -m[d]
                if mn > 1e-12 and (best is None or mn > best[0] + 1e-12):
                    best = (mn, d, side, f)
        if best is None:
            raise GeometryError("no boundary stencil at cell %s phase %d" % (ic, p))
        mn, d, side, f = best
        wall = g.lo[d] + (g.n[d] if side else 0) * h
        dw = max(abs(wall - xb[d]), 0.05 * h)
        return -mn / dw, Form(d={("face", f): mn / dw})

    def dphi_dm(self, ic, p, xb, m, order):
        """Derivative along unit m (into phase p) at xb: (w_B, Form over unknowns)."""
        r = self._ray(ic, p, xb, m, order)
        if r is not None:
            return r
        try:
            return self._lsq(ic, p, xb, m)
        except GeometryError:
            return self._wall(ic, p, xb, m)

    def eb_flux(self, ic, p):
        """Outward EB flux form of a cut unknown, with the EB area fraction."""
        g = self.geo
        cc = g.ph[p].cut.get(_np_ix(ic))
        if cc is None or cc.eb_area <= 0.0:
            return 0.0, None
        b = self.bphase[p]
        obj = self.prob.objects[cc.cutter]
        xb = cc.eb_cent
        n = cc.eb_normal
        if obj.kind == W.OBJ_WALL:
            return cc.eb_area, Form(d={("obj", cc.cutter): b})
        if obj.kind == W.OBJ_ELECTRODE:
            wB, S = self.dphi_dm(ic, p, xb, -n, self.opts.eb_order)
            f = S.scaled(-b)
            f.d[("obj", cc.cutter)] = -b * wB
            return cc.eb_area, f
        # gas / dielectric interface: both sides from the gas facet
        if g.nphase < 2:
            raise GeometryError("interface without dielectric phase")
        ng = n if p == 0 else -n
        mg = -ng
        ms = ng
        eg, es = self.bphase[0], self.bphase[1]
        wg, Sg = self.dphi_dm(ic, 0, xb, mg, 2)
        ws, Ss = self.dphi_dm(ic, 1, xb, ms, 2)
        den = eg * wg + es * ws
        cell = g.lin(_np_ix(ic))
        phiB = Form(d={("sigma", cell): -1.0 / den})
        phiB.axpy(-eg / den, Sg).axpy(-es / den, Ss)
        if p == 0:
            dm = Form().axpy(wg, phiB).axpy(1.0, Sg)
        else:
            dm = Form().axpy(ws, phiB).axpy(1.0, Ss)
        return cc.eb_area, dm.scaled(-self.bphase[p])

    # -- rows ----------------------------------------------------------------
    def row(self, ic, p):
        """(mass coefficient, flux-part Form) of unknown (ic, p); L = mass*phi + flux."""
        g = self.geo
        h = g.h
        beta = self.prob.beta
        idx = _np_ix(ic)
        kap = g.kappa(p, idx)
        mass = kap * self.prob.alpha * self.aphase[p]
        flux = Form()
        for d in range(g.dim):
            for side in (0, 1):
                a, f = self.face_out(ic, p, d, side)
                if f is not None:
                    flux.axpy(beta * a / h, f)
        a, f = self.eb_flux(ic, p)
        if f is not None:
            flux.axpy(beta * a / h, f)
        return mass, flux

    def data_values(self, sigma=None, bc_value=None, obj_value=None):
        pr = self.prob
        bcv = list(pr.bc_value) if bc_value is None else list(bc_value)
        ov = [o.value for o in pr.objects] if obj_value is None else list(obj_value)
        sig = pr.sigma if sigma is None else sigma
        sig = None if sig is None else np.asarray(sig).ravel()

        def val(key):
            if key[0] == "face":
                return bcv[key[1]]
            if key[0] == "obj":
                return ov[key[1]]
            if key[0] == "sigma":
                return 0.0 if sig is None else float(sig[key[1]])
            raise KeyError(key)
        return val


class System:
    """Assembled A (scipy CSR over N + N2 unknowns, covered cells as identity
    rows) and b, with the geometry and the builder that made them."""

    def __init__(self, builder, A, b, mass, dof_rows):
        self.builder = builder
        self.geo = builder.geo
        self.A = A
        self.b = b
        self.mass = mass
        self.N = builder.geo.N
        self.N2 = builder.geo.N2
        self.dof_rows = dof_rows  # boolean mask of real unknowns

    def split(self, x):
        """(cell array of primary values, secondary values)."""
        return x[:self.N].reshape(self.geo.shape), x[self.N:]

    def residual(self, x):
        r = self.b - self.A @ x
        return r

    def rel_residual(self, x):
        return float(np.linalg.norm(self.residual(x)) / np.linalg.norm(self.b))


def _regular_mask(builder):
    """Cells whose primary row is the plain 2D+1 / 2D+1 point template:
    kappa = 1 for the primary phase and every in-box neighbour has the same
    phase as its primary unknown; domain faces with a closure that needs no
    second cell."""
    g = builder.geo
    pr = builder.prob
    prim = g.primary
    ok = np.zeros(g.shape, bool)
    for p in range(g.nphase):
        ok |= (prim == p) & (g.ph[p].kappa == 1.0)
    for d in range(g.dim):
        ax = g.dim - 1 - d
        for side in (0, 1):
            sl_me = [slice(None)] * g.dim
            sl_nb = [slice(None)] * g.dim
            if side:
                sl_me[ax] = slice(0, -1)
                sl_nb[ax] = slice(1, None)
            else:
                sl_me[ax] = slice(1, None)
                sl_nb[ax] = slice(0, -1)
            same = prim[tuple(sl_nb)] == prim[tuple(sl_me)]
            ok[tuple(sl_me)] &= same
            fid = 2 * d + side
            kind = pr.bc_kind[fid]
            needs2 = (kind == W.BC_DIRICHLET and builder.opts.dirichlet_closure == DIRICHLET_QUADRATIC) or \
                     (kind == W.BC_ROBIN and builder.opts.robin_closure == ROBIN_TAYLOR)
            if needs2:
                edge = [slice(None)] * g.dim
                edge[ax] = slice(-1, None) if side else slice(0, 1)
                ok[tuple(edge)] = False
    return ok


def assemble(prob, opts=None, rho=None, sigma=None, bc_value=None, obj_value=None, generic_only=False):
    """Build A and b. Regular template rows are vectorised; every other row
    goes through Builder.row (the two agree; see the tests)."""
    B = Builder(prob, opts)
    g = B.geo
    N, N2 = g.N, g.N2
    h = g.h
    dim = g.dim
    beta = prob.beta
    rho = prob.rho if rho is None else rho
    rho = np.zeros(g.shape) if rho is None else np.asarray(rho, dtype=np.float64).reshape(g.shape)
    val = B.data_values(sigma, bc_value, obj_value)
    rows, cols, vals = [], [], []
    b = np.zeros(N + N2)
    mass = np.zeros(N + N2)
    dof_rows = np.zeros(N + N2, bool)
    reg = np.zeros(g.shape, bool) if generic_only else _regular_mask(B)
    lin = np.arange(N).reshape(g.shape)
    # -- vectorised template rows
    if reg.any():
        prim = g.primary
        bc = np.where(prim == 1, B.bphase[-1], B.bphase[0]).astype(np.float64)
        ac = np.where(prim == 1, B.aphase[-1], B.aphase[0]).astype(np.float64)
        diag = np.zeros(g.shape)
        rhs_bnd = np.zeros(g.shape)
        for d in range(dim):
            ax = dim - 1 - d
            for side in (0, 1):
                sl_me = [slice(None)] * dim
                sl_nb = [slice(None)] * dim
                if side:
                    sl_me[ax] = slice(0, -1)
                    sl_nb[ax] = slice(1, None)
                else:
                    sl_me[ax] = slice(1, None)
                    sl_nb[ax] = slice(0, -1)
                me = reg[tuple(sl_me)]
                coef = (beta / h) * (bc[tuple(sl_me)] / h)
                rows.append(lin[tuple(sl_me)][me])
                cols.append(lin[tuple(sl_nb)][me])
                vals.append(coef[me])
                dg = np.zeros(g.shape)
                dg[tuple(sl_me)] = -(beta / h) * (bc[tuple(sl_me)] / h)
                diag += np.where(reg, dg, 0.0)
                # domain face
                edge = [slice(None)] * dim
                edge[ax] = slice(-1, None) if side else slice(0, 1)
                edge = tuple(edge)
                fid = 2 * d + side
                kind = prob.bc_kind[fid]
                be = bc[edge]
                if kind == W.BC_NEUMANN:
                    dme = 0.0
                    dat = be
                elif kind == W.BC_DIRICHLET:
                    dme = -2.0 * be / h
                    dat = 2.0 * be / h
                else:
                    a1 = prob.robin_a1[fid]
                    a2 = prob.robin_a2[fid]
                    cc = 1.0 / (1.0 + 0.5 * h * a1 / a2)
                    dme = -(be * a1 / a2) * cc
                    dat = (be / a2) * (1.0 - a1 * cc * 0.5 * h / a2)
                dg = np.zeros(g.shape)
                dg[edge] = (beta / h) * dme
                diag += np.where(reg, dg, 0.0)
                rb = np.zeros(g.shape)
                rb[edge] = (beta / h) * dat * val(("face", fid))
                rhs_bnd += np.where(reg, rb, 0.0)
        m_reg = prob.alpha * ac
        rows.append(lin[reg])
        cols.append(lin[reg])
        vals.append((diag + m_reg)[reg])
        b[:N][reg.ravel()] = (rho - rhs_bnd)[reg]
        mass[:N][reg.ravel()] = m_reg[reg]
        dof_rows[:N][reg.ravel()] = True
    # -- covered cells: identity rows
    cov = (g.primary < 0).ravel()
    ci = np.nonzero(cov)[0]
    rows.append(ci)
    cols.append(ci)
    vals.append(np.ones(len(ci)))
    # -- every other unknown through the generic row builder
    rr, cc_, vv = [], [], []
    todo = [(idx, int(g.primary[idx])) for idx in zip(*np.nonzero((~reg) & (g.primary >= 0)))]
    for k in range(N2):
        c = int(g.sec_cells[k])
        idx = np.unravel_index(c, g.shape)
        todo.append((tuple(int(q) for q in idx), 1))
    for idx, p in todo:
        idx = tuple(int(q) for q in idx)
        ic = _cell_ix(g, idx)
        i = g.dof(idx, p)
        m_, f = B.row(ic, p)
        rr.append(i); cc_.append(i); vv.append(m_)
        for j, v in f.c.items():
            rr.append(i); cc_.append(j); vv.append(v)
        kap = g.kappa(p, idx)
        src = kap * rho[idx] if g.primary[idx] == p else 0.0
        b[i] = src - sum(v * val(k) for k, v in f.d.items())
        mass[i] = m_
        dof_rows[i] = True
    rows.append(np.asarray(rr, dtype=np.int64))
    cols.append(np.asarray(cc_, dtype=np.int64))
    vals.append(np.asarray(vv, dtype=np.float64))
    R = np.concatenate(rows)
    C = np.concatenate(cols)
    V = np.concatenate(vals)
    A = sp.csr_matrix((V, (R, C)), shape=(N + N2, N + N2))
    A.sum_duplicates()
    return System(B, A, b, mass, dof_rows)
