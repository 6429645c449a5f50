"""ORACLE (test infrastructure) — one explicit advection step of a density on
the gas phase of a cut-cell grid (Convection-Diffusion-Reaction equations:
Advective discretization and Hybrid divergence).

The step n^{k+1} = n^k - dt D computes, in the paper's order:
  1. face-centred states by an unsplit Godunov predictor with van Leer
     limiting: per cell and axis the monotonised-central slope
     s = sign(dc) min(2|dl|, 2|dr|, |dc|) when dl dr > 0, else 0 (dl, dr, dc
     the one-sided and central differences; 0 where a neighbour along the
     axis carries no gas); the state on a face is taken from the upwind cell
     (the solution of the linear-advection Riemann problem) extrapolated in
     space to the face and in time to the half step, including the
     transverse terms:  n_U + (sigma/2 - u dt/(2h)) s_d
                          - dt/(2h) sum_{d' != d} v_{U,d'} s_{d'},
     sigma = +1 when U is the low cell, -1 when it is the high cell, u the
     face-normal velocity, v_U the cell velocity (mean of its two faces per
     axis); an inflow domain face takes the boundary density;
  2. face-centred fluxes F = u n_f, interpolated to the face centroids as the
     Helmholtz fluxes are (linear in 2D, bilinear in 3D over the open
     parallel faces whose cells both carry gas, falling back to linear along
     the available axis with the larger offset, then to face-centred);
  3. the conservative divergence D^c = (1/(kappa h)) sum +-alpha_f Fbar_f
     (no flux through the embedded boundary);
  4. in cut cells (0 < kappa < 1) the non-conservative divergence D^nc, the
     kappa-weighted mean of D^c over the gas cells of the 3^D block around
     the cell, the hybrid D^H = kappa D^c + (1 - kappa) D^nc and the mass the
     hybrid fails to conserve, dM = kappa (1 - kappa) (D^nc - D^c);
  5. redistribution of dM to the gas cells of the block other than the cell
     itself in proportion to their kappa (weights W = 1): a receiving cell j
     gets the mass dM kappa_j / S, S the sum of kappa over those cells, i.e.
     its rate falls by dM / S. (The paper prints D_j = D^H_j + dM_{i,j}; the
     sign and the division by kappa_j used here are the ones for which the
     total mass sum kappa n h^D changes by exactly the domain-boundary
     fluxes, which the tests check.) A cut cell with no gas neighbour keeps
     its conservative divergence.

Parity: pinned by tests/test_oracle_advection.py (free-stream preservation,
exact translation of linear data in regular cells, mass balance to rounding
with embedded boundaries, second-order convergence of a smooth pulse, the
limiter's closed form on monotone, extremal and step data).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, TINY


def mc_slope(dl, dr):
    """Monotonised-central (van Leer) slope of one-sided differences dl, dr."""
    dc = 0.5 * (dl + dr)
    s = np.sign(dc) * np.minimum(np.minimum(2.0 * np.abs(dl), 2.0 * np.abs(dr)), np.abs(dc))
    return np.where(dl * dr > 0.0, s, 0.0)


class Advection:
    """Gas-phase geometry of a problem (``workloads.Problem``) for advection."""

    def __init__(self, prob):
        self.prob = prob
        self.geo = Geometry(prob)
        g = self.geo
        self.dim = g.dim
        self.h = g.h
        self.shape = g.shape
        ph = g.ph[0]
        self.gas = g.has[0].copy()
        self.kappa = np.where(self.gas, ph.kappa, 0.0)
        self.alpha = [ph.alpha[d] for d in range(self.dim)]

    # numpy axis of physical direction d
    def ax(self, d):
        return self.dim - 1 - d

    def _shift(self, a, d, k, fill=0.0):
        """b[i] = a[i + k e_d] (fill outside)."""
        ax = self.ax(d)
        b = np.full_like(a, fill)
        n = a.shape[ax]
        src = [slice(None)] * a.ndim
        dst = [slice(None)] * a.ndim
        if k > 0:
            src[ax] = slice(k, n)
            dst[ax] = slice(0, n - k)
        else:
            src[ax] = slice(0, n + k)
            dst[ax] = slice(-k, n)
        b[tuple(dst)] = a[tuple(src)]
        return b

    def slopes(self, n):
        out = []
        for d in range(self.dim):
            nl = self._shift(n, d, -1)
            nr = self._shift(n, d, 1)
            gl = self._shift(self.gas, d, -1, False)
            gr = self._shift(self.gas, d, 1, False)
            s = mc_slope(n - nl, nr - n)
            out.append(np.where(self.gas & gl & gr, s, 0.0))
        return out

    def face_states(self, n, u, dt, inflow):
        """Face-centred fluxes F_d (face arrays) of the predictor."""
        h = self.h
        s = self.slopes(n)
        vc = []
        for d in range(self.dim):
            ax = self.ax(d)
            lo = np.take(u[d], range(0, u[d].shape[ax] - 1), axis=ax)
            hi = np.take(u[d], range(1, u[d].shape[ax]), axis=ax)
            vc.append(0.5 * (lo + hi))
        # per cell: extrapolated states to its low and high faces along d
        fluxes = []
        for d in range(self.dim):
            ax = self.ax(d)
            trans = sum((vc[e] * s[e] for e in range(self.dim) if e != d), np.zeros(self.shape))
            base = n - 0.5 * dt / h * trans
            nf = u[d].shape[ax]
            F = np.zeros(u[d].shape)
            for f in range(nf):
                sl = [slice(None)] * self.dim
                sl[ax] = f
                uf = u[d][tuple(sl)]
                # low cell f - 1 (face on its high side), high cell f
                if f - 1 >= 0:
                    cl = [slice(None)] * self.dim
                    cl[ax] = f - 1
                    cl = tuple(cl)
                    stl = base[cl] + (0.5 - uf * dt / (2 * h)) * s[d][cl]
                    gl = self.gas[cl]
                else:
                    stl = np.full(uf.shape, inflow[2 * d])
                    gl = np.ones(uf.shape, bool)
                if f < nf - 1:
                    cr = [slice(None)] * self.dim
                    cr[ax] = f
                    cr = tuple(cr)
                    str_ = base[cr] + (-0.5 - uf * dt / (2 * h)) * s[d][cr]
                    gr = self.gas[cr]
                else:
                    str_ = np.full(uf.shape, inflow[2 * d + 1])
                    gr = np.ones(uf.shape, bool)
                st = np.where(uf >= 0.0, stl, str_)
                ok = np.where(uf >= 0.0, gl, gr)
                F[tuple(sl)] = np.where(ok, uf * st, 0.0)
            fluxes.append(F)
        return fluxes

    def _face_ok(self, d, fidx):
        """Face (d, numpy index) open and both its cells (in the box) with gas."""
        a = self.alpha[d]
        if any(q < 0 or q >= m for q, m in zip(fidx, a.shape)) or a[fidx] <= 0.0:
            return False
        ax = self.ax(d)
        for k in (-1, 0):
            c = list(fidx)
            c[ax] += k
            if 0 <= c[ax] < self.shape[ax] and not self.gas[tuple(c)]:
                return False
        return True

    def centroid_fluxes(self, F):
        """Fluxes interpolated to the face centroids (cut faces only change)."""
        out = [f.copy() for f in F]
        ph = self.geo.ph[0]
        for d in range(self.dim):
            tr = [e for e in range(self.dim) if e != d]
            for fidx, offs in ph.foff[d].items():
                if self.alpha[d][fidx] <= 0.0:
                    continue
                axes = [(tr[k], offs[k]) for k in range(len(tr)) if abs(offs[k]) >= TINY]
                if not axes:
                    continue

                def shifted(shifts):
                    c = list(fidx)
                    for e, sgn in shifts.items():
                        c[self.ax(e)] += sgn
                    c = tuple(c)
                    return F[d][c] if self._face_ok(d, c) else None
                base = F[d][fidx]
                if len(axes) == 1:
                    e, sv = axes[0]
                    f1 = shifted({e: 1 if sv > 0 else -1})
                    out[d][fidx] = base if f1 is None else (1 - abs(sv)) * base + abs(sv) * f1
                    continue
                (e1, s1), (e2, s2) = axes
                d1, d2 = (1 if s1 > 0 else -1), (1 if s2 > 0 else -1)
                f1, f2, f12 = shifted({e1: d1}), shifted({e2: d2}), shifted({e1: d1, e2: d2})
                u1, u2 = abs(s1), abs(s2)
                if f1 is not None and f2 is not None and f12 is not None:
                    out[d][fidx] = ((1 - u1) * (1 - u2) * base + u1 * (1 - u2) * f1 + (1 - u1) * u2 * f2
                                    + u1 * u2 * f12)
                    continue
                cand = [(u1, e1, f1), (u2, e2, f2)]
                cand = [c for c in cand if c[2] is not None]
                if not cand:
                    continue
                cand.sort(key=lambda t: (-t[0], t[1]))
                uu, _, fx = cand[0]
                out[d][fidx] = (1 - uu) * base + uu * fx
        return out

    def divergence(self, n, u, dt, inflow):
        """(final rate D, conservative D^c) of one step."""
        h = self.h
        Fb = self.centroid_fluxes(self.face_states(n, u, dt, inflow))
        net = np.zeros(self.shape)
        for d in range(self.dim):
            ax = self.ax(d)
            aF = self.alpha[d] * Fb[d]
            hi = np.take(aF, range(1, aF.shape[ax]), axis=ax)
            lo = np.take(aF, range(0, aF.shape[ax] - 1), axis=ax)
            net += hi - lo
        k = self.kappa
        Dc = np.where(self.gas, net / (np.where(k > 0, k, 1.0) * h), 0.0)
        D = Dc.copy()
        irr = np.argwhere(self.gas & (k < 1.0))
        rate_fix = np.zeros(self.shape)
        for idx in map(tuple, irr):
            nb = [tuple(np.add(idx, o)) for o in np.ndindex(*(3,) * self.dim)]
            nb = [tuple(int(q) - 1 for q in c) for c in nb]
            nb = [c for c in nb if all(0 <= c[a] < self.shape[a] for a in range(self.dim)) and self.gas[c]]
            others = [c for c in nb if c != idx]
            S = sum(k[c] for c in others)
            if S <= 0.0:
                continue
            Dnc = sum(k[c] * Dc[c] for c in nb) / sum(k[c] for c in nb)
            ki = k[idx]
            D[idx] = ki * Dc[idx] + (1 - ki) * Dnc
            dM = ki * (1 - ki) * (Dnc - Dc[idx])
            for c in others:
                rate_fix[c] -= dM / S
        return D + rate_fix, Dc

    def step(self, n, u, dt, inflow=(0.0,) * 6):
        D, _ = self.divergence(n, u, dt, inflow)
        return np.where(self.gas, n - dt * D, 0.0)

    def boundary_outflux(self, n, u, dt, inflow=(0.0,) * 6):
        """Net flux h^(D-1) sum alpha Fbar out through the box faces."""
        Fb = self.centroid_fluxes(self.face_states(n, u, dt, inflow))
        tot = 0.0
        for d in range(self.dim):
            ax = self.ax(d)
            aF = self.alpha[d] * Fb[d]
            tot += np.take(aF, [aF.shape[ax] - 1], axis=ax).sum() - np.take(aF, [0], axis=ax).sum()
        return tot * self.h ** (self.dim - 1)
