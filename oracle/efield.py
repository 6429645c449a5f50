"""ORACLE (test infrastructure) — flux-based electric field E = -grad(phi).

The paper defines E = -grad(Phi) (electrodynamic-equations section) and
evaluates gradients through the same centroid-interpolated face fluxes as the
operator. Reading used here (the paper gives no cell-centred formula):
  * on an open face the gradient is Fbar/b_p (outward normal derivative), so
    d(phi)/dx_d = +Fbar/b_p on the high face and -Fbar/b_p on the low face;
    domain faces use their closure;
  * cell E_d = -(mean of d(phi)/dx_d over the open low/high faces in d);
  * with neither face open, E_d = -(F_EB/b_p) n_EB,d (the EB normal gradient).
E is reported for the primary unknown of each cell; covered cells get 0.

Parity: the vectorised regular-cell path equals the generic path
(tests/test_oracle_efield.py); the field of the coaxial closed form converges;
a linear field normal to a planar electrode is reproduced exactly in every
cell, and by the EB normal-gradient branch when it is forced
(tests/test_oracle_fallbacks.py).
"""
from __future__ import annotations

import numpy as np

import workloads as W
from .operator import _regular_mask, _cell_ix


def _eval(form, x, val):
    s = 0.0
    for j, v in form.c.items():
        s += v * x[j]
    for k, v in form.d.items():
        s += v * val(k)
    return s


def cell_field_generic(builder, x, val, ic, p):
    g = builder.geo
    b = builder.bphase[p]
    out = np.zeros(g.dim)
    for d in range(g.dim):
        grads = []
        for side in (0, 1):
            a, f = builder.face_out(ic, p, d, side)
            if f is None:
                continue
            go = _eval(f, x, val) / b
            grads.append(go if side else -go)
        if grads:
            out[d] = -sum(grads) / len(grads)
        else:
            a, f = builder.eb_flux(ic, p)
            if f is not None:
                cc = g.ph[p].cut[tuple(reversed(ic))]
                out[d] = -(_eval(f, x, val) / b) * cc.eb_normal[d]
    return out


def efield(system, x, sigma=None, bc_value=None, obj_value=None, generic_only=False):
    """Cell-centred E, array of shape (dim,) + cell shape."""
    B = system.builder
    g = B.geo
    pr = B.prob
    h = g.h
    dim = g.dim
    val = B.data_values(sigma, bc_value, obj_value)
    phi = x[:g.N].reshape(g.shape)
    E = np.zeros((dim,) + g.shape)
    reg = np.zeros(g.shape, bool) if generic_only else _regular_mask(B)
    if reg.any():
        prim = g.primary
        bc = np.where(prim == 1, B.bphase[-1], B.bphase[0]).astype(np.float64)
        for d in range(dim):
            ax = dim - 1 - d
            gsum = np.zeros(g.shape)
            for side in (0, 1):
                gd = np.zeros(g.shape)
                sl_me = [slice(None)] * dim
                sl_nb = [slice(None)] * dim
                if side:
                    sl_me[ax] = slice(0, -1)
                    sl_nb[ax] = slice(1, None)
                else:
                    sl_me[ax] = slice(1, None)
                    sl_nb[ax] = slice(0, -1)
                go = (phi[tuple(sl_nb)] - phi[tuple(sl_me)]) / h
                gd[tuple(sl_me)] = go if side else -go
                edge = [slice(None)] * dim
                edge[ax] = slice(-1, None) if side else slice(0, 1)
                edge = tuple(edge)
                fid = 2 * d + side
                kind = pr.bc_kind[fid]
                v = val(("face", fid))
                pe = phi[edge]
                if kind == W.BC_NEUMANN:
                    ge = np.full(pe.shape, v)
                elif kind == W.BC_DIRICHLET:
                    ge = 2.0 * (v - pe) / h
                else:
                    a1 = pr.robin_a1[fid]
                    a2 = pr.robin_a2[fid]
                    pb = (pe + 0.5 * h * v / a2) / (1.0 + 0.5 * h * a1 / a2)
                    ge = (v - a1 * pb) / a2
                gd[edge] = ge if side else -ge
                gsum += gd
            E[d] = np.where(reg, -0.5 * gsum, 0.0)
    for idx in zip(*np.nonzero((~reg) & (g.primary >= 0))):
        idx = tuple(int(q) for q in idx)
        p = int(g.primary[idx])
        e = cell_field_generic(B, x, val, _cell_ix(g, idx), p)
        for d in range(dim):
            E[(d,) + idx] = e[d]
    return E
