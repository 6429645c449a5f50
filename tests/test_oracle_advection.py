"""Pins of the oracle's advection step (Convection-Diffusion-Reaction
equations: unsplit Godunov with van Leer limiting, hybrid divergence and
redistribution on cut cells)."""
import math

import numpy as np

import workloads as W
from oracle.advection import Advection, mc_slope


def _box(dim, n, objs=(), bc=W.BC_DIRICHLET):
    h = 1.0 / n
    return W.Problem(dim, (n,) * dim, h, (0.0,) * dim, list(objs), *W._bc(bc))


def test_limiter_closed_form():
    dl = np.array([1.0, 1.0, 3.0, 1.0, -2.0, 2.0, 0.0])
    dr = np.array([1.0, 3.0, 1.0, -1.0, -0.5, 2.0, 1.0])
    want = np.array([1.0, 2.0, 2.0, 0.0, -1.0, 2.0, 0.0])
    assert np.array_equal(mc_slope(dl, dr), want)


def test_free_stream_is_preserved():
    pr = _box(2, 24)
    A = Advection(pr)
    u = W.velocity_uniform(2, pr.n, pr.h, pr.lo, (0.7, -0.4))
    n0 = np.full(pr.shape, 2.5)
    n1 = A.step(n0, u, 0.5 * pr.h / 0.7, inflow=(2.5,) * 6)
    assert np.abs(n1 - 2.5).max() <= 1e-14


def test_linear_data_translates_exactly():
    """Linear density, uniform velocity: regular cells away from the inflow
    faces hold the density translated by v dt (the predictor is exact for
    linear data, transverse terms included)."""
    for dim, n in ((2, 20), (3, 10)):
        pr = _box(dim, n)
        A = Advection(pr)
        v = (0.6, -0.3, 0.45)[:dim]
        g = (1.3, -0.7, 0.4)[:dim]
        X = [np.broadcast_to(x, pr.shape) for x in pr.cell_centres()]
        n0 = 2.0 + sum(g[d] * X[d] for d in range(dim))
        dt = 0.4 * pr.h
        u = W.velocity_uniform(dim, pr.n, pr.h, pr.lo, v)
        n1 = A.step(n0, u, dt)
        want = 2.0 + sum(g[d] * (X[d] - v[d] * dt) for d in range(dim))
        inner = tuple(slice(2, -2) for _ in range(dim))
        assert np.abs(n1[inner] - want[inner]).max() <= 1e-13


def test_mass_balance_with_embedded_boundaries():
    """With a sphere electrode and a dielectric plane cutting the box, the
    gas mass sum kappa n h^D changes by exactly the net domain-boundary
    flux over the step: interior faces telescope, the EB carries no flux,
    and the hybrid's defect is redistributed."""
    for dim, n in ((2, 40), (3, 16)):
        h = 1.0 / n
        Xn = W._nodes(dim, (n,) * dim, h, (0.0,) * dim)
        objs = [W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_sphere(Xn, (0.45, 0.55, 0.5)[:dim], 0.21))),
                W.Obj(W.OBJ_DIELECTRIC, 4.0, np.ascontiguousarray(W.sdf_halfspace_below(Xn[1], 0.17)))]
        pr = W.Problem(dim, (n,) * dim, h, (0.0,) * dim, objs, *W._bc(W.BC_DIRICHLET))
        A = Advection(pr)
        assert ((A.kappa > 0) & (A.kappa < 1)).sum() > 20
        rng = np.random.default_rng(dim)
        n0 = np.where(A.gas, rng.uniform(0.5, 1.5, size=pr.shape), 0.0)
        u = W.velocity_rotation(dim, pr.n, h, pr.lo, 1.5, (0.5, 0.5))
        if dim == 3:
            u[2] = np.full(u[2].shape, -0.3)
        dt = 0.5 * h / max(float(np.abs(x).max()) for x in u)
        inflow = tuple(rng.uniform(0.5, 1.5, size=6))
        n1 = A.step(n0, u, dt, inflow)
        m0 = (A.kappa * n0).sum() * h ** dim
        m1 = (A.kappa * n1).sum() * h ** dim
        out = A.boundary_outflux(n0, u, dt, inflow)
        assert abs((m1 - m0) + dt * out) <= 1e-13 * max(abs(m0), 1.0), (m1 - m0, -dt * out)
        # the hybrid differs from the conservative divergence in cut cells
        D, Dc = A.divergence(n0, u, dt, inflow)
        assert np.abs(D - Dc).max() > 1e-6


def test_smooth_pulse_converges_at_second_order():
    """A Gaussian pulse carried a fixed distance by a uniform diagonal
    velocity (CFL 0.5): the L1 error against the translated pulse falls by
    about 4 per halving of h (second order where the limiter is inactive)."""
    errs = []
    v = (1.0, 0.5)
    T = 0.25
    for n in (32, 64, 128):
        pr = _box(2, n)
        A = Advection(pr)
        nt = int(round(T / (0.5 * pr.h / 1.0)))
        dt = T / nt
        u = W.velocity_uniform(2, pr.n, pr.h, pr.lo, v)
        c0 = (0.35, 0.4)
        x = W.gaussian_density(pr, c0, 0.08)
        for _ in range(nt):
            x = A.step(x, u, dt)
        ex = W.gaussian_density(pr, (c0[0] + v[0] * T, c0[1] + v[1] * T), 0.08)
        errs.append(np.abs(x - ex).mean())
    p = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(p) >= 1.7, (errs, p)
