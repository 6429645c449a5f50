"""Pins of the oracle's operator A and right-hand side b.

Each test checks the oracle against something fixed by the mathematics or by
the paper, not against itself:
  * closed-form discrete solution of the manufactured sine problem;
  * polynomial exactness of regular rows (per-variable degree <= 3) and of
    the domain closures (quadratic Dirichlet: degree <= 2; linear closures and
    linear Robin: degree <= 1);
  * exactness for quadratics of 2D cut rows with second-order ray stencils
    and of 3D rows cut by a plane (linearised geometry, centroid interpolation
    and the 3-point normal derivative are each exact for quadratics);
  * a planar dielectric interface with piecewise-linear phi satisfying the
    matching condition gives zero residual in every row;
  * the paper's coaxial multifluid problem converges at second order in the
    volume-weighted L2 norm, and the surface-charge variant converges to its
    closed form (which fixes the sign of sigma);
  * telescoping flux balance, symmetry/definiteness of the regular operator.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import exact
from oracle.operator import assemble, Builder, Options, DIRICHLET_QUADRATIC, _regular_mask
from oracle.solvers import solve_splu, rel_residual


def _row_value(B, f, phi_of_dof, data_of_key):
    s = 0.0
    for j, v in f.c.items():
        s += v * phi_of_dof(j)
    for k, v in f.d.items():
        s += v * data_of_key(k)
    return s


def _dof_centre(g, j):
    c = j if j < g.N else int(g.sec_cells[j - g.N])
    return g.centre(np.unravel_index(c, g.shape))


def test_sine_closed_form():
    """Discrete solution equals (2 pi^2/lambda_h) sin sin; printed factor at n=64."""
    for n in (16, 32, 64):
        S = assemble(W.manufactured_sine(n))
        x = solve_splu(S.A, S.b)
        ex = exact.sine_discrete(n)
        assert np.abs(x.reshape(n, n) - ex).max() <= 1e-12 * np.abs(ex).max()
    h = 1 / 64
    assert abs((2 * math.pi ** 2) / ((8 / h ** 2) * math.sin(math.pi * h / 2) ** 2) - 1.0002008218097047) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_regular_rows_cubic_exact(dim):
    n = 12 if dim == 2 else 6
    h = 1.0 / n
    pr = W.Problem(dim, (n,) * dim, h, (0.0,) * dim, [], *W._bc(W.BC_DIRICHLET), b_gas=2.5)
    S = assemble(pr)
    rng = np.random.default_rng(3)
    c = rng.normal(size=(dim, 4))
    X = [np.broadcast_to(a, pr.shape) for a in pr.cell_centres()]
    phi = sum(c[d, 0] + c[d, 1] * X[d] + c[d, 2] * X[d] ** 2 + c[d, 3] * X[d] ** 3 for d in range(dim))
    lap = sum(2 * c[d, 2] + 6 * c[d, 3] * X[d] for d in range(dim))
    Ax = (S.A @ phi.ravel()).reshape(pr.shape)
    inner = tuple(slice(1, -1) for _ in range(dim))
    # beta = -1: A phi = -b lap phi in interior rows
    assert np.abs(Ax[inner] + 2.5 * lap[inner]).max() < 1e-9 * np.abs(lap).max() * n * n


@pytest.mark.parametrize("closure,deg", [(0, 1), (1, 2)])
def test_dirichlet_closure_exactness(closure, deg):
    """phi = q(x) (degree deg), Dirichlet data q(0), q(1) on x faces, Neumann 0
    on y faces: every row has zero residual for the closure's degree."""
    n = 10
    h = 1.0 / n
    q = [0.3, -1.1, 0.7][:deg + 1]
    kind = [W.BC_DIRICHLET, W.BC_DIRICHLET, W.BC_NEUMANN, W.BC_NEUMANN, 0, 0]
    val = [q[0], sum(q), 0.0, 0.0, 0.0, 0.0]
    rho_c = -2.0 * q[2] * 1.0 if deg == 2 else 0.0   # -div(grad q) with beta=-1, b=1 -> rho = -q''
    pr = W.Problem(2, (n, n), h, (0.0, 0.0), [], kind, val, [0.0] * 6, [1.0] * 6,
                   rho=np.full((n, n), -2.0 * q[2] if deg == 2 else 0.0))
    del rho_c
    S = assemble(pr, Options(dirichlet_closure=closure))
    x, _ = pr.cell_centres()
    phi = sum(q[k] * np.broadcast_to(x, pr.shape) ** k for k in range(deg + 1))
    assert rel_residual(S.A, S.b, phi.ravel()) < 1e-12 or np.abs(S.b - S.A @ phi.ravel()).max() < 1e-10


def test_robin_linear_closure_exact_for_linear():
    n = 10
    h = 1.0 / n
    c0, c1 = 0.4, -0.9
    a1, a2 = 2.0, 0.5
    # x- face: outward normal -x: a1 phi + a2 (-c1) = a3; x+ face: a1 phi + a2 c1 = a3
    a3lo = a1 * c0 - a2 * c1
    a3hi = a1 * (c0 + c1) + a2 * c1
    kind = [W.BC_ROBIN, W.BC_ROBIN, W.BC_NEUMANN, W.BC_NEUMANN, 0, 0]
    pr = W.Problem(2, (n, n), h, (0.0, 0.0), [], kind, [a3lo, a3hi, 0, 0, 0, 0], [a1] * 6, [a2] * 6,
                   alpha=1.0, a_gas=3.0, rho=None)
    x, _ = pr.cell_centres()
    phi = c0 + c1 * np.broadcast_to(x, pr.shape)
    pr.rho = 3.0 * phi  # alpha a phi + beta div(b grad phi) with linear phi
    S = assemble(pr)
    assert np.abs(S.b - S.A @ phi.ravel()).max() < 1e-11


def _quad_exact_rows(dim, n, objs_fn, seed):
    h = 1.0 / n
    lo = (0.0,) * dim
    Xn = W._nodes(dim, (n,) * dim, h, lo)
    pr = W.Problem(dim, (n,) * dim, h, lo, objs_fn(Xn), *W._bc(W.BC_DIRICHLET), b_gas=1.7)
    B = Builder(pr)
    g = B.geo
    used = set()
    orig = B._lsq

    def lsq(ic, p, xb, m):
        used.add((tuple(ic), p))
        return orig(ic, p, xb, m)
    B._lsq = lsq
    rng = np.random.default_rng(seed)
    H = rng.normal(size=(dim, dim))
    H = H + H.T
    gv = rng.normal(size=dim)
    c0 = rng.normal()

    def P(x):
        x = np.asarray(x)
        return c0 + gv @ x + 0.5 * x @ H @ x
    lap = float(np.trace(H))
    worst = 0.0
    count = 0
    for p in range(g.nphase):
        for idx, cc in g.ph[p].cut.items():
            ic = tuple(reversed(idx))
            if any(q < 2 or q >= n - 2 for q in ic):
                continue
            used.clear()
            _, f = B.row(ic, p)
            if used:
                continue
            val = _row_value(B, f, lambda j: P(_dof_centre(g, j)), lambda k: P(cc.eb_cent))
            div = val / pr.beta
            want = cc.kappa * B.bphase[p] * lap
            scale = B.bphase[p] * abs(lap) + 1.0
            worst = max(worst, abs(div - want) / scale)
            count += 1
    return worst, count


def test_cut_rows_quadratic_exact_2d():
    worst, count = _quad_exact_rows(
        2, 64, lambda X: [W.Obj(W.OBJ_ELECTRODE, 0.0, np.ascontiguousarray(W.sdf_sphere(X, (0.52, 0.47), 0.23)))], 11)
    assert count > 80
    assert worst < 1e-11


def test_cut_rows_quadratic_exact_3d_plane():
    nv = np.array([0.3, -0.5, 0.8])
    nv /= np.linalg.norm(nv)
    worst, count = _quad_exact_rows(
        3, 16, lambda X: [W.Obj(W.OBJ_ELECTRODE, 0.0, np.ascontiguousarray(W.sdf_plane(X, (0.51, 0.47, 0.53), nv)))], 12)
    assert count > 100
    assert worst < 1e-11


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 12)])
def test_planar_multifluid_exact(dim, n):
    """Piecewise-linear phi, continuous, with eps_g q_g - eps_s q_s = -sigma:
    every row whose stencils stay clear of the box faces has zero residual
    (sigma constant)."""
    rng = np.random.default_rng(20 + dim)
    nv = rng.normal(size=dim)
    nv /= np.linalg.norm(nv)
    p0 = rng.uniform(0.4, 0.6, size=dim)
    eg, es, sigma = 1.5, 4.0, 0.37
    h = 1.0 / n
    Xn = W._nodes(dim, (n,) * dim, h, (0.0,) * dim)
    pr = W.Problem(dim, (n,) * dim, h, (0.0,) * dim,
                   [W.Obj(W.OBJ_DIELECTRIC, es, np.ascontiguousarray(W.sdf_plane(Xn, p0, nv)))],
                   *W._bc(W.BC_DIRICHLET), b_gas=eg)
    pr.sigma = np.full(pr.shape, sigma)
    t = rng.normal(size=dim)
    t -= (t @ nv) * nv
    qs = 0.8
    qg = (es * qs - sigma) / eg
    gg = t + qg * nv
    gs = t + qs * nv
    c = 0.3
    cs = c + (qg - qs) * float(nv @ p0)
    S = assemble(pr, rho=np.zeros(pr.shape))
    g = S.geo
    x = np.zeros(g.N + g.N2)
    for j in range(g.N + g.N2):
        cell = j if j < g.N else int(g.sec_cells[j - g.N])
        idx = np.unravel_index(cell, g.shape)
        ph = 1 if j >= g.N else int(g.primary[idx])
        if ph < 0:
            continue
        xc = g.centre(idx)
        x[j] = (c + gg @ xc) if ph == 0 else (cs + gs @ xc)
    r = S.b - S.A @ x
    # rows whose stencils cannot reach the box faces (least-squares stencils
    # may use Dirichlet face values up to three cells away)
    mask = np.zeros(g.N + g.N2, bool)
    for j in range(g.N + g.N2):
        cell = j if j < g.N else int(g.sec_cells[j - g.N])
        ic = np.unravel_index(cell, g.shape)
        mask[j] = all(4 <= q < n - 4 for q in ic)
    scale = max(eg, es) / h / h
    assert np.abs(r[mask]).max() < 1e-10 * scale
    assert g.N2 > 0


def _coax_errors(ns, sigma=0.0):
    out = []
    for n in ns:
        pr = W.coaxial(n, sigma=sigma)
        S = assemble(pr)
        x = solve_splu(S.A, S.b)
        g = S.geo
        phi = x[:g.N].reshape(g.shape)
        X, Y = pr.cell_centres()
        r = np.sqrt(X ** 2 + Y ** 2) * np.ones(g.shape)
        prim = g.primary
        k = np.where(prim == 0, g.ph[0].kappa, np.where(prim == 1, g.ph[1].kappa, 0.0))
        eg = exact.coaxial(r, sigma=sigma, branch="gas")
        ed = exact.coaxial(r, sigma=sigma, branch="diel")
        e = np.where(prim == 0, phi - eg, np.where(prim == 1, phi - ed, 0.0))
        out.append(math.sqrt((k * e * e).sum() / k.sum()))
    return out


def test_coaxial_second_order():
    """The paper's multifluid coaxial problem: L2 (volume-weighted) error falls
    at second order from 64^2 to 256^2."""
    e = _coax_errors((64, 128, 256))
    slopes = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(slopes) > 1.8, (e, slopes)
    assert e[-1] < 1e-4
    A, B = exact.coaxial_coefficients()
    assert abs(A - (-1.727856088917657)) < 1e-14


def test_coaxial_surface_charge_closed_form():
    """Uniform sigma = 0.5 on the dielectric surface: converges to the closed
    form of the thin-charged-layer limit (phi(R1) = 0.73700601...); the
    opposite sign of sigma would leave an O(0.07) error."""
    e = _coax_errors((64, 128), sigma=0.5)
    assert e[1] < e[0] / 3 and e[1] < 5e-4
    assert abs(exact.coaxial(np.array(0.6), sigma=0.5) - 0.7370060132015176) < 1e-13


def test_flux_balance_two_disks():
    """Interior fluxes telescope: boundary + electrode fluxes balance the
    source and the interface surface charge, up to the residual."""
    pr = W.two_disks(64, seed=1)
    S = assemble(pr)
    x = solve_splu(S.A, S.b)
    B = S.builder
    g = S.geo
    val = B.data_values()
    h = g.h
    tot = 0.0
    sig_tot = 0.0
    for idx in zip(*np.nonzero(g.primary >= 0)):
        ic = tuple(reversed([int(q) for q in idx]))
        for p in range(g.nphase):
            if not g.has[p][idx]:
                continue
            for d in range(2):
                for side in (0, 1):
                    nb = list(ic)
                    nb[d] += 1 if side else -1
                    if 0 <= nb[d] < g.n[d]:
                        continue
                    a, f = B.face_out(ic, p, d, side)
                    if f is not None:
                        tot += a * _row_value(B, f, lambda j: x[j], val) * h
            cc = g.ph[p].cut.get(idx)
            if cc is not None and pr.objects[cc.cutter].kind == W.OBJ_ELECTRODE:
                a, f = B.eb_flux(ic, p)
                tot += a * _row_value(B, f, lambda j: x[j], val) * h
            if cc is not None and pr.objects[cc.cutter].kind == W.OBJ_DIELECTRIC and p == 0:
                sig_tot += cc.eb_area * pr.sigma[idx] * h
    kr = (g.ph[0].kappa * np.where(g.primary == 0, pr.rho, 0.0)).sum() + \
         (g.ph[1].kappa * np.where(g.primary == 1, pr.rho, 0.0)).sum()
    rhs = -h * h * kr - sig_tot
    r = S.b - S.A @ x
    assert abs(tot - rhs) <= 1e-9 * (abs(rhs) + 1) + h * h * np.abs(r).sum()
    assert abs(sig_tot) > 0


def test_regular_operator_symmetric_positive_definite():
    pr = W.Problem(2, (12, 12), 1 / 12, (0.0, 0.0), [], [0, 0, 1, 1, 0, 0], [0.5] * 6, [0.0] * 6, [1.0] * 6)
    S = assemble(pr)
    A = S.A.toarray()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    pr2 = W.eddington(2, 10, 7.0)
    A2 = assemble(pr2).A.toarray()
    assert np.array_equal(A2, A2.T)
    assert np.linalg.eigvalsh(A2).min() > 0


@pytest.mark.parametrize("make", [lambda: W.two_disks(48, seed=2), lambda: W.pin_plane(16, seed=1),
                                  lambda: W.coaxial(40)])
def test_vectorised_rows_equal_generic(make):
    pr = make()
    S1 = assemble(pr)
    S2 = assemble(pr, generic_only=True)
    assert abs(S1.A - S2.A).max() < 1e-9 * abs(S1.A).max()
    assert np.abs(S1.b - S2.b).max() <= 1e-12 * (np.abs(S1.b).max() + 1)
    assert _regular_mask(S1.builder).sum() > 0
