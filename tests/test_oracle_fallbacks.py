"""Pins of the oracle's fallback boundary stencils against exact linear fields.

Each stencil below is a consistent one-sided derivative or a linear
extrapolation, so it reproduces a linear field exactly (rounding only). A
dropped term, a wrong sign, a wrong distance or a transposed weight fails:

  * the least-squares EB derivative (Helmholtz equations / Boundary
    conditions, "quadrant-based least squares" fallback of the EB Dirichlet
    stencil): for linear p it returns grad(p).m exactly, with or without the
    known Dirichlet wall values it takes in, and with the ray stencil switched
    off every cut row of a linear field has zero flux divergence (the face
    fluxes, the facet flux and the closure of the cut-cell moments together);
  * the wall derivative (last resort against a Dirichlet box face): exact for
    a field linear along that face's normal, and it picks the face that m
    faces most;
  * the first-order ray stencil of figure `raycast` (one plane, linear
    interpolation): exact for linear p;
  * the Taylor Robin closure phi_b = (3 phi_n - phi_nn)/2: exact for linear phi;
  * the cell-centred E of a cell with no open face along an axis uses the EB
    normal gradient: exact for a linear field normal to a planar electrode.
"""
import numpy as np
import pytest

import workloads as W
from oracle.efield import cell_field_generic, efield
from oracle.operator import Builder, Options, ROBIN_TAYLOR, assemble
from oracle.geometry import GeometryError


def _dof_centre(g, j):
    c = j if j < g.N else int(g.sec_cells[j - g.N])
    return g.centre(np.unravel_index(c, g.shape))


def _sphere_problem(dim, n, centre, r, bc_kinds):
    h = 1.0 / n
    lo = (0.0,) * dim
    Xn = W._nodes(dim, (n,) * dim, h, lo)
    obj = W.Obj(W.OBJ_ELECTRODE, 0.0, np.ascontiguousarray(W.sdf_sphere(Xn, centre, r)))
    return W.Problem(dim, (n,) * dim, h, lo, [obj], list(bc_kinds), [0.0] * 6, [0.0] * 6, [1.0] * 6, b_gas=1.3)


def _eval(B, wB, form, P, xb, face_val):
    s = wB * P(xb)
    for j, v in form.c.items():
        s += v * P(_dof_centre(B.geo, j))
    for k, v in form.d.items():
        s += v * face_val(k)
    return s


def _electrode_cells(B, p=0):
    for idx, cc in B.geo.ph[p].cut.items():
        if cc.eb_area > 0 and B.prob.objects[cc.cutter].kind == W.OBJ_ELECTRODE:
            yield tuple(reversed(idx)), cc


ALL_NEUMANN = [W.BC_NEUMANN] * 6


@pytest.mark.parametrize("dim,n,centre,r", [(2, 40, (0.47, 0.53), 0.27), (3, 14, (0.48, 0.52, 0.49), 0.31)])
def test_lsq_derivative_exact_for_linear(dim, n, centre, r):
    """No Dirichlet face: the fit uses unknowns only; g.m for random linear p."""
    B = Builder(_sphere_problem(dim, n, centre, r, ALL_NEUMANN))
    rng = np.random.default_rng(7 + dim)
    gv, c0 = rng.normal(size=dim), rng.normal()
    P = lambda x: c0 + gv @ np.asarray(x)
    count = 0
    for ic, cc in _electrode_cells(B):
        m = -cc.eb_normal
        wB, form = B._lsq(ic, 0, cc.eb_cent, m)
        assert wB < 0.0
        got = _eval(B, wB, form, P, cc.eb_cent, lambda k: pytest.fail(f"unexpected datum {k}"))
        assert abs(got - gv @ m) <= 1e-11 * np.linalg.norm(gv), (ic, got, gv @ m)
        count += 1
    assert count > (60 if dim == 2 else 150)


@pytest.mark.parametrize("dim,n,centre,r", [(2, 32, (0.3, 0.5), 0.245), (2, 32, (0.7, 0.45), 0.245),
                                            (3, 16, (0.28, 0.5, 0.5), 0.22), (3, 16, (0.72, 0.5, 0.47), 0.22)])
def test_lsq_derivative_with_wall_values_exact(dim, n, centre, r):
    """Dirichlet x faces (known values at their centres enter the fit) and
    Neumann elsewhere; p linear in x is constant on both Dirichlet faces."""
    kinds = [W.BC_DIRICHLET, W.BC_DIRICHLET] + [W.BC_NEUMANN] * 4
    B = Builder(_sphere_problem(dim, n, centre, r, kinds))
    c0, gx = 0.37, -1.9
    P = lambda x: c0 + gx * x[0]
    walls = {("face", 0): P([0.0]), ("face", 1): P([1.0])}
    count = with_wall = 0
    for ic, cc in _electrode_cells(B):
        m = -cc.eb_normal
        wB, form = B._lsq(ic, 0, cc.eb_cent, m)
        got = _eval(B, wB, form, P, cc.eb_cent, lambda k: walls[k])
        assert abs(got - gx * m[0]) <= 1e-11 * abs(gx), (ic, got, gx * m[0])
        count += 1
        with_wall += any(k in walls for k in form.d)
    assert count > 30 and with_wall >= 3


@pytest.mark.parametrize("dim,n,centre,r", [(2, 36, (0.3, 0.52), 0.245), (2, 36, (0.7, 0.5), 0.245),
                                            (3, 14, (0.3, 0.5, 0.48), 0.23)])
def test_cut_rows_linear_exact_without_ray(dim, n, centre, r, monkeypatch):
    """With the ray stencil switched off every EB row uses the least-squares
    (or wall) derivative; for a field linear in x (constant on the Dirichlet x
    faces) the flux divergence of every cut row is zero, including rows
    against the Dirichlet face that take its value."""
    monkeypatch.setattr(Builder, "_ray", lambda self, *a: None)
    kinds = [W.BC_DIRICHLET, W.BC_DIRICHLET] + [W.BC_NEUMANN] * 4
    pr = _sphere_problem(dim, n, centre, r, kinds)
    B = Builder(pr)
    c0, gx = -0.6, 2.3
    P = lambda x: c0 + gx * x[0]
    g = B.geo
    walls = {("face", 0): P([0.0]), ("face", 1): P([1.0])}
    worst = 0.0
    count = 0
    for ic, cc in _electrode_cells(B):
        _, f = B.row(ic, 0)
        data = lambda k: P(cc.eb_cent) if k[0] == "obj" else walls.get(k, 0.0)
        s = sum(v * P(_dof_centre(g, j)) for j, v in f.c.items()) + sum(v * data(k) for k, v in f.d.items())
        worst = max(worst, abs(s / pr.beta) / (B.bphase[0] * abs(gx) / g.h))
        count += 1
    assert count > 30
    assert worst < 1e-12


@pytest.mark.parametrize("sx,sy", [(1, 1), (0, 0), (1, 0), (0, 1)])
def test_wall_derivative_exact_and_face_choice(sx, sy):
    """A corner cell against two Dirichlet faces (x side sx, y side sy): the
    derivative toward the face that m faces most is exact for a field linear
    along that face's normal; the other face's datum must not enter."""
    n = 10
    pr = _sphere_problem(2, n, (0.5, 0.5), 0.1, [W.BC_DIRICHLET] * 4)
    B = Builder(pr)
    h = pr.h
    ic = ((n - 1) if sx else 0, (n - 1) if sy else 0)
    wall = (1.0 if sx else 0.0, 1.0 if sy else 0.0)
    out = np.array([1.0 if sx else -1.0, 1.0 if sy else -1.0])   # outward normals of the two faces
    rng = np.random.default_rng(5 + 2 * sx + sy)
    for _ in range(50):
        off = rng.uniform(0.05, 0.95, size=2) * h
        xb = np.array([wall[0] - out[0] * off[0], wall[1] - out[1] * off[1]])
        a = rng.uniform(0.05, 1.5) * 0.5
        m = np.array([np.cos(a), np.sin(a)])                # faces the x face more than the y face
        if rng.random() < 0.5:
            m = m[::-1].copy()
        axis = 0 if m[0] > m[1] else 1
        m = m * out
        q, c0 = rng.normal(), rng.normal()
        P = lambda x: c0 + q * x[axis]
        fx, fy = ("face", 0 + sx), ("face", 2 + sy)
        vals = {fx: P(wall) if axis == 0 else 1e3, fy: P(wall) if axis == 1 else 1e3}
        wB, form = B._wall(ic, 0, xb, m)
        got = wB * P(xb) + sum(v * vals[k] for k, v in form.d.items())
        assert not form.c
        assert abs(got - q * m[axis]) <= 1e-11 * abs(q), (xb, m, got, q * m[axis])


def test_wall_derivative_needs_a_dirichlet_face():
    pr = _sphere_problem(2, 10, (0.2, 0.2), 0.1, [W.BC_NEUMANN] * 4)
    B = Builder(pr)
    with pytest.raises(GeometryError):
        B._wall((9, 9), 0, np.array([0.97, 0.97]), np.array([0.6, 0.8]))


@pytest.mark.parametrize("dim,n,centre,r", [(2, 48, (0.51, 0.47), 0.23), (3, 16, (0.5, 0.49, 0.52), 0.27)])
def test_first_order_ray_exact_for_linear(dim, n, centre, r):
    B = Builder(_sphere_problem(dim, n, centre, r, [W.BC_DIRICHLET] * 6), Options(eb_order=1))
    rng = np.random.default_rng(17 + dim)
    gv, c0 = rng.normal(size=dim), rng.normal()
    P = lambda x: c0 + gv @ np.asarray(x)
    count = 0
    for ic, cc in _electrode_cells(B):
        m = -cc.eb_normal
        res = B._ray(ic, 0, cc.eb_cent, m, 1)
        if res is None:
            continue
        wB, form = res
        got = _eval(B, wB, form, P, cc.eb_cent, lambda k: pytest.fail(f"unexpected datum {k}"))
        assert abs(got - gv @ m) <= 1e-11 * np.linalg.norm(gv), (ic, got, gv @ m)
        count += 1
    assert count > (60 if dim == 2 else 150)


def test_first_order_rows_linear_exact():
    """Assembled with eb_order = 1: the rows of a linear field have zero flux
    divergence wherever the ray stencil applies."""
    pr = _sphere_problem(2, 48, (0.51, 0.47), 0.23, [W.BC_NEUMANN] * 4)
    B = Builder(pr, Options(eb_order=1))
    rng = np.random.default_rng(29)
    gv, c0 = rng.normal(size=2), rng.normal()
    P = lambda x: c0 + gv @ np.asarray(x)
    count = 0
    for ic, cc in _electrode_cells(B):
        _, f = B.row(ic, 0)
        s = sum(v * P(_dof_centre(B.geo, j)) for j, v in f.c.items()) + \
            sum(v * P(cc.eb_cent) for k, v in f.d.items() if k[0] == "obj")
        assert abs(s) <= 1e-12 * B.bphase[0] * np.linalg.norm(gv) / pr.h ** 2
        count += 1
    assert count > 60


@pytest.mark.parametrize("dim", [2, 3])
def test_robin_taylor_closure_exact_for_linear(dim):
    """a1 phi + a2 dphi/dn = a3 on every face with the Taylor closure: linear
    phi (any direction) with the matching a3 per face gives zero residual in
    every row, corners included."""
    n = 10 if dim == 2 else 6
    h = 1.0 / n
    rng = np.random.default_rng(41 + dim)
    gv, c0 = rng.normal(size=dim), rng.normal()
    a1, a2 = 1.7, 0.6
    # a3 is one value per face, so the field is linear along one axis at a
    # time: Robin on that axis's faces, Neumann 0 on the others
    for axis in range(dim):
        q = gv[axis]
        vals = []
        for d in range(3):
            for side in (0, 1):
                if d >= dim:
                    vals.append(0.0)
                    continue
                xf = 1.0 if side else 0.0
                nrm = (1.0 if side else -1.0) if d == axis else 0.0
                if d == axis:
                    vals.append(a1 * (c0 + q * xf) + a2 * q * nrm)
                else:
                    vals.append(None)
        kinds = [W.BC_ROBIN if v is not None else W.BC_NEUMANN for v in vals]
        vals = [0.0 if v is None else v for v in vals]
        pr = W.Problem(dim, (n,) * dim, h, (0.0,) * dim, [], kinds, vals, [a1] * 6, [a2] * 6,
                       alpha=1.0, a_gas=2.0)
        X = pr.cell_centres()
        phi = c0 + q * np.broadcast_to(X[axis], pr.shape)
        pr.rho = 2.0 * phi
        S = assemble(pr, Options(robin_closure=ROBIN_TAYLOR))
        r = S.b - S.A @ phi.ravel()
        assert np.abs(r).max() < 1e-11 * (abs(q) / h ** 2 + 1), (axis, np.abs(r).max())
        # the linear closure is exact too; the Taylor form must differ from it
        # in its coefficients (it reaches the second cell)
        S0 = assemble(pr)
        assert abs(S0.A - S.A).max() > 0.1


@pytest.mark.parametrize("dim", [2, 3])
def test_efield_eb_branch_exact_for_linear(dim):
    """Planar electrode, phi linear along its normal (constant on it): the EB
    normal-gradient branch of the cell field gives -grad(phi) exactly. The
    branch is forced on every cut cell by closing its faces along one axis;
    the unforced field is -grad(phi) in every cell as well."""
    n = 24 if dim == 2 else 10
    h = 1.0 / n
    lo = (0.0,) * dim
    rng = np.random.default_rng(3 + dim)
    nv = rng.normal(size=dim)
    nv /= np.linalg.norm(nv)
    p0 = np.full(dim, 0.5) + 0.03 * rng.normal(size=dim)
    q, c0 = 1.7, -0.4
    P = lambda x: c0 + q * float(nv @ (np.asarray(x) - p0))
    Xn = W._nodes(dim, (n,) * dim, h, lo)
    obj = W.Obj(W.OBJ_ELECTRODE, c0, np.ascontiguousarray(W.sdf_plane(Xn, p0, nv)))
    # Neumann data = outward normal derivative of the linear field per face
    vals = []
    for d in range(3):
        for side in (0, 1):
            vals.append(0.0 if d >= dim else (q * nv[d] if side else -q * nv[d]))
    pr = W.Problem(dim, (n,) * dim, h, lo, [obj], [W.BC_NEUMANN] * 6, vals, [0.0] * 6, [1.0] * 6, b_gas=2.0,
                   rho=np.zeros(tuple(reversed((n,) * dim))))
    S = assemble(pr)
    g = S.geo
    x = np.zeros(g.N + g.N2)
    for j in range(g.N):
        idx = np.unravel_index(j, g.shape)
        if g.primary[idx] >= 0:
            x[j] = P(g.centre(idx))
    E = efield(S, x)
    want = -q * nv
    live = g.primary >= 0
    for d in range(dim):
        assert np.abs(E[d][live] - want[d]).max() <= 1e-11 * abs(q)
    B = S.builder
    val = B.data_values()
    orig = B.face_out
    count = 0
    for axis in range(dim):
        B.face_out = lambda ic, p, d, side, _a=axis: (0.0, None) if d == _a else orig(ic, p, d, side)
        for idx, cc in g.ph[0].cut.items():
            if cc.eb_area <= 0:
                continue
            e = cell_field_generic(B, x, val, tuple(reversed(idx)), 0)
            assert abs(e[axis] - want[axis]) <= 1e-11 * abs(q), (idx, axis, e, want)
            count += 1
    B.face_out = orig
    assert count > 20
