"""Pins of the oracle's cut-cell geometry against closed forms.

* a straight cut is reproduced exactly by the linearised boundary: the wet
  area/volume of a box cut by a line/plane equals the closed-form area/volume
  of the half-plane/half-space inside the box;
* disk areas and perimeters converge at O(h^2) to pi r^2 and 2 pi r; sphere
  volume and area likewise;
* per cell, the phase volumes of gas, dielectric and electrode sum to 1 and
  the facet area vector closes the cell (divergence theorem);
* saddle cells and cells cut by two objects are rejected.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import Geometry, GeometryError


def _prob(dim, n, objs_fn, lo=None, h=None):
    h = h or 1.0 / n
    lo = lo or (0.0,) * dim
    Xn = W._nodes(dim, (n,) * dim, h, lo)
    return W.Problem(dim, (n,) * dim, h, lo, objs_fn(Xn), *W._bc(W.BC_DIRICHLET))


def halfspace_measure(normal, c):
    """Measure of {x in [0,1]^D : normal.x < c} (closed form by inclusion-exclusion,
    valid when every normal component is nonzero)."""
    nv = np.array(normal, dtype=float)
    D = len(nv)
    # reflect axes with negative components: x -> 1 - x
    cc = c
    for d in range(D):
        if nv[d] < 0:
            cc -= nv[d]
            nv[d] = -nv[d]
    tot = 0.0
    for v in itertools.product((0, 1), repeat=D):
        s = cc - float(np.dot(nv, v))
        if s > 0:
            tot += (-1) ** sum(v) * s ** D
    return tot / (math.factorial(D) * float(np.prod(nv)))


@pytest.mark.parametrize("dim,n", [(2, 37), (3, 13)])
def test_planar_cut_is_exact(dim, n):
    rng = np.random.default_rng(7 + dim)
    nv = rng.normal(size=dim)
    nv /= np.linalg.norm(nv)
    p = rng.uniform(0.35, 0.65, size=dim)
    pr = _prob(dim, n, lambda X: [W.Obj(W.OBJ_DIELECTRIC, 3.0, np.ascontiguousarray(W.sdf_plane(X, p, nv)))])
    g = Geometry(pr)
    h = pr.h
    vd = g.ph[1].kappa.sum() * h ** dim
    vg = g.ph[0].kappa.sum() * h ** dim
    exact = halfspace_measure(nv, float(np.dot(nv, p)))
    assert abs(vd - exact) < 1e-13
    assert abs(vg - (1 - exact)) < 1e-13
    # every cut cell carries the same facet for both phases, with normal -nv
    # for the dielectric (outward from it) and total facet area = plane section
    for idx, cd in g.ph[1].cut.items():
        assert np.allclose(cd.eb_normal, nv, atol=1e-12)
        cg = g.ph[0].cut[idx]
        assert np.allclose(cg.eb_normal, -nv, atol=1e-12)
        assert abs(cd.kappa + cg.kappa - 1.0) < 1e-14


def test_disk_area_perimeter_second_order():
    errs = []
    for n in (32, 64, 128):
        pr = _prob(2, n, lambda X: [W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_sphere(X, (0.513, 0.487), 0.3)))])
        g = Geometry(pr)
        h = pr.h
        area = g.ph[0].kappa.sum() * h * h
        per = sum(c.eb_area for c in g.ph[0].cut.values()) * h
        errs.append((abs(area - (1 - math.pi * 0.09)), abs(per - 2 * math.pi * 0.3)))
    for k in range(2):
        r1 = math.log2(errs[0][k] / errs[1][k])
        r2 = math.log2(errs[1][k] / errs[2][k])
        assert r1 > 1.8 and r2 > 1.8, (k, errs)


def test_sphere_volume_area_second_order():
    errs = []
    for n in (12, 24):
        pr = _prob(3, n, lambda X: [W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_sphere(X, (0.51, 0.49, 0.5), 0.3)))])
        g = Geometry(pr)
        h = pr.h
        vol = g.ph[0].kappa.sum() * h ** 3
        area = sum(c.eb_area for c in g.ph[0].cut.values()) * h * h
        errs.append((abs(vol - (1 - 4 / 3 * math.pi * 0.027)), abs(area - 4 * math.pi * 0.09)))
    assert math.log2(errs[0][0] / errs[1][0]) > 1.7
    assert math.log2(errs[0][1] / errs[1][1]) > 1.7


def test_two_disks_areas_and_partition():
    """Gas area 1 - 0.05 pi and dielectric area 0.04 pi (the two-disk workload);
    per cell, gas + dielectric + electrode volume fractions sum to 1."""
    out = []
    for n in (64, 128):
        pr = W.two_disks(n, seed=0)
        g = Geometry(pr)
        h = pr.h
        out.append((g.ph[0].kappa.sum() * h * h - (1 - 0.05 * math.pi),
                    g.ph[1].kappa.sum() * h * h - 0.04 * math.pi))
        # electrode phase: s = -d_electrode
        from oracle.geometry import PhaseGeom
        pe = PhaseGeom(g, -pr.objects[0].sdf)
        tot = g.ph[0].kappa + g.ph[1].kappa + pe.kappa
        assert np.abs(tot - 1.0).max() < 1e-13
    assert abs(out[1][0]) < abs(out[0][0]) / 3
    assert abs(out[1][1]) < abs(out[0][1]) / 3


def test_level_set_zero_on_nodes():
    """h = 1/130 puts grid nodes exactly on both circles of the two-disk
    workload (level set exactly 0 there). Such nodes belong to neither side;
    the geometry still partitions every cell (gas + dielectric + electrode
    volume fractions sum to 1), each cut cell has one cutter, and the phase
    areas stay within O(h^2) of the exact ones."""
    pr = W.two_disks(130, seed=1)
    assert any((o.sdf == 0).any() for o in pr.objects)
    g = Geometry(pr)
    from oracle.geometry import PhaseGeom
    pe = PhaseGeom(g, -pr.objects[0].sdf)
    tot = g.ph[0].kappa + g.ph[1].kappa + pe.kappa
    assert np.abs(tot - 1.0).max() < 1e-13
    h = pr.h
    # a chord across a cell cuts off ~h^3/(12 R) of a circle of radius R, about
    # pi h^2 / 6 over its 2 pi R / h cells: bound each circle by h^2
    assert abs(g.ph[0].kappa.sum() * h * h - (1 - 0.05 * math.pi)) < 2.0 * h * h
    assert abs(g.ph[1].kappa.sum() * h * h - 0.04 * math.pi) < 1.0 * h * h
    for pg in g.ph:
        assert all(cc.cutter in (0, 1) for cc in pg.cut.values())


@pytest.mark.parametrize("dim", [2, 3])
def test_closure_per_cell(dim):
    """alpha_EB n_EB + sum_d (alpha_hi - alpha_lo) e_d = 0 per cut cell, and the
    facet centroid lies in the cell."""
    n = 24 if dim == 2 else 10
    pr = _prob(dim, n, lambda X: [W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_sphere(X, (0.5,) * dim, 0.31)))])
    g = Geometry(pr)
    pg = g.ph[0]
    for idx, cc in pg.cut.items():
        vec = cc.eb_area * cc.eb_normal
        for d in range(dim):
            lo_i = list(idx)
            hi_i = list(idx)
            hi_i[dim - 1 - d] += 1
            vec[d] += pg.alpha[d][tuple(hi_i)] - pg.alpha[d][tuple(lo_i)]
        assert np.abs(vec).max() < 1e-14
        c = g.centre(idx)
        assert np.all(np.abs(cc.eb_cent - c) <= 0.5 * pr.h * (1 + 1e-12))
        assert np.all(np.abs(cc.vcent - c) <= 0.5 * pr.h * (1 + 1e-12))


def test_rejections():
    # two objects cutting one cell
    with pytest.raises(GeometryError):
        Geometry(_prob(2, 16, lambda X: [
            W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_sphere(X, (0.5, 0.5), 0.2))),
            W.Obj(W.OBJ_DIELECTRIC, 2.0, np.ascontiguousarray(W.sdf_sphere(X, (0.5, 0.92), 0.2)))]))
    # saddle: a checkerboard level set
    n = 4
    s = np.array([[1.0, -1.0, 1.0, -1.0, 1.0]] * 5)
    s[1::2] *= -1
    pr = W.Problem(2, (n, n), 0.25, (0.0, 0.0), [W.Obj(W.OBJ_ELECTRODE, 1.0, s)], *W._bc(0))
    with pytest.raises(GeometryError):
        Geometry(pr)
