"""Pins of the oracle's composite AMR operator (oracle/amr.py) against what
the mathematics fixes: quadratic exactness of every valid row (ghosts,
tangential stencils with their one-sided forms, refluxed coarse faces),
telescoping of the area-weighted divergence, second-order convergence of the
composite solution, and reduction to the single-level system when a box
covers the whole domain."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.amr import Composite, AmrError
from oracle.operator import assemble

pytestmark = pytest.mark.filterwarnings("ignore")


def _quad(dim):
    """A quadratic with every mixed term, and its Laplacian."""
    if dim == 2:
        f = lambda x, y: 1 + 0.3 * x - 0.2 * y + 0.7 * x * x - 0.4 * x * y + 0.5 * y * y
        lap = 2 * 0.7 + 2 * 0.5
    else:
        f = lambda x, y, z: (1 + 0.3 * x - 0.2 * y + 0.1 * z + 0.7 * x * x - 0.4 * x * y + 0.5 * y * y
                             + 0.6 * x * z - 0.3 * y * z - 0.8 * z * z)
        lap = 2 * 0.7 + 2 * 0.5 - 2 * 0.8
    return f, lap


def _level_values(amr, f):
    out = []
    for lv in amr.levels:
        X = W._centres(amr.dim, lv.prob.n, lv.prob.h, lv.prob.lo)
        out.append(np.ascontiguousarray(f(*X)).ravel())
    return out


def _interior_valid(C):
    """Mask over valid unknowns: cells whose stencil stays off the domain
    boundary (there the linear Dirichlet closure is not exact for
    quadratics)."""
    masks = []
    for lv in C.amr.levels:
        full = [m * 2 ** lv.level for m in C.amr.levels[0].prob.n]
        idx = np.indices(tuple(reversed(lv.prob.n)))
        m = np.ones(tuple(reversed(lv.prob.n)), bool)
        for d in range(C.dim):
            g = idx[C.dim - 1 - d] + lv.lo[d]
            m &= (g > 0) & (g < full[d] - 1)
        masks.append(m.ravel())
    return np.concatenate(masks)[C.valid]


CASES = {
    "2d two levels": (2, 16, [((8, 10), (12, 14))]),
    "2d three levels": (2, 16, [((8, 8), (16, 16)), ((24, 20), (16, 24))]),
    "2d box on the domain edge": (2, 16, [((8, 0), (12, 14))]),
    "2d box in a corner": (2, 16, [((0, 18), (14, 14))]),
    "3d two levels": (3, 8, [((4, 4, 6), (8, 6, 6))]),
    "3d three levels": (3, 8, [((4, 4, 4), (8, 8, 8)), ((12, 12, 12), (8, 8, 8))]),
    "3d box on two domain faces": (3, 8, [((6, 0, 8), (8, 8, 8))]),
    "2d two boxes on level 1": (2, 16, [(1, (4, 4), (8, 8)), (1, (20, 16), (8, 10))]),
    "2d two boxes, one refined again": (2, 16, [(1, (4, 4), (8, 8)), (1, (20, 16), (10, 12)),
                                                (2, (44, 36), (8, 8))]),
    "3d two boxes on level 1": (3, 12, [(1, (2, 2, 2), (6, 6, 6)), (1, (16, 16, 10), (6, 6, 8))]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_quadratic_exactness_of_every_row(name):
    dim, n0, boxes = CASES[name]
    amr = W.amr_plain(dim, n0, boxes)
    C = Composite(amr)
    f, lap = _quad(dim)
    x = C.gather(_level_values(amr, f))
    y = C.A @ x
    mask = _interior_valid(C)
    # Poisson rows: beta b lap (beta = -1, b = 1)
    err = np.abs(y[mask] - (-lap))
    assert mask.sum() > 50
    assert err.max() < 1e-9 * max(1.0, abs(lap)), (name, err.max())


def test_planted_ghost_weight_fails():
    """The exactness pin catches a wrong ghost weight (planted in the oracle
    module on the CPU, then restored)."""
    import oracle.amr as A
    dim, n0, boxes = CASES["2d two levels"]
    amr = W.amr_plain(dim, n0, boxes)
    f, lap = _quad(dim)
    old = A.GHOST_W
    try:
        A.GHOST_W = (0.5, 0.75, -0.25)
        C = A.Composite(amr)
        y = C.A @ C.gather(_level_values(amr, f))
        mask = _interior_valid(C)
        assert np.abs(y[mask] + lap).max() > 1e-3
    finally:
        A.GHOST_W = old


@pytest.mark.parametrize("name", ["2d two levels", "2d three levels", "3d two levels", "3d three levels",
                                  "3d box on two domain faces", "2d two boxes, one refined again",
                                  "3d two boxes on level 1"])
def test_refluxed_divergence_telescopes(name):
    """With zero-flux Neumann faces, the rows weighted by their cell volumes
    sum to zero for any field: the fluxes through coarse-fine faces cancel."""
    dim, n0, boxes = CASES[name]
    amr = W.amr_plain(dim, n0, boxes, bc=W.BC_NEUMANN)
    C = Composite(amr)
    vol = []
    for i, lv in enumerate(amr.levels):
        s = C.sys[i]
        vol.append(np.full(s.N + s.N2, lv.prob.h ** dim))
    vol = np.concatenate(vol)[C.valid]
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal(C.A.shape[0])
        tot = vol @ (C.A @ x)
        scale = np.abs(vol * (C.A @ x)).sum()
        assert abs(tot) < 1e-12 * scale, (name, tot, scale)


def test_second_order_convergence_2d():
    """phi = sin(pi x) sin(pi y), Dirichlet 0, patch over the middle: the
    composite solution's max error falls by ~4 per refinement of the whole
    hierarchy."""
    errs = []
    for n0 in (16, 32, 64):
        k = n0 // 16
        rho = lambda X: 2 * math.pi ** 2 * np.sin(math.pi * X[0]) * np.sin(math.pi * X[1])
        amr = W.amr_plain(2, n0, [((10 * k, 8 * k), (12 * k, 16 * k))], rho_fn=rho)
        C = Composite(amr)
        x = C.solve()
        ex = C.gather(_level_values(amr, lambda a, b: np.sin(math.pi * a) * np.sin(math.pi * b)))
        errs.append(np.abs(x - ex).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.8, (errs, orders)


def test_second_order_convergence_3d_two_levels():
    errs = []
    for n0 in (8, 16, 32):
        k = n0 // 8
        rho = lambda X: 3 * math.pi ** 2 * np.sin(math.pi * X[0]) * np.sin(math.pi * X[1]) * np.sin(math.pi * X[2])
        amr = W.amr_plain(3, n0, [((4 * k, 4 * k, 6 * k), (8 * k, 6 * k, 6 * k))], rho_fn=rho)
        C = Composite(amr)
        x = C.solve()
        ex = C.gather(_level_values(amr, lambda a, b, c: np.sin(math.pi * a) * np.sin(math.pi * b)
                                    * np.sin(math.pi * c)))
        errs.append(np.abs(x - ex).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.7, (errs, orders)


def test_box_covering_the_domain_is_the_fine_system():
    rho = lambda X: np.exp(-((X[0] - 0.4) ** 2 + (X[1] - 0.6) ** 2) / 0.02)
    amr = W.amr_plain(2, 12, [((0, 0), (24, 24))], rho_fn=rho)
    C = Composite(amr)
    x = C.solve()
    fine = amr.levels[1].prob
    S = assemble(fine)
    import scipy.sparse.linalg as spl
    ref = spl.spsolve(S.A.tocsc(), S.b)
    assert C.A.shape[0] == fine.ncells
    assert np.abs(x - ref).max() < 1e-12 * np.abs(ref).max()


def test_embedded_boundary_at_the_coarse_fine_face_is_rejected():
    """The pin's cut cells may not touch the ghosts' stencils."""
    amr = W.amr_pin_plane(32, 2)
    lv = amr.levels[1]
    # move the patch so that its low z face cuts through the pin tip
    bad = W.amr_hierarchy(3, (32,) * 3, 1.0 / 32, (0.0,) * 3, [((24, 24, 38), (16, 16, 26))],
                          lambda n, h, lo: (amr_objs(n, h, lo), None),
                          [W.BC_NEUMANN] * 4 + [W.BC_DIRICHLET] * 2, [0.0] * 5 + [1.0])
    with pytest.raises(AmrError):
        Composite(bad)
    assert lv.cf[4] and not lv.cf[5]


def amr_objs(n, h, lo):
    Xn = W._nodes(3, n, h, lo)
    return [W.Obj(W.OBJ_ELECTRODE, 1.0, np.ascontiguousarray(W.sdf_pin3(Xn, (0.5, 0.5), 0.6, 0.1)))]


def test_touching_boxes_are_rejected():
    """Two boxes of one level sharing a face: the ghosts of the cells along
    it would need the other box's fine values (fine-fine faces are not part
    of this hierarchy), so their coarse cell is not a valid coarse cell."""
    amr = W.amr_plain(2, 16, [(1, (4, 4), (8, 8)), (1, (12, 4), (8, 8))])
    with pytest.raises(AmrError):
        Composite(amr)
