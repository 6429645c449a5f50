"""Richardson convergence order of the oracle's EB operator where no closed
form exists (Verification tests: the paper checks its multifluid solver by
second-order convergence under refinement).

For three grids h, 2h, 4h the solutions are compared after averaging each
finer solution over the 2^D children of the coarser cell:
    E_4h = |A(phi_2h) - phi_4h|,  E_2h = |A(phi_h) - phi_2h|,
    p = log2(E_4h / E_2h),
over cells that are regular and single-phase on both grids. A second-order
operator gives p -> 2 (cell-centre values and child means differ by O(h^2)
as well, with a resolution-independent constant). An O(1) error anywhere in
the cut-cell rows (a wrong moment, a wrong facet flux) drives p towards 0
or 1.

Workloads: the two-disk class (electrode disk and eps = 4 dielectric disk,
Gaussian space charge) without its per-cell random surface charge, which is
white noise that does not converge; and the pin-plane class with a pin of
radius 0.1 and blobs of standard deviation 0.06-0.1, so that the coarsest
grid (32^3) resolves the pin and the blobs (the production radius 0.02 is
below one cell at 32^3).
"""
import math

import numpy as np

import workloads as W
from oracle.operator import assemble
from oracle.solvers import solve_splu, solve_gmres


def _solution(pr, gmres=False):
    S = assemble(pr)
    x = solve_gmres(S, rtol=1e-12) if gmres else solve_splu(S.A, S.b)
    g = S.geo
    phi = x[:g.N].reshape(g.shape)
    prim = g.primary
    kap = np.where(prim == 0, g.ph[0].kappa, np.where(prim == 1, g.ph[1].kappa, 0.0))
    return phi, prim, kap


def _child_blocks(a, dim):
    n = a.shape[0] // 2
    return a.reshape((n, 2) * dim)


def _difference(fine, coarse, dim):
    pf, prf, kf = fine
    pc, prc, kc = coarse
    axes = tuple(range(1, 2 * dim, 2))
    mean = _child_blocks(pf, dim).mean(axis=axes)
    ok = (kc == 1.0) & (prc >= 0)
    ok &= (_child_blocks(kf, dim) == 1.0).all(axis=axes)
    bshape = tuple(s for n in pc.shape for s in (n, 1))
    ok &= (_child_blocks(prf, dim) == prc.reshape(bshape)).all(axis=axes)
    d = np.abs(mean - pc)[ok]
    return math.sqrt((d * d).mean()), d.mean(), int(ok.sum())


def _orders(sols, dim):
    e1 = _difference(sols[1], sols[0], dim)
    e2 = _difference(sols[2], sols[1], dim)
    assert e2[2] > 3 * e1[2] > 1000
    return math.log2(e1[0] / e2[0]), math.log2(e1[1] / e2[1])


def test_richardson_two_disks_256_512_1024():
    sols = [_solution(W.two_disks(n, seed=0, sigma_std=0.0)) for n in (256, 512, 1024)]
    p_l2, p_l1 = _orders(sols, 2)
    assert p_l2 >= 1.8 and p_l1 >= 1.8, (p_l2, p_l1)


def test_richardson_pin_plane_32_64_128():
    sols = [_solution(W.pin_plane(n, seed=0, r_pin=0.1, blob_sigma=(0.06, 0.1)), gmres=True)
            for n in (32, 64, 128)]
    p_l2, p_l1 = _orders(sols, 3)
    assert p_l2 >= 1.8 and p_l1 >= 1.8, (p_l2, p_l1)
