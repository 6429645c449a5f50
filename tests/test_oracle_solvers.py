"""P1: the oracle's three solution routes agree (dense LU, SuperLU with
refinement, multigrid-preconditioned GMRES), including cut cells and
two-unknown cells; the stopping measure is the paper's relative residual."""
import numpy as np
import pytest

import workloads as W
from oracle.operator import assemble
from oracle import solvers


def _box3(seed):
    rng = np.random.default_rng(seed)
    while True:
        try:
            pr = W.random_box(rng)
        except Exception:
            continue
        if max(pr.n) <= 32:
            return pr


@pytest.mark.parametrize("make", [
    lambda: W.two_disks(16, seed=0),
    lambda: W.coaxial(16),
    lambda: W.manufactured_sine(16),
])
def test_dense_splu_gmres_agree_small(make):
    pr = make()
    S = assemble(pr)
    assert S.A.shape[0] <= 600
    xd = solvers.solve_dense(S.A, S.b)
    xs = solvers.solve_splu(S.A, S.b)
    xg = solvers.solve_gmres(S, rtol=1e-13)
    nd = np.linalg.norm(xd)
    assert np.linalg.norm(xs - xd) <= 1e-12 * nd
    assert np.linalg.norm(xg - xd) <= 1e-10 * nd
    assert solvers.rel_residual(S.A, S.b, xd) < 1e-13


def test_splu_gmres_agree_two_disks():
    pr = W.two_disks(128, seed=3)
    S = assemble(pr)
    assert S.N2 > 0
    xs = solvers.solve_splu(S.A, S.b)
    info = {}
    xg = solvers.solve_gmres(S, rtol=1e-13, info=info)
    assert np.linalg.norm(xg - xs) <= 1e-10 * np.linalg.norm(xs)
    assert info["converged"]


def test_splu_gmres_agree_3d_box():
    pr = W.pin_plane(24, seed=2)
    S = assemble(pr)
    xs = solvers.solve_splu(S.A, S.b)
    xg = solvers.solve_gmres(S, rtol=1e-13)
    assert np.linalg.norm(xg - xs) <= 1e-10 * np.linalg.norm(xs)
    assert solvers.rel_residual(S.A, S.b, xs) < 1e-13
