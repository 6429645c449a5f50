"""Oracle E = -grad(phi): the vectorised regular path equals the generic
face-flux path, and on the coaxial problem the radial field on each side of
the dielectric surface converges to the closed form (-A/r in the gas,
-B/r in the dielectric; their ratio at R1 is the permittivity 4)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact
from oracle.efield import efield
from oracle.operator import assemble
from oracle.solvers import solve_splu


@pytest.mark.parametrize("make", [lambda: W.two_disks(48, seed=4), lambda: W.pin_plane(12, seed=3),
                                  lambda: W.eddington(2, 16, 3.0)])
def test_efield_vectorised_equals_generic(make):
    pr = make()
    S = assemble(pr)
    x = solve_splu(S.A, S.b)
    E1 = efield(S, x)
    E2 = efield(S, x, generic_only=True)
    assert np.abs(E1 - E2).max() <= 1e-12 * (np.abs(E1).max() + 1)


def test_coaxial_field_converges():
    A, B = exact.coaxial_coefficients()
    errs = []
    for n in (64, 128, 256):
        pr = W.coaxial(n)
        S = assemble(pr)
        x = solve_splu(S.A, S.b)
        E = efield(S, x)
        X, Y = pr.cell_centres()
        X = np.broadcast_to(X, pr.shape)
        Y = np.broadcast_to(Y, pr.shape)
        r = np.sqrt(X ** 2 + Y ** 2)
        Er = (E[0] * X + E[1] * Y) / r
        g = S.geo
        gas = (g.primary == 0) & (r > 0.62) & (r < 0.85)
        die = (g.primary == 1) & (r > 0.33) & (r < 0.58)
        eg = np.abs(Er[gas] - (-A / r[gas])).max()
        ed = np.abs(Er[die] - (-B / r[die])).max()
        errs.append(max(eg, ed))
    assert errs[2] < errs[0] / 8
    assert errs[2] < 1e-3
    assert abs((-A / 0.6) / (-B / 0.6) - 4.0) < 1e-12
    assert abs(-A / 0.6 - 2.87976) < 1e-5
