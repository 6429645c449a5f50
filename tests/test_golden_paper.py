"""Pins from values the paper prints (tests/golden/): the multi-fluid coaxial
problem of its verification section.

The fixture holds the printed parameters only; the checks are properties the
closed form and the generator must have, independent of how either is coded:
boundary values on both electrodes, continuity of phi and of eps dphi/dr
across the dielectric surface (zero surface charge), and r dphi/dr constant on
each shell (the cylindrical Poisson equation without space charge).
"""
import math
import os

import numpy as np

import workloads as W
from oracle import exact

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    d = {}
    with open(os.path.join(HERE, "golden", "coaxial_paper.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, *v = line.split()
                d[k] = [float(x) for x in v]
    return d


def test_coaxial_generator_uses_printed_parameters():
    g = _golden()
    n = int(g["grids"][0])
    pr = W.coaxial(n)
    assert pr.lo == (g["domain"][0], g["domain"][0])
    assert math.isclose(pr.h * n, g["domain"][1] - g["domain"][0])
    xs = pr.lo[0] + pr.h * np.arange(n + 1)
    X, Y = np.meshgrid(xs, xs)
    r = np.hypot(X, Y)
    inner, outer, diel = pr.objects
    assert inner.kind == W.OBJ_ELECTRODE and inner.value == g["phi0"][0]
    assert outer.kind == W.OBJ_ELECTRODE and outer.value == 0.0
    assert diel.kind == W.OBJ_DIELECTRIC and diel.value == g["eps"][0]
    # zero sets of the level sets are the printed circles
    for obj, R in ((inner, g["R0"][0]), (outer, g["R2"][0]), (diel, g["R1"][0])):
        s = obj.sdf
        assert np.allclose(np.abs(s), np.abs(r - R), atol=1e-14)


def test_coaxial_closed_form_properties():
    g = _golden()
    R0, R1, R2, eps, phi0 = g["R0"][0], g["R1"][0], g["R2"][0], g["eps"][0], g["phi0"][0]
    kw = dict(R0=R0, R1=R1, R2=R2, eps=eps, phi0=phi0)
    f = lambda r, br=None: float(exact.coaxial(np.array([r]), branch=br, **kw)[0])
    assert abs(f(R0) - phi0) < 1e-15
    assert abs(f(R2)) < 1e-15
    assert abs(f(R1, "gas") - f(R1, "diel")) < 1e-14
    d = 1e-6
    dg = (f(R1 + d, "gas") - f(R1 - d, "gas")) / (2 * d)
    dd = (f(R1 + d, "diel") - f(R1 - d, "diel")) / (2 * d)
    assert abs(dg - eps * dd) < 1e-8
    # r dphi/dr constant on each shell
    for lo, hi in ((R0, R1), (R1, R2)):
        rs = np.linspace(lo + 0.01, hi - 0.01, 7)
        q = [r * (f(r + d) - f(r - d)) / (2 * d) for r in rs]
        assert np.ptp(q) < 1e-7
