"""ORACLE (test infrastructure) — closed forms used as pins.

* ``sine_discrete``: with the linear Dirichlet closure, sin(pi x) sin(pi y)
  sampled at cell centres is an eigenvector of the 5-point operator on the
  unit square (odd reflection across each wall), eigenvalue
  lambda_h = (8/h^2) sin^2(pi h/2); hence the discrete solution for
  rho = 2 pi^2 sin sin is (2 pi^2/lambda_h) sin sin, exactly.
* ``coaxial``: the paper's multifluid coaxial problem (verification
  section): phi = phi0 + (a/eps) ln(r/R0) on R0 <= r <= R1 and a ln(r/R2) on
  R1 <= r <= R2 with a = phi0 / (ln(R1/R2) - ln(R1/R0)/eps). With a uniform
  surface charge sigma on r = R1 (an extension derived here from
  div(eps grad phi) = -rho with a thin charged layer, which gives
  eps_gas dphi/dr(R1+) - eps dphi/dr(R1-) = -sigma), write
  phi = A ln(r/R2) outside and phi0 + B ln(r/R0) inside:
  A - eps B = -sigma R1 and A ln(R1/R2) = phi0 + B ln(R1/R0).
"""
from __future__ import annotations

import math

import numpy as np


def sine_discrete(n):
    h = 1.0 / n
    lam = (8.0 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    x = (np.arange(n) + 0.5) * h
    s = np.sin(math.pi * x)
    return (2 * math.pi ** 2 / lam) * np.outer(s, s)


def coaxial_coefficients(R0=0.3, R1=0.6, R2=0.9, eps=4.0, phi0=1.0, sigma=0.0):
    """(A, B): phi = A ln(r/R2) in the gas, phi0 + B ln(r/R0) in the dielectric."""
    l2 = math.log(R1 / R2)
    l0 = math.log(R1 / R0)
    # A = eps B - sigma R1 ; (eps B - sigma R1) l2 = phi0 + B l0
    B = (phi0 + sigma * R1 * l2) / (eps * l2 - l0)
    A = eps * B - sigma * R1
    return A, B


def coaxial(r, R0=0.3, R1=0.6, R2=0.9, eps=4.0, phi0=1.0, sigma=0.0, branch=None):
    """Closed-form potential; branch 'gas'/'diel' extends one branch past R1."""
    A, B = coaxial_coefficients(R0, R1, R2, eps, phi0, sigma)
    g = A * np.log(r / R2)
    d = phi0 + B * np.log(r / R0)
    if branch == "gas":
        return g
    if branch == "diel":
        return d
    return np.where(r >= R1, g, d)
