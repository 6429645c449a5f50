"""Pins of the oracle's signed distance from a triangle mesh (geometry
generation section): the closed form of a box, sphere bounds of an
icosphere, winding numbers."""
import numpy as np

import workloads as W
from oracle.mesh_sdf import signed_distance, winding_number, node_points


def _box_sdf(P, c, s):
    q = np.abs(P - c) - s
    out = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inn = np.minimum(q.max(axis=1), 0.0)
    return out + inn


def test_cube_matches_box_closed_form():
    """Every feature class: face regions, edge regions and corner regions of
    the 12-triangle cube (the diagonal of each face is an interior edge)."""
    v, t = W.mesh_cube((0.5, 0.5, 0.5), 0.25)
    rng = np.random.default_rng(0)
    P = np.concatenate([rng.uniform(-0.2, 1.2, size=(3000, 3)), node_points((12, 12, 12), 1 / 12, (0, 0, 0))])
    d = signed_distance(P, v, t)
    assert np.abs(d - _box_sdf(P, 0.5, 0.25)).max() <= 1e-13


def test_icosphere_between_inscribed_and_circumscribed_spheres():
    c, r = np.array([0.45, 0.5, 0.55]), 0.3
    v, t = W.mesh_icosphere(c, r, subdiv=2)
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    n /= np.linalg.norm(n, axis=1)[:, None]
    r_in = np.abs(np.einsum("ij,ij->i", v[t[:, 0]] - c, n)).min()
    rng = np.random.default_rng(1)
    P = rng.uniform(0.0, 1.0, size=(2000, 3))
    d = signed_distance(P, v, t)
    rho = np.linalg.norm(P - c, axis=1)
    assert (d >= rho - r - 1e-13).all()
    assert (d <= rho - r_in + 1e-13).all()
    assert r - r_in < 0.02


def test_winding_numbers():
    v, t = W.mesh_torus()
    inside = np.array([[0.5 + 0.28, 0.5, 0.5], [0.5, 0.5 - 0.28, 0.52]])
    outside = np.array([[0.5, 0.5, 0.5], [0.05, 0.05, 0.05], [0.5 + 0.28, 0.5, 0.75]])
    assert np.allclose(winding_number(inside, v, t), 1.0, atol=1e-9)
    assert np.allclose(winding_number(outside, v, t), 0.0, atol=1e-9)
    d = signed_distance(np.concatenate([inside, outside]), v, t)
    assert (d[:2] < 0).all() and (d[2:] > 0).all()
