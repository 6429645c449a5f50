"""ORACLE (test infrastructure) — signed distance from a closed triangle mesh.

Written from the geometry-generation section of the paper: the level set of a
watertight two-manifold tessellation is the signed distance to its closest
polygon, edge or vertex. This is the plain definition, by brute force over
every triangle (no tree, no pseudonormals):
  * distance from p to a triangle: if the foot of the perpendicular from p
    to the triangle's plane lies in the triangle (barycentric coordinates
    from the 2x2 normal equations of the plane's edge vectors), the distance
    to the plane; otherwise the least distance to its three edges (point to
    segment, with the projection parameter clamped to [0, 1]);
  * sign: the generalised winding number of the closed surface around p,
    the sum of the solid angles of its triangles seen from p over 4 pi
    (solid angle of a triangle by the formula of Van Oosterom and
    Strackee); p is inside where it exceeds 1/2, and the distance is then
    negated (> 0 outside, the convention of the node-sampled level sets).

Parity: pinned by tests/test_oracle_mesh_sdf.py against the closed-form
signed distance of a box (faces, edges and corners), the inscribed /
circumscribed sphere bounds of an icosphere, and winding numbers of 1 inside
and 0 outside.
"""
from __future__ import annotations

import numpy as np


def _triangle_distance(P, a, b, c):
    """Distance from every point of P (m, 3) to the triangle (a, b, c)."""
    e1, e2 = b - a, c - a
    n = np.cross(e1, e2)
    n = n / np.linalg.norm(n)
    ap = P - a
    h = ap @ n
    foot = ap - np.outer(h, n)
    g11, g12, g22 = e1 @ e1, e1 @ e2, e2 @ e2
    r1, r2 = foot @ e1, foot @ e2
    det = g11 * g22 - g12 * g12
    l1 = (r1 * g22 - r2 * g12) / det
    l2 = (r2 * g11 - r1 * g12) / det
    inside = (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
    d = np.abs(h)
    edge = np.full(len(P), np.inf)
    for s, t in ((a, b), (b, c), (c, a)):
        v = t - s
        w = P - s
        u = np.clip((w @ v) / (v @ v), 0.0, 1.0)
        q = w - np.outer(u, v)
        edge = np.minimum(edge, np.sqrt(np.einsum("ij,ij->i", q, q)))
    return np.where(inside, d, edge)


def winding_number(P, verts, tris):
    """Generalised winding number of the closed surface around each point."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    w = np.zeros(len(P))
    for t in tris:
        A = verts[t[0]] - P
        B = verts[t[1]] - P
        C = verts[t[2]] - P
        la, lb, lc = (np.linalg.norm(X, axis=1) for X in (A, B, C))
        num = np.einsum("ij,ij->i", A, np.cross(B, C))
        den = la * lb * lc + np.einsum("ij,ij->i", A, B) * lc + np.einsum("ij,ij->i", A, C) * lb + \
            np.einsum("ij,ij->i", B, C) * la
        w += 2.0 * np.arctan2(num, den)
    return w / (4.0 * np.pi)


def signed_distance(P, verts, tris):
    """Signed distance (> 0 outside) of the closed mesh at the points P (m, 3)."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    verts = np.asarray(verts, dtype=np.float64)
    d = np.full(len(P), np.inf)
    for t in tris:
        d = np.minimum(d, _triangle_distance(P, verts[t[0]], verts[t[1]], verts[t[2]]))
    inside = winding_number(P, verts, tris) > 0.5
    return np.where(inside, -d, d)


def node_points(n, h, lo):
    """Nodes lo + (i, j, k) h of an n[0] x n[1] x n[2]-cell box, x fastest."""
    z, y, x = np.meshgrid(*(lo[d] + h * np.arange(n[d] + 1) for d in (2, 1, 0)), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
