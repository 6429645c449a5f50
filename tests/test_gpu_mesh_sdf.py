"""Signed distance from surface tessellations on the GPU (geometry
generation section) through the C ABI, against the oracle's brute force
(distance within 1e-12 of the box scale, the same sign wherever the
distance exceeds 1e-9), on small lattices in full and, at the benchmark's
257^3 nodes, on sampled nodes; the cube also against the box closed form on
every node."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.mesh_sdf import signed_distance, node_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ebmg = pytest.importorskip("paper_1809_03745_amd.ebmg", reason="libebmg.so not built")

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ebmg.Context(0)


MESHES = {
    "cube": lambda: W.mesh_cube((0.47, 0.52, 0.5), 0.26),
    "icosphere": lambda: W.mesh_icosphere((0.5, 0.46, 0.53), 0.31, subdiv=3),
    "torus": lambda: W.mesh_torus(),
    "pin": lambda: W.mesh_pin(),
}


def _gpu_sdf(M, n, h, lo):
    out = torch.full(((n + 1) ** 3,), np.nan, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    vis = M.sdf((n, n, n), h, lo, out)
    return out.cpu().numpy(), vis


def _compare(got, want):
    assert np.isfinite(got).all()
    assert np.abs(np.abs(got) - np.abs(want)).max() <= 1e-12
    far = np.abs(want) > 1e-9
    assert np.array_equal(np.sign(got[far]), np.sign(want[far]))


@pytest.mark.parametrize("name", sorted(MESHES))
def test_mesh_sdf_small_lattice(ctx, name):
    v, t = MESHES[name]()
    M = ebmg.Mesh(ctx, v, t)
    n, h, lo = 20, 1.0 / 20, (0.0, 0.0, 0.0)
    got, vis = _gpu_sdf(M, n, h, lo)
    want = signed_distance(node_points((n, n, n), h, lo), v, t)
    _say(name, "triangles", M.ntri, "tree depth", M.depth, "visits per node", vis / got.size)
    _compare(got, want)
    if M.ntri >= 1000:
        assert vis < 0.1 * got.size * M.ntri      # the tree prunes most of the brute-force work
    M.release()


@pytest.mark.parametrize("name", ["torus", "pin"])
def test_mesh_sdf_full_size_sampled(ctx, name):
    v, t = MESHES[name]()
    M = ebmg.Mesh(ctx, v, t)
    n, h = 256, 1.0 / 256
    got, vis = _gpu_sdf(M, n, h, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(5)
    idx = rng.choice(got.size, size=1500, replace=False)
    P = node_points((n, n, n), h, (0.0, 0.0, 0.0))[idx]
    _compare(got[idx], signed_distance(P, v, t))
    _say(name, "257^3 nodes, visits per node", vis / got.size)
    M.release()


def test_cube_every_node_matches_closed_form(ctx):
    c, s = np.array([0.47, 0.52, 0.5]), 0.26
    v, t = W.mesh_cube(c, s)
    M = ebmg.Mesh(ctx, v, t)
    n, h = 96, 1.0 / 96
    got, _ = _gpu_sdf(M, n, h, (0.0, 0.0, 0.0))
    P = node_points((n, n, n), h, (0.0, 0.0, 0.0))
    q = np.abs(P - c) - s
    want = np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)
    _compare(got, want)
    M.release()


def test_mesh_errors(ctx):
    v, t = W.mesh_cube()
    with pytest.raises(ebmg.EbmgError) as e:        # a hole: one triangle missing
        ebmg.Mesh(ctx, v, t[:-1])
    assert e.value.status == ebmg.ERR_GEOMETRY
    bad = t.copy()
    bad[0, 0] = 99
    with pytest.raises(ebmg.EbmgError) as e:
        ebmg.Mesh(ctx, v, bad)
    assert e.value.status == ebmg.ERR_GEOMETRY
    M = ebmg.Mesh(ctx, v, t)
    with pytest.raises(ebmg.EbmgError) as e:        # too short an output
        M.sdf((8, 8, 8), 0.125, (0, 0, 0), torch.zeros(10, dtype=torch.float64, device=DEV))
    assert e.value.status == ebmg.ERR_ARG
    M.release()
