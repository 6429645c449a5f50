"""Seeded synthetic inputs for the embedded-boundary elliptic solve.

This module is shared by the CPU oracle and the GPU library. It holds only
problem *descriptions*: the box, analytic signed-distance functions sampled at
grid nodes, the per-cell source density, the per-cell surface charge draw and
the boundary data. It contains none of the discretisation arithmetic (no
moments, no stencils, no solves).

Conventions (shared by both sides):
  * cells are indexed (i_x, i_y[, i_z]); arrays are stored C-order with x
    fastest, i.e. numpy shape (ny, nx) or (nz, ny, nx);
  * node-sampled level sets have shape (ny+1, nx+1) or (nz+1, ny+1, nx+1);
  * an object's signed distance is > 0 outside the object;
  * nondimensional units with eps0 = 1, so rho means rho/eps0;
  * all random numbers come from numpy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

OBJ_ELECTRODE = 0   # covered for every phase; Dirichlet value on its surface
OBJ_DIELECTRIC = 1  # region of phase 1 (permittivity = value)
OBJ_WALL = 2        # covered for every phase; Neumann flux (value) on its surface

BC_DIRICHLET = 0
BC_NEUMANN = 1
BC_ROBIN = 2

FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


@dataclasses.dataclass
class Obj:
    kind: int
    value: float
    sdf: np.ndarray  # node-sampled, float64, > 0 outside


@dataclasses.dataclass
class Problem:
    """One elliptic problem: alpha*a*phi + beta*div(b grad phi) = rho."""
    dim: int
    n: tuple            # (nx, ny) or (nx, ny, nz)
    h: float
    lo: tuple
    objects: List[Obj]
    bc_kind: list       # 6 entries (x-, x+, y-, y+, z-, z+)
    bc_value: list      # Dirichlet value / Neumann outward flux / Robin a3
    robin_a1: list
    robin_a2: list
    alpha: float = 0.0
    beta: float = -1.0
    a_gas: float = 0.0
    a_diel: float = 0.0
    b_gas: float = 1.0
    rho: Optional[np.ndarray] = None     # per cell (primary DOF), float64
    sigma: Optional[np.ndarray] = None   # per cell (used on gas/dielectric facets)
    name: str = ""
    seed: Optional[int] = None

    @property
    def shape(self):
        """numpy shape of a cell array."""
        return tuple(reversed(self.n))

    @property
    def ncells(self):
        return int(np.prod(self.n))

    def cell_centres(self):
        """Tuple of coordinate arrays (x, y[, z]) broadcastable to ``shape``."""
        return _axes(self.dim, self.n, self.h, self.lo, 0.5)

    def nodes(self):
        return _axes(self.dim, tuple(m + 1 for m in self.n), self.h, self.lo, 0.0)


def _axes(dim, n, h, lo, off):
    out = []
    for d in range(dim):
        v = lo[d] + (np.arange(n[d], dtype=np.float64) + off) * h
        shp = [1] * dim
        shp[dim - 1 - d] = n[d]
        out.append(v.reshape(shp))
    return tuple(out)


def _bc(kind, value=0.0, a1=0.0, a2=1.0):
    return [kind] * 6, [value] * 6, [a1] * 6, [a2] * 6


# --------------------------------------------------------------------------
# analytic signed distances (exact for the shapes named)
# --------------------------------------------------------------------------

def sdf_sphere(X, centre, r):
    return np.sqrt(sum((X[d] - centre[d]) ** 2 for d in range(len(X)))) - r


def sdf_halfspace_below(coord, level):
    """Region coord < level (signed distance > 0 above)."""
    return coord - level


def sdf_plane(X, point, normal):
    """Half-space {(x - point).normal < 0}; distance > 0 on the +normal side."""
    return sum((X[d] - point[d]) * normal[d] for d in range(len(X)))


def sdf_pin3(X, axis_xy, z_tip, r):
    """Vertical cylinder of radius r on axis (ax, ay) running upward from a
    hemispherical tip whose apex is at z_tip."""
    x, y, z = X
    zc = z_tip + r
    rxy = np.sqrt((x - axis_xy[0]) ** 2 + (y - axis_xy[1]) ** 2)
    cap = np.sqrt(rxy ** 2 + (z - zc) ** 2)
    return np.where(z >= zc, rxy, cap) - r


def sdf_blade2(X, axis_x, y_tip, r):
    """2D blade: strip |x - axis_x| < r above a semicircular tip with apex y_tip."""
    x, y = X
    yc = y_tip + r
    dx = np.abs(x - axis_x)
    cap = np.sqrt(dx ** 2 + (y - yc) ** 2)
    return np.where(y >= yc, dx - r, cap - r)


def _nodes(dim, n, h, lo):
    X = _axes(dim, tuple(m + 1 for m in n), h, lo, 0.0)
    shp = tuple(m + 1 for m in reversed(n))
    return tuple(np.broadcast_to(a, shp) for a in X)


def _centres(dim, n, h, lo):
    X = _axes(dim, n, h, lo, 0.5)
    shp = tuple(reversed(n))
    return tuple(np.broadcast_to(a, shp) for a in X)


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def manufactured_sine(n=64):
    """2D unit square, no embedded boundary, eps = 1, Dirichlet 0 on all sides,
    rho = 2 pi^2 sin(pi x) sin(pi y) at cell centres (manufactured from
    phi = sin(pi x) sin(pi y))."""
    h = 1.0 / n
    x, y = _centres(2, (n, n), h, (0.0, 0.0))
    rho = 2.0 * math.pi ** 2 * np.sin(math.pi * x) * np.sin(math.pi * y)
    k, v, a1, a2 = _bc(BC_DIRICHLET, 0.0)
    return Problem(2, (n, n), h, (0.0, 0.0), [], k, v, a1, a2,
                   rho=np.ascontiguousarray(rho), name=f"sine2d-{n}")


def two_disks(n=1024, seed=0, sigma_std=0.1):
    """2D unit square: conducting disk r=0.1 at (0.5,0.7) held at 1, dielectric
    disk r=0.2 at (0.5,0.3) with eps=4 in gas eps=1, Dirichlet 0 on the box,
    a Gaussian space-charge blob (amplitude 1, standard deviation 0.02) placed
    by the seed at least 0.06 away from both disks, and i.i.d. N(0, sigma_std^2)
    surface charge per cell (used on dielectric facets)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    ce, re = (0.5, 0.7), 0.1
    cd, rd = (0.5, 0.3), 0.2
    while True:
        c = rng.uniform(0.1, 0.9, size=2)
        de = math.hypot(c[0] - ce[0], c[1] - ce[1]) - re
        dd = math.hypot(c[0] - cd[0], c[1] - cd[1]) - rd
        if de >= 0.06 and dd >= 0.06:
            break
    sig = rng.normal(0.0, sigma_std, size=(n, n)) if sigma_std > 0 else None
    Xn = _nodes(2, (n, n), h, (0.0, 0.0))
    objs = [Obj(OBJ_ELECTRODE, 1.0, np.ascontiguousarray(sdf_sphere(Xn, ce, re))),
            Obj(OBJ_DIELECTRIC, 4.0, np.ascontiguousarray(sdf_sphere(Xn, cd, rd)))]
    x, y = _centres(2, (n, n), h, (0.0, 0.0))
    rho = np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2 * 0.02 ** 2))
    k, v, a1, a2 = _bc(BC_DIRICHLET, 0.0)
    return Problem(2, (n, n), h, (0.0, 0.0), objs, k, v, a1, a2,
                   rho=np.ascontiguousarray(rho), sigma=sig,
                   name=f"two-disks-{n}", seed=seed)


def _blobs3(rng, nblob, dists, srange=(0.01, 0.05)):
    cs, ss = [], []
    for _ in range(nblob):
        s = rng.uniform(*srange)
        while True:
            c = np.array([rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9), rng.uniform(0.25, 0.95)])
            if all(f(c) >= 3 * s for f in dists):
                break
        cs.append(c)
        ss.append(s)
    return cs, ss


def _pin_distance_point(c, z_tip=0.6, r=0.02):
    zc = z_tip + r
    rxy = math.hypot(c[0] - 0.5, c[1] - 0.5)
    if c[2] >= zc:
        return rxy - r
    return math.sqrt(rxy ** 2 + (c[2] - zc) ** 2) - r


def pin_plane(n=256, seed=0, nblob=8, r_pin=0.02, blob_sigma=(0.01, 0.05)):
    """3D unit cube: pin of radius r_pin (0.02) on the axis (0.5,0.5) with a
    hemispherical tip whose apex is at z=0.6, held at 1 and reaching the top
    face; dielectric slab eps=4 for z<0.2; z- Dirichlet 0, z+ Dirichlet 1,
    x/y faces homogeneous Neumann; rho = sum of 8 Gaussian blobs (amplitude 1,
    standard deviations U[blob_sigma] = U[0.01,0.05]) kept 3 sigma away from
    pin and slab. The thicker-pin, wider-blob members of the class serve
    convergence studies on coarse grids."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    dists = [lambda c: _pin_distance_point(c, r=r_pin), lambda c: c[2] - 0.2]
    cs, ss = _blobs3(rng, nblob, dists, blob_sigma)
    Xn = _nodes(3, (n, n, n), h, (0.0, 0.0, 0.0))
    objs = [Obj(OBJ_ELECTRODE, 1.0, np.ascontiguousarray(sdf_pin3(Xn, (0.5, 0.5), 0.6, r_pin))),
            Obj(OBJ_DIELECTRIC, 4.0, np.ascontiguousarray(sdf_halfspace_below(Xn[2], 0.2)))]
    X = _centres(3, (n, n, n), h, (0.0, 0.0, 0.0))
    rho = np.zeros(X[0].shape)
    for c, s in zip(cs, ss):
        rho += np.exp(-((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2 + (X[2] - c[2]) ** 2) / (2 * s * s))
    kind = [BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_DIRICHLET, BC_DIRICHLET]
    val = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    return Problem(3, (n, n, n), h, (0.0, 0.0, 0.0), objs, kind, val, [0.0] * 6, [1.0] * 6,
                   rho=np.ascontiguousarray(rho), name=f"pin-plane-{n}", seed=seed)


def _blade_distance_point(c):
    yc = 0.62
    dx = abs(c[0] - 0.5)
    return dx - 0.02 if c[1] >= yc else math.hypot(dx, c[1] - yc) - 0.02


def _blobs_blade(rng, nblob):
    cs, ss = [], []
    for _ in range(nblob):
        s = rng.uniform(0.01, 0.05)
        while True:
            c = np.array([rng.uniform(0.1, 0.9), rng.uniform(0.25, 0.95)])
            if _blade_distance_point(c) >= 3 * s and c[1] - 0.2 >= 3 * s:
                break
        cs.append(c)
        ss.append(s)
    return cs, ss


def _blobs_box(rng, nblob, dim):
    cs, ss = [], []
    for _ in range(nblob):
        s = rng.uniform(0.01, 0.05)
        c = rng.uniform(0.1, 0.9, size=dim)
        cs.append(c)
        ss.append(s)
    return cs, ss


def blade_plane(n=512, seed=0, nblob=8):
    """2D analogue of the pin-plane class: a blade of half-width 0.02 with a
    semicircular tip at y=0.6 reaching the top, dielectric slab y<0.2,
    y- Dirichlet 0, y+ Dirichlet 1, x faces Neumann 0."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n

    cs, ss = _blobs_blade(rng, nblob)
    Xn = _nodes(2, (n, n), h, (0.0, 0.0))
    objs = [Obj(OBJ_ELECTRODE, 1.0, np.ascontiguousarray(sdf_blade2(Xn, 0.5, 0.6, 0.02))),
            Obj(OBJ_DIELECTRIC, 4.0, np.ascontiguousarray(sdf_halfspace_below(Xn[1], 0.2)))]
    X = _centres(2, (n, n), h, (0.0, 0.0))
    rho = np.zeros(X[0].shape)
    for c, s in zip(cs, ss):
        rho += np.exp(-((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2) / (2 * s * s))
    kind = [BC_NEUMANN, BC_NEUMANN, BC_DIRICHLET, BC_DIRICHLET, BC_DIRICHLET, BC_DIRICHLET]
    val = [0.0, 0.0, 0.0, 1.0, 0.0, 0.0]
    return Problem(2, (n, n), h, (0.0, 0.0), objs, kind, val, [0.0] * 6, [1.0] * 6,
                   rho=np.ascontiguousarray(rho), name=f"blade-plane-{n}", seed=seed)


def eddington(dim, n, kappa_abs, seed=0, nblob=8):
    """Eddington (SP1) stationary form kappa*phi - div((1/(3 kappa)) grad phi) = S
    on the unit box, no embedded boundary, Robin outflow
    d(phi)/dn + (3 kappa/2) phi = 0 on every face; S = Gaussian blob sum."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = (n,) * dim
    X = _centres(dim, nn, h, (0.0,) * dim)
    S = np.zeros(X[0].shape)
    for c, s in zip(*_blobs_box(rng, nblob, dim)):
        S += np.exp(-sum((X[d] - c[d]) ** 2 for d in range(dim)) / (2 * s * s))
    pr = eddington_coefficients(dim, n, kappa_abs)
    pr.rho = np.ascontiguousarray(S)
    pr.seed = seed
    return pr


def eddington_coefficients(dim, n, kappa_abs):
    """The Eddington problem's operator and boundary data without a source:
    a = kappa, b = 1/(3 kappa), Robin a1 = 3 kappa/2, a2 = 1 on every face."""
    kind = [BC_ROBIN] * 6
    return Problem(dim, (n,) * dim, 1.0 / n, (0.0,) * dim, [], kind, [0.0] * 6, [1.5 * kappa_abs] * 6,
                   [1.0] * 6, alpha=1.0, beta=-1.0, a_gas=kappa_abs, a_diel=kappa_abs,
                   b_gas=1.0 / (3.0 * kappa_abs), name=f"eddington{dim}d-{n}-k{kappa_abs:.3g}")


# Photoionization model of oxygen (three Eddington groups): lambda_gamma in
# 1/(m Pa), the oxygen partial pressure 0.2 bar, kappa_gamma = lambda_gamma
# p_O2 / sqrt(3), made nondimensional by the 2 cm edge of the pin-plane gap.
PHOTO_LAMBDA = (4.15e-2, 1.09e-1, 6.69e-1)
PHOTO_P_O2 = 2.0e4
PHOTO_L = 0.02


def photo_kappas():
    return [lam * PHOTO_P_O2 / math.sqrt(3.0) * PHOTO_L for lam in PHOTO_LAMBDA]


def tga_mus(dt=1.0, eps=1e-12):
    """mu_1, mu_2 of the TGA scheme, a = 2 - sqrt(2) - eps."""
    a = 2.0 - math.sqrt(2.0) - eps
    r = math.sqrt(a * a - 4.0 * a + 2.0)
    return (a - r) / 2.0 * dt, (a + r) / 2.0 * dt


def photoionization_family(n=128, seed=0, nblob=8, diffusion_number=1.0):
    """Helmholtz operators of one plasma time step on the pin-plane gap
    geometry (pin electrode of radius 0.02 with its tip at z = 0.6, no
    dielectric): the three Eddington groups kappa_g phi - div((1/3kappa_g)
    grad phi) = S with the outflow condition dphi/dn + (3 kappa_g/2) phi = 0
    on every box face, and the two TGA diffusion operators
    phi - div(mu_i D grad phi) = S (zero flux on the box faces; D dt / h^2 =
    diffusion_number). The electrode absorbs (phi = 0 on it) in every member.
    Every member's source is the same blob sum (the photon source is the same
    for all groups). Returns the list of five problems."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    dists = [_pin_distance_point, lambda c: c[2] - 0.05]
    cs, ss = _blobs3(rng, nblob, dists)
    Xn = _nodes(3, (n, n, n), h, (0.0, 0.0, 0.0))
    X = _centres(3, (n, n, n), h, (0.0, 0.0, 0.0))
    src = np.zeros(X[0].shape)
    for c, s in zip(cs, ss):
        src += np.exp(-((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2 + (X[2] - c[2]) ** 2) / (2 * s * s))
    src = np.ascontiguousarray(src)
    pin = np.ascontiguousarray(sdf_pin3(Xn, (0.5, 0.5), 0.6, 0.02))
    out = []
    for kap in photo_kappas():
        out.append(Problem(3, (n, n, n), h, (0.0, 0.0, 0.0), [Obj(OBJ_ELECTRODE, 0.0, pin)],
                           [BC_ROBIN] * 6, [0.0] * 6, [1.5 * kap] * 6, [1.0] * 6,
                           alpha=1.0, beta=-1.0, a_gas=kap, b_gas=1.0 / (3.0 * kap), rho=src,
                           name=f"eddington-group-kappa{kap:.3g}-{n}", seed=seed))
    nu = diffusion_number * h * h          # D dt in units of the box edge squared
    for mu in tga_mus(1.0):
        out.append(Problem(3, (n, n, n), h, (0.0, 0.0, 0.0), [Obj(OBJ_ELECTRODE, 0.0, pin)],
                           [BC_ROBIN] * 6, [0.0] * 6, [0.0] * 6, [1.0] * 6,
                           alpha=1.0, beta=-1.0, a_gas=1.0, b_gas=mu * nu, rho=src,
                           name=f"tga-mu{mu:.4f}-{n}", seed=seed))
    return out


def coaxial(n=256, R0=0.3, R1=0.6, R2=0.9, eps=4.0, phi0=1.0, sigma=0.0):
    """Coaxial cable cross-section on (-1,1)^2: inner electrode r<R0 at phi0,
    dielectric shell R0<r<R1 with permittivity eps, gas R1<r<R2, outer
    electrode r>R2 grounded. Optional uniform surface charge on r=R1."""
    h = 2.0 / n
    lo = (-1.0, -1.0)
    Xn = _nodes(2, (n, n), h, lo)
    r = np.sqrt(Xn[0] ** 2 + Xn[1] ** 2)
    objs = [Obj(OBJ_ELECTRODE, phi0, np.ascontiguousarray(r - R0)),
            Obj(OBJ_ELECTRODE, 0.0, np.ascontiguousarray(R2 - r)),
            Obj(OBJ_DIELECTRIC, eps, np.ascontiguousarray(r - R1))]
    k, v, a1, a2 = _bc(BC_DIRICHLET, 0.0)
    sig = np.full((n, n), float(sigma)) if sigma != 0.0 else None
    return Problem(2, (n, n), h, lo, objs, k, v, a1, a2,
                   rho=np.zeros((n, n)), sigma=sig, name=f"coaxial-{n}")


def random_box(rng):
    """One box of the batched workload: edges 8*round(exp(U[ln16, ln64])/8),
    h = 1/max edge, a random plane splitting eps in {1,2,4,8} (gas side and
    dielectric side), a sphere electrode (phi=1, radius U[0.1,0.3]*shortest
    edge, at least 2h inside the box), the plane redrawn while it passes within
    r+2h of the sphere centre, Dirichlet 0 on the box, and a smooth source of
    4 Fourier modes with wave vectors in {1,2,3}^3."""
    n = tuple(int(8 * round(math.exp(rng.uniform(math.log(16), math.log(64))) / 8)) for _ in range(3))
    h = 1.0 / max(n)
    L = np.array([m * h for m in n])
    lmin = L.min()
    r = rng.uniform(0.1, 0.3) * lmin
    c = np.array([rng.uniform(r + 2 * h, L[d] - r - 2 * h) for d in range(3)])
    while True:
        nv = rng.normal(size=3)
        nv /= np.linalg.norm(nv)
        p = rng.uniform(0.0, 1.0, size=3) * L
        if abs(float(np.dot(c - p, nv))) > r + 2 * h:
            break
    eps_gas, eps_diel = rng.choice([1.0, 2.0, 4.0, 8.0], size=2)
    modes = []
    for _ in range(4):
        k = rng.integers(1, 4, size=3)
        A = rng.normal()
        th = rng.uniform(0, 2 * math.pi)
        modes.append((k, A, th))
    Xn = _nodes(3, n, h, (0.0, 0.0, 0.0))
    objs = [Obj(OBJ_ELECTRODE, 1.0, np.ascontiguousarray(sdf_sphere(Xn, c, r))),
            Obj(OBJ_DIELECTRIC, float(eps_diel), np.ascontiguousarray(sdf_plane(Xn, p, nv)))]
    X = _centres(3, n, h, (0.0, 0.0, 0.0))
    rho = np.zeros(X[0].shape)
    for k, A, th in modes:
        rho += A * np.sin(2 * math.pi * sum(k[d] * X[d] / L[d] for d in range(3)) + th)
    kk, v, a1, a2 = _bc(BC_DIRICHLET, 0.0)
    return Problem(3, n, h, (0.0, 0.0, 0.0), objs, kk, v, a1, a2, b_gas=float(eps_gas),
                   rho=np.ascontiguousarray(rho), name=f"box-{n[0]}x{n[1]}x{n[2]}")


def batched_boxes(nbox=512, seed=0):
    rng = np.random.default_rng(seed)
    return [random_box(rng) for _ in range(nbox)]


def serving_requests(nreq, rate, seed=0):
    """Request stream: Poisson arrivals at ``rate`` per second; each request is
    2D (n in {512,1024,2048}) or 3D (n in {32,64,128,256}) with equal odds, and
    either a pin/blade Poisson solve or an Eddington Helmholtz solve with
    kappa log-uniform in [1,100]. Returns (arrival times, list of specs); a
    spec is materialised with ``make_request``."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    specs = []
    for i in range(nreq):
        dim = 2 if rng.uniform() < 0.5 else 3
        n = int(rng.choice([512, 1024, 2048])) if dim == 2 else int(rng.choice([32, 64, 128, 256]))
        op = "poisson" if rng.uniform() < 0.5 else "helmholtz"
        kappa = math.exp(rng.uniform(0.0, math.log(100.0)))
        specs.append(dict(dim=dim, n=n, op=op, kappa=kappa, seed=int(rng.integers(1 << 31))))
    return t, specs


def request_blobs(spec, nblob=8):
    """(centres, standard deviations) of the source blobs of a served request:
    the same draws ``make_request`` makes, without building the problem."""
    rng = np.random.default_rng(spec["seed"])
    if spec["op"] == "poisson":
        if spec["dim"] == 3:
            return _blobs3(rng, nblob, [_pin_distance_point, lambda c: c[2] - 0.2])
        return _blobs_blade(rng, nblob)
    return _blobs_box(rng, nblob, spec["dim"])


def blob_field(dim, n, centres, sigmas, xp=np, device=None):
    """Sum of unit-amplitude Gaussian blobs at the cell centres of the unit box
    (n^dim cells, x fastest), evaluated with the array module ``xp`` (numpy, or
    torch on ``device``). With numpy it is bitwise the source term of the
    request generators."""
    h = 1.0 / n
    X = _axes(dim, (n,) * dim, h, (0.0,) * dim, 0.5)
    if xp is not np:
        X = tuple(xp.as_tensor(np.ascontiguousarray(a), dtype=xp.float64, device=device) for a in X)
    out = xp.zeros((n,) * dim, dtype=xp.float64, **({} if xp is np else {"device": device}))
    for c, s in zip(centres, sigmas):
        q = (X[0] - float(c[0])) ** 2
        for d in range(1, dim):
            q = q + (X[d] - float(c[d])) ** 2
        out += xp.exp(-q / (2 * s * s))
    return out


def make_request(spec):
    if spec["op"] == "poisson":
        if spec["dim"] == 3:
            return pin_plane(spec["n"], seed=spec["seed"])
        return blade_plane(spec["n"], seed=spec["seed"])
    return eddington(spec["dim"], spec["n"], spec["kappa"], seed=spec["seed"])


# ---------------------------------------------------------------------------
# closed triangle meshes (vertices, triangles counter-clockwise seen from
# outside) for signed distances from surface tessellations
# ---------------------------------------------------------------------------

def mesh_cube(centre=(0.5, 0.5, 0.5), half=0.25):
    c = np.asarray(centre, dtype=np.float64)
    v = np.array([[x, y, z] for z in (-1, 1) for y in (-1, 1) for x in (-1, 1)], dtype=np.float64) * half + c
    # faces as quads (outward, counter-clockwise), two triangles each
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c_, d in quads:
        t.append((a, b, c_))
        t.append((a, c_, d))
    return v, np.array(t, dtype=np.int32)


def mesh_icosphere(centre=(0.5, 0.5, 0.5), r=0.3, subdiv=3):
    """Icosahedron subdivided `subdiv` times, vertices on the sphere."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    v = [np.array(x, dtype=np.float64) / np.linalg.norm(x) for x in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        nf = []
        for a, b, c_ in f:
            ab, bc, ca = mid(a, b), mid(b, c_), mid(c_, a)
            nf += [(a, ab, ca), (b, bc, ab), (c_, ca, bc), (ab, bc, ca)]
        f = nf
    verts = np.array(v) * r + np.asarray(centre, dtype=np.float64)
    return verts, np.array(f, dtype=np.int32)


def mesh_torus(centre=(0.5, 0.5, 0.5), R=0.28, r=0.1, nu=48, nv=24):
    """Torus around the z axis through centre: major radius R, minor r."""
    c = np.asarray(centre, dtype=np.float64)
    verts = []
    for i in range(nu):
        u = 2 * math.pi * i / nu
        for j in range(nv):
            w = 2 * math.pi * j / nv
            verts.append(c + np.array([(R + r * math.cos(w)) * math.cos(u), (R + r * math.cos(w)) * math.sin(u),
                                       r * math.sin(w)]))
    idx = lambda i, j: (i % nu) * nv + (j % nv)
    t = []
    for i in range(nu):
        for j in range(nv):
            a, b, c_, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            t.append((a, b, c_))
            t.append((a, c_, d))
    return np.array(verts), np.array(t, dtype=np.int32)


def mesh_pin(axis_xy=(0.5, 0.5), z_tip=0.6, r=0.02, z_top=1.1, nseg=64, nring=16, nz=32):
    """The pin electrode of the pin-plane gap as a closed tessellation: a
    cylinder of radius r from the hemispherical tip (apex at z_tip) up to a
    flat cap at z_top (above the box, so inside the box it is the pin)."""
    ax, ay = axis_xy
    zc = z_tip + r
    verts = [np.array([ax, ay, z_tip])]              # apex
    rings = []
    for k in range(1, nring + 1):                    # hemisphere rings, polar angle from the apex
        th = 0.5 * math.pi * k / nring
        rings.append([(r * math.sin(th), zc - r * math.cos(th))])
    for k in range(1, nz + 1):                       # cylinder rings
        rings.append([(r, zc + (z_top - zc) * k / nz)])
    ring_idx = []
    for (rad, z), in rings:
        ids = []
        for s in range(nseg):
            ph = 2 * math.pi * s / nseg
            verts.append(np.array([ax + rad * math.cos(ph), ay + rad * math.sin(ph), z]))
            ids.append(len(verts) - 1)
        ring_idx.append(ids)
    verts.append(np.array([ax, ay, z_top]))          # centre of the top cap
    top = len(verts) - 1
    t = []
    first = ring_idx[0]
    for s in range(nseg):                            # fan around the apex (outward = downward side)
        t.append((0, first[(s + 1) % nseg], first[s]))
    for a_ring, b_ring in zip(ring_idx[:-1], ring_idx[1:]):
        for s in range(nseg):
            a0, a1 = a_ring[s], a_ring[(s + 1) % nseg]
            b0, b1 = b_ring[s], b_ring[(s + 1) % nseg]
            t.append((a0, a1, b1))
            t.append((a0, b1, b0))
    last = ring_idx[-1]
    for s in range(nseg):                            # top cap fan
        t.append((top, last[s], last[(s + 1) % nseg]))
    return np.array(verts), np.array(t, dtype=np.int32)


# ---------------------------------------------------------------------------
# advection inputs: a density on cell centres, face-normal velocities on the
# face centres of each axis (face arrays in numpy order, the axis of the
# faces extended by one), a time step from a CFL number on the cell size
# ---------------------------------------------------------------------------

def face_centres(dim, n, h, lo, d):
    """Coordinate arrays (x, y[, z]) of the centres of the faces normal to d."""
    off = tuple(0.0 if e == d else 0.5 for e in range(dim))
    m = tuple(n[e] + (1 if e == d else 0) for e in range(dim))
    axes = []
    for e in range(dim):
        v = lo[e] + (np.arange(m[e]) + off[e]) * h
        shape = [1] * dim
        shape[dim - 1 - e] = m[e]
        axes.append(v.reshape(shape))
    full = tuple(reversed(m))
    return tuple(np.broadcast_to(a, full) for a in axes)


def velocity_uniform(dim, n, h, lo, v):
    return [np.full(face_centres(dim, n, h, lo, d)[0].shape, float(v[d])) for d in range(dim)]


def velocity_rotation(dim, n, h, lo, omega, centre):
    """Rigid rotation about the z axis through centre (in the x-y plane),
    sampled as face-normal components at face centres (discretely
    divergence-free: u_x depends on y only, u_y on x only)."""
    out = []
    for d in range(dim):
        X = face_centres(dim, n, h, lo, d)
        if d == 0:
            out.append(np.ascontiguousarray(-omega * (X[1] - centre[1])))
        elif d == 1:
            out.append(np.ascontiguousarray(omega * (X[0] - centre[0])))
        else:
            out.append(np.zeros(X[0].shape))
    return out


def gaussian_density(prob, centre, width):
    X = prob.cell_centres()
    r2 = sum((np.broadcast_to(X[d], prob.shape) - centre[d]) ** 2 for d in range(prob.dim))
    return np.ascontiguousarray(np.exp(-r2 / (2.0 * width * width)))


def advection_pin_plane(n=128, seed=0):
    """Advection on the gas phase of the pin-plane gap: a density blob near
    the pin tip carried by a rigid rotation about the pin axis plus a
    downward drift (electrons drifting towards the plane), CFL 0.5."""
    pr = pin_plane(n, seed=seed)
    h = pr.h
    rng = np.random.default_rng(seed)
    c = (0.5 + rng.uniform(0.05, 0.1), 0.5, 0.5)
    n0 = gaussian_density(pr, c, 0.05)
    u = velocity_rotation(3, pr.n, h, pr.lo, 2.0, (0.5, 0.5))
    u[2] = np.full(u[2].shape, -0.4)
    vmax = max(float(np.abs(x).max()) for x in u)
    dt = 0.5 * h / vmax
    return pr, n0, u, dt


# --------------------------------------------------------------------------
# nested AMR hierarchies (one box per level, refinement ratio 2)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class AmrLevel:
    """One box of a nested hierarchy: ``prob`` is the box (level 0 the whole
    domain; a box of level l >= 1 one patch) with the domain's boundary
    conditions on faces that lie on the domain boundary and homogeneous
    Dirichlet on coarse-fine faces (flags ``cf``); ``lo`` is the box's first
    cell in its level's global index space (domain cells times 2^level);
    ``parent`` the index of the level - 1 box that contains it (-1 for the
    domain)."""
    prob: Problem
    lo: tuple
    cf: list
    level: int = 0
    parent: int = -1


@dataclasses.dataclass
class AmrProblem:
    levels: List[AmrLevel]
    name: str = ""

    @property
    def dim(self):
        return self.levels[0].prob.dim


def amr_hierarchy(dim, n0, h0, lo0, boxes, sample, bc_kind, bc_value, robin_a1=None, robin_a2=None, name="",
                  **coef):
    """Nested hierarchy over the domain box (n0 cells of size h0 from lo0).
    ``boxes`` lists the patches in that level's global cell indices (even
    corners, inside a box of the next coarser level): (lo, n) entries are one
    box per level, levels 1, 2, ... in order; (level, lo, n) entries name
    their level (several boxes per level). ``sample(n, h, lo)`` returns
    (objects, rho) of a box: its node-sampled level sets and cell-centred
    source."""
    robin_a1 = robin_a1 or [0.0] * 6
    robin_a2 = robin_a2 or [1.0] * 6
    levels = []
    spec = [(0, tuple([0] * dim), tuple(n0))]
    for k, b in enumerate(boxes):
        spec.append((k + 1, tuple(b[0]), tuple(b[1])) if len(b) == 2 else (int(b[0]), tuple(b[1]), tuple(b[2])))
    for lev, lo, n in spec:
        parent = -1
        for q, o in enumerate(levels):
            if o.level == lev - 1 and all(o.lo[d] <= lo[d] // 2 and (lo[d] + n[d]) // 2 <= o.lo[d] + o.prob.n[d]
                                          for d in range(dim)):
                parent = q
                break
        if lev > 0 and parent < 0:
            raise ValueError(f"box {lo} {n} of level {lev} lies in no box of level {lev - 1}")
        l = lev
        h = h0 / (2 ** l)
        full = tuple(m * 2 ** l for m in n0)
        blo = tuple(lo0[d] + lo[d] * h for d in range(dim))
        cf = [False] * 6
        kind, val = list(bc_kind), list(bc_value)
        for d in range(dim):
            for side in (0, 1):
                f = 2 * d + side
                on_domain = (lo[d] == 0) if side == 0 else (lo[d] + n[d] == full[d])
                if not on_domain:
                    cf[f] = True
                    kind[f] = BC_DIRICHLET
                    val[f] = 0.0
        objs, rho = sample(n, h, blo)
        p = Problem(dim, n, h, blo, objs, kind, val, list(robin_a1), list(robin_a2),
                    rho=None if rho is None else np.ascontiguousarray(rho), name=f"{name}-L{l}-{len(levels)}",
                    **coef)
        levels.append(AmrLevel(p, lo, cf, level=lev, parent=parent))
    return AmrProblem(levels, name)


def amr_pin_plane(n0=64, nlev=3, seed=0, r_pin=0.02, nblob=8):
    """The pin-plane gap (pin electrode at 1 with its apex at z = 0.6, eps = 4
    slab below z = 0.2, Neumann x/y faces, Dirichlet 0 / 1 at z-/z+, eight
    Gaussian space-charge blobs) on an n0^3 base grid refined twice around the
    pin: level 1 covers x, y in [0.375, 0.625], z in [0.5, 1] (reaching the
    top face, where the pin meets it), level 2 x, y in [0.4375, 0.5625],
    z in [0.5625, 1]. The finest cells near the tip are those of a uniform
    (4 n0)^3 grid."""
    rng = np.random.default_rng(seed)
    dists = [lambda c: _pin_distance_point(c, r=r_pin), lambda c: c[2] - 0.2]
    cs, ss = _blobs3(rng, nblob, dists)

    def sample(n, h, lo):
        Xn = _nodes(3, n, h, lo)
        objs = [Obj(OBJ_ELECTRODE, 1.0, np.ascontiguousarray(sdf_pin3(Xn, (0.5, 0.5), 0.6, r_pin))),
                Obj(OBJ_DIELECTRIC, 4.0, np.ascontiguousarray(sdf_halfspace_below(Xn[2], 0.2)))]
        X = _centres(3, n, h, lo)
        rho = np.zeros(X[0].shape)
        for c, s in zip(cs, ss):
            rho += np.exp(-((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2 + (X[2] - c[2]) ** 2) / (2 * s * s))
        return objs, rho

    def frac_box(l, xlo, xhi, zlo, zhi):
        m = n0 * 2 ** l
        lo = (int(round(xlo * m)), int(round(xlo * m)), int(round(zlo * m)))
        hi = (int(round(xhi * m)), int(round(xhi * m)), int(round(zhi * m)))
        return lo, tuple(hi[d] - lo[d] for d in range(3))

    boxes = [frac_box(1, 0.375, 0.625, 0.5, 1.0), frac_box(2, 0.4375, 0.5625, 0.5625, 1.0)][:nlev - 1]
    kind = [BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_NEUMANN, BC_DIRICHLET, BC_DIRICHLET]
    val = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    return amr_hierarchy(3, (n0,) * 3, 1.0 / n0, (0.0,) * 3, boxes, sample, kind, val,
                         name=f"amr-pin-plane-{n0}-{nlev}")


def amr_plain(dim, n0, boxes, bc=BC_DIRICHLET, rho_fn=None, **coef):
    """A hierarchy over the unit box with no embedded objects (for the
    operator's exactness and conservation pins); rho_fn(X) gives the source
    at cell centres (None: no source)."""
    def sample(n, h, lo):
        X = _centres(dim, n, h, lo)
        return [], (None if rho_fn is None else rho_fn(X))
    k, v, a1, a2 = _bc(bc, 0.0)
    return amr_hierarchy(dim, (n0,) * dim, 1.0 / n0, (0.0,) * dim, boxes, sample, k, v, a1, a2,
                         name=f"amr-plain-{dim}d-{n0}", **coef)
