"""The smoother kernels against the definition of a red/black Gauss-Seidel
sweep, and against each other.

Every variant (split half-sweeps, fused tile sweep, z-marching sweep in each
tile configuration, one-launch colour phases out of place) must
produce bitwise the same result, and the result must be a red half-sweep
followed by a black half-sweep over the template cells, computed here in
numpy from the level's exported operator rows; explicit-row, covered and
second-phase entries stay untouched.
"""
import sys

import numpy as np
import pytest

import workloads as W

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


def _reference_sweeps(A, tag, n, dim, x, b, sweeps):
    """Red then black half-sweeps over template cells, from the CSR rows."""
    A = A.tocsr()
    N = int(np.prod(n))
    idx = np.arange(N)
    i = idx % n[0]
    j = (idx // n[0]) % n[1]
    k = idx // (n[0] * n[1]) if dim == 3 else 0
    colour = (i + j + k) & 1
    templ = (tag & 3) <= 1
    d = A.diagonal()
    x = x.copy()
    for _ in range(sweeps):
        for c in (0, 1):
            rows = idx[templ & (colour == c)]
            Ar = A[rows]
            off = Ar @ x - d[rows] * x[rows]
            x[rows] = (b[rows] - off) / d[rows]
    return x


CASES = {
    "pin-plane64": lambda: W.pin_plane(64, seed=2),
    "random-box-ragged": lambda: W.random_box(np.random.default_rng(7)),   # 40 x 56 x 48 cells
    "two-disks256": lambda: W.two_disks(256, seed=1),
    "two-disks130": lambda: W.two_disks(130, seed=1),   # level 1 is 65 x 65: odd x extent
    "pin-plane26": lambda: W.pin_plane(26, seed=2),     # level 1 is 13^3: odd x extent
}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_smoother_variants(ctx, name, prec):
    pr = CASES[name]()
    P = ebmg.Problem(ctx, pr, precision=prec)
    rng = np.random.default_rng(7)
    for level in range(min(2, P.levels)):
        n, n2 = P.level_size(level)
        tag, _, _ = P.level_arrays(level)
        shape = [pr.n[d] >> level for d in range(pr.dim)]
        if int(np.prod(shape)) != n:
            continue
        x0 = rng.normal(size=n + n2)
        b = rng.normal(size=n + n2)
        variants = list(range(1, ebmg.SMOOTH_OOP + 1)) if pr.dim == 3 else [1, 2, ebmg.SMOOTH_OOP]
        outs = {}
        for v in variants:
            xt = torch.tensor(x0, dtype=torch.float64, device=DEV)
            bt = torch.tensor(b, dtype=torch.float64, device=DEV)
            torch.cuda.synchronize()
            try:
                P.smooth(level, v, 2, xt, bt)
            except ebmg.EbmgError as e:
                assert e.status == ebmg.ERR_ARG and v > 1   # level too small for the fused sweeps
                continue
            outs[v] = xt.cpu().numpy()
        _say(name, "precision", prec, "level", level, "variants run", sorted(outs))
        for v in outs:
            assert np.array_equal(outs[v], outs[1]), (name, level, v)
        y = outs[1]
        keep = np.concatenate([(tag & 3) > 1, np.ones(n2, bool)])
        if prec == 1:
            keep_ref = x0.astype(np.float32).astype(np.float64)
            assert np.array_equal(y[keep], keep_ref[keep])
        else:
            assert np.array_equal(y[keep], x0[keep])
        if prec == 0:
            A = P.operator(level)
            ref = _reference_sweeps(A, tag, shape, pr.dim, x0, b, 2)
            assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    P.release()


def _reference_phases_with_rows(A, tag, n, dim, sec_cell, x, b, sweeps):
    """Colour phases in which every unknown of the phase's colour (template
    cells by their own parity, explicit rows and second-phase unknowns by the
    parity of their cell) is relaxed from the values before the phase."""
    A = A.tocsr()
    N = int(np.prod(n))
    nd = A.shape[0]
    cell = np.concatenate([np.arange(N), np.asarray(sec_cell, dtype=np.int64)])
    i = cell % n[0]
    j = (cell // n[0]) % n[1]
    k = cell // (n[0] * n[1]) if dim == 3 else 0
    colour = (i + j + k) & 1
    active = np.concatenate([(tag & 3) != 3, np.ones(nd - N, bool)])
    d = A.diagonal()
    x = x.copy()
    for _ in range(sweeps):
        for c in (0, 1):
            rows = np.nonzero(active & (colour == c))[0]
            off = A[rows] @ x - d[rows] * x[rows]
            x[rows] = (b[rows] - off) / d[rows]
    return x


@pytest.mark.parametrize("name", ["two-disks130", "pin-plane26", "random-box-ragged"])
def test_colour_phases_with_rows(ctx, name):
    """The one-launch colour phases as the solver runs them on its small
    levels (explicit rows included) against the numpy definition built from
    the exported level operator, FP64."""
    pr = CASES[name]()
    P = ebmg.Problem(ctx, pr, precision=0)
    rng = np.random.default_rng(3)
    checked = 0
    for level in range(P.levels):
        n, n2 = P.level_size(level)
        tag, _, sec = P.level_arrays(level)
        shape = [max(1, pr.n[d] >> level) for d in range(pr.dim)]
        if int(np.prod(shape)) != n or not ((tag & 3) == 2).any():
            continue
        x0 = rng.normal(size=n + n2)
        b = rng.normal(size=n + n2)
        xt = torch.tensor(x0, dtype=torch.float64, device=DEV)
        bt = torch.tensor(b, dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        try:
            P.smooth(level, ebmg.SMOOTH_OOP_ROWS, 2, xt, bt)
        except ebmg.EbmgError as e:
            assert e.status == ebmg.ERR_ARG
            continue
        y = xt.cpu().numpy()
        ref = _reference_phases_with_rows(P.operator(level), tag, shape, pr.dim, sec, x0, b, 2)
        _say(name, "level", level, "rows", int(((tag & 3) == 2).sum()) + n2, "max diff", np.abs(y - ref).max())
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
        checked += 1
    assert checked >= 1
    P.release()


def _reference_fused_with_rows(A, tag, n, dim, sec_cell, x, b, sweeps):
    """Per sweep: red then black half-sweeps over the template cells, then a
    Jacobi pass over the explicit rows (cut-cell and second-phase unknowns) of
    red cells, then one over those of black cells (seeing the red rows' new
    values) -- the smoothing step of levels that use a fused sweep."""
    A = A.tocsr()
    N = int(np.prod(n))
    nd = A.shape[0]
    cell = np.concatenate([np.arange(N), np.asarray(sec_cell, dtype=np.int64)])
    i = cell % n[0]
    j = (cell // n[0]) % n[1]
    k = cell // (n[0] * n[1]) if dim == 3 else 0
    colour = (i + j + k) & 1
    templ = np.concatenate([(tag & 3) <= 1, np.zeros(nd - N, bool)])
    expl = np.concatenate([(tag & 3) == 2, np.ones(nd - N, bool)])
    d = A.diagonal()
    x = x.copy()
    for _ in range(sweeps):
        for group in (templ, expl):
            for c in (0, 1):
                rows = np.nonzero(group & (colour == c))[0]
                off = A[rows] @ x - d[rows] * x[rows]
                x[rows] = (b[rows] - off) / d[rows]
    return x


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", ["pin-plane64", "random-box-ragged", "two-disks256"])
def test_fused_sweeps_with_rows(ctx, name, prec):
    """The fused sweep followed by the explicit rows' Jacobi passes, as the
    solver smooths its large levels, against the numpy definition built from
    the exported level operator (FP64 to 1e-12; the FP32 sweep to FP32
    rounding of the same)."""
    pr = CASES[name]()
    P = ebmg.Problem(ctx, pr, precision=prec)
    rng = np.random.default_rng(11)
    checked = 0
    for level in range(min(2, P.levels)):
        n, n2 = P.level_size(level)
        tag, _, sec = P.level_arrays(level)
        shape = [max(1, pr.n[d] >> level) for d in range(pr.dim)]
        if int(np.prod(shape)) != n or not ((tag & 3) == 2).any():
            continue
        x0 = rng.normal(size=n + n2)
        b = rng.normal(size=n + n2)
        xt = torch.tensor(x0, dtype=torch.float64, device=DEV)
        bt = torch.tensor(b, dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        try:
            P.smooth(level, ebmg.SMOOTH_FUSED_ROWS, 2, xt, bt)
        except ebmg.EbmgError as e:
            assert e.status == ebmg.ERR_ARG   # level too small for a fused sweep
            continue
        y = xt.cpu().numpy()
        ref = _reference_fused_with_rows(P.operator(level), tag, shape, pr.dim, sec, x0, b, 2)
        err = np.abs(y - ref).max() / np.abs(ref).max()
        _say(name, "precision", prec, "level", level, "rows", int(((tag & 3) == 2).sum()) + n2, "max rel diff", err)
        assert err <= (1e-12 if prec == 0 else 2e-5)
        checked += 1
    assert checked >= 1
    P.release()
