"""The V-cycle's residual restriction (ebmg_restrict_residual) against its
definition built from the exported level operator: the fine residual
r = b - A x, and for every simple coarse cell the mean of its 2^D children's
residuals; covered coarse cells hold 0. The solver's own kernels (the fused
z-marching kernel in its quad or pair form on large 3D levels), the fused
pair kernel and the separate residual and restriction kernels agree
bitwise."""
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


CASES = {
    "pin-plane64": lambda: W.pin_plane(64, seed=2),     # x extent a multiple of 4: quad form
    "pin-plane66": lambda: W.pin_plane(66, seed=2),     # even, not a multiple of 4: pair form
    "random-box-ragged": lambda: W.random_box(np.random.default_rng(7)),   # 40 x 56 x 48: separate kernels
    "two-disks256": lambda: W.two_disks(256, seed=1),   # 2D
}


def _restricted(r, ctag, fshape, cshape, dim):
    """Mean of the children's residuals per coarse cell (NaN where the coarse
    cell is not simple)."""
    nc = int(np.prod(cshape))
    fr = r[:int(np.prod(fshape))].reshape(tuple(reversed(fshape)))
    if dim == 3:
        m = fr.reshape(cshape[2], 2, cshape[1], 2, cshape[0], 2).mean(axis=(1, 3, 5))
    else:
        m = fr.reshape(cshape[1], 2, cshape[0], 2).mean(axis=(1, 3))
    out = m.ravel().copy()
    simple = ((ctag[:nc] & 3) != 3) & ((ctag[:nc] & 4) == 0)
    out[~simple] = np.nan
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_restricted_residual(ctx, name, prec):
    pr = CASES[name]()
    P = ebmg.Problem(ctx, pr, precision=prec)
    rng = np.random.default_rng(5)
    checked = 0
    for level in range(min(2, P.levels - 1)):
        n, n2 = P.level_size(level)
        nc, nc2 = P.level_size(level + 1)
        fshape = [pr.n[d] >> level for d in range(pr.dim)]
        cshape = [pr.n[d] >> (level + 1) for d in range(pr.dim)]
        if int(np.prod(fshape)) != n or int(np.prod(cshape)) != nc or any(v % 2 for v in fshape):
            continue
        x0 = rng.normal(size=n + n2)
        b = rng.normal(size=n + n2)
        # covered cells are identity rows held at 0 by the solver (x = b = 0)
        ftag, _, _ = P.level_arrays(level)
        cov_f = np.concatenate([(ftag & 3) == 3, np.zeros(n2, bool)])
        x0[cov_f] = 0.0
        b[cov_f] = 0.0
        outs = {}
        for form in (0, 1, 2):
            xt = torch.tensor(x0, dtype=torch.float64, device=DEV)
            bt = torch.tensor(b, dtype=torch.float64, device=DEV)
            bc = torch.full((nc + nc2,), np.nan, dtype=torch.float64, device=DEV)
            try:
                P.restrict_residual(level, form, xt, bt, bc)
            except ebmg.EbmgError as e:
                assert e.status == ebmg.ERR_ARG and form == 1   # no fused kernel on this level
                continue
            outs[form] = bc.cpu().numpy()
        _say(name, "precision", prec, "level", level, "forms", sorted(outs))
        for form in outs:
            assert np.array_equal(outs[form], outs[0], equal_nan=True), (name, level, form)
        y = outs[0]
        assert np.isfinite(y).all()
        if prec == 0:
            ctag, _, _ = P.level_arrays(level + 1)
            r = b - P.operator(level) @ x0
            ref = _restricted(r, ctag, fshape, cshape, pr.dim)
            ok = np.isfinite(ref)
            assert ok.sum() > 0.5 * nc
            scale = np.abs(ref[ok]).max()
            err = np.abs(y[:nc][ok] - ref[ok]).max() / scale
            _say("   simple coarse cells", int(ok.sum()), "max rel diff", err)
            assert err <= 1e-12
            cov = (ctag[:nc] & 3) == 3
            assert np.all(y[:nc][cov] == 0.0)
        checked += 1
    assert checked >= 1
    P.release()
