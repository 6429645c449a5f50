"""The entry point that allocates nothing (ebmg_apply_noalloc) against
ebmg_apply, through the C ABI: two calls in a row, the second on a smaller
problem (so stale scratch contents from the first would show), each equal
to ebmg_apply bit for bit (the same kernels on the same values); a problem
beyond the scratch limit is refused with ERR_ARG and its outputs left as
they were."""
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


def _pair(P, x):
    xt = torch.tensor(x[:P.N], dtype=torch.float64, device=DEV)
    x2 = torch.tensor(x[P.N:], dtype=torch.float64, device=DEV) if P.N2 else None
    return xt, x2


def _outs(P):
    return (torch.full((P.N,), np.nan, dtype=torch.float64, device=DEV),
            torch.full((max(1, P.N2),), np.nan, dtype=torch.float64, device=DEV) if P.N2 else None)


def _host(a, b, n2):
    return np.concatenate([a.cpu().numpy(), b.cpu().numpy()[:n2] if b is not None else np.zeros(0)])


def test_apply_noalloc_matches_apply(ctx):
    rng = np.random.default_rng(12)
    for name, make in (("pin-plane 64^3", lambda: W.pin_plane(64, seed=3)),
                       ("two-disks 128^2", lambda: W.two_disks(128, seed=4))):
        pr = make()
        P = ebmg.Problem(ctx, pr)
        _say("apply_noalloc", name, "N", P.N, "N2", P.N2)
        x = rng.normal(size=P.N + P.N2)
        xt, x2 = _pair(P, x)
        o1, o12 = _outs(P)
        o2, o22 = _outs(P)
        torch.cuda.synchronize()
        P.apply(xt, x2, o1, o12)
        P.apply_noalloc(xt, x2, o2, o22)
        torch.cuda.synchronize()
        a = _host(o1, o12, P.N2)
        b = _host(o2, o22, P.N2)
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), (name, np.abs(a - b).max())
        P.release()


def test_apply_noalloc_refuses_beyond_its_scratch(ctx):
    pr = W.manufactured_sine(1100)     # 1,210,000 unknowns > 1,179,648
    P = ebmg.Problem(ctx, pr)
    x = torch.ones(P.N, dtype=torch.float64, device=DEV)
    out = torch.full((P.N,), 7.0, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    with pytest.raises(ebmg.EbmgError) as e:
        P.apply_noalloc(x, None, out, None)
    assert e.value.status == ebmg.ERR_ARG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    P.release()
