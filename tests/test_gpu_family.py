"""A family of Helmholtz operators on one resident hierarchy (the three
photoionization groups and the two TGA diffusion operators of one time step)
through the C ABI: each member against the oracle's own solution of that
member (FP64 within 1e-10, mixed within 1e-8, residual certified by the
oracle's operator at the 1e-10 stopping tolerance), the structure held once,
and each member's result the same (bitwise) alone, with the others, and
solved concurrently."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.operator import assemble
from oracle.solvers import solve_splu, rel_residual

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


def _t(a):
    return torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device=DEV)


def _solve(F, probs, rtol, which=None):
    K = len(probs)
    which = range(K) if which is None else which
    rho = [_t(p.rho) if k in which else None for k, p in enumerate(probs)]
    phi = [torch.zeros(F.N, dtype=torch.float64, device=DEV) for _ in probs]
    phi2 = [torch.zeros(max(1, F.N2), dtype=torch.float64, device=DEV) for _ in probs] if F.N2 else None
    torch.cuda.synchronize()
    st, sts, infos = F.solve(rho, phi, phi2=phi2, rtol=rtol, max_cycles=600, check=False)
    xs = [np.concatenate([phi[k].cpu().numpy(), phi2[k].cpu().numpy()[:F.N2] if F.N2 else np.zeros(0)])
          for k in range(K)]
    return st, sts, infos, xs


FAMILIES = {
    "photoionization-tga 32^3": lambda: W.photoionization_family(32, seed=1),
    "two-disks shifted 64^2": lambda: _two_disk_shifts(64),
}


def _two_disk_shifts(n):
    """Poisson and two shifted operators on the two-disk geometry (two
    phases): alpha a phi + beta div(b grad phi) with a = 0, 10, 1000."""
    base = W.two_disks(n, seed=2, sigma_std=0.0)
    out = []
    for a in (0.0, 10.0, 1000.0):
        p = W.two_disks(n, seed=2, sigma_std=0.0)
        p.alpha, p.a_gas, p.a_diel = (1.0 if a else 0.0), a, a
        p.rho = base.rho
        out.append(p)
    return out


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-8)])
@pytest.mark.parametrize("name", sorted(FAMILIES))
def test_family_members_match_oracle(ctx, name, prec, tol):
    probs = FAMILIES[name]()
    F = ebmg.Family(ctx, probs, precision=prec)
    _say(name, "precision", prec, "members", F.nmem, "device bytes", F.device_bytes, "shared", F.shared_bytes)
    assert F.nmem == len(probs)
    assert F.shared_bytes > 0
    for rtol in (1e-10, 1e-13):
        st, sts, infos, xs = _solve(F, probs, rtol)
        for k, pr in enumerate(probs):
            S = assemble(pr)
            rr = rel_residual(S.A, S.b, xs[k])
            if rtol == 1e-10:
                assert sts[k] == ebmg.OK, (k, sts[k])
                _say("   member", k, "cycles", infos[k]["cycles"], "oracle residual", rr)
                assert rr <= 1.01e-10
            else:
                assert sts[k] in (ebmg.OK, ebmg.ERR_NOCONV)
                ref = solve_splu(S.A, S.b)
                err = np.linalg.norm(xs[k] - ref) / np.linalg.norm(ref)
                _say("   member", k, "error vs oracle", err)
                assert err <= tol
    F.release()


@pytest.mark.parametrize("prec", [0, 1])
def test_family_result_independent_of_the_mix(ctx, prec):
    probs = W.photoionization_family(32, seed=4)
    F = ebmg.Family(ctx, probs, precision=prec)
    _, _, _, first = _solve(F, probs, 1e-10)          # sequential (first call)
    _, _, _, again = _solve(F, probs, 1e-10)          # concurrent members
    for k in range(len(probs)):
        assert np.array_equal(first[k], again[k]), k
        st, sts, _, alone = _solve(F, probs, 1e-10, which=[k])
        assert st == ebmg.OK
        assert np.array_equal(alone[k], first[k]), k
        assert all(not alone[j].any() for j in range(len(probs)) if j != k)   # others untouched (zeros)
    F.release()


def test_family_solve_argument_errors(ctx):
    probs = W.photoionization_family(16, seed=0)
    F = ebmg.Family(ctx, probs)
    phi = [torch.zeros(F.N, dtype=torch.float64, device=DEV) for _ in probs]
    with pytest.raises(ebmg.EbmgError) as e:       # one list entry per member
        F.solve([_t(probs[0].rho)], phi[:1])
    assert e.value.status == ebmg.ERR_ARG
    rho = [_t(p.rho) for p in probs]
    rho[2] = torch.zeros(F.N, dtype=torch.float32, device=DEV)
    with pytest.raises(ebmg.EbmgError) as e:       # a float32 source
        F.solve(rho, phi)
    assert e.value.status == ebmg.ERR_ARG
    F.release()
