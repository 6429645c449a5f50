"""Replayed HIP graphs against direct launches.

Each Krylov iteration / refinement cycle (and each batched iteration) is
captured once as a graph and replayed; with graphs switched off the same
kernels run in the same order, so the solutions must agree bitwise. Every
replay is checked, with other eager work and synchronisations between the
replays, and across a coefficient change (which drops the captured graphs)
and a change of the stopping parameters (which recaptures the batched one).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ebmg = pytest.importorskip("paper_1809_03745_amd.ebmg", reason="libebmg.so not built")

DEV = "cuda:0"
# kernel choices fixed without timing, so both problems run the same kernels
PIN = dict(smoother=4, tail=1)


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


def _solve(P, pr, rtol=1e-10):
    phi = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    phi2 = torch.zeros(max(1, P.N2), dtype=torch.float64, device=DEV)
    sig = _t(pr.sigma) if pr.sigma is not None else None
    st, info = P.solve(_t(pr.rho), phi, sigma=sig, phi2=phi2 if P.N2 else None, rtol=rtol, max_cycles=400,
                       check=False)
    assert st == ebmg.OK, info
    torch.cuda.synchronize()
    return np.concatenate([phi.cpu().numpy(), phi2.cpu().numpy()[:P.N2]]), info


CASES = {
    "pin-plane64-mixed-bicgstab": (lambda: W.pin_plane(64, seed=3), ebmg.MIXED),
    "two-disks128-fp64-bicgstab": (lambda: W.two_disks(128, seed=2), ebmg.FP64),
    "sine64-fp64-refinement": (lambda: W.manufactured_sine(64), ebmg.FP64),
    "eddington3d-mixed-refinement": (lambda: W.eddington(3, 32, 5.0, seed=1), ebmg.MIXED),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replays_equal_direct_launches(ctx, name):
    make, prec = CASES[name]
    pr = make()
    Pg = ebmg.Problem(ctx, pr, precision=prec, graphs=0, **PIN)
    Pe = ebmg.Problem(ctx, pr, precision=prec, graphs=1, **PIN)
    ref, info_e = _solve(Pe, pr)
    for rep in range(3):
        x, info_g = _solve(Pg, pr)
        _say(name, "replay", rep, "cycles", info_g["cycles"], "eager cycles", info_e["cycles"])
        assert info_g["cycles"] == info_e["cycles"]
        assert np.array_equal(x, ref), (name, rep)
        # eager work between the replays
        ref2, _ = _solve(Pe, pr)
        assert np.array_equal(ref2, ref)
    Pg.release()
    Pe.release()


def test_graphs_dropped_on_coefficient_change(ctx):
    pr1 = W.eddington(3, 32, 2.0, seed=4)
    pr2 = W.eddington(3, 32, 40.0, seed=4)
    Pg = ebmg.Problem(ctx, pr1, precision=ebmg.MIXED, graphs=0, **PIN)
    Pe = ebmg.Problem(ctx, pr1, precision=ebmg.MIXED, graphs=1, **PIN)
    for pr in (pr1, pr2, pr1):
        Pg.set_coefficients(pr)
        Pe.set_coefficients(pr)
        xg, _ = _solve(Pg, pr)
        xe, _ = _solve(Pe, pr)
        _say("coefficients", pr.name, "max |diff|", float(np.abs(xg - xe).max()))
        assert np.array_equal(xg, xe)
    Pg.release()
    Pe.release()


def test_batched_graph_replays_equal_direct_launches(ctx):
    probs = W.batched_boxes(12, seed=5)
    rho = [_t(p.rho) for p in probs]
    out = {}
    for graphs in (1, 0):
        B = ebmg.Batch(ctx, probs, precision=ebmg.MIXED, graphs=graphs)
        res = []
        for rtol in (1e-10, 1e-10, 1e-8, 1e-10):
            phi = [torch.zeros(int(np.prod(p.shape)), dtype=torch.float64, device=DEV) for p in probs]
            phi2 = [torch.zeros(4096 * 64, dtype=torch.float64, device=DEV) for _ in probs]
            st, infos = B.solve(rho, phi, phi2=phi2, rtol=rtol, max_cycles=400, check=False)
            assert st == ebmg.OK, infos
            torch.cuda.synchronize()
            res.append(([x.cpu().numpy() for x in phi], [i["cycles"] for i in infos]))
        out[graphs] = res
        B.release()
    for k, ((xe, ce), (xg, cg)) in enumerate(zip(out[1], out[0])):
        _say("batched solve", k, "cycles", cg)
        assert ce == cg
        for a, b in zip(xe, xg):
            assert np.array_equal(a, b), k


def test_in_solve_kernel_timing_runs_the_same_kernels(ctx):
    pr = W.pin_plane(64, seed=3)
    P = ebmg.Problem(ctx, pr, precision=ebmg.MIXED, **PIN)
    ref, info = _solve(P, pr)
    P.kernel_timing(0, 0, True)
    P.kernel_timing(1, 0, True)
    x, info2 = _solve(P, pr)
    n, ms, by = P.kernel_timing(0, 0, False)
    nr, msr, byr = P.kernel_timing(1, 0, False)
    _say("sweeps timed", n, "mean ms", ms, "residuals timed", nr, "mean ms", msr)
    # direct launches with events between them: the same kernels, the same bits
    assert info2["cycles"] == info["cycles"]
    assert np.array_equal(x, ref)
    # one fused sweep launch per smoothing sweep on the finest level, except
    # the first of a V-cycle when the z-marching sweep takes it from x = 0;
    # two colour-phase launches per sweep where the level uses those
    var = P.tuning(0)[0]
    if 2 <= var < ebmg.OOP_VARIANT:
        assert n == info["cycles"] * 3 and by == P.N * 13
    else:
        assert var == ebmg.OOP_VARIANT
        assert n == info["cycles"] * 8 and by == (P.N + 1) // 2 * 13
    assert ms > 0
    assert nr >= 1 and msr > 0 and byr == P.N * 25
    with pytest.raises(ebmg.EbmgError):
        P.kernel_timing(0, 0, False)
    # graphs again after the timing
    x3, _ = _solve(P, pr)
    assert np.array_equal(x3, ref)
    P.release()
