"""GPU parity of the batched persistent solver (many independent boxes, one
launch) against the FP64 oracle and against the single-box path.

Bars as for one box: FP64 within 1e-10 relative L2 of the oracle's direct
solution, mixed within 1e-8, residual <= 1e-10 by the oracle's operator. A
box's result must not depend on the other boxes in the batch (bitwise).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.operator import assemble
from oracle.solvers import rel_residual, solve_splu

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


def _batch_solve(B, probs, rtol, max_cycles=400):
    rho = [_t(p.rho) for p in probs]
    sig = [(_t(p.sigma) if p.sigma is not None else None) for p in probs]
    phi = [torch.zeros(int(np.prod(p.shape)), dtype=torch.float64, device=DEV) for p in probs]
    phi2 = [torch.zeros(4096 * 64, dtype=torch.float64, device=DEV) for _ in probs]
    torch.cuda.synchronize()
    st, infos = B.solve(rho, phi, sigma=sig, phi2=phi2, rtol=rtol, max_cycles=max_cycles, check=False)
    return st, infos, [p.cpu().numpy() for p in phi], [q.cpu().numpy() for q in phi2]


def _full(x, x2, N2):
    return np.concatenate([x, x2[:N2]])


def _n2(ctx, pr):
    P = ebmg.Problem(ctx, pr)
    n2 = P.N2
    P.release()
    return n2


# 3D boxes of the batched workload (random sizes 16..64 per edge, sphere
# electrode, dielectric half-space): the four smallest of a seeded draw go to
# the oracle, the rest to the single-box library path.
BOXES = W.batched_boxes(16, seed=11)
ORACLE_IDX = [12, 2, 11, 0]


MODES = [ebmg.BATCH_LEVELSYNC, ebmg.BATCH_PERSISTENT]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_3d_vs_oracle(ctx, prec, mode):
    _say("batch 3d vs oracle, precision", prec, "mode", mode)
    B = ebmg.Batch(ctx, BOXES, precision=prec, batch=mode)
    assert B.cells == sum(int(np.prod(p.shape)) for p in BOXES)
    st, infos, xs, x2s = _batch_solve(B, BOXES, 1e-10)
    assert st == ebmg.OK, infos
    for i in range(len(BOXES)):
        assert infos[i]["rel_residual"] <= 1e-10, (i, infos[i])
    st, infos13, xs13, x2s13 = _batch_solve(B, BOXES, 1e-13)
    assert st == ebmg.OK
    for i in ORACLE_IDX:
        pr = BOXES[i]
        S = assemble(pr)
        N2 = S.N2
        x = _full(xs[i], x2s[i], N2)
        assert rel_residual(S.A, S.b, x) <= 1.01e-10, i
        ref = solve_splu(S.A, S.b)
        x13 = _full(xs13[i], x2s13[i], N2)
        err = np.linalg.norm(x13 - ref) / np.linalg.norm(ref)
        _say("   box", i, pr.shape, "error vs oracle", err, "cycles", infos13[i]["cycles"])
        assert err <= (1e-10 if prec == 0 else 1e-8)
    B.release()


@pytest.mark.parametrize("mode", MODES)
def test_batch_3d_vs_single_box(ctx, mode):
    _say("batch 3d vs single-box path, mode", mode)
    B = ebmg.Batch(ctx, BOXES, batch=mode)
    st, infos, xs, x2s = _batch_solve(B, BOXES, 1e-13)
    assert st == ebmg.OK
    for i, pr in enumerate(BOXES):
        if i in ORACLE_IDX:
            continue
        P = ebmg.Problem(ctx, pr)
        phi = torch.zeros(P.N, dtype=torch.float64, device=DEV)
        phi2 = torch.zeros(max(1, P.N2), dtype=torch.float64, device=DEV)
        st1, info = P.solve(_t(pr.rho), phi, phi2=phi2 if P.N2 else None, rtol=1e-13, max_cycles=400, check=False)
        assert st1 == ebmg.OK
        a = _full(xs[i], x2s[i], P.N2)
        b = _full(phi.cpu().numpy(), phi2.cpu().numpy(), P.N2)
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b), i
        P.release()
    B.release()


@pytest.mark.parametrize("mode", MODES)
def test_batch_2d_mixed_kinds(ctx, mode):
    """A 2D batch mixing Poisson with surface charge, blade-plane with a
    dielectric and an Eddington Helmholtz box with Robin faces (plain
    V-cycle refinement and BiCGStab boxes side by side)."""
    _say("batch 2d mixed kinds, mode", mode)
    probs = [W.two_disks(64, seed=3), W.blade_plane(96, seed=4), W.eddington(2, 64, 10.0, seed=5),
             W.coaxial(48, sigma=0.5), W.manufactured_sine(32)]
    for prec, bar in ((0, 1e-10), (1, 1e-8)):
        B = ebmg.Batch(ctx, probs, precision=prec, batch=mode)
        st, infos, xs, x2s = _batch_solve(B, probs, 1e-13, max_cycles=600)
        assert st == ebmg.OK, infos
        for i, pr in enumerate(probs):
            S = assemble(pr)
            ref = solve_splu(S.A, S.b)
            x = _full(xs[i], x2s[i], S.N2)
            err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
            _say("   ", pr.name, "precision", prec, "error", err)
            assert err <= bar
        B.release()


@pytest.mark.parametrize("mode", MODES)
def test_batch_result_independent_of_mix(ctx, mode):
    _say("batch mix invariance, mode", mode)
    probs = BOXES[:8]
    B = ebmg.Batch(ctx, probs, precision=ebmg.MIXED, batch=mode)
    _, _, xs, _ = _batch_solve(B, probs, 1e-10)
    B.release()
    for i in (1, 5):
        Bi = ebmg.Batch(ctx, [probs[i]], precision=ebmg.MIXED, batch=mode)
        _, _, xi, _ = _batch_solve(Bi, [probs[i]], 1e-10)
        assert np.array_equal(xi[0], xs[i])
        Bi.release()
    # and a reordered batch
    perm = [7, 3, 0, 5, 1, 6, 2, 4]
    Bp = ebmg.Batch(ctx, [probs[k] for k in perm], precision=ebmg.MIXED, batch=mode)
    _, _, xp, _ = _batch_solve(Bp, [probs[k] for k in perm], 1e-10)
    for j, k in enumerate(perm):
        assert np.array_equal(xp[j], xs[k])
    Bp.release()


@pytest.mark.parametrize("mode", MODES)
def test_batch_errors(ctx, mode):
    _say("batch error paths, mode", mode)
    probs = BOXES[:3]
    B = ebmg.Batch(ctx, probs, batch=mode)
    st, infos, _, _ = _batch_solve(B, probs, 1e-10, max_cycles=2)
    assert st == ebmg.ERR_NOCONV
    assert all(i["cycles"] <= 2 for i in infos)
    bad = [p for p in probs]
    rho = [_t(p.rho) for p in bad]
    rho[1].fill_(float("nan"))
    phi = [torch.zeros(int(np.prod(p.shape)), dtype=torch.float64, device=DEV) for p in bad]
    phi2 = [torch.zeros(4096 * 64, dtype=torch.float64, device=DEV) for _ in bad]
    st, infos = B.solve(rho, phi, phi2=phi2, rtol=1e-10, max_cycles=100, check=False)
    assert st == ebmg.ERR_NUMERIC
    assert infos[0]["rel_residual"] <= 1e-10 and infos[2]["rel_residual"] <= 1e-10
    B.release()
    with pytest.raises(ebmg.EbmgError):
        ebmg.Batch(ctx, [W.two_disks(32, seed=0), W.pin_plane(16, seed=0)])


def test_batch_levelsync_tuning_and_modes_agree(ctx):
    """The level-synchronous setup reports its coarse-part choice, and both
    batched modes reach the same solution (to the solve tolerance)."""
    _say("batch modes agree")
    probs = BOXES[:6]
    Bw = ebmg.Batch(ctx, probs, precision=ebmg.MIXED, batch=ebmg.BATCH_LEVELSYNC)
    tu = Bw.tuning()
    _say("   tuning", tu)
    assert tu["mode"] == 2 and len(tu["candidates"]) >= 1
    assert tu["tail_cells"] in [c for c, _ in tu["candidates"]]
    st, iw, xw, x2w = _batch_solve(Bw, probs, 1e-12)
    assert st == ebmg.OK
    Bw.release()
    Bp = ebmg.Batch(ctx, probs, precision=ebmg.MIXED, batch=ebmg.BATCH_PERSISTENT)
    assert Bp.tuning()["mode"] == 1
    st, ip, xp, x2p = _batch_solve(Bp, probs, 1e-12)
    assert st == ebmg.OK
    Bp.release()
    for i in range(len(probs)):
        assert np.linalg.norm(xw[i] - xp[i]) <= 1e-9 * np.linalg.norm(xp[i]), i


@pytest.mark.parametrize("tail,cells", [(1, 0), (2, 32768)])
def test_batch_fixed_coarse_part(ctx, tail, cells):
    """A pinned coarse-part rule (options.tail 1 or 2) times nothing: the
    threshold is the rule's, the only candidate, and the solve still meets
    the tolerance (the serving loop relies on this for mix invariance)."""
    _say("batch fixed coarse part", tail)
    probs = BOXES[:4]
    B = ebmg.Batch(ctx, probs, precision=ebmg.MIXED, batch=ebmg.BATCH_LEVELSYNC, tail=tail)
    tu = B.tuning()
    _say("   tuning", tu)
    assert tu["tail_cells"] == cells
    assert [c for c, _ in tu["candidates"]] == [cells]
    st, infos, xs, x2s = _batch_solve(B, probs, 1e-10)
    assert st == ebmg.OK
    assert all(i["rel_residual"] <= 1e-10 for i in infos)
    B.release()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_edge_cases(ctx, mode, prec):
    """A single-level box (its whole system solved by the bottom inverse), a
    box whose coarsest level is too large for an inverse (relaxation bottom),
    an EB box, and a box with a zero right-hand side, all from a nonzero
    initial guess: each result matches the oracle (the zero box gives exactly
    zero)."""
    _say("batch edge cases, precision", prec, "mode", mode)
    zero = W.manufactured_sine(16)
    zero.rho = np.zeros_like(zero.rho)
    probs = [W.manufactured_sine(16), W.manufactured_sine(130), W.two_disks(32, seed=6), zero]
    B = ebmg.Batch(ctx, probs, precision=prec, batch=mode)
    rho = [_t(p.rho) for p in probs]
    sig = [(_t(p.sigma) if p.sigma is not None else None) for p in probs]
    rng = np.random.default_rng(3)
    phi = [_t(rng.normal(size=int(np.prod(p.shape)))) for p in probs]
    phi2 = [torch.zeros(4096, dtype=torch.float64, device=DEV) for _ in probs]
    # 1e-12: the 130^2 box's FP64 round-off floor is a few 1e-13
    st, infos = B.solve(rho, phi, sigma=sig, phi2=phi2, rtol=1e-12, max_cycles=600, check=False)
    assert st == ebmg.OK, infos
    xs = [x.cpu().numpy() for x in phi]
    x2s = [x.cpu().numpy() for x in phi2]
    assert np.all(xs[3] == 0.0) and infos[3]["rel_residual"] == 0.0
    for i in range(3):
        S = assemble(probs[i])
        ref = solve_splu(S.A, S.b)
        x = _full(xs[i], x2s[i], S.N2)
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        _say("   ", probs[i].name, "levels", infos[i]["levels"], "cycles", infos[i]["cycles"], "error", err)
        assert err <= (1e-10 if prec == 0 else 1e-8)
    assert infos[0]["levels"] == 1
    B.release()


def test_batch_level0_timing_hook_leaves_solves_unchanged(ctx):
    """The finest-level timing hook runs the batch's template sweeps and
    explicit-row passes on its cycle vectors; a solve after it gives the
    same result, bitwise, as the one before, and the persistent mode refuses
    the hook."""
    B = ebmg.Batch(ctx, BOXES, precision=1)
    st, infos, xs, x2s = _batch_solve(B, BOXES, 1e-10)
    assert st == ebmg.OK
    for which in (0, 1):
        ms, by = B.time_level0(which, reps=3)
        _say("   level-0 kernels", which, "ms", ms, "bytes", by)
        assert ms > 0 and by > 0
    st2, infos2, xs2, x2s2 = _batch_solve(B, BOXES, 1e-10)
    assert st2 == ebmg.OK
    for a, b in zip(xs, xs2):
        assert np.array_equal(a, b)
    B.release()
    P = ebmg.Batch(ctx, BOXES[:2], batch=ebmg.BATCH_PERSISTENT)
    with pytest.raises(ebmg.EbmgError) as e:
        P.time_level0(0)
    assert e.value.status == ebmg.ERR_ARG
    P.release()
