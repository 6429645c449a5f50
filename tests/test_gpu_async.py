"""Submitted (asynchronous) solves against blocking ones.

A submitted solve runs the same kernels as ``ebmg_solve`` on the same
problem, only on the context's worker thread, so its solution must equal the
blocking one bitwise, whatever else is queued on the context or runs on
another context's stream at the same time.
"""
import sys
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ebmg = pytest.importorskip("paper_1809_03745_amd.ebmg", reason="libebmg.so not built")

DEV = "cuda:0"
PIN = dict(smoother=4, tail=1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    a, b = ebmg.Context(0), ebmg.Context(0)
    yield a, b
    a.close()
    b.close()


def _bufs(P, guess=None):
    phi = torch.zeros(P.N, dtype=torch.float64, device=DEV) if guess is None else guess.clone()
    phi2 = torch.zeros(max(1, P.N2), dtype=torch.float64, device=DEV) if P.N2 else None
    return phi, phi2


def _host(phi, phi2, n2):
    h = phi.cpu().numpy()
    return np.concatenate([h, phi2.cpu().numpy()[:n2]]) if n2 else h


def _blocking(P, pr, rtol=1e-10, **kw):
    phi, phi2 = _bufs(P)
    sig = _t(pr.sigma) if pr.sigma is not None else None
    st, info = P.solve(_t(pr.rho), phi, sigma=sig, phi2=phi2, rtol=rtol, max_cycles=400, check=False, **kw)
    assert st == ebmg.OK, info
    torch.cuda.synchronize()
    return _host(phi, phi2, P.N2), info


def test_submitted_solves_equal_blocking_on_two_contexts(ctxs):
    c1, c2 = ctxs
    pr1 = W.pin_plane(64, seed=3)
    pr2 = W.two_disks(128, seed=2)
    P1 = ebmg.Problem(c1, pr1, precision=ebmg.MIXED, **PIN)
    P2 = ebmg.Problem(c2, pr2, precision=ebmg.FP64, **PIN)
    ref1, i1 = _blocking(P1, pr1)
    ref2, i2 = _blocking(P2, pr2)
    jobs = []
    for rep in range(3):
        for c, P, pr, ref, inf in ((c1, P1, pr1, ref1, i1), (c2, P2, pr2, ref2, i2)):
            b = _bufs(P)
            sig = _t(pr.sigma) if pr.sigma is not None else None
            t = P.submit(_t(pr.rho), b[0], sigma=sig, phi2=b[1], rtol=1e-10, max_cycles=400)
            jobs.append((c, P, t, b, ref, inf))
    _say("submitted", len(jobs), "solves on two contexts")
    pending = list(jobs)
    t0 = time.perf_counter()
    while pending and time.perf_counter() - t0 < 60:
        for j in list(pending):
            r = j[0].poll(j[2])
            if r is not None:
                st, info = r
                _say("ticket", j[2], "status", st, "cycles", info["cycles"])
                assert st == ebmg.OK
                assert info["cycles"] == j[5]["cycles"]
                pending.remove(j)
        time.sleep(0.002)
    assert not pending, "submitted solves did not finish within 60 s"
    torch.cuda.synchronize()
    for c, P, t, (phi, phi2), ref, _ in jobs:
        assert np.array_equal(_host(phi, phi2, P.N2), ref), t
        with pytest.raises(ebmg.EbmgError):  # collected already
            c.poll(t)
    assert not c1._held and not c2._held
    P1.release()
    P2.release()


def test_boundary_values_copied_at_submit(ctxs):
    c1, _ = ctxs
    pr = W.pin_plane(64, seed=5)
    P = ebmg.Problem(c1, pr, precision=ebmg.FP64, **PIN)
    bcv = np.array(pr.bc_value, dtype=np.float64) * 0.5 + 0.25
    ref, _ = _blocking(P, pr, bc_values=bcv)
    phi, phi2 = _bufs(P)
    t = P.submit(_t(pr.rho), phi, phi2=phi2, rtol=1e-10, max_cycles=400, bc_values=bcv)
    bcv[:] = 123.0  # the queued solve must not see this
    st, info = c1.wait(t)
    assert st == ebmg.OK, info
    torch.cuda.synchronize()
    assert np.array_equal(_host(phi, phi2, P.N2), ref)
    P.release()


def test_blocking_calls_wait_for_submitted_ones(ctxs):
    c1, _ = ctxs
    pr = W.manufactured_sine(64)
    P = ebmg.Problem(c1, pr, precision=ebmg.FP64, **PIN)
    ref, _ = _blocking(P, pr)
    rho = _t(pr.rho)
    bufs = [_bufs(P) for _ in range(4)]
    tickets = [P.submit(rho, b[0], phi2=b[1], rtol=1e-10, max_cycles=400) for b in bufs]
    # a blocking solve on the same problem runs after the queued ones
    x, _ = _blocking(P, pr)
    assert np.array_equal(x, ref)
    for t, b in zip(tickets, bufs):
        r = c1.poll(t)
        assert r is not None and r[0] == ebmg.OK  # finished before the blocking solve started
        assert np.array_equal(_host(b[0], b[1], P.N2), ref)
    # release with a queued solve: it completes first, and its ticket stays collectable
    phi, phi2 = _bufs(P)
    t = P.submit(rho, phi, phi2=phi2, rtol=1e-10, max_cycles=400)
    P.release()
    st, _ = c1.wait(t)
    assert st == ebmg.OK
    assert np.array_equal(_host(phi, phi2, 0), ref)


def test_failed_submitted_solve_reports_its_status(ctxs):
    _, c2 = ctxs
    pr = W.two_disks(128, seed=4)
    P = ebmg.Problem(c2, pr, precision=ebmg.FP64, **PIN)
    phi, phi2 = _bufs(P)
    t = P.submit(_t(pr.rho), phi, phi2=phi2, rtol=1e-14, max_cycles=1)
    st, info = c2.wait(t)
    _say("max_cycles=1:", ebmg.STATUS_NAMES[st], info["cycles"], info["rel_residual"])
    assert st == ebmg.ERR_NOCONV
    assert info["cycles"] <= 1 and info["rel_residual"] > 1e-14
    # the context stays usable
    x, _ = _blocking(P, pr)
    assert np.isfinite(x).all()
    P.release()


def test_release_and_close_run_queued_solves(ctxs):
    pr = W.pin_plane(64, seed=3)
    c = ebmg.Context(0)
    P = ebmg.Problem(c, pr, precision=ebmg.MIXED, **PIN)
    ref, _ = _blocking(P, pr)
    rho = _t(pr.rho)
    bufs = [_bufs(P) for _ in range(3)]
    for b in bufs:
        P.submit(rho, b[0], phi2=b[1], rtol=1e-10, max_cycles=400)
    P.release()
    c.close()
    torch.cuda.synchronize()
    for b in bufs:
        assert np.array_equal(_host(b[0], b[1], P.N2), ref)


def test_problem_outlives_its_context_handle():
    pr = W.manufactured_sine(64)
    c = ebmg.Context(0)
    P = ebmg.Problem(c, pr, precision=ebmg.FP64, **PIN)
    ref, _ = _blocking(P, pr)
    c.close()  # the stream stays until P is released
    x, _ = _blocking(P, pr)
    assert np.array_equal(x, ref)
    P.release()
