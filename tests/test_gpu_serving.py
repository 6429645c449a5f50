"""GPU tests of the serving loop: each served result is bitwise the same alone
and in a concurrent mix, served results meet the parity bar against the
oracle, and admission keeps the footprint within the byte budget."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.operator import assemble
from oracle.solvers import rel_residual, solve_splu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ebmg = pytest.importorskip("paper_1809_03745_amd.ebmg", reason="libebmg.so not built")
from paper_1809_03745_amd import serving  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SPECS = [dict(dim=2, n=128, op="poisson", kappa=1.0, seed=11),
         dict(dim=3, n=32, op="poisson", kappa=1.0, seed=12),
         dict(dim=2, n=128, op="helmholtz", kappa=3.0, seed=13),
         dict(dim=3, n=32, op="helmholtz", kappa=50.0, seed=14),
         dict(dim=2, n=128, op="poisson", kappa=1.0, seed=15),
         dict(dim=3, n=32, op="helmholtz", kappa=7.0, seed=16),
         dict(dim=2, n=256, op="helmholtz", kappa=20.0, seed=17),
         dict(dim=3, n=64, op="poisson", kappa=1.0, seed=18)]


def _serve(specs, slots, budget=None, bytes_per_cell=256, measured=None):
    srv = serving.Server(0, slots=slots, budget_bytes=budget, bytes_per_cell=bytes_per_cell)
    if measured:
        srv.sched.measured.update(measured)
    reqs = [srv.submit(serving.request_from_spec(i, sp)) for i, sp in enumerate(specs)]
    for r in reqs:
        assert r.done.wait(300), "request did not finish"
    out = []
    for r in reqs:
        assert r.status == ebmg.OK, (r.rid, r.status, r.error, r.info)
        out.append(r.phi.cpu().numpy())
    summ = srv.summary(min(r.arrival for r in reqs), max(r.t_end for r in reqs))
    summ["measured"] = dict(srv.sched.measured)
    srv.close()
    return out, reqs, summ


def test_alone_equals_mix():
    _say("serving: alone vs mix")
    alone = []
    for i, sp in enumerate(SPECS):
        phi, reqs, _ = _serve([sp], slots=1)
        alone.append(phi[0])
    mixed, reqs, summ = _serve(SPECS, slots=4)
    _say("   mix summary", summ)
    assert summ["completed"] == len(SPECS)
    # two requests share the 2D Poisson hierarchy, three the 3D Helmholtz one
    assert summ["hierarchy_misses"] <= len(SPECS)
    for i in range(len(SPECS)):
        assert np.array_equal(alone[i], mixed[i]), SPECS[i]


@pytest.mark.parametrize("case", ["blade-poisson", "helmholtz-recoefficiented"])
def test_served_result_vs_oracle(case):
    """A Poisson request on the blade geometry (with second-phase unknowns at
    the slab), and a Helmholtz request served on a hierarchy that was set up
    for another absorption and re-coefficiented: residual by the oracle's own
    operator with the same source, and the error against its direct solve."""
    _say("serving: vs oracle", case)
    specs = [SPECS[0]] if case == "blade-poisson" else [SPECS[5], SPECS[3]]
    srv = serving.Server(0, slots=1)
    reqs = [srv.submit(serving.request_from_spec(i, sp)) for i, sp in enumerate(specs)]
    for r in reqs:
        assert r.done.wait(300) and r.status == ebmg.OK, (r.status, r.error)
    req = reqs[-1]
    x = req.phi.cpu().numpy()
    x2 = req.phi2.cpu().numpy() if req.phi2 is not None else np.zeros(0)
    rho = req.make_rho(torch.device("cuda:0")).cpu().numpy()
    srv.close()
    pr = W.make_request(specs[-1])
    pr.rho = rho.reshape(pr.rho.shape)
    S = assemble(pr)
    assert S.N2 == len(x2)
    xf = np.concatenate([x, x2])
    assert rel_residual(S.A, S.b, xf) <= 1.01e-10
    ref = solve_splu(S.A, S.b)
    err = np.linalg.norm(xf - ref) / np.linalg.norm(ref)
    _say("   error vs oracle", err)
    assert err <= 1e-8


def test_admission_within_budget():
    """With hierarchy sizes known from solo runs, a budget that holds the
    largest request but never two: everything completes, serially, with
    evictions, the footprint never exceeds the budget, and each result equals
    its solo result."""
    _say("serving: admission")
    specs = [SPECS[7], SPECS[6], SPECS[1], SPECS[3]]
    alone, sizes, needs = [], {}, []
    for i, sp in enumerate(specs):
        phi, reqs, summ = _serve([sp], slots=1)
        alone.append(phi[0])
        sizes.update(summ["measured"])
        needs.append(summ["measured"][reqs[0].key] + reqs[0].vec_bytes())
    budget = max(needs) + (1 << 20)
    phis, reqs, summ = _serve(specs, slots=4, budget=budget, measured=sizes)
    _say("   summary", summ)
    assert summ["completed"] == len(specs)
    assert summ["footprint_high_water_bytes"] <= budget
    assert summ["evicted"] >= 1
    for a, b in zip(alone, phis):
        assert np.array_equal(a, b)
    # a request that cannot fit an empty device is rejected, not queued
    srv = serving.Server(0, slots=1, budget_bytes=1 << 20)
    r = srv.submit(serving.request_from_spec(0, SPECS[7]))
    assert r.done.wait(10) and r.rejected
    srv.close()


def test_small_poisson_requests_are_coalesced():
    """Six small 3D Poisson requests of one grid arriving together are solved
    in batched groups (one batched solve per group), each result bitwise
    equal to the same request served alone."""
    _say("serving: coalescing")
    specs = [dict(dim=3, n=32, op="poisson", kappa=1.0, seed=100 + i) for i in range(6)]
    alone = []
    for sp in specs:
        phi, _, _ = _serve([sp], slots=1)
        alone.append(phi[0])
    phis, reqs, summ = _serve(specs, slots=1)
    _say("   summary", summ)
    assert summ["completed"] == len(specs)
    assert summ["coalesced_groups"] >= 1 and summ["coalesced_requests"] >= 2
    for a, b in zip(alone, phis):
        assert np.array_equal(a, b)
