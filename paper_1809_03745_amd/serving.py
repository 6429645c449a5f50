"""Serving loop: continuous batching of Poisson and Helmholtz solves on one
GPU over device-resident multigrid hierarchies, with admission by HBM
footprint.

Requests name a *key* (same key = same grid, same geometry, hence the same
hierarchy up to coefficients). A hierarchy, once set up, stays resident on
the device and is reused by later requests of its key; a Helmholtz request
whose coefficients differ from the resident ones re-coefficients it in place
(``ebmg_set_coefficients``) instead of a new setup. Every resident hierarchy
owns its own HIP stream, so requests running on different hierarchies
overlap on the device; ``slots`` worker threads drive them (the library
releases the interpreter lock inside every call).

Admission: a request is admitted when a slot is free and its footprint (its
device vectors, plus the hierarchy when none of its key is resident) fits the
byte budget together with everything resident; idle hierarchies are evicted
least-recently-used to make room. A request whose key's hierarchy is busy
waits for it (a new setup costs far more than one solve) while later
requests of other keys may pass. A request that cannot fit even into an
empty device is rejected. Admission is first-fit over the queue in arrival
order, except that a request waiting longer than ``max_bypass_s`` blocks all
later ones (no starvation of large requests).

Coalescing: small Poisson requests (3D grids up to 64^3, 2D up to 512^2)
of one key are served by a resident batch of ``coalesce`` copies of the
box; when one is admitted, up to ``coalesce - 1`` more queued requests of
the key join it and the group is solved by one batched solve (one
level-synchronous launch sequence over the boxes, unused boxes with a zero
source). A small request alone is solved the same way, as a group of one.

Results do not depend on the mix: every hierarchy is set up with fixed
smoother and coarse-tail choices (no timing-based autotuning, which would
depend on what else runs), a batched box's result is bitwise the same
whatever the other boxes hold, all reductions are deterministic, and a
request's work touches only its own hierarchy and vectors (or its own box
of a batch).

The scheduler (``Scheduler``) is plain Python with no device calls, so its
policy is testable on the CPU; ``Server`` executes admitted requests.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Any, Callable, Optional


@dataclasses.dataclass
class Request:
    """One solve. ``make_problem()`` returns the ``workloads.Problem`` that sets
    up the hierarchy of ``key`` on a miss; ``coeffs`` (optional) is a problem
    whose coefficients and boundary data are applied to a resident hierarchy
    before the solve; ``make_rho(device)`` returns the source as a device
    tensor of the grid's cells. ``cells`` / ``cells2`` size the footprint."""
    rid: int
    key: Any
    cells: int
    make_problem: Callable[[], Any]
    make_rho: Callable[[Any], Any]
    coeffs: Any = None
    coeff_sig: Any = None
    group_key: Any = None       # requests of one group key may share a batched solve
    dim: int = 3
    arrival: float = 0.0
    want_phi: bool = True
    # filled by the server
    status: int = -1
    info: Optional[dict] = None
    phi: Any = None
    phi2: Any = None
    t_admit: float = 0.0
    t_start: float = 0.0
    t_end: float = 0.0
    hit: bool = False
    setup_s: float = 0.0
    rejected: bool = False
    error: str = ""
    members: Any = None         # the group a coalesced request leads (itself first)
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    def vec_bytes(self):
        # source, solution, second-phase unknowns (bounded by the cell count)
        return 8 * (2 * self.cells + max(1, self.cells // 8))


@dataclasses.dataclass
class Entry:
    key: Any
    bytes: int
    busy: bool = False
    last_used: float = 0.0
    coeff_sig: Any = None
    handle: Any = None          # executor state (problem, context, stream)
    ready: bool = False


class Scheduler:
    """Admission and residency bookkeeping (no device calls)."""

    def __init__(self, budget_bytes, slots, bytes_per_cell=160, max_bypass_s=0.5, clock=time.perf_counter,
                 coalesce=1):
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.coalesce = max(1, int(coalesce))
        self.bytes_per_cell = bytes_per_cell
        self.max_bypass_s = max_bypass_s
        self.clock = clock
        self.queue = collections.deque()
        self.entries = []
        self.running = 0
        self.vec_reserved = 0
        self.releasing = 0       # bytes of evicted hierarchies not yet freed
        self.high_water = 0
        self.measured = {}       # key -> bytes of a set-up hierarchy
        self.stats = collections.Counter()

    # -- footprint ----------------------------------------------------------
    def reserved(self):
        return self.vec_reserved + self.releasing + sum(e.bytes for e in self.entries)

    def hier_estimate(self, req):
        boxes = self.coalesce if req.group_key is not None else 1
        return self.measured.get(req.key, self.bytes_per_cell * req.cells * boxes)

    def offer(self, req):
        """Queue a request, or reject it when it cannot fit an empty device."""
        if req.vec_bytes() + self.hier_estimate(req) > self.budget:
            req.rejected = True
            self.stats["rejected"] += 1
            return False
        self.queue.append(req)
        self.stats["queued"] += 1
        return True

    def _plan(self, req):
        """(entry to use or None for a new one, idle entries to evict) if the
        request fits now, else None."""
        same = [e for e in self.entries if e.key == req.key]
        idle = [e for e in same if not e.busy and e.ready]
        if same and not idle:
            return None     # wait for the resident hierarchy rather than set up a second one
        use = max(idle, key=lambda e: e.last_used) if idle else None
        need = req.vec_bytes() + (0 if use is not None else self.hier_estimate(req))
        free = self.budget - self.reserved()
        evict = []
        if need > free:
            victims = sorted((e for e in self.entries if not e.busy and e.ready and e is not use),
                             key=lambda e: e.last_used)
            for e in victims:
                evict.append(e)
                free += e.bytes
                if need <= free:
                    break
            if need > free:
                return None
        return use, evict

    def next_admissible(self):
        """Pick the next request to run: (request, entry, evictions) or None."""
        if self.running >= self.slots or not self.queue:
            return None
        now = self.clock()
        for i, req in enumerate(self.queue):
            plan = self._plan(req)
            if plan is not None:
                del self.queue[i]
                use, evict = plan
                for e in evict:
                    self.entries.remove(e)
                    self.releasing += e.bytes   # still held until the executor frees it
                    self.stats["evicted"] += 1
                if use is None:
                    use = Entry(req.key, self.hier_estimate(req))
                    self.entries.append(use)
                    self.stats["misses"] += 1
                    req.hit = False
                else:
                    self.stats["hits"] += 1
                    req.hit = True
                use.busy = True
                self.running += 1
                self.vec_reserved += req.vec_bytes()
                req.t_admit = now
                req.members = [req]
                if req.group_key is not None and self.coalesce > 1:
                    self._gather(req, now)
                # the admitting worker frees its evictions before it sets up
                # the new hierarchy, so they do not add to the peak
                self.high_water = max(self.high_water, self.reserved() - self.releasing)
                return req, use, evict
            if now - req.arrival > self.max_bypass_s and i == 0:
                return None     # the head has waited too long: nothing may pass it
        return None

    def _gather(self, req, now):
        """Queued requests of the admitted one's group join it (queue order,
        up to the batch's size, while their vectors fit)."""
        free = self.budget - self.reserved()
        for other in list(self.queue):
            if len(req.members) >= self.coalesce:
                break
            if other.group_key != req.group_key or other.vec_bytes() > free:
                continue
            self.queue.remove(other)
            self.vec_reserved += other.vec_bytes()
            free -= other.vec_bytes()
            other.t_admit = now
            other.hit = req.hit
            other.members = None
            req.members.append(other)
        if len(req.members) > 1:
            self.stats["coalesced_groups"] += 1
            self.stats["coalesced_requests"] += len(req.members)

    def reset_stats(self):
        self.stats.clear()
        self.high_water = self.reserved()

    def set_up(self, entry, actual_bytes):
        """A new hierarchy is resident: replace the estimate by its size."""
        entry.bytes = int(actual_bytes)
        entry.ready = True
        self.measured[entry.key] = int(actual_bytes)
        # evictions still being freed by other workers are covered by the
        # reservations that replace them (a worker frees its evictions before
        # it allocates), so they are not counted twice
        self.high_water = max(self.high_water, self.reserved() - self.releasing)

    def released(self, entry):
        """An evicted hierarchy's device memory has been freed."""
        self.releasing -= entry.bytes

    def failed_setup(self, entry):
        if entry in self.entries:
            self.entries.remove(entry)

    def finish(self, req, entry):
        """The admitted request (and the group it leads) is done."""
        group = req.members or [req]
        if entry in self.entries:
            entry.busy = False
            entry.last_used = self.clock()
        self.running -= 1
        for m in group:
            self.vec_reserved -= m.vec_bytes()
        self.stats["completed"] += len(group)


class Server:
    """Executes requests on one GPU with ``slots`` worker threads."""

    def __init__(self, device=0, slots=4, budget_bytes=None, precision=None, rtol=1e-10, max_cycles=400,
                 bytes_per_cell=160, coalesce=8):
        import torch
        from . import ebmg
        self.torch = torch
        self.ebmg = ebmg
        self.device = device
        self.dev = torch.device(f"cuda:{device}")
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            budget_bytes = int(0.5 * free)
        self.precision = ebmg.MIXED if precision is None else precision
        self.rtol = rtol
        self.max_cycles = max_cycles
        self.sched = Scheduler(budget_bytes, slots, bytes_per_cell=bytes_per_cell, coalesce=coalesce)
        self.coalesce = max(1, int(coalesce))
        self.cv = threading.Condition()
        self.closed = False
        self.records = []
        self.workers = [threading.Thread(target=self._work, daemon=True) for _ in range(slots)]
        for w in self.workers:
            w.start()

    # -- client side ----------------------------------------------------------
    def submit(self, req):
        with self.cv:
            if req.arrival == 0.0:
                req.arrival = time.perf_counter()
            ok = self.sched.offer(req)
            if not ok:
                req.t_end = time.perf_counter()
                self.records.append(req)
                req.done.set()
            self.cv.notify_all()
        return req

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()
        for e in list(self.sched.entries):
            self._release(e)
        self.sched.entries.clear()

    # -- executor -------------------------------------------------------------
    def _release(self, e):
        h = e.handle
        if h is not None:
            (h.get("problem") or h.get("batch")).release()
            h["ctx"].close()
            e.handle = None

    def _setup(self, req, entry):
        torch, ebmg = self.torch, self.ebmg
        stream = torch.cuda.Stream(device=self.dev)
        ctx = ebmg.Context(self.device, stream=stream.cuda_stream)
        try:
            prob = req.make_problem()
            t0 = time.perf_counter()
            if req.group_key is not None and self.coalesce > 1:
                # a batch of copies of the box (its results do not depend on
                # what the other boxes hold or on its coarse-part choice)
                B = ebmg.Batch(ctx, [prob] * self.coalesce, precision=self.precision, batch=ebmg.BATCH_LEVELSYNC,
                               tail=1)
                req.setup_s = time.perf_counter() - t0
                entry.handle = {"batch": B, "ctx": ctx, "stream": stream}
                return B.device_bytes
            # fixed kernel choices (no timing: a result is the same alone and
            # in any mix) and direct launches (a Helmholtz request
            # re-coefficients the hierarchy, which would drop a captured
            # graph every time)
            P = ebmg.Problem(ctx, prob, precision=self.precision, smoother=4, tail=1, graphs=1)
        except Exception:
            ctx.close()
            raise
        req.setup_s = time.perf_counter() - t0
        entry.handle = {"problem": P, "ctx": ctx, "stream": stream}
        entry.coeff_sig = req.coeff_sig
        return P.device_bytes

    def _run_group(self, req, entry):
        torch = self.torch
        h = entry.handle
        B, stream = h["batch"], h["stream"]
        group = req.members or [req]
        n, n2 = B.sizes[0]
        with torch.cuda.stream(stream):
            rho = [m.make_rho(self.dev) for m in group]
            rho += [torch.zeros(n, dtype=torch.float64, device=self.dev) for _ in range(self.coalesce - len(group))]
            phi = [torch.zeros(n, dtype=torch.float64, device=self.dev) for _ in range(self.coalesce)]
            phi2 = [torch.zeros(max(1, n2), dtype=torch.float64, device=self.dev) for _ in range(self.coalesce)]
        t = time.perf_counter()
        for m in group:
            m.t_start = t
        st, infos = B.solve(rho, phi, phi2=phi2, rtol=self.rtol, max_cycles=self.max_cycles, check=False)
        for i, m in enumerate(group):
            ok = st == self.ebmg.OK or infos[i]["rel_residual"] <= self.rtol
            m.status, m.info = (self.ebmg.OK if ok else st), infos[i]
            if m.want_phi:
                m.phi = phi[i]
                m.phi2 = phi2[i][:n2] if n2 else None
        del rho

    def _run(self, req, entry):
        torch = self.torch
        h = entry.handle
        P, stream = h["problem"], h["stream"]
        if req.coeffs is not None and entry.coeff_sig != req.coeff_sig:
            P.set_coefficients(req.coeffs)
            entry.coeff_sig = req.coeff_sig
        with torch.cuda.stream(stream):
            rho = req.make_rho(self.dev)
            phi = torch.zeros(P.N, dtype=torch.float64, device=self.dev)
            phi2 = torch.zeros(max(1, P.N2), dtype=torch.float64, device=self.dev)
        # the library works on the same stream, so the source is ready in order
        req.t_start = time.perf_counter()
        st, info = P.solve(rho, phi, phi2=phi2 if P.N2 else None, rtol=self.rtol, max_cycles=self.max_cycles,
                           check=False)
        req.status, req.info = st, info
        if req.want_phi:
            req.phi = phi
            req.phi2 = phi2[:P.N2] if P.N2 else None
        del rho

    def _work(self):
        while True:
            with self.cv:
                pick = None
                while not self.closed:
                    pick = self.sched.next_admissible()
                    if pick is not None:
                        break
                    self.cv.wait(0.01)
                if pick is None:
                    return
            req, entry, evict = pick
            for e in evict:
                try:
                    self._release(e)
                finally:
                    with self.cv:
                        self.sched.released(e)
                        self.cv.notify_all()
            group = req.members or [req]
            try:
                if entry.handle is None:
                    nbytes = self._setup(req, entry)
                    with self.cv:
                        self.sched.set_up(entry, nbytes)
                if "batch" in entry.handle:
                    self._run_group(req, entry)
                else:
                    self._run(req, entry)
            except Exception as exc:  # a failed request must not stop the server
                for m in group:
                    m.status = -2
                    m.error = repr(exc)
                if entry.handle is None:
                    with self.cv:
                        self.sched.failed_setup(entry)
            t_end = time.perf_counter()
            with self.cv:
                self.sched.finish(req, entry)
                for m in group:
                    m.t_end = t_end
                    self.records.append(m)
                self.cv.notify_all()
            for m in group:
                m.done.set()

    # -- reporting ------------------------------------------------------------
    def summary(self, t0, t1):
        done = [r for r in self.records if not r.rejected and r.status == self.ebmg.OK]
        lat = sorted(1000.0 * (r.t_end - r.arrival) for r in done)

        def pct(q):
            if not lat:
                return None
            return lat[min(len(lat) - 1, int(round(q / 100.0 * (len(lat) - 1))))]

        st = self.sched.stats
        bad = [r for r in self.records if not r.rejected and r.status != self.ebmg.OK]
        return {"completed": len(done), "rejected": st["rejected"],
                "failed": len(bad),
                "failed_detail": [{"key": list(r.key), "status": r.status,
                                   "rel_residual": (r.info or {}).get("rel_residual"),
                                   "cycles": (r.info or {}).get("cycles"), "error": r.error[:200]}
                                  for r in bad[:10]],
                "solves_per_s": len(done) / max(t1 - t0, 1e-9),
                "latency_ms": {"p50": pct(50), "p99": pct(99)},
                "hierarchy_hits": st["hits"], "hierarchy_misses": st["misses"], "evicted": st["evicted"],
                "coalesced_groups": st["coalesced_groups"], "coalesced_requests": st["coalesced_requests"],
                "footprint_high_water_bytes": self.sched.high_water, "budget_bytes": self.sched.budget}


def request_from_spec(rid, spec, arrival=0.0, torch_module=None):
    """A ``Request`` for a spec of ``workloads.serving_requests``: Poisson
    requests key on (dim, n) (the pin-plane / blade geometry of that size),
    Helmholtz requests on (dim, n) with the absorption applied by
    re-coefficienting; the source is evaluated on the device."""
    import workloads as W
    torch = torch_module
    if torch is None:
        import torch
    dim, n = spec["dim"], spec["n"]
    cells = n ** dim
    centres, sigmas = W.request_blobs(spec)

    def make_rho(device):
        return W.blob_field(dim, n, centres, sigmas, xp=torch, device=device).reshape(-1)

    if spec["op"] == "poisson":
        key = ("poisson", dim, n)
        small = (dim == 3 and n <= 64) or (dim == 2 and n <= 512)
        return Request(rid, key, cells, make_problem=lambda: W.make_request(dict(spec, seed=0)),
                       make_rho=make_rho, dim=dim, arrival=arrival, group_key=key if small else None)
    kappa = spec["kappa"]
    key = ("helmholtz", dim, n)
    coeffs = W.eddington_coefficients(dim, n, kappa)
    return Request(rid, key, cells, make_problem=lambda: coeffs, make_rho=make_rho, coeffs=coeffs,
                   coeff_sig=kappa, dim=dim, arrival=arrival)


def replay(server, arrivals, specs, t_scale=1.0):
    """Submit ``specs`` at their (relative) arrival times in real time and wait
    for all of them; returns (records in submission order, t0, t1)."""
    reqs = []
    t0 = time.perf_counter()
    for i, (ta, spec) in enumerate(zip(arrivals, specs)):
        target = t0 + t_scale * (ta - arrivals[0])
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        r = request_from_spec(i, spec, arrival=target)
        reqs.append(server.submit(r))
    for r in reqs:
        r.done.wait()
    t1 = max(r.t_end for r in reqs) if reqs else t0
    return reqs, t0, t1
