"""Serving loop: continuous batching of projection-step and PPE-solve requests.

Requests arrive over time (a Poisson stream, or any list of arrival times).
The server keeps plans and their device workspaces resident, one pool of plan
instances per (kind, shape, precision), and admits work against a fixed HBM
budget: a request is admitted when a plan instance of its shape is idle (or a
new one fits in the budget) and its buffers fit.  Admitted requests are packed
into a batch (grouped launches, `api.Batch`) on one of several lanes (each
lane: its own context stream and batch object), so requests that arrive while
other batches run are issued as soon as a lane is free and their work
overlaps on the device with the batches already in flight.  Each plan
instance is bound to one lane's context: a request that is alone on its
plan's own lane runs as the plain call on that lane's stream (no grouping,
argument upload or stream fork / join), any other work as a batch.
Completion is observed by polling an event per launch (every poll_s seconds
while idle); latency = completion - arrival.

Every result equals the plain call on the same plan bitwise (the batch
launches the same kernels on the same data), so a request gives the same
output alone and in the mix.

Failure handling (each request ends with a status):
* "ok";
* "nonfinite": with check_finite set, every output is checked by the
  library's finiteness count when its batch completes; a request whose
  inputs or outputs hold NaN / infinities fails alone (batch items share no
  data, so the others in its batch are unaffected);
* "rejected": a request whose plan workspace and buffers exceed the whole HBM
  budget can never be admitted and is refused on arrival;
* "timeout": not admitted within its deadline (seconds after arrival);
* "cancelled": cancelled (Server.cancel, or its cancel_at time) while still
  queued; work already issued to the device runs to completion.
Latency statistics cover the "ok" requests.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import api, synth


@dataclass
class Request:
    rid: int
    t_arrival: float          # seconds from the start of the stream
    kind: str                 # 'step' | 'ppe'
    dims: int                 # 2 | 3
    n: int                    # lattice points per axis
    seed: int
    t_done: float = math.nan
    out: list = field(default_factory=list)
    status: str = "pending"
    deadline: float = math.inf     # admission deadline, seconds after arrival
    cancel_at: float = math.inf    # cancelled if still queued at this time (from the stream start)
    poison: bool = False           # inputs carry a NaN (failure-path tests)


def make_requests(lam: float, count: int, seed: int = 40, p_step: float = 0.5, p_2d: float = 0.75,
                  n2=(64, 1024), n3=(64, 192), quantum2: int = 16, quantum3: int = 16) -> list:
    """Poisson arrivals at rate lam; per request (in this order): inter-arrival
    gap ~ Exp(lam), kind step w.p. p_step, 2D w.p. p_2d, size log-uniform over
    the range rounded to a multiple of the quantum (a finite set of shapes
    keeps the plan cache finite)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / lam)
        kind = "step" if rng.random() < p_step else "ppe"
        dims = 2 if rng.random() < p_2d else 3
        lo, hi = n2 if dims == 2 else n3
        q = quantum2 if dims == 2 else quantum3
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / q) * q)
        n = min(max(n, lo), hi)
        out.append(Request(i, t, kind, dims, n, int(rng.integers(1 << 30))))
    return out


def problem_for(dims: int, n: int, precision: str, op_eval: str = "fft_window") -> api.Problem:
    """2D: walls on all four sides, Dirichlet velocity and pressure; 3D: the
    channel (walls on y, Dirichlet velocity, Neumann pressure)."""
    if dims == 2:
        return api.Problem(n=(n, n), walled=(True, True), dx=1.0 / (n - 1),
                           vel_bc=(("D", "D"), ("D", "D")), prs_bc=(("D", "D"), ("D", "D")),
                           precision=precision, op_eval=op_eval, batched=True)
    return api.Problem(n=(n, n, n), walled=(False, True, False), dx=1.0 / (n - 1),
                       vel_bc=(None, ("D", "D"), None), prs_bc=(None, ("N", "N"), None),
                       precision=precision, op_eval=op_eval, batched=True)


class Server:
    def __init__(self, precision: str = "fp64", hbm_budget: float = 200e9, max_batch: int = 16,
                 lanes: int = 4, op_eval: str = "fft_window", dt: float = 1e-4, nu: float = 1e-3,
                 max_batch_3d: int = 2, check_finite: bool = False, poll_s: float = 2e-5):
        import torch
        self.precision, self.op_eval = precision, op_eval
        self.check_finite = check_finite
        # idle wait of the loop between polls (arrivals, completions): it adds
        # about half of itself (plus the OS wake-up) to a lone request's latency
        self.poll_s = poll_s
        self.cancelled: set = set()
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.max_batch_3d = max(1, min(max_batch_3d, max_batch))
        self.dt, self.nu = dt, nu
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.ctxs = [api.Context(0, s) for s in self.streams]
        self.batches = [api.Batch(c, max_batch) for c in self.ctxs]
        self.inflight = [None] * lanes          # (event, [(request, plan instance, bufs)])
        self.pool: dict = {}                    # shape key -> idle plans
        self.count: dict = {}                   # shape key -> plan instances
        self.used = 0.0                         # bytes: plan workspaces + request buffers in flight
        self.resident = 0.0                     # bytes: plan workspaces (resident until the server ends)
        self.templates: dict = {}
        self.stats = {"plans_created": 0, "admitted": 0, "max_queue": 0, "batches": 0}

    # ---- resident state
    def _key(self, r: Request):
        return (r.dims, r.n)

    def _template(self, dims, n):
        import torch
        k = (dims, n)
        if k not in self.templates:
            if dims == 2:
                f = [synth.poly_trig_2d(n, 2 * n), synth.poly_trig_2d(n, 2 * n + 1)]
            else:
                f = list(synth.ChannelFlow3D((n, n, n), 20, 21).u)
            self.templates[k] = [torch.from_numpy(c).cuda() for c in f]
        return self.templates[k]

    def _new_plan(self, dims, n, lane: int = 0):
        # bound to a lane's context: a lone request on that lane runs as the
        # plain call on the lane's stream; in batches any lane can run it
        ctx = self.ctxs[lane % len(self.ctxs)]
        plan = api.Plan(ctx, problem_for(dims, n, self.precision, self.op_eval))
        plan.lane = lane % len(self.ctxs)
        ctx.sync()                     # tables resident before any lane stream uses the plan
        self.used += plan.workspace.numel()
        self.resident += plan.workspace.numel()
        self.stats["plans_created"] += 1
        return plan

    def warm(self, shapes):
        """Create the resident plans (one per lane) and the input template per shape."""
        for dims, n in shapes:
            self._template(dims, n)
            for lane in range(len(self.streams)):
                self.pool.setdefault((dims, n), []).append(self._new_plan(dims, n, lane))
            self.count[(dims, n)] = len(self.streams)

    def _request_bytes(self, r: Request) -> int:
        pts = r.n ** r.dims
        return pts * 8 * (2 * r.dims + 1 if r.kind == "step" else 2)

    def cancel(self, rid: int):
        """Cancel a request that is still queued (no effect once issued)."""
        self.cancelled.add(rid)

    def _never_fits(self, r: Request) -> bool:
        """Resident plans are never evicted, so the room a request can ever get
        is the budget less every plan workspace."""
        room = self.budget - self.resident
        need = self._request_bytes(r)
        if self.count.get(self._key(r), 0) > 0:
            return need > room
        ws = api.workspace_bytes(problem_for(r.dims, r.n, self.precision, self.op_eval))
        return ws + need > room

    def _acquire(self, r: Request, lane: int = 0):
        idle = self.pool.setdefault(self._key(r), [])
        need = self._request_bytes(r)
        if idle:
            if self.used + need > self.budget:
                return None
            # an instance bound to this lane when one is idle
            for i in range(len(idle) - 1, -1, -1):
                if getattr(idle[i], "lane", -1) == lane:
                    return idle.pop(i)
            return idle.pop()
        # a new instance only while a shape has fewer than one per lane
        # (otherwise the request waits for an instance to return)
        if self.count.get(self._key(r), 0) >= len(self.streams):
            return None
        ws = api.workspace_bytes(problem_for(r.dims, r.n, self.precision, self.op_eval))
        if self.used + ws + need > self.budget:
            return None
        self.count[self._key(r)] = self.count.get(self._key(r), 0) + 1
        return self._new_plan(r.dims, r.n, lane)

    def _inputs(self, r: Request):
        import torch
        tpl = self._template(r.dims, r.n)
        s = 1.0 + (r.seed % 97) / 97.0
        if r.kind == "step":
            u = [(c * s).contiguous() for c in tpl]
            wall = [c.clone() for c in u]
            if r.poison:
                u[0][tuple(k // 2 for k in u[0].shape)] = float("nan")   # an interior point
            p = torch.empty_like(u[0])
            return {"u": u, "wall": wall, "p": p}
        rhs = (tpl[0] * s).contiguous()
        if r.poison:
            rhs[tuple(k // 2 for k in rhs.shape)] = float("nan")     # an interior point
        if self.precision == "fp32":
            rhs = rhs.float()
        return {"rhs": rhs, "phi": torch.empty_like(tpl[0])}

    # ---- the loop
    def _poll(self, now_fn):
        done = 0
        for k, fl in enumerate(self.inflight):
            if fl is None or not fl[0].query():
                continue
            t = now_fn()
            for r, plan, bufs in fl[1]:
                r.out = [bufs["u"], bufs["p"]] if r.kind == "step" else [bufs["phi"]]
                r.status = "ok"
                if self.check_finite:
                    outs = (bufs["u"] + [bufs["p"]]) if r.kind == "step" else [bufs["phi"]]
                    if any(plan.nonfinite_count(o) for o in outs):
                        r.status = "nonfinite"
                    t = now_fn()
                r.t_done = t
                self.pool[self._key(r)].append(plan)
                self.used -= self._request_bytes(r)
                done += 1
            self.inflight[k] = None
        return done

    def _launch(self, lane: int, work):
        if len(work) == 1 and getattr(work[0][1], "lane", -1) == lane:
            # a lone request on its plan's own lane: the plain call (the same
            # kernels and bitwise the same result as a batch of one, without
            # the grouping, argument upload and stream fork / join)
            r, plan, bufs = work[0]
            if r.kind == "step":
                plan.project_step(bufs["u"], self.dt, self.nu, p_out=bufs["p"], wall=bufs["wall"])
            else:
                plan.ppe_solve(bufs["rhs"], bufs["phi"])
            self.stats["plain_launches"] = self.stats.get("plain_launches", 0) + 1
        else:
            b = self.batches[lane]
            b.clear()
            for r, plan, bufs in work:
                if r.kind == "step":
                    b.add_step(plan, bufs["u"], self.dt, self.nu, p_out=bufs["p"], wall=bufs["wall"])
                else:
                    b.add_ppe(plan, bufs["rhs"], bufs["phi"])
            b.launch()
        ev = self.streams[lane].record_event()
        self.inflight[lane] = (ev, work)
        self.stats["batches"] += 1

    def run(self, requests: list, realtime: bool = True, keep_outputs: bool = False) -> dict:
        """Serve the requests (arrival times relative to the start); returns
        throughput and latency statistics."""
        import torch
        torch.cuda.synchronize()
        self.stats.update(admitted=0, max_queue=0, batches=0)
        pending = deque(sorted(requests, key=lambda r: r.t_arrival))
        queue: deque = deque()
        if not realtime:                     # burst: every request arrives at once
            for r in pending:
                r.t_arrival = 0.0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0
        remaining = len(requests)
        for r in requests:
            r.status = "pending"

        def finish(r, status):
            r.status, r.t_done = status, now()
            return 1
        while remaining:
            t = now()
            while pending and pending[0].t_arrival <= t:
                r = pending.popleft()
                if self._never_fits(r):
                    remaining -= finish(r, "rejected")
                else:
                    queue.append(r)
            # queued requests past their deadline or cancelled leave the queue
            if queue:
                keep = deque()
                for r in queue:
                    if r.rid in self.cancelled or t >= r.cancel_at:
                        remaining -= finish(r, "cancelled")
                    elif t - r.t_arrival >= r.deadline:
                        remaining -= finish(r, "timeout")
                    else:
                        keep.append(r)
                queue = keep
            self.stats["max_queue"] = max(self.stats["max_queue"], len(queue))
            remaining -= self._poll(now)
            free = [k for k, fl in enumerate(self.inflight) if fl is None]
            if free and queue:
                lane = free[0]
                work, skipped = [], deque()
                cls = queue[0].dims                             # batches of one class (2D or 3D): a
                limit = self.max_batch if cls == 2 else self.max_batch_3d   # large 3D solve does not
                with torch.cuda.stream(self.streams[lane]):     # hold small ones
                    while queue and len(work) < limit:
                        r = queue.popleft()
                        if r.dims != cls:
                            skipped.append(r)
                            continue
                        plan = self._acquire(r, lane)
                        if plan is None:
                            skipped.append(r)
                            continue
                        self.used += self._request_bytes(r)
                        work.append((r, plan, self._inputs(r)))
                        self.stats["admitted"] += 1
                queue.extendleft(reversed(skipped))
                if work:
                    self._launch(lane, work)
                    continue
            if not free or not queue:
                time.sleep(self.poll_s)
        wall = now()
        ok = [r for r in requests if r.status == "ok"]
        lat = np.array([r.t_done - r.t_arrival for r in ok]) if ok else np.array([math.nan])
        if not keep_outputs:
            for r in requests:
                r.out = []
        status = {}
        for r in requests:
            status[r.status] = status.get(r.status, 0) + 1
        return {"requests": len(requests), "wall_s": round(wall, 3),
                "solves_per_s": round(len(ok) / wall, 1),
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                "status": status,
                "plans_created": self.stats["plans_created"], "batches": self.stats["batches"],
                "max_queue": self.stats["max_queue"], "hbm_used_GB": round(self.used / 1e9, 2)}


def run_plain(requests: list, srv: Server, realtime: bool = True) -> dict:
    """The plain per-request path at the same arrival times on the server's
    resident plans: one request at a time, each call synchronised before the
    next."""
    import torch
    dt, nu = srv.dt, srv.nu
    pending = deque(sorted(requests, key=lambda r: r.t_arrival))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in pending:
        if realtime:
            while time.perf_counter() - t0 < r.t_arrival:
                time.sleep(srv.poll_s)
        plan = srv._acquire(r)
        bufs = srv._inputs(r)
        if r.kind == "step":
            plan.project_step(bufs["u"], dt, nu, p_out=bufs["p"], wall=bufs["wall"])
        else:
            plan.ppe_solve(bufs["rhs"], bufs["phi"])
        torch.cuda.synchronize()
        r.t_done = time.perf_counter() - t0
        srv.pool[srv._key(r)].append(plan)
    wall = time.perf_counter() - t0
    lat = np.array([r.t_done - r.t_arrival for r in requests])
    return {"requests": len(requests), "wall_s": round(wall, 3),
            "solves_per_s": round(len(requests) / wall, 1),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3)}
