"""Warm-start serving on top of the native serving context (hjr_ctx).

Requests are reachability solves whose model parameters change from one request to the next
(mass, disturbance bound, control bound).  The native context admits requests while their
working memory fits its HBM budget and advances every admitted request in the same batched
launches (continuous batching).  This module adds the warm-start policy: solutions stay resident
on the device, and a new request is started from the resident solution of the nearest earlier
request of the same kind, preferring one whose problem dominates the new one (more control
authority, less disturbance, a smaller target).  By Theorem 2 and Propositions 1-2 a dominating
warm start converges to the new problem's value function exactly; any other warm start is still
conservative by Theorem 1.

Only converged results (status OK) are kept as warm starts: Theorem 2's exactness assumes the
prior is the converged value function of its problem.  Every request records whether its warm
start came from a dominating prior (``exact_warm``: exact by Theorem 2) or not (conservative
only); with ``only_dominating=True`` requests without a dominating prior start cold instead.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Optional

from . import hjr


@dataclass
class Request:
    kind: str                 # requests of one kind share grid, target and scheme
    grid: object
    dyn: object
    key: tuple                # parameters the warm-start policy compares
    dominates: Callable       # dominates(prior_key, key) -> True if the prior's problem dominates
    l_dev: object             # FP64 device tensor (shared by the kind)
    opts: dict
    arrival: float = 0.0      # seconds after the start of the stream
    ticket: int = -1
    submitted: float = 0.0
    done: float = 0.0
    status: int = 0
    result: dict = field(default_factory=dict)
    warm_from: Optional[tuple] = None
    exact_warm: Optional[bool] = None   # None: cold; True: dominating prior; False: any other prior
    V: object = None


class WarmStartServer:
    """Drive an hjr.Context with a request stream; keep solutions resident as warm starts."""

    def __init__(self, ctx: "hjr.Context", warm: bool = True, resident_per_kind: int = 8,
                 only_dominating: bool = False, keep_outputs: bool = True):
        """keep_outputs=False drops each request's result array once it is done, unless it stays
        resident as a warm start (for long streams of large grids)."""
        self.ctx = ctx
        self.warm = warm
        self.only_dominating = only_dominating
        self.keep_outputs = keep_outputs
        self.resident_per_kind = resident_per_kind
        self.resident = {}     # kind -> list of (key, V tensor, last use)

    def pick_warm_start(self, req: Request):
        """(k, prior key, exact): the nearest resident prior of the request's kind, preferring
        dominating ones (exact = True); (None, None, None) for a cold start."""
        if not self.warm:
            return None, None, None
        cands = self.resident.get(req.kind, [])

        def dist(a, b):
            return math.sqrt(sum((x - y) ** 2 for x, y in zip(a, b)))
        dom = [c for c in cands if req.dominates(c[0], req.key)]
        pool = dom if dom else ([] if self.only_dominating else cands)
        if not pool:
            return None, None, None
        best = min(pool, key=lambda c: dist(c[0], req.key))
        best[2] = time.perf_counter()
        return best[1], best[0], bool(dom)

    def keep(self, req: Request):
        lst = self.resident.setdefault(req.kind, [])
        lst.append([req.key, req.V, time.perf_counter()])
        if len(lst) > self.resident_per_kind:
            lst.sort(key=lambda c: c[2])
            lst.pop(0)

    def run(self, requests, torch, device, poll_interval=2e-4, max_in_flight=None, on_done=None):
        """Submit each request at its arrival time (at most max_in_flight submitted and not yet
        done; later arrivals wait, and their latency counts the wait); returns the requests with
        timings filled.  on_done(request, finished_count) is called as each request finishes."""
        pending = sorted(requests, key=lambda r: r.arrival)
        active = {}
        t0 = time.perf_counter()
        i = 0
        finished = 0
        while i < len(pending) or active:
            now = time.perf_counter() - t0
            while (i < len(pending) and pending[i].arrival <= now
                   and (max_in_flight is None or len(active) < max_in_flight)):
                r = pending[i]
                k, key, exact = self.pick_warm_start(r)
                r.warm_from = key
                r.exact_warm = exact
                r.V = torch.empty_like(r.l_dev)
                r.submitted = time.perf_counter() - t0
                r.ticket = self.ctx.submit(r.grid, r.dyn, r.l_dev, k, r.V, **r.opts)
                active[r.ticket] = r
                i += 1
            for t in list(active):
                res = self.ctx.poll(t)
                if res is None:
                    continue
                r = active.pop(t)
                r.status, r.result = res
                r.done = time.perf_counter() - t0
                if r.status == hjr.OK:
                    self.keep(r)
                if not self.keep_outputs:
                    r.V = None
                finished += 1
                if on_done is not None:
                    on_done(r, finished)
            time.sleep(poll_interval)
        return requests


def latency_stats(requests):
    """Latency percentiles over all requests; solves/s counts converged results only (status OK),
    and the others are reported apart."""
    lat = sorted(r.done - r.arrival for r in requests)

    def pct(q):
        if not lat:
            return float("nan")
        return lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    ok = sum(1 for r in requests if r.status == hjr.OK)
    return {"requests": len(requests), "converged": ok, "not_converged": len(requests) - ok, "seconds": span,
            "solves_per_s": ok / span, "p50_s": pct(0.50), "p99_s": pct(0.99), "mean_s": sum(lat) / len(lat)}
