"""Continuous-batching server for fluctuating lattice Boltzmann solves.

Requests (model, box, steps, relaxation rate, mean density, seed) arrive
over time.  The server keeps one batch (flb_batch_*) of resident lattices:
a request is admitted as soon as its device memory (populations + workspace,
from flb_required_bytes) fits in the HBM budget, joins the running batch at
the next tick, and is retired when it has done its steps; its final
statistics are read and its memory released, which lets queued requests in.
Every tick advances all active lattices by the same number of steps in
batched launches (at least tick_steps, as many more as fit a wall-time
budget at the measured rate, never past the earliest completion), so work
of requests that arrived at different times overlaps on the device.  Because the batch is bit-identical to stepping
each lattice alone, a request's result does not depend on what it was
batched with.

    python -m paper_1606_07801_amd.serve --requests 48 --rate 200
"""

import argparse
import json
import math
import time
from collections import deque

import numpy as np

from . import flb, inputs


class Request:
    __slots__ = ("id", "arrival", "d", "dims", "steps", "omega", "rho", "seed", "precision",
                 "lat", "bytes", "start", "done", "remaining", "result", "error", "keep_state", "layout",
                 "alt_bytes")

    def __init__(self, rid, arrival, d, dims, steps, omega, rho, seed, precision=4, keep_state=False):
        self.id, self.arrival, self.d, self.dims = rid, float(arrival), int(d), tuple(int(x) for x in dims)
        self.steps, self.omega, self.rho, self.seed = int(steps), float(omega), float(rho), int(seed)
        self.precision = precision
        self.lat = None
        self.bytes = 0
        self.start = self.done = None
        self.remaining = self.steps
        self.result = None
        self.error = None
        self.keep_state = keep_state
        self.layout = "two"
        self.alt_bytes = None

    @property
    def sites(self):
        return int(np.prod(self.dims))

    @classmethod
    def from_dict(cls, r, precision=4, keep_state=False):
        return cls(r["id"], r["arrival"], r["d"], r["dims"], r["steps"], r["omega"], r["rho"],
                   r["seed"], precision, keep_state)


def request_bytes(req):
    p = flb.make_params(req.d, req.dims, precision=req.precision, omega=req.omega, seed=req.seed,
                        layout=req.layout)
    pop, work = flb.required_bytes(p)
    return pop + work + 512


def aa_eligible(req):
    """The AA layout steps with the flat kernel, which needs Q N precision < 2^32."""
    return req.sites * (2 * req.d + 1) * req.precision < (1 << 32)


def pick_layout(req, policy):
    """Preferred storage layout of a request.  "two": two buffers for every
    request; "aa": one buffer (AA layout, half the population memory) for
    every request that can take it; "auto": the faster layout per model --
    one buffer for D1Q3 (as fast or faster), two for D2Q5 (a two-step pass
    per two steps) and D3Q7 (its in-place steps run 10 % slower) -- with the
    single buffer as a fallback under memory pressure (fallback_bytes)."""
    if policy == "two" or not aa_eligible(req):
        return "two"
    if policy == "aa" or req.d == 1:
        return "aa"
    return "two"


def fallback_bytes(req, policy):
    """Device bytes of the request in the AA layout when policy "auto" may
    admit it that way because its preferred two-buffer footprint does not fit
    the free budget (None when there is no such fallback)."""
    if policy != "auto" or req.layout != "two" or not aa_eligible(req):
        return None
    keep = req.layout
    req.layout = "aa"
    try:
        return request_bytes(req)
    finally:
        req.layout = keep


def initial_state(torch, req, device):
    """Uniform equilibrium f_i = w_i rho (the library's weights), built on
    the device."""
    w, _ = flb.constants(req.d)
    dt = torch.float32 if req.precision == 4 else torch.float64
    wt = torch.tensor(w, dtype=dt, device=device).reshape((-1,) + (1,) * req.d)
    shape = tuple(reversed(req.dims))
    return (wt * req.rho).expand((len(w),) + shape).contiguous()


def start_request(torch, req, device):
    L = flb.Lattice(req.d, req.dims, precision=req.precision, omega=req.omega, seed=req.seed,
                    noise="local", layout=req.layout)
    f0 = initial_state(torch, req, device)
    L.set_populations(f0)
    del f0
    req.lat = L


def finish_request(req):
    L = req.lat
    m = L.moments()
    res = {"id": req.id, "steps": L.t, "mass": m["mass"], "mass0": m["mass0"],
           "var_rho": m["sum_rho2"] / m["nsite"] - (m["mass"] / m["nsite"]) ** 2,
           "n_negative": m["n_negative"], "nonfinite": m["nonfinite"]}
    if req.keep_state:
        res["state"] = L.get_populations()
    L.close()
    req.lat = None
    req.result = res


class Server:
    """Admission by HBM budget, continuous batching by ticks."""

    def __init__(self, budget_bytes=None, tick_steps=64, chunk=None, use_graph=True, device=None, layout="auto",
                 tick_ms=20.0):
        import torch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.8 * free)
        self.budget = int(budget_bytes)
        self.used = 0
        self.tick_steps = int(tick_steps)
        # a tick runs at least tick_steps steps and as many more as fit
        # tick_ms of wall time at the batch's measured rate (admission waits
        # at most about that long; each tick ends with a synchronisation)
        self.tick_ms = float(tick_ms)
        self._step_s = None        # wall seconds per batch step, measured on the current members
        from . import tune
        bcfg = tune.batch_config()
        if chunk is not None:
            bcfg["chunk"] = chunk
        self.batch = flb.Batch(use_graph=use_graph, **bcfg)
        self.queue = deque()
        self.active = []
        self.finished = []
        self.rejected = []
        self.ticks = 0
        self.site_updates = 0
        self.layout = layout
        self.fallbacks = 0         # requests admitted in the AA layout under memory pressure
        self.peak_active = 0
        self.active_ticks = 0      # sum over ticks of the number of active requests

    def submit(self, req):
        req.layout = pick_layout(req, self.layout)
        req.bytes = request_bytes(req)
        req.alt_bytes = fallback_bytes(req, self.layout)
        if min(req.bytes, req.alt_bytes or req.bytes) > self.budget:
            req.error = f"needs {req.bytes} bytes, budget is {self.budget}"
            self.rejected.append(req)
            return False
        self.queue.append(req)
        return True

    def _admit(self, now):
        while self.queue:
            req = self.queue[0]
            free = self.budget - self.used
            if req.bytes > free:
                # the single-buffer footprint, when the preferred one does not fit
                if req.alt_bytes is None or req.alt_bytes > free:
                    break
                req.layout, req.bytes = "aa", req.alt_bytes
                self.fallbacks += 1
            self.queue.popleft()
            start_request(self.torch, req, self.device)
            self.used += req.bytes
            req.start = now
            if req.remaining == 0:
                self._retire(req, now)
                continue
            self.batch.admit(req.lat)
            self.active.append(req)
            self._step_s = None

    def _retire(self, req, now):
        if req in self.active:
            self.active.remove(req)
            self.batch.retire(req.lat)
            self._step_s = None
        finish_request(req)
        self.used -= req.bytes
        req.done = now
        self.finished.append(req)

    def tick(self, now):
        """One scheduling step: admit what fits, advance the batch, retire."""
        self._admit(now)
        if not self.active:
            return 0
        left = min(r.remaining for r in self.active)
        n = min(self.tick_steps, left)
        if self.tick_ms > 0 and self._step_s:
            n = min(left, max(n, int(self.tick_ms * 1e-3 / self._step_s)))
        t0 = time.perf_counter()
        self.batch.step(n)
        self.batch.sync()
        self._step_s = (time.perf_counter() - t0) / n
        self.ticks += 1
        self.peak_active = max(self.peak_active, len(self.active))
        self.active_ticks += len(self.active)
        t = time.perf_counter()
        for r in list(self.active):
            r.remaining -= n
            self.site_updates += r.sites * n
            if r.remaining == 0:
                self._retire(r, t)
        return n

    def run(self, requests, clock=time.perf_counter, progress=0.0):
        """Serve `requests` (sorted by arrival time, seconds from now) until
        all are finished.  Arrivals are released by the wall clock.  With
        progress > 0 a status line goes to stderr every `progress` seconds."""
        import sys
        t0 = clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            r.arrival += t0
        last = t0
        while pending or self.queue or self.active:
            if progress > 0 and clock() - last >= progress:
                last = clock()
                print(f"[serve] t={last - t0:.0f}s finished {len(self.finished)}, active {len(self.active)}, "
                      f"queued {len(self.queue)}, pending {len(pending)}", file=sys.stderr, flush=True)
            now = clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.queue and not self.active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - clock(), 0.01)))
                continue
            self.tick(now)
        return clock() - t0

    def close(self):
        self.batch.close()


def summary(server, makespan):
    lat = np.array([r.done - r.arrival for r in server.finished])
    ups = server.site_updates
    return {
        "requests": len(server.finished), "rejected": len(server.rejected),
        "makespan_s": round(makespan, 3),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4) if len(lat) else None,
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4) if len(lat) else None,
        "mlups": round(ups / makespan / 1e6, 1) if makespan > 0 else None,
        "ticks": server.ticks, "layout": server.layout, "aa_fallbacks": server.fallbacks,
        "peak_resident": server.peak_active,
        "mean_resident": round(server.active_ticks / server.ticks, 2) if server.ticks else 0,
        "budget_gb": round(server.budget / 2 ** 30, 2),
    }


def make_requests(n, rate, seed=0, sites=(1e3, 1e8), steps=(1e2, 1e5), precision=4):
    return [Request.from_dict(r, precision) for r in
            inputs.request_stream(n, rate, seed=seed, sites=sites, steps=steps)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-sites", type=float, default=1e8)
    ap.add_argument("--max-steps", type=float, default=1e5)
    ap.add_argument("--budget-gb", type=float, default=0.0)
    ap.add_argument("--tick", type=int, default=64, help="least steps per tick")
    ap.add_argument("--tick-ms", type=float, default=20.0, help="wall-time budget of a tick (0: tick steps only)")
    ap.add_argument("--layout", default="auto", choices=["auto", "aa", "two"])
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    reqs = make_requests(args.requests, args.rate, args.seed, sites=(1e3, args.max_sites),
                         steps=(1e2, args.max_steps))
    S = Server(budget_bytes=int(args.budget_gb * 2 ** 30) if args.budget_gb else None, tick_steps=args.tick,
               layout=args.layout, tick_ms=args.tick_ms)
    mk = S.run(reqs)
    out = summary(S, mk)
    out.update({"rate_per_s": args.rate, "work_site_updates": S.site_updates,
                "budget_gb": round(S.budget / 2 ** 30, 1)})
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
