"""Continuous-batching request loop for guaranteed-bound requests.

Requests (microstructures of any d and N) arrive over time.  A request is
admitted when the batch has free slots for its solves and its plan's workspace
fits the HBM budget (plans are pooled per (d, N, precision) and kept on the
device, so a later request of the same shape reuses one).  An admitted
request's material fields are built at once; its 2d CG solves then join a
shared batch (fftgal_batch_*) together -- plans of grids up to 2^20 points
are made with FFTGAL_CONCURRENT, one buffer set per solve -- and every launch
of the batch advances all active solves of all requests.  Larger grids, whose
single solve already fills the GPU, keep one buffer set (a request's solves
then run one after another), and so does every plan with concurrent=False.
When a request's last solve retires, its bounds are evaluated (FP64
quadrature) and its latency recorded.  Plans are made with FFTGAL_FAST_GRID
by default: orders whose smallest double grid has no specialised kernels run
on a slightly larger grid that has them, with the same bounds.

All scheduling is host logic; every step of the computation runs in the HIP
library.
"""

from __future__ import annotations

import collections
import time

import numpy as np

from . import fftgal


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, float), q)) if len(xs) else float("nan")


class Server:
    def __init__(self, precision="fp32", rtol=5e-6, maxit=20000, capacity=256, hbm_budget=64 << 30,
                 iters_per_step=8, device="cuda:0", concurrent="auto", fast_grid=True):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.rtol = rtol
        self.maxit = maxit
        self.iters_per_step = iters_per_step
        self.hbm_budget = int(hbm_budget)
        self.batch = fftgal.Batch(capacity, device=self.device)
        self.capacity = capacity
        self.pool = collections.defaultdict(list)
        self.used_bytes = 0
        self.peak_bytes = 0
        self.plans_created = 0
        self.concurrent = concurrent
        self.fast_grid = bool(fast_grid)

    def concurrent_for(self, d, N):
        """Whether plans of this shape hold one buffer set per solve."""
        if self.concurrent == "auto":
            return int(np.prod([2 * n - 1 for n in N])) <= (1 << 20)
        return bool(self.concurrent)

    def flags_for(self, d, N):
        return fftgal.PRECISIONS[self.precision] | (fftgal.CONCURRENT if self.concurrent_for(d, N) else 0) | \
            (fftgal.FAST_GRID if self.fast_grid else 0)

    def _plan(self, d, N):
        key = (d, N)
        if self.pool[key]:
            return self.pool[key].pop()
        need = fftgal.fftgal_workspace_bytes(d, N, self.flags_for(d, N))
        if need > self.hbm_budget:
            raise ValueError("a plan of d = %d, N = %s needs %d bytes, more than the HBM budget %d"
                             % (d, N, need, self.hbm_budget))
        # release idle plans of other shapes until the new one fits
        for k in list(self.pool):
            while self.used_bytes + need > self.hbm_budget and self.pool[k]:
                p = self.pool[k].pop()
                self.used_bytes -= p.nbytes
                p.close()
                p.workspace = None
        if self.used_bytes + need > self.hbm_budget:
            return None
        self.used_bytes += need
        self.peak_bytes = max(self.peak_bytes, self.used_bytes)
        self.plans_created += 1
        return fftgal.Plan(d, N, self.precision, device=self.device, stream=self.batch.stream,
                           concurrent=self.concurrent_for(d, N), fast_grid=self.fast_grid)

    def run(self, requests, realtime=True):
        """Serve `requests` (dicts with id, arrival_s, N, micro); returns per-request records."""
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival_s"]))
        waiting = collections.deque()
        active = {}
        by_sid = {}
        n_solves = 0  # batch members
        records = []
        iter_points = 0.0
        deferred = set()  # requests that waited for memory with a slot free
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        sim_now = 0.0
        while pending or waiting or active:
            now = clock() if realtime else sim_now
            while pending and pending[0]["arrival_s"] <= now:
                waiting.append(pending.popleft())
            while waiting:
                req = waiting[0]
                d = int(req["micro"]["d"])
                N = (int(req["N"]),) * d
                width = 2 * d if self.concurrent_for(d, N) else 1  # solves the request adds at once
                if n_solves + width > self.capacity:
                    break
                plan = self._plan(d, N)
                if plan is None:
                    deferred.add(req["id"])
                    break  # wait until a plan's memory is released
                waiting.popleft()
                plan.set_material(req["micro"])
                seq = [(0, a) for a in range(d)] + [(1, a) for a in range(d)]
                st = {"req": req, "plan": plan, "seq": seq, "k": width, "left": len(seq), "t_admit": now,
                      "iters": [], "status": [], "key": (d, N), "pts": float(np.prod([2 * n - 1 for n in N]))}
                for j in range(width):
                    by_sid[self.batch.add(plan, *seq[j], self.rtol, self.maxit)] = st
                n_solves += width
                active[id(plan)] = st
            if active:
                self.batch.step(self.iters_per_step)
                for sid, info, status in self.batch.poll():
                    st = by_sid.pop(sid)
                    n_solves -= 1
                    st["iters"].append(info["iters"])
                    st["status"].append(status)
                    iter_points += info["iters"] * st["pts"]
                    st["left"] -= 1
                    if st["k"] < len(st["seq"]):  # one solve at a time: start the next
                        by_sid[self.batch.add(st["plan"], *st["seq"][st["k"]], self.rtol, self.maxit)] = st
                        st["k"] += 1
                        n_solves += 1
                        continue
                    if st["left"] > 0:
                        continue
                    up, lo, gap = st["plan"].bounds()
                    t_done = clock() if realtime else sim_now
                    req = st["req"]
                    records.append({"id": req["id"], "N": req["N"], "arrival_s": req["arrival_s"],
                                    "admit_s": st["t_admit"], "done_s": t_done,
                                    "latency_s": t_done - req["arrival_s"], "iters": st["iters"],
                                    "status": st["status"],
                                    "upper": up, "lower": lo})
                    del active[id(st["plan"])]
                    self.pool[st["key"]].append(st["plan"])
            elif pending:
                if realtime:
                    time.sleep(max(0.0, pending[0]["arrival_s"] - clock()))
                else:
                    sim_now = pending[0]["arrival_s"]
        wall = time.perf_counter() - t0
        return records, {"wall_s": wall, "Mpoint_iter_per_s": iter_points / wall / 1e6,
                         "plans_created": self.plans_created, "hbm_bytes": self.used_bytes,
                         "peak_hbm_bytes": self.peak_bytes, "deferred_requests": len(deferred)}

    def close(self):
        for plans in self.pool.values():
            for p in plans:
                p.close()
        self.pool.clear()
        self.batch.close()


def sequential(requests, precision="fp64", rtol=1e-10, maxit=20000, device="cuda:0"):
    """The same requests solved one at a time with the plain (unbatched) path:
    one request after another, its solves one after another."""
    import torch
    out = []
    t0 = time.perf_counter()
    plans = {}
    for req in requests:
        d = int(req["micro"]["d"])
        N = (int(req["N"]),) * d
        if N not in plans:
            plans[N] = fftgal.Plan(d, N, precision, device=torch.device(device))
        t = time.perf_counter()
        res = plans[N].run(req["micro"], rtol=rtol, maxit=maxit)
        out.append({"id": req["id"], "seconds": time.perf_counter() - t, "upper": res["upper"],
                    "lower": res["lower"]})
    wall = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    return out, wall
