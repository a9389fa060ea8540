"""Continuous-batching server for independent hydro problems on one GPU.

Requests (a problem, a step count, an arrival time) arrive as a Poisson
stream. The server admits waiting requests in arrival order whenever the sum
of resident workspaces stays within an HBM budget (each problem's workspace
is exactly ``hy.workspace_bytes``, because the library allocates nothing
else), keeps admitted states resident, and advances all resident problems
together in epochs of at most ``epoch_steps`` steps with ``hy.batch_advance``
(one launch per RK stage and kernel for the whole resident set). After every
epoch, finished problems are copied back and their memory is released, and
new requests join: requests that arrive while others run are admitted as
soon as memory frees up, and their work shares launches with the running
ones.

Initial states are produced by a client-side thread pool (the stand-in for
clients sending data), ahead of the arrival time; their generation is not
part of the measured latency, which runs from the scheduled arrival to the
result being on the host.

Every problem's per-cell arithmetic is independent of which other problems
share a launch, so a served result equals the result of running the request
alone (tested bitwise).
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np

from . import hy
from . import problems as P


@dataclasses.dataclass
class Request:
    index: int
    pb: object                 # problems.Problem without U until generated
    steps: int
    arrival: float             # seconds after the start of the run
    ws_bytes: int = 0
    status: int = hy.HY_OK
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: np.ndarray | None = None
    dt_next: float = float("nan")
    t_final: float = float("nan")

    @property
    def latency(self):
        return self.t_done - self.arrival

    @property
    def cell_updates(self):
        return self.pb.cells * self.steps


def make_stream(seed: int, count: int, rate: float, max_n: int | None = None):
    """``count`` requests of the seeded stream with Poisson arrivals at ``rate``
    per second (exponential gaps from PCG64(seed)). The problems themselves
    come from ``problems.serving_request``; ``max_n`` caps the mesh size."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(count):
        pb, steps = P.serving_request(seed, q, max_n=max_n, generate=False)
        r = Request(index=q, pb=pb, steps=steps, arrival=float(arrivals[q]))
        r.ws_bytes = hy.workspace_bytes(pb)
        out.append(r)
    return out


class _Client:
    """Generates the initial states of upcoming requests ahead of time."""

    def __init__(self, requests, threads=8, lookahead=32):
        self.reqs = list(requests)
        self.pool = cf.ThreadPoolExecutor(max_workers=threads)
        self.fut = {}
        self.lookahead = lookahead
        self.next = 0

    def prefetch(self, upto):
        while self.next < len(self.reqs) and self.next < upto + self.lookahead:
            r = self.reqs[self.next]
            self.fut[r.index] = self.pool.submit(P.generate_state, r.pb)
            self.next += 1

    def take(self, r):
        U = self.fut.pop(r.index).result()
        return U

    def close(self):
        self.pool.shutdown(wait=False, cancel_futures=True)


class Server:
    """Continuous batching by HBM budget (see the module docstring)."""

    def __init__(self, budget_bytes: int, epoch_steps: int = 10, client_threads: int = 8,
                 tuned: dict | None = None):
        self.budget = int(budget_bytes)
        self.epoch = int(epoch_steps)
        self.client_threads = client_threads
        self.tuned = tuned if tuned is not None else {}
        self.peak_bytes = 0

    def _launch_shape(self, g, pb):
        key = (pb.block, pb.recon, pb.precision)
        if key in self.tuned:
            g.set_launch(*self.tuned[key])

    def run(self, requests):
        """Serve ``requests`` in real time. Returns them (sorted by arrival)
        with status, admission/completion times and results filled in."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        client = _Client(reqs, threads=self.client_threads)
        pending = collections.deque(reqs)
        queue = collections.deque()
        resident = []            # [request, Problem, remaining steps]
        used = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        client.prefetch(0)
        done_count = 0
        try:
            while pending or queue or resident:
                now = clock()
                while pending and pending[0].arrival <= now:
                    queue.append(pending.popleft())
                client.prefetch(done_count + len(resident) + len(queue))
                # admission in arrival order; stop at the first that does not fit
                while queue:
                    r = queue[0]
                    if r.ws_bytes > self.budget:
                        queue.popleft()
                        client.take(r)
                        r.status = hy.HY_ERR_BUDGET
                        r.t_done = clock()
                        done_count += 1
                        continue
                    if used + r.ws_bytes > self.budget:
                        break
                    queue.popleft()
                    U = client.take(r)
                    g = hy.Problem(r.pb)
                    self._launch_shape(g, r.pb)
                    g.set_state(U)
                    del U
                    used += r.ws_bytes
                    self.peak_bytes = max(self.peak_bytes, used)
                    r.t_admit = clock()
                    resident.append([r, g, r.steps])
                if resident:
                    ks = [min(rem, self.epoch) for _, _, rem in resident]
                    hy.batch_advance([g for _, g, _ in resident], ks)
                    for item, k in zip(resident, ks):
                        item[2] -= k
                    keep = []
                    for r, g, rem in resident:
                        if rem == 0:
                            st, U = g.get_state_status()
                            q = g.query(raise_on_state=False)
                            r.status, r.result = st, U
                            r.dt_next, r.t_final = q["dt"], q["t"]
                            g.close()
                            used -= r.ws_bytes
                            r.t_done = clock()
                            done_count += 1
                        else:
                            keep.append([r, g, rem])
                    resident = keep
                elif pending:
                    wait = pending[0].arrival - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.02))
        finally:
            for _, g, _ in resident:
                g.close()
            client.close()
        return reqs


def run_fifo(requests, tuned=None, client_threads=8):
    """One request at a time in arrival order (the plain path)."""
    tuned = tuned or {}
    reqs = sorted(requests, key=lambda r: r.arrival)
    client = _Client(reqs, threads=client_threads)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    client.prefetch(0)
    try:
        for n, r in enumerate(reqs):
            client.prefetch(n)
            wait = r.arrival - clock()
            if wait > 0:
                time.sleep(wait)
            U = client.take(r)
            g = hy.Problem(r.pb)
            key = (r.pb.block, r.pb.recon, r.pb.precision)
            if key in tuned:
                g.set_launch(*tuned[key])
            g.set_state(U)
            r.t_admit = clock()
            g.advance(r.steps)
            st, res = g.get_state_status()
            q = g.query(raise_on_state=False)
            r.status, r.result = st, res
            r.dt_next, r.t_final = q["dt"], q["t"]
            g.close()
            r.t_done = clock()
    finally:
        client.close()
    return reqs


def summarize(reqs, wall=None):
    ok = [r for r in reqs if r.status == hy.HY_OK]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    if wall is None:
        wall = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    cu = sum(r.cell_updates for r in ok)
    return {
        "requests": len(reqs),
        "completed": len(ok),
        "rejected": sum(r.status == hy.HY_ERR_BUDGET for r in reqs),
        "failed": sum(r.status not in (hy.HY_OK, hy.HY_ERR_BUDGET) for r in reqs),
        "wall_s": wall,
        "cell_updates_per_s": cu / wall if wall > 0 else float("nan"),
        "requests_per_s": len(ok) / wall if wall > 0 else float("nan"),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
    }
