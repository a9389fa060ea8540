"""Continuous-batching server for independent hydro problems on one GPU.

Requests (a problem, a step count, an arrival time) arrive as a Poisson
stream. The server admits waiting requests in arrival order whenever the sum
of resident workspaces stays within an HBM budget (each problem's workspace
is exactly ``hy.workspace_bytes``, because the library allocates nothing
else), keeps admitted states resident, and advances resident problems
together in epochs of at most ``epoch_steps`` steps with ``hy.batch_advance``
(one launch per RK stage and kernel for all problems of the epoch). Requests
that arrive while others run join an epoch as soon as memory frees up and the
scheduling policy (below) lets them in, so their work shares launches with the
running ones.

Transfers overlap compute: epochs run on a compute stream, while initial
states go up and results come back through page-locked buffers on separate
upload and download streams, ordered by events (a problem joins an epoch only after its upload
has landed; a result is read only after its last epoch). At most two epochs
are in flight, so newly admitted work waits for at most one queued epoch.

Initial states are produced by a client-side thread pool (the stand-in for
clients sending data) ahead of the arrival time; their generation is not part
of the measured latency, which runs from the scheduled arrival to the result
being on the host.

Scheduling policy ("oldest-first", the default): each epoch advances the
oldest resident problem by its full epoch, and younger resident problems join
it, in arrival order, while the epoch's work (cells x steps) stays within
(1 + slack) x max(the oldest's work, a floor of ``min_epoch_work``). The
oldest request therefore runs at close to its solo speed, as it would on the
one-at-a-time path (which bounds the latency of the largest requests), while
smaller requests ride in the slack instead of queueing behind it. Policy
"all" advances every resident problem in every epoch (processor sharing: the
best median, but a large request then shares the GPU with everything that
arrives while it runs).

Every problem's per-cell arithmetic is independent of which other problems
share a launch, so a served result equals the result of running the request
alone (tested bitwise).
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import hashlib
import time

import numpy as np

from . import hy
from . import problems as P


@dataclasses.dataclass
class Request:
    index: int
    pb: object                 # problems.Problem (U is None until generated)
    steps: int
    arrival: float             # seconds after the start of the run
    ws_bytes: int = 0
    status: int = hy.HY_OK
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: np.ndarray | None = None
    digest: str | None = None
    dt_next: float = float("nan")
    t_final: float = float("nan")

    @property
    def latency(self):
        return self.t_done - self.arrival

    @property
    def cell_updates(self):
        return self.pb.cells * self.steps

    @property
    def state_bytes(self):
        return self.pb.cells * 40


def make_stream(seed: int, count: int, rate: float, max_n: int | None = None,
                inputs: dict | None = None):
    """``count`` requests of the seeded stream with Poisson arrivals at ``rate``
    per second (exponential gaps from PCG64(seed), first arrival at 0). The
    problems come from ``problems.serving_request``; ``max_n`` caps the size.
    ``inputs`` (from ``generate_inputs``) attaches pre-generated states."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(count):
        pb, steps = P.serving_request(seed, q, max_n=max_n, generate=False)
        if inputs is not None and q in inputs:
            pb = pb.with_(U=inputs[q])
        r = Request(index=q, pb=pb, steps=steps, arrival=float(arrivals[q]))
        r.ws_bytes = hy.workspace_bytes(pb)
        out.append(r)
    return out


def generate_inputs(seed: int, count: int, max_n: int | None = None, threads: int = 16):
    """Initial states of the first ``count`` requests of the stream, generated
    in parallel ahead of a run (host memory, keyed by request index)."""
    pbs = [P.serving_request(seed, q, max_n=max_n, generate=False)[0] for q in range(count)]
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return dict(enumerate(ex.map(P.generate_state, pbs)))


def _prepare(pb):
    """A request's initial state in page-locked host memory (generated here
    unless the request carries it already)."""
    import torch
    U = pb.U if pb.U is not None else P.generate_state(pb)
    return torch.from_numpy(U).pin_memory()


class _Client:
    """Generates the initial states of upcoming requests ahead of time, within a
    byte budget of prepared inputs; also digests results off the main thread."""

    def __init__(self, requests, threads=8, max_bytes=8 << 30):
        self.reqs = list(requests)
        self.pool = cf.ThreadPoolExecutor(max_workers=threads)
        self.fut = {}
        self.next = 0
        self.max_bytes = max_bytes
        self.prepared_bytes = 0
        self.post = []

    def prefetch(self):
        while self.next < len(self.reqs):
            r = self.reqs[self.next]
            if self.fut and self.prepared_bytes + r.state_bytes > self.max_bytes:
                break
            self.fut[r.index] = self.pool.submit(_prepare, r.pb)
            self.prepared_bytes += r.state_bytes
            self.next += 1

    def ready(self, r):
        f = self.fut.get(r.index)
        return f is not None and f.done()

    def take(self, r):
        while r.index not in self.fut:
            self.prefetch()
            if r.index not in self.fut:
                time.sleep(0.001)
        t = self.fut.pop(r.index).result()
        self.prepared_bytes -= r.state_bytes
        return t

    def finish(self, r, out, keep):
        """Store or digest a result (pinned tensor) without blocking."""
        def work():
            a = out.numpy()
            if keep == "array":
                r.result = a.copy()
            elif keep == "digest":
                r.digest = hashlib.blake2b(a.tobytes(), digest_size=16).hexdigest()
        self.post.append(self.pool.submit(work))

    def close(self):
        for f in self.post:
            f.result()
        self.pool.shutdown(wait=False, cancel_futures=True)


class Server:
    """Continuous batching by HBM budget (see the module docstring)."""

    def __init__(self, budget_bytes: int, epoch_steps: int = 10, client_threads: int = 8,
                 tuned: dict | None = None, keep: str = "array", policy: str = "oldest-first",
                 slack: float = 0.25, min_epoch_work: float = 4e7):
        if policy not in ("oldest-first", "all"):
            raise ValueError("policy must be 'oldest-first' or 'all'")
        self.budget = int(budget_bytes)
        self.epoch = int(epoch_steps)
        self.policy = policy
        self.slack = float(slack)
        self.min_work = float(min_epoch_work)
        self.client_threads = client_threads
        self.tuned = tuned if tuned is not None else {}
        self.keep = keep
        self.peak_bytes = 0
        self.epochs = 0

    def _launch_shape(self, g, pb):
        key = (tuple(pb.block), pb.recon, pb.precision)
        if key in self.tuned:
            g.set_launch(*self.tuned[key])

    def _select(self, resident):
        """Indices (into the arrival-ordered resident list) of the problems that
        advance in this epoch."""
        if self.policy == "all":
            return list(range(len(resident)))
        work = [r.pb.cells * min(rem, self.epoch) for r, _, rem in resident]
        cap = (1.0 + self.slack) * max(work[0], self.min_work)
        sel, tot = [], 0.0
        for i, w in enumerate(work):
            if not sel or tot + w <= cap:
                sel.append(i)
                tot += w
        return sel

    def run(self, requests, progress=None):
        """Serve ``requests`` in real time; returns them sorted by arrival with
        status, admission/completion times and results (or digests) filled in.
        ``progress(done, total)`` is called after every 100th completion."""
        import torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        client = _Client(reqs, threads=self.client_threads)
        # uploads and downloads on their own streams, so an upload never queues
        # behind a download that is waiting for the running epoch
        compute, up, down = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
        pending = collections.deque(reqs)
        queue = collections.deque()
        admitting, resident, retiring, inflight = [], [], [], collections.deque()
        used = 0
        finished = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        try:
            while pending or queue or admitting or resident or retiring:
                progressed = False
                now = clock()
                while pending and pending[0].arrival <= now:
                    queue.append(pending.popleft())
                client.prefetch()
                gpu_busy = bool(resident or admitting or retiring)
                # admission in arrival order by budget; do not stall a busy GPU
                # waiting for an input that is still being prepared
                while queue:
                    r = queue[0]
                    if r.ws_bytes > self.budget:
                        queue.popleft()
                        client.take(r)
                        r.status = hy.HY_ERR_BUDGET
                        r.t_done = clock()
                        continue
                    if used + r.ws_bytes > self.budget:
                        break
                    if gpu_busy and not client.ready(r):
                        break
                    queue.popleft()
                    t = client.take(r)
                    g = hy.Problem(r.pb)
                    self._launch_shape(g, r.pb)
                    g.set_state_pinned(t, stream=up)
                    ev = torch.cuda.Event()
                    ev.record(up)
                    admitting.append((r, g, ev, t))
                    used += r.ws_bytes
                    self.peak_bytes = max(self.peak_bytes, used)
                    gpu_busy = progressed = True
                # uploads that have landed join the resident set
                if admitting and not resident and not any(a[2].query() for a in admitting):
                    admitting[0][2].synchronize()
                still = []
                for r, g, ev, t in admitting:
                    if ev.query():
                        compute.wait_event(ev)
                        r.t_admit = clock()
                        resident.append([r, g, r.steps])
                        progressed = True
                    else:
                        still.append((r, g, ev, t))
                admitting = still
                # one epoch of the resident set (at most two epochs in flight)
                if resident:
                    while len(inflight) >= 2:
                        inflight.popleft().synchronize()
                    sel = self._select(resident)
                    ks = [min(resident[i][2], self.epoch) for i in sel]
                    hy.batch_advance([resident[i][1] for i in sel], ks, stream=compute)
                    ev_c = torch.cuda.Event()
                    ev_c.record(compute)
                    inflight.append(ev_c)
                    self.epochs += 1
                    keep = []
                    step_of = dict(zip(sel, ks))
                    for i, item in enumerate(resident):
                        item[2] -= step_of.get(i, 0)
                        r, g, rem = item
                        if i in step_of and rem == 0:
                            down.wait_event(ev_c)
                            out = torch.empty(g.shape, dtype=torch.float64, pin_memory=True)
                            g.get_state_pinned(out, stream=down)
                            ev_r = torch.cuda.Event()
                            ev_r.record(down)
                            retiring.append((r, g, ev_r, out))
                        else:
                            keep.append(item)
                    resident = keep
                    progressed = True
                # results that have reached the host
                still = []
                for r, g, ev_r, out in retiring:
                    if ev_r.query():
                        q = g.query(raise_on_state=False)
                        r.status = q["status"]
                        r.dt_next, r.t_final = q["dt"], q["t"]
                        g.close()
                        used -= r.ws_bytes
                        r.t_done = clock()
                        client.finish(r, out, self.keep)
                        progressed = True
                        finished += 1
                        if progress and finished % 100 == 0:
                            progress(finished, len(reqs))
                    else:
                        still.append((r, g, ev_r, out))
                retiring = still
                if not progressed:
                    if pending and not (queue or admitting or resident or retiring):
                        time.sleep(max(0.0, min(pending[0].arrival - clock(), 0.01)))
                    else:
                        time.sleep(0.0002)
        finally:
            torch.cuda.synchronize()
            for item in resident:
                item[1].close()
            for a in admitting + retiring:
                a[1].close()
            client.close()
        return reqs


def run_fifo(requests, tuned=None, client_threads=8, keep="array", progress=None):
    """The plain path: one request at a time in arrival order, the same
    page-locked transfers, no overlap between requests. ``progress(done,
    total)`` is called after every 100th completion."""
    import torch
    tuned = tuned or {}
    reqs = sorted(requests, key=lambda r: r.arrival)
    client = _Client(reqs, threads=client_threads)
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    try:
        for r in reqs:
            client.prefetch()
            wait = r.arrival - clock()
            if wait > 0:
                time.sleep(wait)
            t = client.take(r)
            g = hy.Problem(r.pb)
            key = (tuple(r.pb.block), r.pb.recon, r.pb.precision)
            if key in tuned:
                g.set_launch(*tuned[key])
            g.set_state_pinned(t, stream=s)
            r.t_admit = clock()
            g.advance(r.steps, stream=s)
            out = torch.empty(g.shape, dtype=torch.float64, pin_memory=True)
            g.get_state_pinned(out, stream=s)
            s.synchronize()
            q = g.query(raise_on_state=False)
            r.status = q["status"]
            r.dt_next, r.t_final = q["dt"], q["t"]
            g.close()
            r.t_done = clock()
            client.finish(r, out, keep)
            if progress and (r.index + 1) % 100 == 0:
                progress(r.index + 1, len(reqs))
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
