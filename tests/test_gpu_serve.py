"""Serving: continuous batching by HBM budget on the GPU.

Checks that the budget is never exceeded, oversize requests are refused with
HY_ERR_BUDGET, every served result is bitwise equal to running the same
request alone, and served results match the CPU reference solver.
"""
import numpy as np
import pytest

import oracle
from paper_2409_16053_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_16053_amd import hy as _hy
    _hy.lib()
    return _hy


def _stream(count, rate, max_n=64, seed=21):
    from paper_2409_16053_amd import serve
    reqs = serve.make_stream(seed, count, rate, max_n=max_n)
    for r in reqs:           # keep the test short: at most 30 steps per request
        r.steps = min(r.steps, 30)
    return reqs


@pytest.mark.parametrize("policy", ["oldest-first", "all"])
def test_continuous_batching_equals_alone(hy, policy):
    from paper_2409_16053_amd import serve
    reqs = _stream(14, rate=400.0)
    budget = 3 * max(r.ws_bytes for r in reqs)
    srv = serve.Server(budget_bytes=budget, epoch_steps=7, client_threads=4, policy=policy)
    served = srv.run(reqs)
    assert all(r.status == hy.HY_OK for r in served)
    assert srv.peak_bytes <= budget
    # requests shared launches: some were admitted before others finished
    overlaps = sum(1 for a in served for b in served
                   if a is not b and a.t_admit < b.t_done and b.t_admit < a.t_done)
    assert overlaps > 0
    alone = serve.run_fifo(_stream(14, rate=400.0), client_threads=4)
    for a, b in zip(served, alone):
        assert a.index == b.index
        assert np.array_equal(a.result, b.result), a.index
        assert a.dt_next == b.dt_next and a.t_final == b.t_final
    s = serve.summarize(served)
    assert s["completed"] == 14 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_served_results_match_reference(hy):
    from paper_2409_16053_amd import serve
    reqs = _stream(6, rate=1000.0, max_n=48, seed=22)
    served = serve.Server(budget_bytes=2 * max(r.ws_bytes for r in reqs), epoch_steps=4).run(reqs)
    for r in served:
        pb = r.pb.with_(U=P.generate_state(r.pb))
        ref = oracle.advance(pb, r.steps)
        rel = np.abs(r.result - ref["U"]).sum() / np.abs(ref["U"]).sum()
        tol = 1e-12 if pb.precision == P.FP64 else 1e-5
        print(f"[serve {r.index} {pb.meta['kind']} {pb.n[0]}^3 prec {pb.precision}] rel L1 {rel:.3e}")
        assert rel <= tol


def test_oversize_request_refused(hy):
    from paper_2409_16053_amd import serve
    reqs = _stream(4, rate=1000.0, max_n=48, seed=23)
    big = max(reqs, key=lambda r: r.ws_bytes)
    budget = big.ws_bytes - 1
    served = serve.Server(budget_bytes=budget, epoch_steps=5).run(reqs)
    for r in served:
        if r.ws_bytes > budget:
            assert r.status == hy.HY_ERR_BUDGET and r.result is None
        else:
            assert r.status == hy.HY_OK
