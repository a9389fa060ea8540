"""The batched and served workloads at their real sizes.

* 48 Sedov problems of seeded sizes (32^3..128^3), outflow, PLM, mixed
  precision, 50 steps, advanced together in one launch per stage (and
  replayed from a captured HIP graph): every 32^3 and 48^3 member against the
  FP64 CPU reference solver within the mixed-precision gate (rel L1 <= 1e-5),
  and the graph replay equal to the eager batch bitwise.
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


def test_sedov_batch_of_48(hy):
    import torch
    pbs, steps = P.workload_sedov_batch()
    print(f"[sedov batch] {len(pbs)} problems, {sum(p.cells for p in pbs)} cells, {steps} steps",
          flush=True)
    gs = [hy.Problem(pb).set_state() for pb in pbs]
    hy.batch_advance(gs, steps)
    eager = [g.get_state() for g in gs]
    small = [q for q, pb in enumerate(pbs) if pb.n[0] <= 48]
    assert small
    worst = 0.0
    for q in small:
        ref = oracle.advance(pbs[q].with_(precision=P.FP64), steps)
        assert ref["status"] == 0
        r = float(np.abs(eager[q] - ref["U"]).sum() / np.abs(ref["U"]).sum())
        worst = max(worst, r)
        assert r <= 1e-5, (q, pbs[q].n, r)
    print(f"[sedov batch] {len(small)} members checked, worst rel L1 vs FP64 reference {worst:.2e}",
          flush=True)
    s = torch.cuda.Stream()
    for g in gs:
        g.set_state(stream=s)
    hy.batch_advance_graph(gs, [steps] * len(gs), stream=s)
    s.synchronize()
    for g, U in zip(gs, eager):
        assert np.array_equal(g.get_state(), U)
        g.close()
