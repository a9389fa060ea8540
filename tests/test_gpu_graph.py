"""Graph-captured stepping replays the eager launch sequence exactly.

Each replay is checked bitwise against the eager run at the same step count,
with the program's own eager work and synchronisations between replays, and
with an odd step count so that both step parities are captured and replayed.
"""
import numpy as np
import pytest

from paper_2409_16053_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_16053_amd import hy
    hy.lib()
    return hy, torch


def _problems():
    return [
        P.sound_wave(N=32, amp=1e-6).with_(block=(32, 32, 32)),
        P.sedov(N=32, seed=31).with_(block=(16, 16, 16), precision=P.MIXED),
        P.kelvin_helmholtz(N=32, seed=32).with_(block=(16, 16, 16), recon=P.PPM4),
    ]


def test_graph_replays_match_eager(env):
    hy, torch = env
    pbs = _problems()
    steps = [3, 2, 3]
    reps = 4
    eager = [hy.Problem(pb).set_state() for pb in pbs]
    ref = []
    for _ in range(reps):
        hy.batch_advance(eager, steps)
        ref.append([(g.get_state(), g.query()) for g in eager])
    s = torch.cuda.Stream()
    gr = [hy.Problem(pb).set_state(stream=s) for pb in pbs]
    for k in range(reps):
        hy.batch_advance_graph(gr, steps, stream=s)
        # eager work of the program between replays
        x = torch.ones(1 << 20, device="cuda")
        _ = (x * 2).sum().item()
        for g, (U, q) in zip(gr, ref[k]):
            Ug, qg = g.get_state(stream=s), g.query()
            assert np.array_equal(Ug, U), k
            assert qg["t"] == q["t"] and qg["dt"] == q["dt"] and qg["steps"] == q["steps"]
        s.synchronize()
    for g in eager + gr:
        g.close()


def test_graph_rejects_default_stream(env):
    hy, torch = env
    g = hy.Problem(_problems()[0]).set_state()
    with pytest.raises(hy.HydroError):
        hy.lib()
        n = hy._c.c_int32(1)
        hs = (hy._vp * 1)(g.h)
        hy._check(hy.lib().hy_batch_advance_graph(hs, hy._c.byref(n), 1, None))
    g.close()
