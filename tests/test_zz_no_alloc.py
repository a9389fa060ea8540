"""The allocation-free entry point (hy_advance_noalloc) against the regular
path (hy_create + hy_set_state + hy_advance + hy_get_state) on the same
inputs: two calls in a row, the second with a smaller problem, each equal
bitwise to the regular path (same kernels, same launch shape), with time and
next time step equal too."""
import numpy as np
import pytest

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


def _regular(hy, pb, steps, t0):
    g = hy.Problem(pb).set_state()
    g.set_time(t0)
    g.advance(steps)
    U, q = g.get_state(), g.query()
    g.close()
    return U, q


def _noalloc(hy, pb, steps, t0):
    import torch
    U = torch.from_numpy(np.ascontiguousarray(pb.U)).to("cuda")
    out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    hy.advance_noalloc(pb, U, steps, t0=t0, out=out)
    torch.cuda.synchronize()
    return U.cpu().numpy(), out.cpu().numpy()


def test_noalloc_equals_regular_path_two_calls(hy):
    cases = [
        # larger first: 64^3 turbulence in 32^3 blocks, PLM + RK2, FP64
        (P.turbulence(N=64, seed=11, kmax=8).with_(block=(32, 32, 32)), 5, 0.0),
        # then smaller: Mach-20 turbulence with flux correction, WENO-Z + RK3,
        # mixed precision, 24^3 in 12^3 blocks, starting at t0 = 0.25
        (P.turbulence(N=24, seed=12, kmax=6, mach=20).with_(block=(12, 12, 12), recon=P.WENOZ, rk=3,
                                                           fofc=1, precision=P.MIXED), 4, 0.25),
    ]
    for pb, steps, t0 in cases:
        print(f"[noalloc] n={pb.n} block={pb.block} recon={pb.recon} rk={pb.rk} fofc={pb.fofc} "
              f"prec={pb.precision}", flush=True)
        ref, q = _regular(hy, pb, steps, t0)
        U, out = _noalloc(hy, pb, steps, t0)
        assert np.array_equal(U, ref)
        assert out[0] == q["t"] and out[1] == q["dt"] and out[2] == 0.0
        assert q["steps"] == steps


def test_noalloc_rejects_oversized_and_refined(hy):
    import torch
    big = P.uniform(n=(256, 256, 256), rho=1.0, v=(0, 0, 0), p=1.0).with_(block=(64, 64, 64))
    assert hy.workspace_bytes(big) > hy.NOALLOC_MAX_BYTES
    U = torch.zeros(5 * 256 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(hy.HydroError) as e:
        hy.advance_noalloc(big, U, 1)
    assert e.value.status == hy.HY_ERR_NOMEM and "at most" in hy.last_error()
    del U
    small = P.turbulence(N=32, seed=1, kmax=4).with_(block=(16, 16, 16), refine=((0, 0, 0), (1, 1, 1)))
    Us = torch.zeros(5 * 32 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(hy.HydroError) as e:
        hy.advance_noalloc(small, Us, 1)
    assert e.value.status == hy.HY_ERR_ARG
