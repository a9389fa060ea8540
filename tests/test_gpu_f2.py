"""GPU parity of the higher-order options: WENO-Z and PPMX reconstruction
and the one-, three- and ten-stage SSP-RK integrators (RK1, RK3 and the
fourth-order SSPRK(10,4)), against the CPU reference solver.

FP64 gate: rel L1 <= 1e-12 and per-variable elementwise agreement <= 1e-9 of
the variable's largest magnitude; mixed precision: rel L1 <= 1e-5 against the
FP64 reference.
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


def _rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def _elem(a, b):
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    return float((np.abs(a - b).reshape(5, -1).max(axis=1) / scale).max())


def _run(hy, pb, steps, variant=None, kc=None):
    g = hy.Problem(pb).set_state()
    if variant is not None:
        g.set_launch(variant, kc)
    g.advance(steps)
    U, q = g.get_state(), g.query()
    g.close()
    return U, q


def _check(hy, pb, steps, label, **kw):
    print(f"[{label}] n={pb.n} block={pb.block} recon={pb.recon} rk={pb.rk} fofc={pb.fofc}",
          flush=True)
    U, q = _run(hy, pb, steps, **kw)
    ref = oracle.advance(pb, steps)
    r, e = _rel(U, ref["U"]), _elem(U, ref["U"])
    print(f"[{label}] rel L1 {r:.3e} elem {e:.3e} dt {q['dt']:.15g}/{ref['dt']:.15g} "
          f"floors {q['floor_hits']}/{ref['floor_hits']} fofc {q['fofc_cells']}/{ref['fofc_cells']}",
          flush=True)
    assert r <= 1e-12 and e <= 1e-9
    assert abs(q["dt"] / ref["dt"] - 1) <= 1e-11
    assert abs(q["t"] - ref["t"]) <= 1e-13 * max(1.0, abs(ref["t"]))
    assert q["floor_hits"] == ref["floor_hits"] and q["fofc_cells"] == ref["fofc_cells"]
    return U, q, ref


@pytest.mark.parametrize("recon,rk", [(P.WENOZ, 3), (P.WENOZ, 2), (P.PLM, 3), (P.PPM4, 3), (P.PPMX, 3),
                                     (P.PPMX, 2), (P.WENOZ, 4), (P.PLM, 4), (P.PPMX, 4),
                                     (P.PLM, 1), (P.WENOZ, 1)])
def test_turbulence_schemes(hy, recon, rk):
    pb = P.turbulence(N=48, seed=3, kmax=8).with_(block=(16, 16, 24), recon=recon, rk=rk)
    _check(hy, pb, 8, f"turb {recon}/{rk}")


@pytest.mark.parametrize("recon,noise", [(P.WENOZ, 0.0), (P.PPMX, 1e-6)])
def test_kh_rk3_ragged_tiles(hy, recon, noise):
    # 40 x 24 x 24 blocks: no tile shape divides 40, so the x tiles are ragged.
    # WENO-Z runs on the exact layer (the reference solver's one-ulp
    # sensitivity there is 2e-16). PPMX's extremum test switches
    # discontinuously where a cell equals its neighbour exactly (the layer's
    # untouched plateaus next to the noisy band: sensitivity 2e-8), so this
    # case perturbs every cell by 1e-6 (sensitivity 2e-16 again); the exact
    # layer with PPMX is checked below against what stays well defined there
    pb = P.kelvin_helmholtz(n=(80, 48, 24), seed=5, bg_noise=noise).with_(block=(40, 24, 24),
                                                                          recon=recon, rk=3)
    _check(hy, pb, 6, f"kh {recon} ragged noise {noise}")


def _kh_exact_ppmx(rk):
    return P.kelvin_helmholtz(n=(80, 48, 24), seed=5).with_(block=(40, 24, 24), recon=P.PPMX, rk=rk)


def test_kh_ppmx_exact_plateaus_tiles_and_conservation(hy):
    # the exact KH layer with PPMX: every tile shape and z-chunk gives the same
    # bits, totals stay constant to roundoff, and the distance to the
    # reference solver stays within 100 x its own one-ulp sensitivity
    from smr_cases import one_ulp_sensitivity
    pb = _kh_exact_ppmx(3)
    outs = [_run(hy, pb, 6, variant=v, kc=kc)[0] for v in range(len(hy.variants())) for kc in (24, 5, 1)]
    for U in outs[1:]:
        assert np.array_equal(U, outs[0])
    U = outs[0]
    s0, s1 = pb.U.reshape(5, -1).sum(1), U.reshape(5, -1).sum(1)
    a = np.abs(pb.U).reshape(5, -1).sum(1)
    a[1:4] = a[1:4].sum()  # momentum roundoff relative to the momentum magnitude (M_z starts at 0)
    cells = U[0].size
    assert np.all(np.abs(s1 - s0) <= 4 * np.finfo(float).eps * np.sqrt(cells * 18) * a), (s1 - s0) / a
    ref = oracle.advance(pb, 6)
    sens = one_ulp_sensitivity(oracle.advance, pb, 6)
    r = _rel(U, ref["U"])
    print(f"[kh ppmx exact] rel L1 {r:.3e}, reference one-ulp sensitivity {sens:.3e}", flush=True)
    assert r <= max(1e-12, 100 * sens)


def _near_ties(W, tol):
    """Cells where, along some axis and for some primitive, the PPMX stencil
    (two cells each side) is not constant but holds two neighbours equal to
    within tol x the variable's scale: there the extremum switch can take
    either branch under rounding-level changes."""
    mask = np.zeros(W.shape[1:], dtype=bool)
    for v in range(5):
        w = W[v]
        scale = max(float(np.abs(w).max()), 1e-300)
        for ax in range(3):
            sh = [np.roll(w, -o, axis=2 - ax) for o in (-2, -1, 0, 1, 2)]
            eq = np.zeros_like(mask)
            for a_, b_ in zip(sh[:-1], sh[1:]):
                eq |= np.abs(b_ - a_) <= tol * scale
            const = np.ones_like(mask)
            for x in sh[1:]:
                const &= x == sh[0]
            mask |= eq & ~const
    return mask


def _dilate_axes(mask, r):
    out = mask.copy()
    for ax in range(3):
        for o in range(1, r + 1):
            out |= np.roll(mask, o, axis=ax) | np.roll(mask, -o, axis=ax)
    return out


def test_kh_ppmx_exact_plateaus_differ_only_near_ties(hy):
    # one forward-Euler step from the exact layer agrees to rounding; in the
    # second, the GPU and the reference solver may take different (equally
    # valid) PPMX branches, but only within a flux stencil (3 cells along an
    # axis) of a cell whose PPMX stencil holds a near-exact tie in the
    # reference solver's state after step 1
    pb = _kh_exact_ppmx(1)
    ref1 = oracle.advance(pb, 1)
    U1, _ = _run(hy, pb, 1)
    assert _rel(U1, ref1["U"]) <= 1e-12
    ref2 = oracle.advance(pb, 2)
    U2, _ = _run(hy, pb, 2)
    scale = np.abs(ref2["U"]).reshape(5, -1).max(1)[:, None, None, None]
    diff = (np.abs(U2 - ref2["U"]) > 1e-12 * scale).any(axis=0)
    u = ref1["U"]
    W = np.empty_like(u)
    W[0] = u[0]
    W[1:4] = u[1:4] / u[0]
    W[4] = u[4] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]
    ties = _near_ties(W, 1e-13)
    allowed = _dilate_axes(ties, 3)
    print(f"[kh ppmx exact] cells differing after 2 steps: {int(diff.sum())}, near-tie cells "
          f"{int(ties.sum())}, outside the tie reach: {int((diff & ~allowed).sum())}", flush=True)
    assert not (diff & ~allowed).any()


@pytest.mark.parametrize("recon", [P.WENOZ, P.PPMX])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sod_rk3_each_axis(hy, axis, recon):
    pb = P.sod(N=64, axis=axis, ntrans=8).with_(block=(8, 8, 8), recon=recon, rk=3)
    pb = pb.with_(block=tuple(32 if pb.n[d] == 64 else 8 for d in range(3)))
    _check(hy, pb, 20, f"sod {recon} axis {axis}")


def test_sedov_outflow_ppmx_rk3(hy):
    # PPMX's extremum tests compare products with 0, which an exactly
    # symmetric blast puts exactly at 0: break the symmetry as for WENO-Z
    pb = P.sedov(N=32, seed=7, noise=1e-6).with_(block=(16, 16, 16), recon=P.PPMX, rk=3)
    _check(hy, pb, 12, "sedov ppmx")


def test_sedov_outflow_wenoz_rk3(hy):
    # WENO-Z's tau5 vanishes on exactly mirror-symmetric stencils, which makes
    # the weights at the centre of an exactly symmetric blast a ratio of
    # rounding errors; a 1e-6 density and pressure perturbation makes the problem well
    # conditioned, so two correct implementations agree to rounding
    pb = P.sedov(N=32, seed=7, noise=1e-6).with_(block=(16, 16, 16), recon=P.WENOZ, rk=3)
    _check(hy, pb, 12, "sedov wenoz")


@pytest.mark.parametrize("recon,rk", [(P.WENOZ, 3), (P.PPM4, 3), (P.PPMX, 3), (P.WENOZ, 4),
                                     (P.PLM, 4), (P.PLM, 1), (P.PPM4, 1)])
def test_fofc_hypersonic_rk3(hy, recon, rk):
    pb = P.turbulence(N=32, seed=5, kmax=8, mach=20).with_(block=(16, 16, 16), recon=recon, rk=rk,
                                                           fofc=1)
    U, q, ref = _check(hy, pb, 12, f"fofc rk{rk} {recon}")
    assert ref["fofc_cells"] > 0


@pytest.mark.parametrize("rk", [1, 4])
def test_sod_rk1_rk4(hy, rk):
    # the mix after stage 5 and the V -> U copy of RK1 run between stages:
    # a discontinuity across several blocks checks their indexing
    pb = P.sod(N=64, axis=1, ntrans=8).with_(block=(8, 32, 8), recon=P.PLM, rk=rk)
    _check(hy, pb, 15, f"sod rk{rk}")


@pytest.mark.parametrize("recon,order", [(P.WENOZ, 4.5), (P.PPMX, 3.8)])
def test_entropy_wave_high_order_on_gpu(hy, recon, order):
    # entropy waves are exact at any amplitude: the GPU path on its own
    # reproduces the fifth order of WENO-Z and the fourth of PPMX (y-axis
    # wave, several blocks)
    errs = []
    for N in (16, 32, 64):
        pb = P.entropy_wave(N=N, amp=0.2, axis=1, ntrans=8).with_(block=(8, N // 2, 8),
                                                                   recon=recon, rk=3, cfl=0.05)
        g = hy.Problem(pb).set_state()
        while True:
            q = g.query()
            if q["t"] + q["dt"] > 1.0:
                break
            g.advance(1)
        U = g.get_state()
        g.close()
        ex = P.entropy_wave(N=N, amp=0.2, axis=1, ntrans=8, t=q["t"]).U
        errs.append(float(np.abs(U[0] - ex[0]).mean() / 0.2))
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(f"[entropy wave gpu {recon}] errs {errs} rates {r}", flush=True)
    assert np.all(r >= order)


@pytest.mark.parametrize("case", ["turb_wenoz", "kh_wenoz", "sedov_wenoz", "turb_ppmx", "sedov_ppmx"])
def test_mixed_rk3_vs_fp64_reference(hy, case):
    recon = P.PPMX if case.endswith("ppmx") else P.WENOZ
    if case.startswith("turb"):
        pb, steps = P.turbulence(N=48, seed=1).with_(block=(24, 24, 24)), 10
    elif case.startswith("kh"):
        pb, steps = P.kelvin_helmholtz(N=48, seed=2).with_(block=(24, 24, 24)), 10
    else:
        # FP32 cannot resolve a 1e-6 break of the blast's mirror symmetry well
        # enough for WENO-Z's weights (tau5 ~ 0 on near-symmetric stencils):
        # there mixed precision departs from FP64 at the 1e-4 level; a 1e-3
        # break keeps it at 1e-7
        noise = 1e-3 if recon == P.WENOZ else 1e-6
        pb, steps = P.sedov(N=32, seed=3, noise=noise).with_(block=(16, 16, 16)), 20
    pb = pb.with_(recon=recon, rk=4 if case == "turb_wenoz" else 3)
    ref = oracle.advance(pb, steps)
    U, _ = _run(hy, pb.with_(precision=P.MIXED), steps)
    r = _rel(U, ref["U"])
    print(f"[mixed {case}] rel L1 vs FP64 reference {r:.3e}", flush=True)
    assert r <= 1e-5


@pytest.mark.xfail(strict=False, reason=(
    "FP32 primitives (6e-8 relative) cannot resolve a 1e-6 break of the blast's mirror "
    "symmetry, where WENO-Z's tau5 is the difference of two nearly equal indicators: the "
    "mixed path departs from FP64 at ~1e-4. Computing the indicators and weights in FP64 "
    "from the same FP32 values leaves it at 7e-5 (CPU build of the kernel), so the loss is "
    "in the FP32 rounding of the inputs, not in the weight arithmetic"))
def test_mixed_wenoz_sedov_small_symmetry_break(hy):
    pb = P.sedov(N=32, seed=3, noise=1e-6).with_(block=(16, 16, 16), recon=P.WENOZ, rk=3)
    ref = oracle.advance(pb, 20)
    U, _ = _run(hy, pb.with_(precision=P.MIXED), 20)
    r = _rel(U, ref["U"])
    print(f"[mixed sedov wenoz 1e-6 break] rel L1 vs FP64 reference {r:.3e}", flush=True)
    assert r <= 1e-5


@pytest.mark.parametrize("recon", [P.WENOZ, P.PPMX])
def test_rk3_every_tile_shape_bitwise(hy, recon):
    pb = P.turbulence(N=32, seed=9, kmax=8).with_(block=(32, 32, 32), recon=recon, rk=3)
    outs = [_run(hy, pb, 5, variant=v, kc=kc)[0]
            for v in range(len(hy.variants())) for kc in (32, 7, 1)]
    for U in outs[1:]:
        assert np.array_equal(U, outs[0])


@pytest.mark.parametrize("recon", [P.PLM, P.PPM4, P.WENOZ, P.PPMX])
@pytest.mark.parametrize("prec", [P.FP64, P.MIXED])
@pytest.mark.parametrize("rk", [1, 3, 4])
def test_uniform_state_rk3(hy, recon, prec, rk):
    # the weights of RK3 and RK4 are not all exact in binary: a few ulps per
    # stage, the same bound the reference solver's own pin uses
    pb = P.uniform(n=(32, 24, 16), rho=1.3, v=(0.3, -0.2, 0.4), p=0.8, bc=P.PERIODIC)
    pb = pb.with_(block=(16, 8, 8), recon=recon, precision=prec, rk=rk)
    U, q = _run(hy, pb, 3)
    nst = {1: 1, 3: 3, 4: 10}[rk]
    ulp = np.spacing(np.abs(pb.U))
    assert np.all(np.abs(U - pb.U) <= 4 * nst * 3 * ulp)
    if rk == 1:
        assert np.array_equal(U, pb.U)
    assert q["floor_hits"] == 0


def test_batch_mixing_integrators_equals_alone(hy):
    pbs = [P.turbulence(N=32, seed=21, kmax=8).with_(block=(16, 16, 16), recon=P.WENOZ, rk=3),
           P.turbulence(N=32, seed=22, kmax=8).with_(block=(16, 16, 16), recon=P.WENOZ, rk=2),
           P.sedov(N=32, seed=23).with_(block=(32, 32, 32), rk=3),
           P.sedov(N=32, seed=24).with_(block=(32, 32, 32)),
           P.kelvin_helmholtz(N=32, seed=25).with_(block=(16, 16, 16), recon=P.PPM4, rk=3,
                                                   precision=P.MIXED),
           P.turbulence(N=32, seed=27, kmax=8).with_(block=(16, 16, 16), recon=P.WENOZ, rk=4),
           P.turbulence(N=32, seed=28, kmax=8, mach=20).with_(block=(16, 16, 16), rk=1, fofc=1),
           P.sedov(N=32, seed=29).with_(block=(16, 32, 16), rk=4, fofc=1)]
    steps = [5, 7, 4, 6, 3, 2, 6, 3]
    alone = [_run(hy, pb, n) for pb, n in zip(pbs, steps)]
    gs = [hy.Problem(pb).set_state() for pb in pbs]
    hy.batch_advance(gs, steps)
    for g, (U, q), n in zip(gs, alone, steps):
        Ub, qb = g.get_state(), g.query()
        assert np.array_equal(Ub, U) and qb["dt"] == q["dt"] and qb["t"] == q["t"]
        assert qb["steps"] == n
        g.close()


@pytest.mark.parametrize("rk", [1, 3, 4])
def test_graph_replay_rk3(hy, rk):
    import torch
    # RK1 and RK4 at Mach 20 so that the flux correction also replays
    extra = {} if rk == 3 else {"mach": 20}
    pb = P.turbulence(N=32, seed=26, kmax=8, **extra).with_(block=(16, 16, 16), recon=P.WENOZ,
                                                           rk=rk, fofc=1)
    ref, qref = _run(hy, pb, 6)
    g = hy.Problem(pb).set_state()
    s = torch.cuda.Stream()
    for r in range(3):  # replays with eager copies and synchronisations between them
        hy.batch_advance_graph([g], [2], stream=s)
        s.synchronize()
        assert g.query()["steps"] == 2 * (r + 1)
    q = g.query()
    assert np.array_equal(g.get_state(), ref)
    assert q["dt"] == qref["dt"] and q["t"] == qref["t"] and q["fofc_cells"] == qref["fofc_cells"]
    g.close()


def test_workspace_has_third_register(hy):
    pb = P.turbulence(N=16, seed=1, kmax=4).with_(block=(8, 8, 8))
    n2 = hy.workspace_bytes(pb)
    n3 = hy.workspace_bytes(pb.with_(rk=3))
    assert n3 - n2 == (16 ** 3 * 5 * 8 + 255) // 256 * 256
    assert hy.workspace_bytes(pb.with_(rk=4)) == n3  # SSPRK(10,4) is low-storage: 3 registers
    assert hy.workspace_bytes(pb.with_(rk=1)) == n2
    for bad in (-1, 5):
        with pytest.raises(hy.HydroError):
            hy.workspace_bytes(pb.with_(rk=bad))


@pytest.mark.parametrize("rk", [1, 4])
def test_state_reload_between_advances(hy, rk):
    # the time-step slot the next step reduces into must start cleared after
    # hy_set_state at either step parity (RK1 has no earlier launch in its
    # step to clear it); each segment is compared with the reference solver
    pa = P.turbulence(N=32, seed=31, kmax=8).with_(block=(16, 16, 16), rk=rk)
    pb = P.sedov(N=32, seed=32).with_(block=(16, 16, 16), rk=rk)
    g = hy.Problem(pa).set_state()
    for k, (pp, n) in enumerate(((pa, 3), (pb, 2), (pa, 1))):
        if k:
            g.set_state(pp.U)
        g.advance(n)
        U, q = g.get_state(), g.query()
        ref = oracle.advance(pp, n)
        assert _rel(U, ref["U"]) <= 1e-12
        assert abs(q["dt"] / ref["dt"] - 1) <= 1e-11, (k, q["dt"], ref["dt"])
    g.close()
