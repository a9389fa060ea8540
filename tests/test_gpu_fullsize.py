"""Parity at the full benchmark sizes, in the launch shape the benchmark
times (chosen by the same whole-step autotuning on a scratch copy).

* 256^3 turbulence in 64 MeshBlocks of 64^3, PLM, 20 steps: the whole state
  against the CPU reference solver, FP64 (rel L1 <= 1e-12) and mixed
  precision (<= 1e-5).
* 512^3 Kelvin-Helmholtz in 64 MeshBlocks of 128^3, PPM4: the whole state
  after 2 steps against the reference solver (10 steps of the reference at
  this size take minutes of host time), and over the full 10 steps the
  properties that hold at any size: conservation to roundoff on the periodic
  grid, no floor firings, and FP64 vs mixed agreement within the mixed gate.
* The refined 256^3 mesh of the benchmark (central 2^3 root blocks refined
  once): one step against the reference solver, 20 steps for the same
  properties.
* First-order flux correction on the benchmark's rms Mach 20 turbulence
  (256^3, structure down to 4 cells): 20 steps uniform and 2 steps with the
  central root blocks refined, against the reference solver, corrected-cell
  and floor counts equal.
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


def _run_tuned(hy, pb, steps):
    g = hy.Problem(pb).set_state()
    v, kc, _ = g.autotune_steps(2)
    g.advance(steps)
    U, q = g.get_state(), g.query()
    g.close()
    return U, q, (v, kc)


def test_turbulence_256_full_size(hy):
    pb, steps = P.workload_turbulence_256()
    print(f"[turb256] reference solver, {steps} steps", flush=True)
    ref = oracle.advance(pb, steps)
    for prec, gate in ((P.FP64, 1e-12), (P.MIXED, 1e-5)):
        U, q, shape = _run_tuned(hy, pb.with_(precision=prec), steps)
        r = _rel(U, ref["U"])
        print(f"[turb256 prec {prec}] launch {shape} rel L1 {r:.3e} "
              f"dt {q['dt']:.15g}/{ref['dt']:.15g}", flush=True)
        assert r <= gate
        assert q["steps"] == steps and q["floor_hits"] == 0
        if prec == P.FP64:
            assert abs(q["dt"] / ref["dt"] - 1) <= 1e-11
        del U


def test_kh_512_full_size(hy):
    pb, steps = P.workload_kh_512()
    print("[kh512] reference solver, 2 steps", flush=True)
    ref = oracle.advance(pb, 2)
    U2, q2, shape = _run_tuned(hy, pb, 2)
    r = _rel(U2, ref["U"])
    print(f"[kh512 2 steps] launch {shape} rel L1 {r:.3e}", flush=True)
    assert r <= 1e-12
    del ref, U2
    U, q, _ = _run_tuned(hy, pb, steps)
    assert q["floor_hits"] == 0 and np.isfinite(U).all()
    eps = np.finfo(np.float64).eps
    bound = 4 * eps * np.sqrt(pb.cells * 2 * steps)
    for v in range(5):
        scale = np.abs(pb.U[v]).sum() + np.abs(U[v]).sum()
        assert abs(U[v].sum() - pb.U[v].sum()) <= bound * scale, v
    Um, qm, _ = _run_tuned(hy, pb.with_(precision=P.MIXED), steps)
    r = _rel(Um, U)
    print(f"[kh512 {steps} steps] mixed vs FP64 rel L1 {r:.3e}", flush=True)
    assert r <= 1e-5


def test_turbulence_256_refined_full_size(hy):
    # the refined benchmark mesh (central 2^3 root blocks on level 1, 120
    # leaves of 64^3): one whole step (both stages and the time step) against
    # the reference solver (about 10 s of host time per step at this size),
    # 20 steps for conservation, floors and FP64 vs mixed agreement
    base, steps = P.workload_turbulence_256()
    pb, _ = P.workload_turbulence_refined(hy.leaves(base.with_(refine=P.REFINED_BOX_256)))
    lv = hy.leaves(pb)
    U2, q2, launch = _run_tuned(hy, pb, 1)
    ref = oracle.advance(pb, 1)
    r = _rel(U2, ref["U"])
    print(f"[refined 256 full] launch {launch} rel L1 after 1 step {r:.3e}", flush=True)
    assert r <= 1e-12
    assert abs(q2["dt"] / ref["dt"] - 1) <= 1e-11
    U, q, _ = _run_tuned(hy, pb, steps)
    vol = np.prod(pb.dx) * np.where(lv[:, 0] == 0, 1.0, 0.125)
    s0 = np.einsum("q,qv->v", vol, pb.U.reshape(len(lv), 5, -1).sum(-1))
    s1 = np.einsum("q,qv->v", vol, U.reshape(len(lv), 5, -1).sum(-1))
    a = np.einsum("q,qv->v", vol, np.abs(U).reshape(len(lv), 5, -1).sum(-1))
    assert np.all(np.abs(s1 - s0) <= 1e-13 * a), (s1 - s0) / a
    assert q["floor_hits"] == 0
    Um, _, _ = _run_tuned(hy, pb.with_(precision=P.MIXED), steps)
    rm = _rel(Um, U)
    print(f"[refined 256 full] 20 steps: mixed vs FP64 rel L1 {rm:.3e}", flush=True)
    assert rm <= 1e-5


def _mach20():
    return P.turbulence(N=256, seed=1, kmax=64, mach=20).with_(block=(64, 64, 64), recon=P.PLM, fofc=1)


def test_fofc_mach20_full_size(hy):
    pb = _mach20()
    U, q, launch = _run_tuned(hy, pb, 20)
    ref = oracle.advance(pb, 20)
    r = _rel(U, ref["U"])
    print(f"[fofc mach20 256 full] launch {launch} rel L1 {r:.3e} cells {q['fofc_cells']}/{ref['fofc_cells']} "
          f"floors {q['floor_hits']}/{ref['floor_hits']}", flush=True)
    assert ref["fofc_cells"] > 0 and q["fofc_cells"] == ref["fofc_cells"]
    assert q["floor_hits"] == ref["floor_hits"]
    assert r <= 1e-12 and abs(q["dt"] / ref["dt"] - 1) <= 1e-11


def test_fofc_mach20_refined_full_size(hy):
    m20 = _mach20()
    pb = P.inject_to_leaves(m20, P.REFINED_BOX_256, hy.leaves(m20.with_(refine=P.REFINED_BOX_256)))
    U, q, launch = _run_tuned(hy, pb, 2)
    ref = oracle.advance(pb, 2)
    r = _rel(U, ref["U"])
    print(f"[fofc mach20 refined 256 full] launch {launch} rel L1 {r:.3e} cells {q['fofc_cells']}/"
          f"{ref['fofc_cells']} floors {q['floor_hits']}/{ref['floor_hits']}", flush=True)
    assert ref["fofc_cells"] > 0 and q["fofc_cells"] == ref["fofc_cells"]
    assert q["floor_hits"] == ref["floor_hits"]
    assert r <= 1e-12 and abs(q["dt"] / ref["dt"] - 1) <= 1e-11
