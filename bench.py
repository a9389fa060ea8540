"""Throughput of the 3D hydro update on one MI355X.

Workload: 256^3 periodic turbulence (seeded solenoidal velocity field, k^-5/3
over k = 1..16, rms Mach 0.5) in 64 MeshBlocks of 64^3, PLM + HLLC, SSP-RK2,
CFL 0.3. One "step" is one full RK2 time step through the whole hot path
(ghost zones, cons-to-prim, reconstruction, HLLC in x/y/z, divergence, both
RK stages, CFL reduction). `value` is cell-updates/s in FP64 (interior cells x
steps / wall seconds, state resident in HBM); the mixed-precision path is
timed the same way and reported beside it.

Prints one JSON line. Beside the headline it reports, unless switched off:
  fofc      first-order flux correction: idle cost on the headline state, and
            rms Mach 20 turbulence (uniform, and refined) where it fires
  kh512     the 512^3 Kelvin-Helmholtz workload (64 MeshBlocks of 128^3, PPM4,
            10 steps), FP64 and mixed
  schemes   the 256^3 workload with WENO-Z + SSP-RK3 and PPMX + SSP-RK3 (FP64
            and mixed) and PPM4 + RK2 (FP64)
  batch     48 Sedov problems of seeded sizes, one launch per stage for all
  serving   a seeded Poisson stream of requests, continuous batching by HBM
            budget against one request at a time (p50/p99 latency)
  small_problem, cpu_baseline
Options:
  --copy-probe BYTES   run the library's plain copy kernel on a buffer of BYTES
                       (used to calibrate rocprofv3 byte counters)
  --skip-cpu           skip the CPU reference-solver baseline
  --headline-only      only the 256^3 FP64/mixed lines (profiling runs)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s 3D PLM+HLLC RK2, FP64 vs mixed; % HBM roofline; p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per interior cell and launch: stage 1 reads U and
# writes V (2 x 40 B); stage 2 reads V and U and writes U (3 x 40 B)
BYTES_STAGE = {1: 80.0, 2: 120.0}
COUNTERS = os.path.join(ROOT, "profiles", "stage_turbulence256_counters.json")
# FP64 vector lanes per second: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz
# (one FP64 add, mul or fma per lane per clock; 78.6 TFLOP/s counts an fma
# as two flops)
FP64_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank lines removed (a
    comment edit does not change the kernels the counters were taken on) and
    of the compiler flags other than include paths."""
    import re
    from paper_2409_16053_amd import build
    h = hashlib.sha256()
    h.update(" ".join(f for f in build.CFLAGS if not f.startswith("-I")).encode())
    for f in ("hy_kernels.hip", "hy_internal.h"):
        with open(os.path.join(ROOT, "paper_2409_16053_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        src = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(src.encode())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--launch", default="auto",
                    help="tile variant and z-chunk as V,KC (FP64 and mixed), or 'auto' to autotune")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 48-problem Sedov batch (mixed, 50 steps)")
    ap.add_argument("--serve", type=int, default=1000, metavar="COUNT",
                    help="serve COUNT requests of the seeded Poisson stream (0: skip)")
    ap.add_argument("--skip-kh", action="store_true", help="skip the 512^3 PPM4 workload")
    ap.add_argument("--skip-schemes", action="store_true", help="skip WENO-Z/RK3 and PPM4 at 256^3")
    ap.add_argument("--skip-refined", action="store_true",
                    help="skip the statically refined 256^3 workload")
    ap.add_argument("--refined-only", action="store_true",
                    help="time only the statically refined workload (for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the two batch workloads (for profiling)")
    ap.add_argument("--skip-fofc", action="store_true", help="skip the first-order flux correction lines")
    ap.add_argument("--fofc-only", action="store_true",
                    help="time only the first-order flux correction workloads (for profiling)")
    ap.add_argument("--schemes-only", action="store_true",
                    help="time only the higher-order schemes at 256^3 (for profiling)")
    ap.add_argument("--kh-only", action="store_true",
                    help="time only the 512^3 PPM4 workload (for profiling)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 256^3 FP64 (and mixed) lines")
    ap.add_argument("--serve-budget-gb", default="16,8,64",
                    help="HBM budget(s) in GiB for continuous batching, comma-separated")
    ap.add_argument("--serve-policies", default="oldest-first",
                    help="continuous-batching policies to run (oldest-first, all), comma-separated")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(halo exchange across GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_16053_amd import hy
    from paper_2409_16053_amd import problems as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe:
        nb = args.copy_probe // 16 * 16
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            hy.copy_probe(dst, src, nb)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {nb} bytes")

    log(f"building workload: turbulence {args.N}^3 in blocks of {args.block}^3")
    pb, _ = P.workload_turbulence_256(N=args.N, block=args.block)
    cells = pb.cells

    def run(precision, prob=None, steps=None):
        prob = pb if prob is None else prob
        steps = args.steps if steps is None else steps
        g = hy.Problem(prob.with_(precision=precision)).set_state()
        if args.launch == "auto":
            g.autotune_steps(2)
        else:
            v, kc = (int(x) for x in args.launch.split(","))
            g.set_launch(v, kc)
        g.advance(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms1, ms2 = g.advance_timed(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        q = g.query()
        U = g.get_state()
        launch = g.get_launch()
        g.close()
        sec = t1 - t0
        return dict(sec=sec, ms1=ms1, ms2=ms2, q=q, U=U, launch=launch)

    if args.batch_only:
        print(json.dumps({"batch": run_batch_workload(hy, P, torch),
                          "batch_small": run_batch_workload(hy, P, torch, seed=5, sizes=(32, 48),
                                                            label="small")}), flush=True)
        return

    if args.refined_only:
        print(json.dumps({"refined": run_refined(run, hy, P, None, args.steps, cpu=not args.skip_cpu)}),
              flush=True)
        return

    if args.kh_only:
        print(json.dumps({"kh512": run_kh512(run, P, hy, cpu=not args.skip_cpu)}), flush=True)
        return

    if args.schemes_only:
        print(json.dumps({"schemes": run_schemes(run, pb, P, args.steps)}), flush=True)
        return

    if args.fofc_only:
        print(json.dumps({"fofc": run_fofc(run, hy, P, args.steps, None)}), flush=True)
        return

    log("timing FP64")
    r64 = run(P.FP64)
    value = cells * args.steps / r64["sec"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r64["sec"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"turbulence {args.N}^3 periodic, {(args.N // args.block) ** 3} MeshBlocks of "
                        f"{args.block}^3, PLM+HLLC, SSP-RK2, CFL 0.3, rho=1 P=1, rms Mach 0.5, seed 1",
            "cells": cells,
            "tile_variant": list(hy.variants()[r64["launch"][0]]) + [r64["launch"][1]],
            "launch": list(r64["launch"]),
        },
    }

    # live per-kernel times from HIP events on the launch stream
    a1 = r64["ms1"] / args.steps * 1e-3
    a2 = r64["ms2"] / args.steps * 1e-3
    dom = 2 if a2 >= a1 else 1
    avg = a2 if dom == 2 else a1
    achieved = BYTES_STAGE[dom] * cells / avg / 1e9
    launch_key = "{},{}".format(*r64["launch"])
    counters = launch_counters(cells, launch_key)
    traffic = counters.get(f"stage{dom}_hbm_bytes_per_launch") if counters else None
    out["roofline"] = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "k_stage<0, double, {}, {}, {}, {}, false>".format(*hy.variants_full()[r64["launch"][0]], dom),
        "avg_launch_ms": avg * 1e3,
        "other_stage_avg_launch_ms": (a1 if dom == 2 else a2) * 1e3,
        "bytes_per_cell": BYTES_STAGE[dom],
    }

    if not args.skip_mixed:
        log("timing mixed precision")
        rmx = run(P.MIXED)
        rel = float(np.abs(rmx["U"] - r64["U"]).sum() / np.abs(r64["U"]).sum())
        out["mixed"] = {
            "value": cells * args.steps / rmx["sec"],
            "ms_per_step": 1e3 * rmx["sec"] / args.steps,
            "stage1_ms": rmx["ms1"] / args.steps,
            "stage2_ms": rmx["ms2"] / args.steps,
            "tile_variant": list(hy.variants()[rmx["launch"][0]]) + [rmx["launch"][1]],
            "rel_l1_vs_fp64_gpu": rel,
            "dtype": "f32 reconstruct/Riemann, f64 state/divergence/dt",
        }

    if not args.skip_cpu and not args.headline_only:
        import oracle
        oracle.build(force=False)
        nsteps = args.cpu_steps
        log(f"timing the CPU reference solver ({nsteps} steps on the full mesh)")
        t0 = time.perf_counter()
        r = oracle.advance(pb, nsteps)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": cells * nsteps / (t1 - t0),
            "unit": "cell-updates/s",
            "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"{nsteps} RK2 steps of the same {args.N}^3 turbulence state (FP64, PLM+HLLC), "
                      f"{t1 - t0:.1f} s wall",
        }
        assert r["status"] == 0
        # full-size parity on the same steps: the FP64 and mixed GPU paths
        # against the reference solver's result
        ref_rel = rel_l1_vs_reference(hy, P, pb, nsteps, r["U"])
        out["parity_full_size"] = {"steps": nsteps, "fp64_rel_l1_vs_oracle": ref_rel["fp64"],
                                   "mixed_rel_l1_vs_oracle": ref_rel["mixed"],
                                   "gates": {"fp64": 1e-12, "mixed": 1e-5}}
        if "mixed" in out:
            out["mixed"]["rel_l1_vs_oracle"] = ref_rel["mixed"]
            out["mixed"]["rel_l1_vs_oracle_steps"] = nsteps
        # one host thread, on a 128^3 cut of the same workload (one step)
        threads = oracle.get_threads()
        small, _ = P.workload_turbulence_256(N=128, block=64)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.advance(small, 1)
        t1 = time.perf_counter()
        oracle.set_threads(threads)
        out["cpu_baseline"]["single_thread"] = {
            "value": small.cells / (t1 - t0), "unit": "cell-updates/s", "cores": 1,
            "sample": f"1 RK2 step of 128^3 turbulence (same recipe), {t1 - t0:.1f} s wall"}

    valu = valu_summary(counters, cells, a1 if dom == 1 else a2, dom)
    if valu is not None:
        out["roofline"]["valu"] = valu

    if not args.headline_only:
        out["small_problem"] = run_small_workload(hy, P, torch)
        if not args.skip_schemes:
            out["schemes"] = run_schemes(run, pb, P, args.steps)
        if not args.skip_kh:
            out["kh512"] = run_kh512(run, P, hy, cpu=not args.skip_cpu)
        if not args.skip_refined:
            out["refined"] = run_refined(run, hy, P, value, args.steps, cpu=not args.skip_cpu)
        if not args.skip_fofc:
            out["fofc"] = run_fofc(run, hy, P, args.steps, value)
        if not args.no_batch:
            out["batch"] = run_batch_workload(hy, P, torch)
            out["batch_small"] = run_batch_workload(hy, P, torch, seed=5, sizes=(32, 48),
                                                    label="small")
        if args.serve:
            out["serving"] = run_serving_workload(hy, P, args.serve, args.serve_budget_gb,
                                                  policies=args.serve_policies)

    print(json.dumps(out), flush=True)


def launch_counters(cells, launch):
    """The committed counter summary of the dominant stage kernels for one
    launch shape ("variant,kc"), if it was taken on the current kernel source
    and workload size; else None."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("kernel_source_hash") != kernel_source_hash() or c.get("cells") != cells:
        return None
    return c.get("by_launch", {}).get(launch)


def valu_summary(c, cells, avg_s, stage):
    """FP64 vector work of the dominant stage kernel from the committed SQ
    counters of its launch shape (instructions per launch, wave-level):
    issued FP64 lane operations per second against the chip's FP64 lane
    rate."""
    if not c:
        return None
    n = c.get(f"stage{stage}_fp64_valu_insts_per_launch")
    if n is None:
        return None
    ops = 64.0 * n / avg_s
    # wave-level instruction counts x 64 lanes = per-cell lane instructions
    return {"fp64_lane_ops_per_s": ops, "peak": FP64_LANE_OPS_PEAK, "frac": ops / FP64_LANE_OPS_PEAK,
            "fp64_lane_insts_per_cell": 64.0 * n / cells,
            "valu_lane_insts_per_cell": 64.0 * c.get(f"stage{stage}_valu_insts_per_launch", 0) / cells}


def run_schemes(run, pb, P, steps):
    """The 256^3 workload with the paper's higher-order options (RK4 is the
    ten-stage SSPRK(10,4): a step costs five RK2 steps but allows a CFL up to
    six times larger; the rate here is per step at the same CFL 0.3)."""
    res = {}
    for name, kw, precs in (("wenoz_rk3", dict(recon=P.WENOZ, rk=3), (P.FP64, P.MIXED)),
                            ("ppmx_rk3", dict(recon=P.PPMX, rk=3), (P.FP64, P.MIXED)),
                            ("ppm4_rk2", dict(recon=P.PPM4, rk=2), (P.FP64,)),
                            ("plm_rk4", dict(recon=P.PLM, rk=4), (P.FP64,)),
                            ("wenoz_rk4", dict(recon=P.WENOZ, rk=4), (P.FP64,))):
        for prec in precs:
            log(f"timing {name} {'fp64' if prec == P.FP64 else 'mixed'}")
            r = run(prec, prob=pb.with_(**kw), steps=steps)
            res[f"{name}_{'fp64' if prec == P.FP64 else 'mixed'}"] = {
                "value": pb.cells * steps / r["sec"], "unit": "cell-updates/s",
                "ms_per_step": 1e3 * r["sec"] / steps, "launch": list(r["launch"])}
    return res


def run_refined(run, hy, P, uniform_value, steps, cpu=True):
    """The 256^3 turbulence mesh with its central 2^3 root blocks refined once
    (120 leaf MeshBlocks of 64^3), FP64 and mixed: throughput over all leaf
    cells, its ratio to the uniform headline rate per cell-update (the cost of
    the ghost slabs, the flux correction and the extra time step), and the
    reference solver's rate on one step of the same mesh."""
    log("building the refined 256^3 turbulence mesh")
    base, _ = P.workload_turbulence_256()
    base = base.with_(refine=P.REFINED_BOX_256)
    pb, _ = P.workload_turbulence_refined(hy.leaves(base))
    lv = hy.leaves(pb)
    out = {"workload": "turbulence 256^3 periodic, central 2^3 of 4^3 root blocks refined once: "
                       f"{int((lv[:, 0] == 0).sum())} MeshBlocks of 64^3 on level 0, "
                       f"{int((lv[:, 0] == 1).sum())} on level 1, PLM+HLLC, SSP-RK2",
           "cells": pb.cells, "steps": steps}
    for prec in (P.FP64, P.MIXED):
        name = "fp64" if prec == P.FP64 else "mixed"
        log(f"timing refined {name}")
        r = run(prec, prob=pb, steps=steps)
        out[name] = {"value": pb.cells * steps / r["sec"], "unit": "cell-updates/s",
                     "ms_per_step": 1e3 * r["sec"] / steps, "launch": list(r["launch"])}
    if uniform_value:
        out["fp64"]["rate_vs_uniform"] = out["fp64"]["value"] / uniform_value
    if cpu:
        import oracle
        oracle.build(force=False)
        log("timing the CPU reference solver on one step of the refined mesh")
        t0 = time.perf_counter()
        oracle.advance(pb, 1)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {"value": pb.cells / (t1 - t0), "unit": "cell-updates/s",
                               "cores": oracle.get_threads(), "kind": "oracle",
                               "sample": f"1 RK2 step of the refined mesh, {t1 - t0:.1f} s wall"}
    return out


def run_fofc(run, hy, P, steps, uniform_value):
    """First-order flux correction (Sec. 3) on 256^3 meshes of 64^3 blocks,
    PLM+HLLC, SSP-RK2, FP64: the headline state with FOFC on (a flow that
    stays positive, so the cost of FOFC when it never fires), and rms Mach 20
    turbulence with structure down to 4 cells (k = 1..64), where the plain
    scheme needs the floors
    and FOFC fires, without and with FOFC, uniform and with the central 2^3
    root blocks refined once (fine leaves injected from their parents)."""
    out = {"steps": steps}
    base, _ = P.workload_turbulence_256()
    log("timing FOFC on the headline state")
    r = run(P.FP64, prob=base.with_(fofc=1), steps=steps)
    out["idle"] = {"workload": "the headline turbulence 256^3 (rms Mach 0.5) with FOFC on",
                   "value": base.cells * steps / r["sec"], "unit": "cell-updates/s",
                   "ms_per_step": 1e3 * r["sec"] / steps, "fofc_cells": r["q"]["fofc_cells"]}
    if uniform_value:
        out["idle"]["rate_vs_fofc_off"] = out["idle"]["value"] / uniform_value
    log("building rms Mach 20 turbulence 256^3")
    m20 = P.turbulence(N=256, seed=1, kmax=64, mach=20).with_(block=(64, 64, 64), recon=P.PLM)
    for name, prob in (("mach20_off", m20), ("mach20", m20.with_(fofc=1))):
        log(f"timing {name}")
        r = run(P.FP64, prob=prob, steps=steps)
        out[name] = {"value": m20.cells * steps / r["sec"], "unit": "cell-updates/s",
                     "ms_per_step": 1e3 * r["sec"] / steps, "fofc_cells": r["q"]["fofc_cells"],
                     "floor_hits": r["q"]["floor_hits"]}
    out["mach20"]["workload"] = ("turbulence 256^3 periodic, k^-5/3 over k = 1..64, rms Mach 20, "
                                 "64 MeshBlocks of 64^3, FOFC on")
    log("timing refined rms Mach 20 with FOFC")
    pr = P.inject_to_leaves(m20, P.REFINED_BOX_256, hy.leaves(m20.with_(refine=P.REFINED_BOX_256)))
    r = run(P.FP64, prob=pr.with_(fofc=1), steps=steps)
    out["mach20_refined"] = {"workload": "the rms Mach 20 state with the central 2^3 of 4^3 root blocks "
                                         "refined once (120 leaves of 64^3), FOFC on",
                             "value": pr.cells * steps / r["sec"], "unit": "cell-updates/s",
                             "ms_per_step": 1e3 * r["sec"] / steps, "fofc_cells": r["q"]["fofc_cells"],
                             "floor_hits": r["q"]["floor_hits"]}
    return out


def rel_l1_vs_reference(hy, P, pb, nsteps, ref):
    """Relative L1 (five variables pooled) of the FP64 and mixed GPU paths
    after nsteps steps from pb's initial state, against the reference
    solver's result ``ref`` for the same steps."""
    out = {}
    for prec, name in ((P.FP64, "fp64"), (P.MIXED, "mixed")):
        g = hy.Problem(pb.with_(precision=prec)).set_state()
        g.advance(nsteps)
        Ug = g.get_state()
        g.close()
        out[name] = float(np.abs(Ug - ref).sum() / np.abs(ref).sum())
    return out


def run_kh512(run, P, hy=None, cpu=False):
    """512^3 periodic Kelvin-Helmholtz layer in 64 MeshBlocks of 128^3, PPM4,
    10 steps: FP64 and mixed throughput."""
    log("building 512^3 Kelvin-Helmholtz")
    pb, steps = P.workload_kh_512()
    out = {"workload": "Kelvin-Helmholtz 512^3 periodic, 64 MeshBlocks of 128^3, PPM4+HLLC, SSP-RK2, "
                       "CFL 0.3, seed 2", "steps": steps}
    res = {}
    for prec in (P.FP64, P.MIXED):
        log(f"timing kh512 {'fp64' if prec == P.FP64 else 'mixed'}")
        res[prec] = run(prec, prob=pb, steps=steps)
    out["fp64"] = {"value": pb.cells * steps / res[P.FP64]["sec"], "unit": "cell-updates/s",
                   "ms_per_step": 1e3 * res[P.FP64]["sec"] / steps, "launch": list(res[P.FP64]["launch"])}
    out["mixed"] = {"value": pb.cells * steps / res[P.MIXED]["sec"], "unit": "cell-updates/s",
                    "ms_per_step": 1e3 * res[P.MIXED]["sec"] / steps,
                    "launch": list(res[P.MIXED]["launch"]),
                    "rel_l1_vs_fp64_gpu": float(np.abs(res[P.MIXED]["U"] - res[P.FP64]["U"]).sum()
                                                / np.abs(res[P.FP64]["U"]).sum())}
    if cpu:
        import oracle
        oracle.build(force=False)
        log("kh512: one step of the reference solver for the L1 comparison")
        t0 = time.perf_counter()
        ref = oracle.advance(pb, 1)
        t1 = time.perf_counter()
        rel = rel_l1_vs_reference(hy, P, pb, 1, ref["U"])
        out["fp64"]["rel_l1_vs_oracle"] = rel["fp64"]
        out["mixed"]["rel_l1_vs_oracle"] = rel["mixed"]
        out["oracle_step_s"] = t1 - t0
        out["rel_l1_vs_oracle_steps"] = 1
    return out


def run_small_workload(hy, P, torch, reps=20):
    """The 32^3 single-MeshBlock eigenmode (10 steps, FP64): time per step with
    eager launches and replayed from a captured HIP graph (launch-bound size)."""
    pb, steps = P.workload_eigenmode_32()
    s = torch.cuda.Stream()
    g = hy.Problem(pb).set_state(stream=s)
    g.advance(steps, stream=s)
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.advance(steps, stream=s)
    s.synchronize()
    eager = (time.perf_counter() - t0) / (reps * steps)
    hy.batch_advance_graph([g], [steps], stream=s)
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        hy.batch_advance_graph([g], [steps], stream=s)
    s.synchronize()
    graph = (time.perf_counter() - t0) / (reps * steps)
    g.close()
    # accuracy of the same 10 steps against the closed-form eigenmode
    g = hy.Problem(pb).set_state(stream=s)
    g.advance(steps, stream=s)
    s.synchronize()
    q = g.query()
    U = g.get_state()
    g.close()
    amp = pb.meta["amp"]
    ex = P.sound_wave(N=pb.n[0], amp=amp, t=q["t"]).U
    return {"workload": "sound-wave eigenmode 32^3, one MeshBlock, FP64, PLM+HLLC, 10 steps",
            "us_per_step_eager": eager * 1e6, "us_per_step_graph": graph * 1e6,
            "cell_updates_per_s_graph": pb.cells / graph,
            "l1_rho_vs_closed_form_over_amplitude": float(np.abs(U[0] - ex[0]).mean() / amp)}


def run_batch_workload(hy, P, torch, count=48, seed=3, sizes=None, label="sedov_c4"):
    """``count`` independent Sedov problems (sizes drawn by seed, by default
    from 32..128^3), outflow, PLM + HLLC, RK2, 50 steps each, mixed precision:
    aggregate cell-updates/s with one launch per RK stage for all problems,
    against the same problems advanced one at a time (also per size class)."""
    kw = {} if sizes is None else {"sizes": sizes}
    pbs, steps = P.workload_sedov_batch(count=count, seed=seed, **kw)
    cells = sum(p.cells for p in pbs)
    log(f"batch {label}: {count} Sedov problems, {cells} cells, {steps} steps")
    gs = [hy.Problem(p) for p in pbs]
    tuned = {}
    for g, p in zip(gs, pbs):       # autotune once per size class
        g.set_state()
        key = p.n
        if key not in tuned:
            tuned[key] = g.autotune_steps(2)
        else:
            g.set_launch(*tuned[key][:2])
    torch.cuda.synchronize()
    # one at a time, each in its own tuned shape; time per size class too
    per_class = {}
    t0 = time.perf_counter()
    for g, p in zip(gs, pbs):
        t1 = time.perf_counter()
        g.advance(steps)
        torch.cuda.synchronize()
        c = per_class.setdefault(f"{p.n[0]}^3", [0, 0.0])
        c[0] += 1
        c[1] += time.perf_counter() - t1
    t_one = time.perf_counter() - t0
    # the batch shares one tile shape per launch: tune it for the batch as a
    # whole (each problem keeps its own z-chunk), timing two batched steps
    own = [g.get_launch() for g in gs]
    best = None
    for v in range(len(hy.variants())):
        for g, (_, kc) in zip(gs, own):
            g.set_launch(v, kc)
        hy.batch_advance(gs, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hy.batch_advance(gs, 2)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        if best is None or t < best[0]:
            best = (t, v)
    for g, (_, kc) in zip(gs, own):
        g.set_launch(best[1], kc)
    for g in gs:
        g.set_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hy.batch_advance(gs, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ref = [g.get_state() for g in gs[:4]]
    # the same batch captured once into a HIP graph (capture, then a timed replay)
    s = torch.cuda.Stream()
    for g in gs:
        g.set_state(stream=s)
    hy.batch_advance_graph(gs, [steps] * len(gs), stream=s)
    s.synchronize()
    for g in gs:
        g.set_state(stream=s)
    s.synchronize()
    t0 = time.perf_counter()
    hy.batch_advance_graph(gs, [steps] * len(gs), stream=s)
    s.synchronize()
    t_graph = time.perf_counter() - t0
    same = all(np.array_equal(g.get_state(), r) for g, r in zip(gs[:4], ref))
    floors = sum(g.query()["floor_hits"] for g in gs)
    for g in gs:
        g.close()
    n_of = {f"{p.n[0]}^3": p.cells for p in pbs}
    return {
        "workload": f"{count} Sedov problems, sizes drawn from "
                    f"{sorted(set(int(p.n[0]) for p in pbs))} (cubed), outflow, PLM+HLLC, SSP-RK2, mixed, "
                    f"{steps} steps each, seed {seed}",
        "value": cells * steps / t_batch,
        "unit": "cell-updates/s",
        "graph_replay": cells * steps / t_graph,
        "graph_equals_eager": bool(same),
        "one_by_one": cells * steps / t_one,
        "speedup": t_one / t_batch,
        "speedup_graph": t_one / t_graph,
        "problems": count,
        "cells": cells,
        "steps": steps,
        "dtype": "mixed",
        "one_by_one_per_class": {k: {"problems": v[0], "cell_updates_per_s": v[0] * n_of[k] * steps / v[1],
                                     "us_per_step": 1e6 * v[1] / (v[0] * steps)}
                                 for k, v in sorted(per_class.items(), key=lambda kv: n_of[kv[0]])},
        "size_classes": {f"{k[0]}^3": list(v[:2]) for k, v in tuned.items()},
        "batch_tile_variant": list(hy.variants()[best[1]]),
        "floor_hits": floors,
    }


def run_serving_workload(hy, P, count, budgets_gb, seed=4, epoch=10, calib=200,
                         policies="oldest-first"):
    """Poisson stream of Sod / KH / Sedov requests (32^3..256^3, 10..200
    steps, FP64 or mixed), admitted by an HBM budget: continuous batching
    against one request at a time. Initial states are generated by the
    client's thread pool ahead of their arrival (a bounded amount of host
    memory; generating all of them first would take ~150 GiB for 1000
    requests). The arrival rate is 0.8 / (mean service time of the
    one-at-a-time path over the first ``calib`` requests, all queued at once,
    results fetched and digested as in the measured runs), so the offered load
    is 80% of what that path can serve. Every run serves the same ``count``
    requests; a served result is compared with the one-at-a-time result by
    digest."""
    from paper_2409_16053_amd import serve
    calib = min(calib, count)
    probe = serve.make_stream(seed, calib, rate=1e9)
    log(f"serving: calibrating on {calib} requests one at a time")
    t0 = time.perf_counter()
    serve.run_fifo(probe, keep="digest", client_threads=16)  # the measured runs' own work
    mean_service = (time.perf_counter() - t0) / calib
    rate = 0.8 / mean_service
    log(f"serving: mean one-at-a-time service {mean_service * 1e3:.1f} ms -> rate {rate:.1f}/s")
    log(f"serving: {count} requests one at a time")
    prog = lambda d, n: log(f"serving: {d}/{n} done")
    fifo = serve.run_fifo(serve.make_stream(seed, count, rate), keep="digest", client_threads=16,
                          progress=prog)
    sf = serve.summarize(fifo)
    budgets = [float(b) for b in str(budgets_gb).split(",")]
    runs = []
    for policy in str(policies).split(","):
        for budget_gb in budgets:
            log(f"serving: {count} requests, continuous batching ({policy}), budget {budget_gb} GiB")
            srv = serve.Server(budget_bytes=int(budget_gb * 2 ** 30), epoch_steps=epoch, keep="digest",
                               client_threads=16, policy=policy)
            cont = srv.run(serve.make_stream(seed, count, rate), progress=prog)
            runs.append({"policy": policy, "budget_gb": budget_gb, "continuous": serve.summarize(cont),
                         "peak_resident_gb": srv.peak_bytes / 2 ** 30, "epochs": srv.epochs,
                         "results_equal_alone": bool(all(a.digest == b.digest for a, b in zip(cont, fifo)))})
    out = {"requests": count, "rate_per_s": rate, "mean_service_ms_one_at_a_time": mean_service * 1e3,
           "calibration_requests": calib, "epoch_steps": epoch, "fifo": sf}
    out.update(runs[0])
    if len(runs) > 1:
        out["sweep"] = runs
    return out


if __name__ == "__main__":
    main()
