#!/usr/bin/env python3
"""Throughput of the fused collide-and-stream step on one MI355X.

Workload (one "step" = one fused collide-and-stream launch over the whole
grid: load, moments, flux, equilibrium, sources including the in-kernel
manufactured-solution forcing, BGK, streamed store): the 3D compressible
Navier-Stokes-Fourier cascade with 5 conserved fields (rho, rho u, E) and
12 gradient trackers (velocity gradient, temperature gradient), D3Q7
populations per field, 256^3 periodic, FP32 shifted populations, smooth
manufactured solution at Mach 0.1, Re 100, Pr 0.71, dt = 0.05 dx,
tau = 1/2 + 20 dt, tracker relaxation g_tau = 3.  The population pair is
16 GB, far beyond the 256 MB Infinity Cache, so the step is HBM-bound.
Inputs are resident in HBM before the timed region.

Printed: one JSON line with MLUPS x variables (the metric), the HBM
roofline of the step kernel (algorithmic 2*K*Q*4 = 952 bytes per cell
update over the kernel's average launch duration: HIP events on the stream
the kernel runs on bracket the K back-to-back launches), the FP64 CPU oracle on a
bounded sample of the same workload, and the adjoint/forward time ratio of
the checkpointed shallow-water rollout (512^2, 500 steps, snapshot every 50).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E nameplate
KERNEL_SOURCES = ["paper_2607_05668_amd/csrc/step_kernels.hpp", "paper_2607_05668_amd/csrc/sys_nsf17.hip",
                  "paper_2607_05668_amd/csrc/kernels.hip", "paper_2607_05668_amd/csrc/systems.hpp",
                  "paper_2607_05668_amd/csrc/lattices.hpp", "paper_2607_05668_amd/csrc/impl.hpp",
                  "paper_2607_05668_amd/csrc/dual.hpp", "paper_2607_05668_amd/csrc/device_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nsf256.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def time_steps(torch, g, k, per_launch):
    """Run k steps on the stepper's stream; returns (total_ms, mean kernel ms)."""
    st = g.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)] \
        if per_launch else []
    torch.cuda.synchronize()
    t0.record(st)
    if per_launch:
        for a, b in evs:
            a.record(st)
            g.step(1)
            b.record(st)
    else:
        g.step(k)
    t1.record(st)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1)
    kern = sum(a.elapsed_time(b) for a, b in evs) / k if per_launch else total / k
    return total, kern


def cpu_baseline(target_s=10.0):
    """The FP64 C oracle on a bounded sample of the benchmark workload: the
    same 17-field D3Q7 system, recipe and manufactured forcing (evaluated
    with numpy from the SymPy residual at t + dt/2 each step) on a 64^3
    grid, for about target_s seconds of steps."""
    import numpy as np
    import oracle
    from oracle import mms
    from paper_2607_05668_amd import inputs
    p = inputs.PRESETS["nsf256"]
    m = inputs.NsfMms()
    n = 64
    o = oracle.make(p, n=n, Q0=m.reference())
    _, fS = mms.nsf17(m.gamma, m.rho0, m.p0, m.u0, m.amp, m.mu, m.kappa, o.params["tau_grad"])
    X, Y, Z = inputs.grid3(n)
    o.init(inputs.nsf_exact(n, 0.0, m))
    src = lambda t: fS(X, Y, Z, t)   # noqa: E731
    t = time.perf_counter()
    o.step(1, source=src)
    one = time.perf_counter() - t
    k = max(1, min(2000, int(target_s / max(one, 1e-3))))
    t = time.perf_counter()
    o.step(k, source=src)
    dt = time.perf_counter() - t
    cells = n ** 3
    assert np.isfinite(o.moments()).all()
    return {"value": round(cells * k * 17 / dt / 1e6, 3), "unit": "MLUPS x variables", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 C oracle (OpenMP over cells) on the same 17-field D3Q7 NSF cascade with its "
                      f"manufactured forcing at 64^3 instead of 256^3 (per-cell work does not depend on the grid), "
                      f"{k} steps ({dt:.1f} s), forcing evaluated with numpy each step"}


def adjoint_ratio(torch):
    from paper_2607_05668_amd import inputs, rollout
    p = inputs.PRESETS["sweadj512"]
    run = rollout.SweRollout(n=p.n, steps=p.steps, ckpt=50)
    h0 = torch.tensor(inputs.swe_height(p.n), device="cuda")
    b = torch.tensor(inputs.topography_gradient(p.n), device="cuda", dtype=torch.float32)
    tgt = torch.tensor(inputs.swe_height(p.n, seed=inputs.SEED_SWE_TARGET), device="cuda")
    hN = run.forward(h0, b)                      # warm-up
    run.backward((hN - tgt) / hN.numel())
    torch.cuda.synchronize()
    reps = 3
    fw = bw = 0.0
    for _ in range(reps):
        t = time.perf_counter()
        hN = run.forward(h0, b)
        torch.cuda.synchronize()
        fw += time.perf_counter() - t
        g = (hN - tgt) / hN.numel()
        torch.cuda.synchronize()
        t = time.perf_counter()
        run.backward(g)
        torch.cuda.synchronize()
        bw += time.perf_counter() - t
    return {"adjoint_forward_ratio": round(bw / fw, 3), "forward_ms": round(1e3 * fw / reps, 3),
            "backward_ms": round(1e3 * bw / reps, 3),
            "workload": "swe2d D2Q9 512x512 FP32, 500 steps, snapshot every 50, topography source; "
                        "backward = recompute with moment history + adjoint steps"}


def probe_peak(torch, lbm):
    n = 4 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    lbm.bw_copy(b, a, n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        lbm.bw_copy(b, a, n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * n / ms / 1e6, 1)


def probe_pattern3(torch, lbm, n, fields=17, reps=10):
    """The 3D step's memory-access pattern without arithmetic at n^3 (7
    fields float planes pulled and stored, the step's launch shape): GB/s
    of 2 x 28 fields n^3 bytes."""
    nbytes = 28 * fields * n ** 3
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        lbm.bw_streams3(b, a, n, n, n, fields)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.bw_streams3(b, a, n, n, n, fields)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * nbytes / ms / 1e6, 1)


def probe_pattern(torch, lbm, n, fields=3, reps=20):
    """The D2Q9 step's memory-access pattern without arithmetic at n x n
    (9 fields float planes pulled and stored): GB/s of 2 x 36 fields n^2 bytes."""
    nbytes = 36 * fields * n * n
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(3):
        lbm.bw_streams(b, a, n, n, fields)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.bw_streams(b, a, n, n, fields)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * nbytes / ms / 1e6, 1)


def extra_runs(torch, lbm, inputs):
    out = {}

    def one(name, preset, n, storage, steps, bytes_per_cell, init, coef=None, params=None):
        g = lbm.from_preset(preset, n=n, storage=storage, params=params)
        if coef is not None:
            g.set_field("coef", coef)
        g.init(init)
        g.step(steps)      # warm-up with the timed call itself (small grids capture their launch graphs here)
        total, kern = time_steps(torch, g, steps, per_launch=False)
        cells = g.C
        out[name] = {"mlups": round(cells / kern / 1e3, 1), "mlups_x_vars": round(cells * g.K / kern / 1e3, 1),
                     "ms_per_step": round(kern, 5), "algorithmic_GBps": round(bytes_per_cell * cells / kern / 1e6, 1)}
        del g

    p = inputs.PRESETS["swe1024"]
    # the shallow-water configuration's own grid: its 226 MB population pair
    # fits the 256 MB Infinity Cache, so this line is cache-resident, not HBM
    one("swe2d_D2Q9_f32_1024_cache_resident", p, 1024, "f32", 1000, 216, inputs.swe_initial(1024))
    one("swe2d_D2Q9_f32_2048", p, 2048, "f32", 200, 216, inputs.swe_initial(2048))
    # two-relaxation-time collision (magic parameter 3/16) on the same workload
    one("swe2d_D2Q9_f32_2048_trt", p, 2048, "f32", 200, 216, inputs.swe_initial(2048),
        params={"trt_lambda": 3.0 / 16.0})
    p = inputs.PRESETS["neohooke2048"]
    one("neohooke2d_D2Q9_f16_2048", p, 2048, "f16", 200, 216, inputs.neohooke_initial(2048))
    # binary16 non-equilibrium deviations + FP32 moments: 2 (K Q 2 + K 4) bytes
    one("neohooke2d_D2Q9_f16ne_2048", p, 2048, "f16ne", 200, 264, inputs.neohooke_initial(2048))
    p = inputs.PRESETS["burgers2048"]
    one("burgers2d_D2Q5_f32_2048", p, 2048, "f32", 200, 40, inputs.burgers_initial(2048))
    p = inputs.PRESETS["euler2048"]
    one("euler2d_D2Q5_f32_2048", p, 2048, "f32", 200, 160, inputs.euler_initial(2048))
    # the same Euler workload with the functor the compiler slice emitted from
    # the declared conservation law (flux deviation formed as Phi(Q) - F0)
    import dataclasses
    one("gen_euler2d_D2Q5_f32_2048", dataclasses.replace(p, system="gen_euler2d"), 2048, "f32", 200, 160,
        inputs.euler_initial(2048))
    p = inputs.PRESETS["maxwell2048"]
    one("maxwell2d_D2Q5_f32_2048", p, 2048, "f32", 200, 120, inputs.maxwell_initial(2048))
    p = inputs.PRESETS["allencahn2048"]
    one("allencahn_trk2d_D2Q5_f32_2048", p, 2048, "f32", 200, 120, inputs.allencahn_initial(2048))
    p = inputs.PRESETS["relhydro2048"]
    one("relhydro2d_D2Q5_f32_2048", p, 2048, "f32", 200, 120, inputs.relhydro_initial(2048))
    p = inputs.PRESETS["nse2048"]
    one("nse_trk2d_D2Q5_f32_2048", p, 2048, "f32", 200, 280, inputs.nse_initial(2048))
    p = inputs.PRESETS["cnsf2048"]
    one("cnsf_trk2d_D2Q5_f32_2048", p, 2048, "f32", 100, 480, inputs.cnsf2d_initial(2048))
    p = inputs.PRESETS["mhd2048"]
    one("mhd_trk2d_D2Q5_f32_2048", p, 2048, "f32", 100, 720, inputs.mhd_initial(2048))
    p = inputs.PRESETS["hcnsf256"]
    # 2 x 14 x 7 x 4 B of populations + 4 x 4 B of porosity and solid velocity
    one("hcnsf3d_trk14_D3Q7_f32_256", p, 256, "f32", 50, 800, inputs.hcnsf_exact(256, 0.0),
        coef=inputs.hcnsf_coefficients(256, 0.0))
    p = inputs.PRESETS["advdiff64"]
    one("advdiff_D2Q5_f64_64", p, 64, "f64", 200, 240, inputs.advdiff_initial(64))
    # one GPU's share of the 3D NSF workload split over eight GPUs along z:
    # a 256 x 256 x 32 slab at the 256^3 spacing (periodic here; a sharded
    # run would exchange the z faces instead)
    p = inputs.PRESETS["nsf256"]
    dx, dt, tau = lbm.recipe(256, p.scaling, p.f, p.tau_r)
    g = lbm.Stepper(p.system, p.lattice, (32, 256, 256), tau, dt, dx, "f32", dict(p.params, g_tau=p.g_tau))
    g.init(inputs.nsf_exact(256, 0.0)[:, :32])
    g.step(100)
    total, kern = time_steps(torch, g, 100, per_launch=False)
    out["nsf3d_trk17_D3Q7_f32_256x256x32_share"] = {
        "mlups": round(g.C / kern / 1e3, 1), "mlups_x_vars": round(g.C * g.K / kern / 1e3, 1),
        "ms_per_step": round(kern, 5), "algorithmic_GBps": round(952 * g.C / kern / 1e6, 1)}
    del g
    return out


# The paper's roofline table, row for row: every system on its lattice
# (D2Q5 in 2D, D3Q7 for the homogenized NSF) in single and double
# precision, on a saturating grid (2048^2, 256^3), with the paper's
# single-precision recipes.  Bytes per cell update: 2 K Q sizeof (+ the
# porosity / solid-velocity field the homogenized NSF reads).
TABLE_ROWS = [
    # (row, preset, initial-state function, extra values per cell)
    ("Inviscid Burgers", "burgers2048", "burgers_initial", 0),
    ("Compressible Euler", "euler2048", "euler_initial", 0),
    ("Shallow Water (SWE)", "swe1024", "swe_initial", 0),
    ("Ideal Ultrarelativistic Fluid", "relhydro2048", "relhydro_initial", 0),
    ("Maxwell (TM)", "maxwell2048", "maxwell_initial", 0),
    ("Nonlinear Elasticity", "neohooke2048", "neohooke_initial", 0),
    ("Scalar ADR", "advdiff64", "advdiff_initial", 0),
    ("Allen-Cahn Phase-Field", "allencahn2048", "allencahn_initial", 0),
    ("Incompressible NSE", "nse2048", "nse_initial", 0),
    ("Compressible NSF", "cnsf2048", "cnsf2d_initial", 0),
    ("Resistive MHD", "mhd2048", "mhd_initial", 0),
    ("HCNSF", "hcnsf256", "hcnsf_exact", 4),
]


def roofline_table(torch, lbm, inputs, steps):
    copy_peak = probe_peak(torch, lbm)
    rows = []
    for row, pre_name, init_name, extra in TABLE_ROWS:
        pre = inputs.PRESETS[pre_name]
        three_d = pre.lattice == "D3Q7"
        n = 256 if three_d else 2048
        lat = "D3Q7" if three_d else "D2Q5"
        init = getattr(inputs, init_name)
        Q = init(n, 0.0) if init_name == "hcnsf_exact" else init(n)
        for storage, size in (("f32", 4), ("f64", 8)):
            g = lbm.from_preset(pre, n=n, storage=storage, lattice=lat)
            if extra:
                g.set_field("coef", inputs.hcnsf_coefficients(n, 0.0))
            g.init(Q)
            g.step(5)
            _, kern = time_steps(torch, g, steps, per_launch=False)
            bpc = (2 * g.K * g.Q + extra) * size
            gbps = bpc * g.C / kern / 1e6
            rows.append({"system": row, "lattice": lat, "fields": g.K, "precision": storage, "cells": g.C,
                         "byte_per_cell": bpc, "mlups": round(g.C / kern / 1e3, 1),
                         "mlups_x_vars": round(g.C * g.K / kern / 1e3, 1), "ms_per_step": round(kern, 5),
                         "GBps": round(gbps, 1), "frac_of_8TBps": round(gbps / HBM_PEAK_GBPS, 4),
                         "frac_of_copy_probe": round(gbps / copy_peak, 4)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del g
            torch.cuda.empty_cache()
    return {"table": "all systems, paper's lattices, FP32 and FP64", "copy_probe_GBps": copy_peak,
            "steps": steps, "rows": rows}


def counters_run(torch, lbm, inputs, workload, warmup):
    """For rocprofv3 --pmc: warm-up and ten launches of one workload's step
    (or adjoint) kernel, then five copies of exactly 1 GiB with the
    library's copy kernel, whose counter readings scale the step kernel's."""
    launches = warmup + 10
    if workload == "adjoint512":
        from paper_2607_05668_amd import rollout
        run = rollout.SweRollout(n=512, steps=launches, ckpt=launches)
        h0 = torch.tensor(inputs.swe_height(512), device="cuda")
        b = torch.tensor(inputs.topography_gradient(512), device="cuda", dtype=torch.float32)
        hN = run.forward(h0, b)
        run.backward(hN / hN.numel())
        del run
    else:
        if workload == "nsf256":
            p = inputs.PRESETS["nsf256"]
            g = lbm.from_preset(p)
            g.init(inputs.nsf_exact(p.n, 0.0))
        elif workload == "swe2048":
            g = lbm.from_preset(inputs.PRESETS["swe1024"], n=2048)
            g.init(inputs.swe_initial(2048))
        else:
            g = lbm.from_preset(inputs.PRESETS["neohooke2048"], storage=workload.split("_")[1])
            g.init(inputs.neohooke_initial(2048))
        g.step(launches)
        del g
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    n = 1 << 30
    a = torch.zeros(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(5):
        lbm.bw_copy(b, a, n)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": workload, "launches": launches, "copy_bytes": n, "copies": 5}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the adjoint ratio, probe and extra workloads")
    ap.add_argument("--counters", nargs="?", const="nsf256", default=None,
                    choices=["nsf256", "swe2048", "neohooke_f16", "neohooke_f16ne", "adjoint512"],
                    help="short run of one workload for rocprofv3 counter collection (default: the benchmark's)")
    ap.add_argument("--table", action="store_true",
                    help="instead of the benchmark: every system in FP32 and FP64 on the paper's lattices")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); nothing was run.", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, ROOT)
    import torch
    from paper_2607_05668_amd import inputs, lbm

    if args.table:
        print(json.dumps(roofline_table(torch, lbm, inputs, min(args.steps, 50))))
        return
    if args.counters:
        counters_run(torch, lbm, inputs, args.counters, args.warmup)
        return
    p = inputs.PRESETS["nsf256"]
    g = lbm.from_preset(p)
    g.init(inputs.nsf_exact(p.n, 0.0))
    g.step(args.warmup)
    # the timed region: K back-to-back launches on the stepper's stream
    # bracketed by HIP events on that stream; the average launch duration is
    # the region's time over K
    total_ms, kern_ms = time_steps(torch, g, args.steps, per_launch=False)
    cells = g.C
    K = g.K
    ms_step = total_ms / args.steps
    value = cells * K * args.steps / total_ms / 1e3          # MLUPS x variables
    bytes_per_launch = 2 * K * g.Q * 4 * cells
    achieved = bytes_per_launch / kern_ms / 1e6              # GB/s
    traffic = measured_traffic()
    nonfinite = g.reduce(lbm.RED_NONFINITE)[0]
    if nonfinite:
        raise SystemExit("non-finite populations after the timed steps")

    line = {
        "metric": "MLUPS x variables and % HBM roofline per step; adjoint/forward time ratio",
        "value": round(value, 1),
        "unit": "MLUPS x variables",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D compressible Navier-Stokes-Fourier cascade, 5 conserved + 9 velocity-gradient "
                               "+ 3 temperature-gradient trackers, D3Q7 per field, 256^3 periodic, FP32 shifted "
                               "populations, manufactured solution (Mach 0.1, Re 100, Pr 0.71) forced in-kernel, "
                               "one fused collide-and-stream launch per step",
                   "cells": cells, "fields": K, "lattice": "D3Q7", "storage": "f32",
                   "bytes_per_cell_update": 2 * K * g.Q * 4},
        "mlups": round(cells * args.steps / total_ms / 1e3, 1),
        "hbm_roofline_pct": round(100.0 * achieved / HBM_PEAK_GBPS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "k_step<SysNSF17, D3Q7, float>", "kernel_ms": round(kern_ms, 5),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        # the paper's own roofline figure for the nearest system it measures
        # (its 3D homogenized NSF, 14 fields on D3Q7 in FP32; Performance
        # section, roofline table), on the hardware it names: context only
        "paper_roofline_context": {"hardware": "NVIDIA RTX A5000, 680 GB/s measured (BabelStream Triad)",
                                   "system": "homogenized compressible NSF, 14 fields, D3Q7, FP32",
                                   "mlups": 546, "bytes_per_cell": 784, "bw_saturation": 0.630},
    }
    del g
    torch.cuda.empty_cache()
    if not args.no_extra:
        line.update(adjoint_ratio(torch))
        line["probe_peak_GBps"] = probe_peak(torch, lbm)
        # the steps' own access patterns without arithmetic: the benchmark's
        # (119 pulled + 119 stored float planes on D3Q7 at 256^3), and the
        # shallow-water step's (27 + 27 on D2Q9, at 1024^2 cache-resident and
        # at 2048^2)
        pat = {"nsf256": probe_pattern3(torch, lbm, 256), "swe1024": probe_pattern(torch, lbm, 1024),
               "swe2048": probe_pattern(torch, lbm, 2048)}
        line["probe_pattern_GBps"] = pat
        line["roofline"]["frac_of_copy_probe"] = round(achieved / line["probe_peak_GBps"], 4)
        line["roofline"]["frac_of_pattern_probe"] = round(achieved / pat["nsf256"], 4)
        line["extra"] = extra_runs(torch, lbm, inputs)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
