"""Throughput of the fused Shan-Chen D3Q19 step on one MI355X.

Default workload: the large single ligament, 256 x 256 x 1024 nodes, FP32
storage and arithmetic, tau 0.8, G -5.5, R0 24, five waves along z,
amplitude 0.05 R0, density noise +-1e-4 (seed 1); liquid/vapour densities
from the library's FP64 flat-interface coexistence run on the GPU.  Inputs
are synthetic and resident in HBM before timing starts.

One step = one launch of the fused psi/force/collide/stream kernel over the
whole grid.  Prints one JSON line (metric MLUPS) with a roofline object for
that kernel (algorithmic bytes 19 loads + 19 stores per node, timed with
HIP events on the kernel's own stream) and the FP64 CPU oracle timed on a
bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--storage f32|f64|f16s|bf16s]
                  [--form single|batch] [--no-cpu-baseline]

Studies (one JSON line each, not the benchmark line):
  --form precision    FP16/BF16 shifted storage against FP32/FP64
  --form shift        FP16 storage error against the shift density rho_ref
  --form convergence  t_b / t_cap against 1/R, FP32 and FP64
  --form paper        the paper's Table 1 sweep (G = -5.3, Oh = 0.1)
  --form small        the small FP64 ligament and R = 8, 16 of the convergence
                      series on the GPU and in the CPU oracle (MLUPS of both)
  --collision mrt     the MRT collision (single form and --form paper)
  --sweep             every compiled tile shape and several z chunks
  --slab N            the single form on the first N z planes (one GPU's share
                      of a z-slab decomposition, without the exchange)
  --grid NX,NY,NZ     the single form on another grid, up to 2^31 - 1 nodes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# bytes one lattice holds per node (19 populations; the FP32-rest kinds keep
# the rest population in FP32 and the 18 moving ones in 16 bits)
BYTES_PER_NODE = {"f64": 152, "f32": 76, "f16s": 38, "bf16s": 38, "f16m": 40, "bf16m": 40}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# The step kernel, and the host code that sets its lattice layout and default
# launch: a change to any of them invalidates the stored traffic figures.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1904_11792_amd", "csrc", f)
                  for f in ("lbm_step.hip", "lbm_device.h", "lbm_internal.h", "lbm_capi.hip")]


def kernel_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, nodes: int):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = t.get(storage)
    if not e or e.get("kernel_digest") != kernel_digest() or e.get("nodes") != nodes:
        return None
    return e.get("bytes_per_launch")


STORAGE_ID = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3, "f16m": 4, "bf16m": 5}


def traffic_from_counters(fetch_csv: str, write_csv: str, storage: str) -> dict:
    """HBM bytes per launch of the fused step from two rocprofv3 --pmc runs of
    this benchmark (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each
    counter is scaled by what it reads for the plain copy kernel of the same
    run, whose bytes are known (19 n b read and written)."""
    import csv

    spec = __import__("workloads").LARGE_FP32
    copy_kib = spec.n * BYTES_PER_NODE[storage] / 1024.0
    tag = f"k_step_bgk<{STORAGE_ID[storage]},"

    def per_dispatch(path, counter):
        step, copy = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            if tag in r["Kernel_Name"]:
                step.append(float(r["Counter_Value"]))
            elif "k_copy16" in r["Kernel_Name"]:
                copy.append(float(r["Counter_Value"]))
        return sum(step) / len(step), sum(copy) / len(copy)

    fs, fc = per_dispatch(fetch_csv, "FETCH_SIZE")
    ws, wc = per_dispatch(write_csv, "WRITE_SIZE")
    fscale, wscale = copy_kib / fc, copy_kib / wc
    total = (fs * fscale + ws * wscale) * 1024.0
    return {"kernel_digest": kernel_digest(), "nodes": spec.n, "bytes_per_launch": round(total),
            "bytes_per_node": round(total / spec.n, 2), "fetch_scale": round(fscale, 4),
            "write_scale": round(wscale, 4), "fetch_kib_raw": fs, "write_kib_raw": ws}


def cpu_baseline(spec, rho_l, rho_v, budget_s=18.0):
    """The FP64 oracle on a z-slab of the same ligament (bounded sample)."""
    import oracle

    nz_s = 64
    f = oracle.init_ligament(spec.nx, spec.ny, nz_s, R0=spec.R0, amp_rel=spec.amp_rel,
                             wavelength=spec.wavelength, rho_l=rho_l, rho_v=rho_v,
                             noise_amp=spec.noise_amp, seed=spec.seed)
    f = oracle.run(f, 2, spec.tau, spec.G)  # pages the arrays in, starts the threads
    t0 = time.perf_counter()
    f = oracle.run(f, 3, spec.tau, spec.G)  # calibration
    t1 = (time.perf_counter() - t0) / 3
    steps = max(2, min(400, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    f = oracle.run(f, steps, spec.tau, spec.G)
    el = time.perf_counter() - t0
    nodes = spec.nx * spec.ny * nz_s
    return {"value": round(nodes * steps / el / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, {steps} steps on a {spec.nx}x{spec.ny}x{nz_s} periodic z-slab "
                      f"of the same ligament ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_NODE))
    ap.add_argument("--form", default="single",
                    choices=["single", "batch", "precision", "shift", "convergence", "paper", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kinds", default="f64,f32,f16s,bf16s,f16m,bf16m",
                    help="--form precision: storage kinds to run (f64 first: it is the reference)")
    ap.add_argument("--cases", default="base,G-6,tau1",
                    help="--form precision: cases to run (base, G-6, tau1)")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"],
                    help="mrt: the multiple-relaxation-time collision with the suggested rates "
                         "of d'Humieres et al. and s_j = 1/tau")
    ap.add_argument("--graph-chunk", type=int, default=0)
    ap.add_argument("--launch", default="", help="tile_x,tile_y,zchunk (default: library's choice; "
                                                 "for --form batch the autotuner's)")
    ap.add_argument("--slab", type=int, default=0,
                    help="run the large ligament's first SLAB z planes only (one GPU's share of a "
                         "z-slab decomposition; periodic in z, no halo exchange)")
    ap.add_argument("--grid", default="",
                    help="NX,NY,NZ: the single form on another grid (same ligament, five waves along z; "
                         "no CPU baseline), e.g. 1024,1024,1024 to fill most of the HBM")
    ap.add_argument("--sweep", action="store_true",
                    help="time every compiled tile and a set of z chunks, print a markdown table")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        try:
            table = json.load(open(TRAFFIC_FILE))
        except (OSError, ValueError):
            table = {}
        table[args.storage] = traffic_from_counters(*args.traffic_from, args.storage)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(table, fh, indent=1)
        print(json.dumps(table[args.storage]))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU z-slab "
              "decomposition is a design only; it is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1904_11792_amd import lbm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    if args.form == "batch":
        return bench_batch(args, lbm, workloads, stream)
    if args.form == "precision":
        return study_precision(args, lbm, workloads, stream)
    if args.form == "shift":
        return study_shift(args, lbm, workloads, stream)
    if args.form == "convergence":
        return study_convergence(args, lbm, workloads, stream)
    if args.form == "paper":
        return study_paper(args, lbm, workloads, stream)
    if args.form == "small":
        return study_small(args, lbm, workloads, stream)

    spec = workloads.LARGE_FP32
    if args.slab:
        import dataclasses

        spec = dataclasses.replace(spec, name=f"large_fp32 slab 256x256x{args.slab}", nz=args.slab)
    if args.grid:
        import dataclasses

        gx, gy, gz = [int(v) for v in args.grid.split(",")]
        spec = dataclasses.replace(spec, name=f"large ligament {gx}x{gy}x{gz}", nx=gx, ny=gy, nz=gz,
                                   wavelength=gz / 5.0)
    print(f"# workload {spec.name}, storage {args.storage}", file=sys.stderr, flush=True)
    rho_l, rho_v = lbm.lbm_coexistence(spec.G, spec.tau)
    mrt = {} if args.collision == "mrt" else None
    if mrt is not None:
        rho_l, rho_v = lbm.lbm_coexistence(spec.G, spec.tau, mrt=mrt)
    lat = lbm.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, spec.G, storage=args.storage,
                      rho_ref=rho_v, stream=stream, mrt=mrt)
    lat.init_ligament(R0=spec.R0, amp_rel=spec.amp_rel, wavelength=spec.wavelength,
                      rho_l=rho_l, rho_v=rho_v, noise_amp=spec.noise_amp, seed=spec.seed)
    if args.sweep:
        return sweep(lat, spec, stream, args.storage)
    if args.launch:
        lat.set_launch(*[int(v) for v in args.launch.split(",")])
    if args.graph_chunk:
        lat.set_graph_chunk(args.graph_chunk)
    launch = lat.get_launch()

    # plain copy kernel of the same size as one lattice pass (at most that of
    # the 256x256x1024 grid): practical HBM ceiling
    nbytes = min(spec.n, workloads.LARGE_FP32.n) * BYTES_PER_NODE[args.storage]
    with torch.cuda.stream(stream):
        a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        lbm.lbm_device_copy(b.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    e0.record(stream)
    for _ in range(10):
        lbm.lbm_device_copy(b.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    copy_gbs = 2 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b

    lat.step(args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    mlups = spec.n * args.steps / (ms * 1e-3) / 1e6
    d = lat.diagnostics()
    alg_bytes = 2 * BYTES_PER_NODE[args.storage] * spec.n
    achieved = alg_bytes / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic(args.storage, spec.n) if mrt is None else None
    out = {
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": spec.name + f" R0=24 tau=0.8 G=-5.5 storage={args.storage}"
                               + (" collision=mrt" if mrt is not None else ""),
                   "grid": [spec.nx, spec.ny, spec.nz], "launch": list(launch),
                   "graph_chunk": args.graph_chunk},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "copy_kernel_GBps": round(copy_gbs, 1),
        "state_check": {"mass": d["mass"], "nonfinite": d["nonfinite"], "step": d["step"]},
    }
    print(f"# {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic, copy {copy_gbs:.0f} GB/s",
          file=sys.stderr, flush=True)
    if args.storage == "f32" and mrt is None and not args.grid and not args.slab and not args.launch:
        # the metric's second half: 16-bit storage against FP32 on the same
        # workload, timed the same way (its error against FP64 is the study
        # of --form precision)
        lat.close()
        out["fp16_store"] = fp16_store_line(lbm, spec, rho_l, rho_v, stream, args, ms_per_step)
    if not args.no_cpu_baseline and mrt is None and not args.grid:
        out["cpu_baseline"] = cpu_baseline(spec, rho_l, rho_v)
    print(json.dumps(out), flush=True)


def fp16_store_line(lbm, spec, rho_l, rho_v, stream, args, ms_f32):
    """Step throughput of the F16M storage (moving populations in half
    precision, stochastically rounded; rest population in FP32) on the
    benchmark workload: ms per step, MLUPS, HBM fraction at its 80 B per
    node, and the speed-up over the FP32 step of the same run."""
    import torch

    lat = lbm.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, spec.G, storage="f16m", rho_ref=rho_v,
                      stream=stream)
    lat.init_ligament(R0=spec.R0, amp_rel=spec.amp_rel, wavelength=spec.wavelength,
                      rho_l=rho_l, rho_v=rho_v, noise_amp=spec.noise_amp, seed=spec.seed)
    lat.step(args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    lat.close()
    gbs = 2 * BYTES_PER_NODE["f16m"] * spec.n / (ms * 1e-3) / 1e9
    return {"storage": "f16m", "ms_per_step": round(ms, 4), "MLUPS": round(spec.n / ms / 1e3, 1),
            "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "speedup_vs_f32": round(ms_f32 / ms, 3), "error_study": "bench.py --form precision"}


def sweep(lat, spec, stream, storage):
    """Per-launch time of every compiled tile shape and several z chunks."""
    import torch

    from paper_1904_11792_amd import lbm

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    zcs = (32, 64, 128, 256)
    bpn = 2 * BYTES_PER_NODE[storage]
    print(f"| tile | " + " | ".join(f"z {z} ms" for z in zcs) + " | best GB/s |")
    print("|---|" + "---:|" * (len(zcs) + 1))
    for tx, ty in lbm.lbm_list_tiles():
        row = []
        for zc in zcs:
            lat.set_launch(tx, ty, zc)
            lat.step(3)
            e0.record(stream)
            lat.step(10)
            e1.record(stream)
            e1.synchronize()
            row.append(e0.elapsed_time(e1) / 10)
        best = min(row)
        name = f"{tx}x{ty}" if tx else f"run-time, {ty} threads"
        print(f"| {name} | " + " | ".join(f"{v:.3f}" for v in row) +
              f" | {bpn * spec.n / best / 1e6:.0f} |", flush=True)


def _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, max_steps, every, extra_after=0,
                  mrt=None, rho_ref=None):
    """Step one ligament to break-up (neck sampled every `every` steps), then
    `extra_after` more steps; returns t_b, time per step, droplets, mass drift.
    Shifted storage uses rho_ref (default: the vapour density)."""
    import torch

    from paper_1904_11792_amd import analysis

    lat = lbm.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, spec.G, storage=storage,
                      rho_ref=rho_v if rho_ref is None else rho_ref, stream=stream, mrt=mrt)
    lat.init_ligament(R0=spec.R0, amp_rel=spec.amp_rel, wavelength=spec.wavelength, rho_l=rho_l,
                      rho_v=rho_v, noise_amp=spec.noise_amp, seed=spec.seed)
    m0 = lat.diagnostics()["mass"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tb, steps, neck, last = analysis.run_to_breakup(lat, rho_l, rho_v, max_steps, every=every)
    e1.record(stream)
    e1.synchronize()
    n_done = lat.step_count
    ms_step = e0.elapsed_time(e1) / max(n_done, 1)
    if extra_after:
        lat.step(extra_after)
    d = lat.diagnostics()
    drops = lat.droplets(0.5 * (rho_l + rho_v), max_out=8)  # labelled on the device
    lat.close()
    return {"t_b": tb, "steps": n_done + extra_after,
            "ms_per_step_incl_diag": round(ms_step, 4),
            "droplets": drops["count"], "volumes": drops["volumes"].tolist(),
            "mass_drift": (d["mass"] - m0) / m0, "nonfinite": d["nonfinite"]}


def study_precision(args, lbm, workloads, stream):
    """Shifted FP16/BF16 storage against FP32 and FP64 on the large ligament
    (and a stronger-attraction case): break-up time, droplets, mass drift and
    step throughput.  The FP64 GPU run is the reference (itself held to the
    oracle within 1e-11 over 200 steps by the parity tests)."""
    import dataclasses

    import torch

    base = workloads.LARGE_FP32
    all_cases = {"base": base, "G-6": dataclasses.replace(base, name="large G=-6.0", G=-6.0),
                 "tau1": dataclasses.replace(base, name="large tau=1.0", tau=1.0)}
    cases = [all_cases[c] for c in args.cases.split(",")]
    out = []
    for spec in cases:
        rho_l, rho_v = lbm.lbm_coexistence(spec.G, spec.tau)
        res = {}
        for storage in args.kinds.split(","):
            print(f"# {spec.name} {storage}", file=sys.stderr, flush=True)
            r = _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, spec.steps, every=10,
                              extra_after=1000)
            # pure step throughput (no diagnostics) on the same grid
            lat = lbm.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, spec.G, storage=storage,
                              rho_ref=rho_v, stream=stream)
            lat.init_ligament(R0=spec.R0, amp_rel=spec.amp_rel, wavelength=spec.wavelength,
                              rho_l=rho_l, rho_v=rho_v, noise_amp=spec.noise_amp, seed=spec.seed)
            lat.step(5)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.step(50)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / 50
            lat.close()
            r["ms_per_step"] = round(ms, 4)
            r["MLUPS"] = round(spec.n / ms / 1e3, 1)
            res[storage] = r
            print(f"# {json.dumps(r)}", file=sys.stderr, flush=True)
        ref = res["f64"]["t_b"]
        for st, r in res.items():
            r["t_b_rel_err_vs_f64"] = None if (ref is None or r["t_b"] is None) else (r["t_b"] - ref) / ref
        out.append({"case": spec.name, "G": spec.G, "tau": spec.tau, "rho_l": rho_l, "rho_v": rho_v,
                    "results": res})
    print(json.dumps({"study": "precision", "grid": [base.nx, base.ny, base.nz], "cases": out}))


def study_shift(args, lbm, workloads, stream):
    """Shifted 16-bit storage (--storage f16s, bf16s, f16m or bf16m; default
    f16m): break-up time and mass drift against the FP64 run
    for several shift densities rho_ref (vapour, 0, the mean of the two phases,
    1) on the large ligament (two noise seeds, G -6.0, tau 1.0) and the R = 32
    grid of the convergence series."""
    import dataclasses

    base = workloads.LARGE_FP32
    cases = [base, dataclasses.replace(base, name=base.name + " seed 2", seed=2),
             dataclasses.replace(base, name=base.name + " G=-6.0", G=-6.0),
             dataclasses.replace(base, name=base.name + " tau=1.0", tau=1.0), workloads.convergence(32)]
    out = []
    for spec in cases:
        rho_l, rho_v = lbm.lbm_coexistence(spec.G, spec.tau)
        kind = args.storage if args.storage in ("f16s", "bf16s", "f16m", "bf16m") else "f16m"
        runs = [("f64", None, "-")] + [(kind, r, name) for name, r in
                                      (("rho_v", rho_v), ("0", 0.0), ("mid", 0.5 * (rho_l + rho_v)), ("1", 1.0))]
        ref, rows = None, []
        for storage, rref, name in runs:
            print(f"# {spec.name} {storage} rho_ref={name}", file=sys.stderr, flush=True)
            r = _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, 30000, every=10, rho_ref=rref)
            if storage == "f64":
                ref = r["t_b"]
            err = None if (ref is None or r["t_b"] is None) else (r["t_b"] - ref) / ref
            rows.append({"storage": storage, "rho_ref": name, "t_b": r["t_b"], "t_b_rel_err_vs_f64": err,
                         "mass_drift": r["mass_drift"], "droplets": r["droplets"]})
            print(f"# {json.dumps(rows[-1])}", file=sys.stderr, flush=True)
        out.append({"case": spec.name, "G": spec.G, "tau": spec.tau, "rho_l": rho_l, "rho_v": rho_v,
                    "rows": rows})
    print(json.dumps({"study": "shift_density", "storage": kind, "cases": out}))


def study_convergence(args, lbm, workloads, stream):
    """Grid-convergence series: break-up time over the capillary time against
    1/R for R = 8, 16, 32, 64 in FP32 and FP64 (sigma from Laplace runs)."""
    from paper_1904_11792_amd import analysis

    G, tau = -5.5, 1.0
    rho_l, rho_v = lbm.lbm_coexistence(G, tau)
    sigma, icpt = analysis.laplace_sigma(lbm, G, tau, rho_l, rho_v)
    rows = []
    for R in (8, 16, 32, 64):
        spec = workloads.convergence(R)
        tcap = analysis.capillary_time(rho_l, R, sigma)
        for storage in ("f32", "f64"):
            print(f"# R={R} {storage}", file=sys.stderr, flush=True)
            r = _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, max_steps=int(40 * tcap) + 2000,
                              every=max(1, R // 8))
            r.update({"R": R, "grid": [spec.nx, spec.ny, spec.nz], "storage": storage,
                      "t_cap": tcap, "t_b_over_t_cap": None if r["t_b"] is None else r["t_b"] / tcap,
                      "kR": 2 * 3.141592653589793 * R / spec.nz})
            rows.append(r)
            print(f"# {json.dumps(r)}", file=sys.stderr, flush=True)
    print(json.dumps({"study": "convergence", "G": G, "tau": tau, "rho_l": rho_l, "rho_v": rho_v,
                      "sigma": sigma, "laplace_intercept": icpt, "rows": rows}))


def study_small(args, lbm, workloads, stream):
    """The small FP64 ligament (32 x 32 x 64, 2000 steps) and the two smallest
    grid-convergence cases run to break-up, each on the GPU and in the FP64
    CPU oracle on all host threads: MLUPS of both, break-up time, droplets,
    mass drift.  These grids live in the MI355X's 256 MB Infinity Cache, so
    only their MLUPS are meaningful, not an HBM fraction."""
    import torch

    import oracle
    from paper_1904_11792_amd import analysis

    rows = []
    cases = [(workloads.SMALL_FP64, 2000)]
    rho_l, rho_v = lbm.lbm_coexistence(-5.5, 1.0)
    sigma, _ = analysis.laplace_sigma(lbm, -5.5, 1.0, rho_l, rho_v)
    for R in (8, 16):
        spec = workloads.convergence(R)
        cases.append((spec, int(12 * analysis.capillary_time(rho_l, R, sigma))))
    for spec, steps in cases:
        for storage in ("f64", "f32"):
            print(f"# {spec.name} {storage}, {steps} steps", file=sys.stderr, flush=True)
            r = _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, steps, every=1)
            lat = lbm.Lattice(spec.nx, spec.ny, spec.nz, spec.tau, spec.G, storage=storage, rho_ref=rho_v,
                              stream=stream)
            lat.init_ligament(R0=spec.R0, amp_rel=spec.amp_rel, wavelength=spec.wavelength, rho_l=rho_l,
                              rho_v=rho_v)
            lat.step(20)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.step(steps)
            e1.record(stream)
            e1.synchronize()
            plain_ms = e0.elapsed_time(e1)
            # the same steps replayed as captured graphs of 100 steps (launch-bound grids)
            lat.set_graph_chunk(100)
            lat.step(200)
            e0.record(stream)
            lat.step(steps // 100 * 100)
            e1.record(stream)
            e1.synchronize()
            graph_ms = e0.elapsed_time(e1) / (steps // 100 * 100) * steps
            # and with the autotuned launch shape, in graphs
            launch, _ = lat.autotune(20)
            lat.step(200)
            e0.record(stream)
            lat.step(steps // 100 * 100)
            e1.record(stream)
            e1.synchronize()
            tuned_ms = e0.elapsed_time(e1) / (steps // 100 * 100) * steps
            lat.close()
            r.update({"case": spec.name, "storage": storage, "steps_timed": steps,
                      "gpu_MLUPS": round(spec.n * steps / plain_ms / 1e3, 1),
                      "gpu_MLUPS_graph": round(spec.n * steps / graph_ms / 1e3, 1),
                      "gpu_MLUPS_tuned": round(spec.n * steps / tuned_ms / 1e3, 1),
                      "tuned_launch": list(launch)})
            rows.append(r)
        f = oracle.init_ligament(spec.nx, spec.ny, spec.nz, R0=spec.R0, amp_rel=spec.amp_rel,
                                 wavelength=spec.wavelength, rho_l=rho_l, rho_v=rho_v)
        t0 = time.perf_counter()
        oracle.run(f, steps, spec.tau, spec.G)
        el = time.perf_counter() - t0
        rows.append({"case": spec.name, "storage": "oracle f64", "steps_timed": steps,
                     "oracle_MLUPS": round(spec.n * steps / el / 1e6, 1), "cores": oracle.num_threads(),
                     "seconds": round(el, 2)})
        print(f"# {json.dumps(rows[-3:])}", file=sys.stderr, flush=True)
    print(json.dumps({"study": "small_grids", "rho_l": rho_l, "rho_v": rho_v, "sigma": sigma, "rows": rows}))


def study_paper(args, lbm, workloads, stream):
    """The paper's sweep (Section 4): G = -5.3, tau from Oh = 0.1, R0 = 7 ... 84.
    Per radius: flat-interface coexistence and Laplace surface tension on the
    GPU against Table 1, then the ligament (FP32 storage unless --storage
    says otherwise) run to break-up: t_b / t_cap against R0, the trend the
    paper's Fig. 2 shows (its data points are not printed).

    With --collision mrt: the comparison the paper's conclusion proposes, the
    same sweep with the MRT collision at s_j and the other non-viscous rates
    fixed to 1, which keeps the density ratio (and sigma) the same at every
    viscosity: one coexistence and one Laplace fit serve all radii, and tau
    follows from Oh = 0.1 with them."""
    from paper_1904_11792_amd import analysis

    storage = args.storage
    if args.collision == "mrt":
        return study_paper_mrt(args, lbm, workloads, stream, analysis)
    rows = []
    specs = [workloads.paper_table1(row[0]) for row in workloads.TABLE1]
    co_l, co_v, co_st = lbm.lbm_coexistence_many([s.G for s in specs], [s.tau for s in specs])
    if (co_st != lbm.LBM_OK).any():
        raise RuntimeError(f"flat-interface run diverged for R0 = {[r[0] for r, s in zip(workloads.TABLE1, co_st) if s]}")
    for (R0, rl_p, rv_p, sg_p), spec, rho_l, rho_v in zip(workloads.TABLE1, specs, co_l, co_v):
        rho_l, rho_v = float(rho_l), float(rho_v)
        try:
            sigma, icpt = analysis.laplace_sigma(lbm, spec.G, spec.tau, rho_l, rho_v, width=4.0)
        except RuntimeError as exc:
            sigma, icpt = None, str(exc)
        sg = sigma if sigma is not None else sg_p
        tcap = analysis.capillary_time(rho_l, R0, sg)
        print(f"# R0={R0} tau={spec.tau:.4f} rho_l={rho_l:.5f} rho_v={rho_v:.5f} sigma={sigma} "
              f"grid {spec.nx}x{spec.ny}x{spec.nz}", file=sys.stderr, flush=True)
        r = _run_ligament(lbm, spec, storage, rho_l, rho_v, stream, max_steps=int(40 * tcap) + 2000,
                          every=max(1, R0 // 8))
        r.update({
            "R0": R0, "grid": [spec.nx, spec.ny, spec.nz], "tau": spec.tau, "storage": storage,
            "rho_l": rho_l, "rho_v": rho_v, "sigma": sigma, "laplace_intercept": icpt,
            "paper": {"rho_l": rl_p, "rho_v": rv_p, "sigma": sg_p},
            "rel_err": {"rho_l": (rho_l - rl_p) / rl_p, "rho_v": (rho_v - rv_p) / rv_p,
                        "sigma": None if sigma is None else (sigma - sg_p) / sg_p},
            "Oh": analysis.ohnesorge(spec.tau, rho_l, sg, R0), "t_cap": tcap,
            "t_b_over_t_cap": None if r["t_b"] is None else r["t_b"] / tcap,
            "t_b_over_t_cap_paper_scales": None if r["t_b"] is None
            else r["t_b"] / analysis.capillary_time(rl_p, R0, sg_p),
            "MLUPS_incl_diag": round(spec.n / r["ms_per_step_incl_diag"] / 1e3, 1)})
        rows.append(r)
        print(f"# {json.dumps(r)}", file=sys.stderr, flush=True)
    print(json.dumps({"study": "paper_table1", "G": workloads.TABLE1_G, "Oh": workloads.TABLE1_OH,
                      "rows": rows}))


def study_paper_mrt(args, lbm, workloads, stream, analysis):
    import dataclasses

    mrt = {k: 1.0 for k in ("s_e", "s_eps", "s_q", "s_pi", "s_m", "s_j")}
    G = workloads.TABLE1_G
    rho_l, rho_v = lbm.lbm_coexistence(G, 1.0, mrt=mrt)
    sigma, icpt = analysis.laplace_sigma(lbm, G, 1.0, rho_l, rho_v, width=4.0, mrt=mrt)
    print(f"# MRT G={G}: rho_l={rho_l:.6f} rho_v={rho_v:.6f} sigma={sigma:.5f}", file=sys.stderr, flush=True)
    rows = []
    for R0, _, _, _ in workloads.TABLE1:
        tau = analysis.tau_for_ohnesorge(workloads.TABLE1_OH, rho_l, sigma, R0)
        spec = dataclasses.replace(workloads.paper_table1(R0), tau=tau)
        co_l, co_v = lbm.lbm_coexistence(G, tau, mrt=mrt)  # the same densities at this tau
        tcap = analysis.capillary_time(rho_l, R0, sigma)
        print(f"# R0={R0} tau={tau:.4f} grid {spec.nx}x{spec.ny}x{spec.nz}", file=sys.stderr, flush=True)
        r = _run_ligament(lbm, spec, args.storage, rho_l, rho_v, stream, max_steps=int(40 * tcap) + 2000,
                          every=max(1, R0 // 8), mrt=mrt)
        r.update({"R0": R0, "grid": [spec.nx, spec.ny, spec.nz], "tau": tau, "storage": args.storage,
                  "rho_l_at_tau": co_l, "rho_v_at_tau": co_v, "t_cap": tcap,
                  "t_b_over_t_cap": None if r["t_b"] is None else r["t_b"] / tcap})
        rows.append(r)
        print(f"# {json.dumps(r)}", file=sys.stderr, flush=True)
    print(json.dumps({"study": "paper_table1_mrt", "G": G, "Oh": workloads.TABLE1_OH, "mrt": mrt,
                      "rho_l": rho_l, "rho_v": rho_v, "sigma": sigma, "laplace_intercept": icpt,
                      "rows": rows}))


def bench_batch(args, lbm, workloads, stream):
    """64 ligaments of uneven size and parameters: one launch per step over
    all cases (autotuned tile, hipGraph chunks) against the same cases run one
    after another with separate launches of the single-grid kernel."""
    import torch

    cases = workloads.batch64()
    params = [lbm.make_params(c.nx, c.ny, c.nz, c.tau, c.G, storage=args.storage) for c in cases]
    specs = [lbm.make_ligament(c.nx, c.ny, c.nz, R0=c.R0, amp_rel=c.amp_rel,
                               wavelength=c.wavelength, seed=c.seed) for c in cases]
    print(f"# batch of {len(cases)}, {sum(c.n for c in cases)} nodes: coexistence per case",
          file=sys.stderr, flush=True)
    b = lbm.Batch(params, stream=stream)
    b.init(specs)
    # The first 1000 steps include the batch's first divergence check, which
    # freezes the cases whose drawn (tau, G) leave the scheme's stability
    # region; the timed steps then run the live cases only, and only their
    # nodes are counted.
    b.step(1000)
    diags = b.diagnostics()
    live = [i for i, d in enumerate(diags) if d["nonfinite"] == 0]
    nodes = sum(cases[i].n for i in live)
    if args.launch:  # a fixed launch (profiling runs), else the autotuner's pick
        launch = tuple(int(v) for v in args.launch.split(","))
        b.set_launch(*launch)
    else:
        launch, tuned = b.autotune(20)
    print(f"# {len(live)} live cases, {nodes} nodes; launch {launch}", file=sys.stderr,
          flush=True)
    chunk = args.graph_chunk or 100
    b.set_graph_chunk(chunk)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.step(max(args.warmup, chunk))  # also captures the graph
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    # sequential baseline: the live cases one after another, separate launches
    seq_ms = 0.0
    for i in live:
        c = cases[i]
        lat = lbm.Lattice(c.nx, c.ny, c.nz, c.tau, c.G, storage=args.storage, stream=stream)
        lat.init_ligament(R0=c.R0, amp_rel=c.amp_rel, wavelength=c.wavelength, rho_l=2.2, rho_v=0.1,
                          seed=c.seed)
        lat.step(3)
        e0.record(stream)
        lat.step(args.steps)
        e1.record(stream)
        e1.synchronize()
        seq_ms += e0.elapsed_time(e1)
        lat.close()
    seq_mlups = nodes * args.steps / (seq_ms * 1e-3) / 1e6
    out = {"metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.storage, "data": "synthetic",
           "config": {"workload": f"batch64: {len(cases)} ligaments, {sum(c.n for c in cases)} nodes, "
                                  f"R0 6-20, kR 0.3-0.9, tau 0.6-1.2, G -6 to -5",
                      "launch": list(launch), "graph_chunk": chunk,
                      "live_cases": len(live), "frozen_cases": len(cases) - len(live),
                      "live_nodes": nodes},
           "sequential_MLUPS": round(seq_mlups, 1),
           "speedup_vs_sequential": round(mlups / seq_mlups, 3),
           "roofline": {"bound": "hbm", "achieved": round(2 * BYTES_PER_NODE[args.storage] * nodes *
                                                          args.steps / (ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s"}}
    out["roofline"]["frac"] = round(out["roofline"]["achieved"] / HBM_PEAK_GBS, 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
