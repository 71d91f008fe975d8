#!/usr/bin/env python3
"""Throughput of the fused peridynamics step on one MI355X.

Default workload: the 100 x 100 x 100 simple-cubic cube (1,000,000 nodes, horizon
3.015 dx, 117,844,248 directed bond slots), FP64, Euler-Cromer, face z = 0 clamped and
face z = 99 pulled at 1e-8 m per step, Morton node order.  One "step" is one full
time step of every node (gather, stretch, break check, PMB force, per-node sum,
integration, boundary conditions).  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2105_04150_amd", "csrc", "pdmi_kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, steps: int, threads: int):
    """The FP64 oracle as it stands, on the host cores, over a bounded prefix."""
    from oracle.oracle import from_workload
    sim = from_workload(w, nthreads=threads)
    sim.run(1)  # first step outside the timing (page-in)
    t0 = time.perf_counter()
    sim.run(steps)
    dt = time.perf_counter() - t0
    return {"value": sim.nnz * steps / dt, "unit": "bond-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} Euler-Cromer steps of the same {w.n}-node workload after one untimed step "
                      f"(family built by the oracle, not timed)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cube100", choices=["cube100", "cube100_wide", "block10", "beam3pb"])
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--lanes", type=int, default=0, help="lanes per node of the sliced mapping")
    ap.add_argument("--mapping", default="auto", choices=["auto", "sliced", "staged"],
                    help="step-kernel mapping (auto: the library's autotuner picks)")
    ap.add_argument("--order", default="auto", choices=["auto", "natural", "morton"],
                    help="device node order (auto: the autotuner tries both)")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8,
                          "copies": 3}), flush=True)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import pd_inputs as pi
    import paper_2105_04150_amd as P

    w = pi.workload(args.workload)
    w.order = args.order
    prec = P.PD_FP64 if args.precision == "f64" else P.PD_FP32
    t0 = time.perf_counter()
    if args.mapping == "auto":
        sim = P.simulation_for(w, precision=prec)
        sim.autotune(trial_steps=10)
    else:
        sim = P.simulation_for(w, precision=prec, lanes=args.lanes, mapping=args.mapping)
    setup_s = time.perf_counter() - t0
    info = sim.info()
    mapping = "staged" if info["mapping"] == P.PD_MAP_STAGED else "sliced"
    order = "morton" if info["order"] == P.PD_ORDER_MORTON else "natural"
    lanes = info["lanes_per_node"]
    print(f"# setup {setup_s:.1f} s, nodes {info['n_nodes']}, slots {info['n_slots']}, "
          f"device slots {info['n_slots_dev']}, mapping {mapping}, lanes {lanes}, order {order}",
          file=sys.stderr, flush=True)

    try:
        import torch
        torch_sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        torch_sync = lambda: None  # noqa: E731

    sim.step(args.warmup)
    sim.sync()
    torch_sync()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch_sync()
    wall = time.perf_counter() - t0
    dev_ms = sim.last_step_ms()

    nnz = info["n_slots"]
    value = nnz * args.steps / wall
    per_launch_s = dev_ms / 1e3 / args.steps
    model_bytes = info["model_bytes_per_step"]
    achieved = model_bytes / per_launch_s / 1e9
    traffic = measured_traffic(args.workload, args.precision)
    out = {
        "metric": "bond-updates/s (bonds*steps/s) & % HBM peak; batched/adjoint vs plain step",
        "value": value,
        "unit": "bond-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {w.dims[0]}x{w.dims[1]}x{w.dims[2]} lattice, "
                               f"horizon {w.horizon / w.dx:.3f} dx, {w.scheme}",
                   "nodes": info["n_nodes"], "bond_slots": nnz, "mapping": mapping, "lanes_per_node": lanes,
                   "device_node_order": order,
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": model_bytes,
                     "avg_launch_ms": per_launch_s * 1e3},
    }
    sim.close()
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
