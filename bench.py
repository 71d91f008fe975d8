#!/usr/bin/env python3
"""Throughput of the fused peridynamics step on one MI355X.

Default workload: the 100 x 100 x 100 simple-cubic cube (1,000,000 nodes, horizon
3.015 dx, 117,844,248 directed bond slots), FP64, Euler-Cromer, face z = 0 clamped and
face z = 99 pulled at 1e-8 m per step; the library's autotuner picks the mapping and the
device node order (natural or Morton).  One "step" is one full time step of every node
(gather, stretch, break check, PMB force, per-node sum, integration, boundary
conditions).  Prints one JSON line.
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

PEAK_HBM_GBS = 8000.0
# MI355X vector peaks (256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz)
PEAK_VALU_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Algorithmic flops of one slot update, the method's own arithmetic in its direct form
# (Eqs. microelastic and simpleBond, Algorithm 2; a square root counts one): bond vector,
# displacement difference and deformed bond (9), |y|^2 and |xi|^2 (10), the two square
# roots (2), s = (r - L)/L (2), the coefficient c s V_j / r (3), the force update (6).
ALGO_FLOPS_PER_SLOT = 32
# the committed rocprofv3 counter summary of the headline kernel (VALU instructions per
# slot row), used when it was taken on the current kernel source
COUNTERS = os.path.join(ROOT, "profiles", "counters_step_cube100_f64.txt")
STEP_SOURCES = [os.path.join(ROOT, "paper_2105_04150_amd", "csrc", f)
                for f in ("pdmi_step.h", "pdmi_device.h", "pdmi_internal.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in STEP_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_values(path: str) -> dict:
    """key: value lines of a committed profile summary, or {} if it was taken on another
    kernel source than the current one."""
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals if vals.get("kernel_source_sha256_16") == kernel_hash() else {}


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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps: int, threads: int, single_steps: int):
    """The FP64 oracle as it stands, on the host cores, over bounded prefixes of the same
    workload: all `threads` cores (the reported value) and one core; the oracle's family
    build (cell list) is timed on its own."""
    import oracle.oracle as O
    t0 = time.perf_counter()
    O.family(w.coords, w.horizon)
    family_s = time.perf_counter() - t0
    rates = {}
    for nt, k in ((threads, steps), (1, single_steps)):
        sim = O.from_workload(w, nthreads=nt)
        sim.run(1)  # first step outside the timing (page-in)
        t0 = time.perf_counter()
        sim.run(k)
        rates[nt] = sim.nnz * k / (time.perf_counter() - t0)
        nnz = sim.nnz
        del sim
    return {"value": rates[threads], "unit": "bond-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} Euler-Cromer steps of the same {w.n}-node, {nnz}-slot workload on {threads} "
                      f"threads and {single_steps} on one, each after one untimed step; the family build "
                      f"timed separately",
            "single_core": {"value": rates[1], "unit": "bond-updates/s", "cores": 1},
            "family_build_s": family_s, "nproc": os.cpu_count(), "cpu_model": cpu_model()}


SETTLE = True  # cleared by --no-settle (counter runs, which time nothing)


def settle(sim, seconds: float = 0.4):
    """Bring the GPU to its steady clock before a measurement: run steps for about
    `seconds` of device time, then put the problem back exactly as it was (u, v, a,
    broken flags and the step counter), so the timed steps start from the state the
    warm-up steps leave, as without this.  Part of setup, outside every timed region."""
    if not SETTLE:
        return
    u, v, a, br, k = sim.u(), sim.v(), sim.a(), sim.broken(), sim.step_count
    sim.step(8)
    sim.sync()
    per = max(sim.last_step_ms() / 8, 1e-3)
    sim.step(max(8, int(seconds * 1e3 / per)))
    sim.sync()
    sim.set_state(u=u, v=v, a=a, broken=br)
    sim.set_step(k)
    sim.prepare()
    # the restore above left the GPU idle while the host copied the state; keep it busy
    # again until the caller's warm-up starts, with force evaluations, which read the
    # state and change none of it (no bond breaks, no integration)
    t_end = time.perf_counter() + 0.1
    while time.perf_counter() < t_end:
        sim.resultant(np.array([0], dtype=np.int64))


def _timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    fn()
    sync()
    return time.perf_counter() - t0


def adjoint_extra(P, pi, sync, steps: int, ckpt: int, mapping: str = "auto"):
    """Adjoint on the 100 x 25 x 20 beam (Euler-Cromer, stiffness field, tip load, 200
    sensors): plain steps, the recording forward run and the reverse pass, timed on the
    same problem.  Rates are bond-updates per second of simulated forward steps.
    mapping "staged" fixes four wavefronts per slice instead of asking the autotuner (the
    counter runs do, since counter collection serialises the trial launches)."""
    w = pi.workload("adjoint_beam", steps=steps)
    sim = P.simulation_for(w, lanes=4)
    if mapping == "staged":
        sim.set_mapping("staged", 4)
    else:
        sim.autotune(trial_steps=10)
    sim.prepare()
    info = sim.info()
    nnz = info["n_slots"]
    sensors, target = pi.adjoint_sensors(w)
    z = np.zeros((w.n, 3))
    sim.step(50)  # warm-up (graphs, caches)
    sim.sync()
    sim.set_state(u=z, v=z, a=z)
    sim.set_step(0)
    t_plain = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    sim.set_state(u=z, v=z, a=z, broken=np.zeros(nnz, dtype=np.uint8))
    sim.set_step(0)
    t_fwd = _timed(lambda: (sim.adj_forward(steps, ckpt), sim.sync()), sync)
    dldu = 2.0 * (sim.u()[sensors] - target)
    t_bwd = _timed(lambda: sim.adj_backward(sensors, dldu), sync)
    # the whole trajectory kept in HBM (a checkpoint at every level: no recompute)
    sim.set_state(u=z, v=z, a=z, broken=np.zeros(nnz, dtype=np.uint8))
    sim.set_step(0)
    t_fwd1 = _timed(lambda: (sim.adj_forward(steps, 1), sim.sync()), sync)
    dldu1 = 2.0 * (sim.u()[sensors] - target)
    t_bwd1 = _timed(lambda: sim.adj_backward(sensors, dldu1), sync)
    traj_bytes = steps * info["n_nodes_dev"] * 48
    mapping = "staged" if info["mapping"] == P.PD_MAP_STAGED else f"sliced-{info['lanes_per_node']}"
    sim.close()
    plain = nnz * steps / t_plain
    return {"config": f"adjoint_beam {w.dims[0]}x{w.dims[1]}x{w.dims[2]}, {steps} Euler-Cromer steps, "
                      f"checkpoint every {ckpt}, {len(sensors)} sensors, f64",
            "bond_slots": nnz, "mapping": mapping,
            "plain_step_rate": plain, "plain_ms": t_plain * 1e3,
            "forward_recording_ms": t_fwd * 1e3, "backward_ms": t_bwd * 1e3,
            "adjoint_rate": nnz * steps / (t_fwd + t_bwd),
            "adjoint_vs_plain": (nnz * steps / (t_fwd + t_bwd)) / plain,
            "backward_vs_plain_step": t_plain / t_bwd,
            "full_trajectory": {"trajectory_bytes": traj_bytes, "forward_recording_ms": t_fwd1 * 1e3,
                                "backward_ms": t_bwd1 * 1e3, "adjoint_rate": nnz * steps / (t_fwd1 + t_bwd1),
                                "adjoint_vs_plain": (nnz * steps / (t_fwd1 + t_bwd1)) / plain}}


def batched_extra(P, pi, sync, count: int, steps: int, seq_sample: int, tune: bool = True):
    """Many uneven uncertainty-quantification beams advanced together, against the same
    instances advanced one problem at a time (a sample of them) on the same GPU.  The
    mapping and node order come from the library's autotuner run on four of the beams
    (the full batch takes tens of seconds per layout build).  Each beam's log-normal
    stiffness field is passed as its node values (bond stiffness sqrt(k_i k_j))."""
    ws = pi.batch_instances(count=count, steps=steps)
    t0 = time.perf_counter()
    mapping, lanes, order = "staged", 1, "natural"
    if tune:
        sub = [ws[b] for b in np.unique(np.linspace(0, count - 1, min(4, count)).round().astype(int))]
        tun = P.Simulation()
        tun.build_family_batch([w.coords for w in sub], [w.horizon for w in sub], order="auto")
        tun.set_integrator("euler_cromer", ws[0].dt)
        for b, w in enumerate(sub):
            P.apply_workload(tun, w, inst=b, stiffness="node")
        tun.autotune(trial_steps=5)
        ti = tun.info()
        tun.close()
        mapping = "staged" if ti["mapping"] == P.PD_MAP_STAGED else "sliced"
        lanes = ti["lanes_per_node"]
        order = "morton" if ti["order"] == P.PD_ORDER_MORTON else "natural"
        print(f"# batched: autotuned on {len(sub)} beams: {mapping}-{lanes}, {order}", file=sys.stderr, flush=True)
    sim = P.Simulation()
    sim.set_mapping(mapping, lanes)
    sim.build_family_batch([w.coords for w in ws], [w.horizon for w in ws], order=order)
    print(f"# batched: {count} families built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    sim.set_integrator("euler_cromer", ws[0].dt)
    for b, w in enumerate(ws):
        P.apply_workload(sim, w, inst=b, stiffness="node")
    sim.prepare()
    setup = time.perf_counter() - t0
    info = sim.info()
    nnz = info["n_slots"]
    sim.step(20)
    sim.sync()
    t_b = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    sim.close()
    idx = np.unique(np.linspace(0, count - 1, min(seq_sample, count)).round().astype(int))
    seq_slots, seq_t = 0, 0.0
    print(f"# batched: {t_b * 1e3 / steps:.3f} ms/step; sequential sample next", file=sys.stderr, flush=True)
    for b in (idx if seq_sample > 0 else []):
        s1 = P.simulation_for(ws[b], lanes=lanes, mapping=mapping, order=order, stiffness="node")
        s1.prepare()
        s1.step(20)
        s1.sync()
        seq_t += _timed(lambda: (s1.step(steps), s1.sync()), sync)
        seq_slots += s1.info()["n_slots"]
        s1.close()
    batched = nnz * steps / t_b
    seq = seq_slots * steps / seq_t if seq_t > 0 else float("nan")
    return {"config": f"{count} beams, dims {ws[0].dims}..{ws[-1].dims}, {steps} Euler-Cromer steps, f64",
            "instances": count, "nodes": info["n_nodes"], "bond_slots": nnz,
            "mapping": mapping if mapping == "staged" else f"sliced-{lanes}", "node_order": order,
            "setup_s": setup, "batched_rate": batched, "ms_per_step": t_b * 1e3 / steps,
            "sequential_rate": seq, "sequential_sample": [int(b) for b in idx],
            "batched_vs_sequential": batched / seq}


def quasistatic_extra(P, pi, sync, steps: int, every: int):
    """The quasi-static toolkit on the notched three-point bend of Sec. 6 (175 x 50 x 50
    lattice, velocity Verlet with damping, fifth-order load ramp, no-failure zones on the
    support and load nodes): the step rate with the zones (zone-aware kernels), the same
    with a load readout (device resultant of the load set) every `every` steps, and the
    rate once the zones are removed (plain kernels), each over `steps` steps of one
    continuing run."""
    w = pi.workload("qs_beam")
    sim = P.simulation_for(w)
    sim.autotune(trial_steps=10)
    sim.prepare()
    info = sim.info()
    nnz = info["n_slots"]
    _, _, load = pi.qs_beam_sets(w.ijk, w.dims)
    sim.step(20)
    sim.sync()
    t_zone = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    loads = []

    every = max(1, min(every, steps // 4))  # at least four readouts in the timed steps

    def with_readout():
        for _ in range(steps // every):
            sim.step(every)
            loads.append(float(sim.resultant(load)[2]))
    t_read = _timed(with_readout, sync)
    n_read = steps // every
    sim.set_no_fail(None)
    sim.prepare()
    sim.step(5)
    sim.sync()
    t_plain = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    mapping = (f"staged-{info['waves_per_slice']}" if info["mapping"] == P.PD_MAP_STAGED
               else f"sliced-{info['lanes_per_node']}")
    sim.close()
    return {"config": f"qs_beam {w.dims[0]}x{w.dims[1]}x{w.dims[2]}, velocity Verlet, eta {w.eta:g}, "
                      f"ramp {w.ramp_T:g} s, {len(w.nofail)} zone nodes, f64",
            "nodes": info["n_nodes"], "bond_slots": nnz, "mapping": mapping, "steps": steps,
            "value": nnz * steps / t_zone, "unit": "bond-updates/s", "avg_launch_ms": dev_ms,
            "hbm_frac": info["model_bytes_per_step"] / (dev_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
            "rate_with_load_readout": nnz * n_read * every / t_read, "readout_every": every,
            "readout_ms": max(t_read - t_zone * n_read * every / steps, 0.0) * 1e3 / max(n_read, 1),
            "last_load_N": loads[-1] if loads else None,
            "rate_without_zones": nnz * steps / t_plain,
            "zones_vs_plain": t_plain / t_zone}


def damage_law_extra(P, pi, sync, steps: int):
    """The trilinear damage law of Sec. 6 on the full-size notched bend (the qs_beam
    workload with its zones, ramp and damping): K steps from the start of loading, then
    K steps with every slot marked softened (each slot takes the bond-model branch every
    step: the worst case), both against the rate of the same problem with the brittle law."""
    w = pi.workload("qs_beam", law="trilinear")
    sim = P.simulation_for(w)
    sim.autotune(trial_steps=10)
    sim.prepare()
    info = sim.info()
    nnz = info["n_slots"]
    sim.step(20)
    sim.sync()
    t_law = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    soft = float((sim.max_stretch() > 0).mean())
    # a fracture process zone: every bond of the nodes within 3 spacings of the notch
    # plane softened to the middle of the second branch; then the worst case, every slot
    s_mid = 0.5 * (pi.LAW_TRILINEAR[0][1] + pi.LAW_TRILINEAR[0][2])
    rp, _ = sim.family()
    band_nodes = np.abs(w.ijk[:, 0] - w.dims[0] // 2) <= 3
    band = np.repeat(band_nodes, np.diff(rp))
    sim.set_max_stretch(np.where(band, s_mid, 0.0))
    sim.prepare()
    sim.step(5)
    sim.sync()
    t_band = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    sim.set_max_stretch(np.full(nnz, s_mid))
    sim.prepare()
    sim.step(5)
    sim.sync()
    t_all = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    mapping = (f"staged-{info['waves_per_slice']}" if info["mapping"] == P.PD_MAP_STAGED
               else f"sliced-{info['lanes_per_node']}")
    sim.close()
    return {"config": f"qs_beam {w.dims[0]}x{w.dims[1]}x{w.dims[2]}, trilinear law {pi.LAW_TRILINEAR}, velocity "
                      f"Verlet, zones, f64",
            "bond_slots": nnz, "mapping": mapping, "steps": steps,
            "value": nnz * steps / t_law, "unit": "bond-updates/s", "avg_launch_ms": dev_ms,
            "softened_fraction_after": soft,
            "band_softened_fraction": float(band.mean()), "rate_band_softened": nnz * steps / t_band,
            "band_softened_vs_start": t_law / t_band,
            "rate_all_softened": nnz * steps / t_all, "all_softened_vs_start": t_law / t_all}


def corrections_extra(P, pi, sync, workload: str, steps: int, plain_ms: float):
    """The headline workload with the conical micromodulus and the volume-method surface
    correction (peak 5c for the same bulk stiffness): the corrected stiffness streams per
    slot, 8 more bytes per slot than the plain step."""
    w = pi.workload(workload)
    w.order = "natural"
    w.c = 5.0 * w.c
    w.corrections = dict(micro="conical", surface=True, delta=w.horizon, dx=w.dx)
    sim = P.simulation_for(w, mapping="staged")
    sim.prepare()
    settle(sim)
    info = sim.info()
    sim.step(20)
    sim.sync()
    t = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    sim.close()
    nnz = info["n_slots"]
    return {"config": f"{workload}, conical micromodulus + surface correction, staged mapping, natural order",
            "steps": steps, "value": nnz * steps / t, "unit": "bond-updates/s", "avg_launch_ms": dev_ms,
            "model_bytes_per_step": info["model_bytes_per_step"],
            "hbm_frac": info["model_bytes_per_step"] / (dev_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
            "vs_plain_step": plain_ms / dev_ms}


def state_based_extra(P, pi, sync, workload: str, steps: int, plain_ms: float):
    """The headline workload on the ordinary state-based linear solid (same bulk modulus,
    Poisson ratio 0.2): two kernels per step, the dilation pass then the force pass, each
    gathering the whole family; one bond update per slot and step as for the PMB."""
    w = pi.workload(workload, model="state_based")
    w.order = "natural"
    sim = P.simulation_for(w, mapping="staged")
    sim.prepare()
    settle(sim)
    info = sim.info()
    sim.step(20)
    sim.sync()
    t = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    sim.close()
    nnz = info["n_slots"]
    # the FP32 build of the same step
    sim = P.simulation_for(w, precision=P.PD_FP32, mapping="staged")
    sim.prepare()
    settle(sim)
    sim.step(20)
    sim.sync()
    t32 = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev32 = sim.last_step_ms() / steps
    sim.close()
    return {"config": f"{workload}, state-based linear solid (K, nu = 0.2), staged mapping, natural order",
            "steps": steps, "value": nnz * steps / t, "unit": "bond-updates/s", "step_ms": dev_ms,
            "model_bytes_per_step": info["model_bytes_per_step"],
            "hbm_frac": info["model_bytes_per_step"] / (dev_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
            "vs_plain_step": plain_ms / dev_ms,
            "fp32": {"value": nnz * steps / t32, "step_ms": dev32, "vs_fp64": dev_ms / dev32}}


def wide_extra(P, pi, sync, steps: int):
    """The 1M-node cube at the wider horizon 5.015 dx (514 neighbours per node, 485,972,824
    slots), FP64, Euler-Cromer, one wavefront per slice of the staged mapping, natural
    order (the headline's choice on the 3.015 dx cube)."""
    w = pi.workload("cube100_wide")
    w.order = "natural"
    t0 = time.perf_counter()
    sim = P.simulation_for(w, mapping="staged")
    sim.prepare()
    settle(sim)
    setup = time.perf_counter() - t0
    info = sim.info()
    sim.step(5)
    sim.sync()
    t = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    sim.close()
    nnz = info["n_slots"]
    return {"config": "cube100_wide 100x100x100 lattice, horizon 5.015 dx, euler_cromer, staged-1, natural order, f64",
            "bond_slots": nnz, "steps": steps, "setup_s": setup, "value": nnz * steps / t, "unit": "bond-updates/s",
            "ms_per_step": t * 1e3 / steps, "avg_launch_ms": dev_ms,
            "model_bytes_per_step": info["model_bytes_per_step"],
            "hbm_frac": info["model_bytes_per_step"] / (dev_ms / 1e3) / 1e9 / PEAK_HBM_GBS}


def fp32_extra(P, pi, sync, workload: str, steps: int):
    """The FP32 build (f32 bond arithmetic, f64 master displacement) on the headline
    workload with the staged mapping, the only mapping it runs."""
    w = pi.workload(workload)
    w.order = "natural"
    sim = P.simulation_for(w, precision=P.PD_FP32, mapping="staged")
    sim.prepare()
    settle(sim)
    info = sim.info()
    sim.step(20)
    sim.sync()
    t = _timed(lambda: (sim.step(steps), sim.sync()), sync)
    dev_ms = sim.last_step_ms() / steps
    sim.close()
    nnz = info["n_slots"]
    return {"config": f"{workload}, FP32 build, staged mapping, natural order", "steps": steps,
            "value": nnz * steps / t, "unit": "bond-updates/s", "ms_per_step": t * 1e3 / steps,
            "avg_launch_ms": dev_ms,
            "hbm_frac": info["model_bytes_per_step"] / (dev_ms / 1e3) / 1e9 / PEAK_HBM_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cube100",
                    choices=["cube100", "cube100_wide", "block10", "beam3pb", "qs_beam"])
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--model", default="pmb", choices=["pmb", "state_based"],
                    help="constitutive model of the timed line (state_based: profiling runs of "
                         "the two-pass step; the state-based extra line covers it otherwise)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per node of the sliced mapping")
    ap.add_argument("--mapping", default="auto", choices=["auto", "sliced", "staged"],
                    help="step-kernel mapping (auto: the library's autotuner picks)")
    ap.add_argument("--order", default="auto", choices=["auto", "natural", "morton"],
                    help="device node order (auto: the autotuner tries both)")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-single-steps", type=int, default=2, help="oracle steps timed on one core")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32, adjoint, batched and quasi-static measurements")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-mapping", default="auto", choices=["auto", "staged"],
                    help="adjoint line: the autotuner's mapping, or staged with four wavefronts per slice")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=300)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--extra", default="", choices=["", "adjoint", "batched", "corrections", "quasistatic"],
                    help="profiling runs: only this extra measurement, in a process with one library "
                         "context (batched: staged-1, natural order, no sequential sample); prints its line")
    ap.add_argument("--no-settle", action="store_true",
                    help="skip the clock warm-up before each measurement (counter-collection runs)")
    args = ap.parse_args()
    global SETTLE
    SETTLE = not args.no_settle

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
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import pd_inputs as pi
    import paper_2105_04150_amd as P

    if args.extra:
        try:
            import torch
            sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
        except Exception:
            sync = lambda: None  # noqa: E731
        if args.extra == "adjoint":
            line = adjoint_extra(P, pi, sync, args.adjoint_steps, 100, args.adjoint_mapping)
        elif args.extra == "batched":
            line = batched_extra(P, pi, sync, args.batch_count, args.batch_steps, 0, tune=False)
        elif args.extra == "corrections":
            line = corrections_extra(P, pi, sync, args.workload, args.steps, float("nan"))
        else:
            line = quasistatic_extra(P, pi, sync, args.steps, 50)
        print(json.dumps({"extra": args.extra, **line}), flush=True)
        return

    try:  # imported before the problem is built: no import pause between setup and timing
        import torch
        torch_sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        torch_sync = lambda: None  # noqa: E731

    w = pi.workload(args.workload, model=args.model)
    if args.model == "state_based" and (args.mapping != "staged" or args.precision != "f64"):
        sys.exit("the state-based model runs with --mapping staged --precision f64")
    w.order = args.order
    prec = P.PD_FP64 if args.precision == "f64" else P.PD_FP32
    t0 = time.perf_counter()
    if args.mapping == "auto":
        sim = P.simulation_for(w, precision=prec)
        sim.autotune(trial_steps=10)
    else:
        sim = P.simulation_for(w, precision=prec, lanes=args.lanes, mapping=args.mapping)
    sim.prepare()  # step graphs built before the warm-up, not inside the timed region
    settle(sim)
    setup_s = time.perf_counter() - t0
    info = sim.info()
    mapping = "staged" if info["mapping"] == P.PD_MAP_STAGED else "sliced"
    order = "morton" if info["order"] == P.PD_ORDER_MORTON else "natural"
    lanes = info["lanes_per_node"]
    print(f"# setup {setup_s:.1f} s, nodes {info['n_nodes']}, slots {info['n_slots']}, "
          f"device slots {info['n_slots_dev']}, mapping {mapping}, lanes {lanes}, order {order}",
          file=sys.stderr, flush=True)

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
    achieved_gbs = model_bytes / per_launch_s / 1e9
    traffic = measured_traffic(args.workload, args.precision)
    tflops = nnz * ALGO_FLOPS_PER_SLOT / per_launch_s / 1e12
    peak = PEAK_VALU_TFLOPS[args.precision]
    counters = profile_values(COUNTERS) if (args.workload, args.precision) == ("cube100", "f64") else {}
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
                               f"horizon {w.horizon / w.dx:.3f} dx, {w.scheme}"
                               + (", state-based linear solid" if args.model == "state_based" else ""),
                   "nodes": info["n_nodes"], "bond_slots": nnz, "mapping": mapping, "lanes_per_node": lanes,
                   "device_node_order": order,
                   "parallelism": "1 GPU"},
        # the method's roofline is HBM bandwidth over its compulsory bytes per step (4 B
        # per slot, node state read and written); beside it the method's own FP64
        # arithmetic against the vector peak and the instructions the kernel issues
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / PEAK_HBM_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": model_bytes, "avg_launch_ms": per_launch_s * 1e3,
                     "alu": {"achieved": tflops, "peak": peak, "unit": "TFLOP/s", "frac": tflops / peak,
                             "algorithmic_flops_per_slot": ALGO_FLOPS_PER_SLOT,
                             "valu_instructions_per_slot_row":
                                 float(counters["valu_wave_instructions_per_slot_row"])
                                 if "valu_wave_instructions_per_slot_row" in counters else None}},
    }
    sim.close()
    if args.model == "state_based":  # a profiling run: the PMB roofline does not apply
        out["roofline"] = {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": achieved_gbs / PEAK_HBM_GBS, "traffic": None, "step_ms": per_launch_s * 1e3,
                           "note": "two kernels per step; step time over the algorithmic bytes of both"}
    if not args.no_extras and args.model == "pmb":
        if args.precision == "f64":
            out["fp32"] = fp32_extra(P, pi, torch_sync, args.workload, args.steps)
            out["fp32"]["vs_fp64"] = out["fp32"]["value"] / value
            print(f"# fp32 {out['fp32']}", file=sys.stderr, flush=True)
        out["corrections"] = corrections_extra(P, pi, torch_sync, args.workload, args.steps, per_launch_s * 1e3)
        print(f"# corrections {out['corrections']}", file=sys.stderr, flush=True)
        out["state_based"] = state_based_extra(P, pi, torch_sync, args.workload, args.steps, per_launch_s * 1e3)
        print(f"# state_based {out['state_based']}", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_extra(P, pi, torch_sync, args.adjoint_steps, 100)
        out["adjoint"]["adjoint_vs_headline_step"] = out["adjoint"]["adjoint_rate"] / value
        print(f"# adjoint {out['adjoint']}", file=sys.stderr, flush=True)
        out["batched"] = batched_extra(P, pi, torch_sync, args.batch_count, args.batch_steps, 8)
        out["batched"]["batched_vs_headline_step"] = out["batched"]["batched_rate"] / value
        print(f"# batched {out['batched']}", file=sys.stderr, flush=True)
        out["quasistatic"] = quasistatic_extra(P, pi, torch_sync, args.steps, 50)
        print(f"# quasistatic {out['quasistatic']}", file=sys.stderr, flush=True)
        out["damage_law"] = damage_law_extra(P, pi, torch_sync, args.steps)
        out["damage_law"]["vs_brittle_zones"] = out["damage_law"]["value"] / out["quasistatic"]["value"]
        print(f"# damage_law {out['damage_law']}", file=sys.stderr, flush=True)
        if args.workload == "cube100" and args.precision == "f64":
            out["cube100_wide"] = wide_extra(P, pi, torch_sync, args.steps)
            print(f"# cube100_wide {out['cube100_wide']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        # the oracle on the box's share of host cores (16 on the GPU machine) and on one
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, threads, args.cpu_single_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
