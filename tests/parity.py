"""Shared helpers for GPU-vs-oracle parity tests (no arithmetic of the method here)."""
import sys

import numpy as np

import oracle
from oracle.oracle import from_workload

# FP64 tolerance: norm-wise relative displacement error (max over nodes and components,
# divided by the largest reference displacement component).
TOL_FP64 = 1e-10
TOL_FP32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


def oracle_run(w, steps, nthreads=0, record_breaks=False):
    sim = from_workload(w, nthreads=nthreads, record_breaks=record_breaks)
    rc = sim.run(steps)
    assert rc == 0
    return sim


def gpu_run(w, steps, precision=0, lanes=0, order=None, chunks=None, mapping="sliced"):
    from paper_2105_04150_amd import simulation_for
    sim = simulation_for(w, precision=precision, lanes=lanes, order=order, mapping=mapping)
    if chunks:
        for c in chunks:
            sim.step(c)
    else:
        sim.step(steps)
    sim.sync()
    return sim


def rate_err(x, ref, dt, uref, power=1):
    """Error of a rate (velocity: power 1, acceleration: power 2) in displacement units:
    max |x - ref| dt^power / max |u_ref|, the size of its contribution to the next step."""
    den = np.abs(uref).max()
    return float(np.abs(x - ref).max() * dt ** power / den) if den > 0 else 0.0


def compare(gsim, osim, tol, what="", check_v=True, inst=0):
    u = gsim.u(inst)
    eu = rel_err(u, osim.u)
    dt = osim.P.dt
    ev = rate_err(gsim.v(inst), osim.v, dt, osim.u) if check_v else 0.0
    gb = gsim.broken(inst).astype(bool)
    ob = osim.broken_mask
    mism = int((gb != ob).sum())
    phi_err = float(np.abs(gsim.damage(inst) - osim.damage()).max())
    say(f"[parity] {what}: u rel {eu:.3e}  v (dt-scaled) {ev:.3e}  broken {int(ob.sum())} "
        f"mismatched {mism}  damage abs {phi_err:.2e}")
    return eu, ev, mism, phi_err
