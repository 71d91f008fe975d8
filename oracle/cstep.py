"""Independent NumPy re-statement of the Euler-Cromer forward run (test infrastructure).

Written separately from ``pd_oracle.c`` and vectorised over slots, it accepts complex
inputs so that complex-step derivatives (Squire and Trapp, SIAM Review 40, 1998) of a
run with respect to the per-slot stiffness or the body-force magnitude can be taken:
d f/d p = Im f(p + i h) / h, exact to rounding for real-analytic f.  Breaking follows a
frozen schedule (slot b acts in pass k iff k < frozen[b]).  Damping follows the damped
equation of motion (Sec. 2.3): the acceleration is (F - eta v)/rho with the velocity of
the start of the step.
"""
from __future__ import annotations

import numpy as np


def ec_forward(x, row_ptr, col, kslot, vol, rho, dt, frozen, steps, *, bhat=None, bmag=0.0,
               bc_kind=None, bc_sched=None, bc_val=None, u0=None, v0=None, step0=0, dtype=complex,
               eta=0.0):
    """Displacement after `steps` Euler-Cromer steps (f = k s V_j y/|y|, Eq. simpleBond)."""
    n = x.shape[0]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    cols = np.asarray(col, dtype=np.int64)
    xi = x[cols] - x[rows]
    L = np.sqrt((xi * xi).sum(1))
    vj = np.asarray(vol, dtype=float)[cols] if np.ndim(vol) else np.full(cols.shape[0], float(vol))
    kk = np.asarray(kslot).astype(dtype)
    u = np.zeros((n, 3), dtype=dtype) if u0 is None else np.array(u0, dtype=dtype)
    v = np.zeros((n, 3), dtype=dtype) if v0 is None else np.array(v0, dtype=dtype)
    b = None if bhat is None else np.asarray(bhat, dtype=float) * bmag
    kind = np.zeros((n, 3), dtype=np.uint8) if bc_kind is None else bc_kind
    for k in range(step0, step0 + steps):
        alive = (k < np.asarray(frozen)).astype(float)
        y = xi + (u[cols] - u[rows])
        r = np.sqrt((y * y).sum(1))
        s = (r - L) / L
        f = ((kk * s * vj / r) * alive)[:, None] * y
        F = np.zeros((n, 3), dtype=dtype)
        np.add.at(F, rows, f)
        if b is not None:
            F = F + b
        vn = v + dt * ((F - eta * v) / rho)
        un = u + dt * vn
        t1 = (k + 1) * dt
        if bc_kind is not None:
            g = np.where(bc_sched == 1, t1, 1.0)
            dg = np.where(bc_sched == 1, 1.0, 0.0)
            disp, vel = kind == 1, kind == 2
            vn = np.where(disp, bc_val * dg, np.where(vel, bc_val * g, vn))
            un = np.where(disp, bc_val * g, np.where(vel, u + dt * (bc_val * g), un))
        u, v = un, vn
    return u, v


def force_cs(x, row_ptr, col, kslot, vol, u, frozen, k):
    """Force density (no body force) for a complex displacement; used for J v by complex step."""
    n = x.shape[0]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    cols = np.asarray(col, dtype=np.int64)
    xi = x[cols] - x[rows]
    L = np.sqrt((xi * xi).sum(1))
    vj = np.asarray(vol, dtype=float)[cols] if np.ndim(vol) else np.full(cols.shape[0], float(vol))
    y = xi + (u[cols] - u[rows])
    r = np.sqrt((y * y).sum(1))
    s = (r - L) / L
    alive = (k < np.asarray(frozen)).astype(float)
    f = ((kslot * s * vj / r) * alive)[:, None] * y
    F = np.zeros((n, 3), dtype=u.dtype)
    np.add.at(F, rows, f)
    return F
