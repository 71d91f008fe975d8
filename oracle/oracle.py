"""ctypes marshalling for the C oracle (``pd_oracle.c``).  No arithmetic here."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
lib_path = os.path.join(_HERE, "liboracle.so")

SCHEMES = {"euler_cromer": 0, "velocity_verlet": 1, "forward_euler": 2}


def build(force_rebuild: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math, OpenMP over rows)."""
    if force_rebuild or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            build(force_rebuild=False)
        _lib = C.CDLL(lib_path)
        P = C.c_void_p
        i64 = C.c_int64
        _lib.pdo_family_brute.restype = i64
        _lib.pdo_family_brute.argtypes = [i64, P, C.c_double, P, P]
        _lib.pdo_family_cells.restype = i64
        _lib.pdo_family_cells.argtypes = [i64, P, C.c_double, P, P]
        _lib.pdo_force.restype = None
        _lib.pdo_force.argtypes = [P, P, P, i64, P]
        _lib.pdo_run.restype = C.c_int
        _lib.pdo_run.argtypes = [P, P, i64]
        _lib.pdo_family_volumes.restype = C.c_double
        _lib.pdo_family_volumes.argtypes = [P, P]
        _lib.pdo_weighted_volumes.restype = None
        _lib.pdo_weighted_volumes.argtypes = [P, P]
        _lib.pdo_damage.restype = None
        _lib.pdo_damage.argtypes = [P, P, P, P]
        _lib.pdo_apply_jt.restype = None
        _lib.pdo_apply_jt.argtypes = [P, P, P, i64, P, P]
        _lib.pdo_adjoint_ec.restype = C.c_int
        _lib.pdo_adjoint_ec.argtypes = [P, P, i64, P, P, i64, i64, P, P, P, P]
    return _lib


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("vol", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("kslot", C.c_void_p),
                ("c", C.c_double), ("s0", C.c_double), ("rho", C.c_double),
                ("eta", C.c_double), ("dt", C.c_double), ("bhat", C.c_void_p),
                ("bmag", C.c_double), ("bc_kind", C.c_void_p), ("bc_sched", C.c_void_p),
                ("bc_val", C.c_void_p), ("scheme", C.c_int32), ("nthreads", C.c_int32),
                ("ramp_T", C.c_double), ("nofail", C.c_void_p),
                ("ncls", C.c_int32), ("pad2_", C.c_int32), ("cls_nb", C.c_void_p), ("cls_s", C.c_void_p),
                ("cls_r", C.c_void_p), ("slot_cls", C.c_void_p),
                ("micro", C.c_int32), ("pvol", C.c_int32), ("delta", C.c_double), ("pv_dx", C.c_double),
                ("surf", C.c_int32), ("pad3_", C.c_int32), ("famvol", C.c_void_p), ("v0", C.c_double),
                ("model", C.c_int32), ("pad4_", C.c_int32), ("K", C.c_double), ("G", C.c_double),
                ("m", C.c_void_p), ("theta", C.c_void_p)]


class _State(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("a", C.c_void_p),
                ("broken", C.c_void_p), ("break_step", C.c_void_p), ("frozen", C.c_void_p),
                ("step", C.c_int64), ("a_valid", C.c_int32), ("pad_", C.c_int32), ("smax", C.c_void_p)]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def family(coords: np.ndarray, delta: float, method: str = "cells"):
    """CSR family (row_ptr int64[n+1], col int32[nnz]) of Eq. family, self excluded."""
    lib = _load()
    x = np.ascontiguousarray(coords, dtype=np.float64)
    n = x.shape[0]
    fn = lib.pdo_family_cells if method == "cells" else lib.pdo_family_brute
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    nnz = fn(n, _ptr(x), float(delta), _ptr(row_ptr), None)
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    fn(n, _ptr(x), float(delta), _ptr(row_ptr), _ptr(col))
    return row_ptr, col[:nnz]


def bc_arrays(n: int, bcs: Sequence) -> tuple:
    """Per-node, per-component BC tables from a list of pd_inputs.BCSpec (later specs win)."""
    kind = np.zeros((n, 3), dtype=np.uint8)
    sched = np.zeros((n, 3), dtype=np.uint8)
    val = np.zeros((n, 3), dtype=np.float64)
    for bc in bcs:
        for d in range(3):
            if bc.comp_mask >> d & 1:
                kind[bc.nodes, d] = bc.kind
                sched[bc.nodes, d] = bc.sched
                val[bc.nodes, d] = bc.value[d]
    return kind, sched, val


class OracleSim:
    """One oracle simulation: problem data plus state, advanced by ``run``."""

    def __init__(self, coords, row_ptr, col, *, c, s0, rho, dt, vol, scheme="euler_cromer",
                 eta=0.0, kslot=None, bhat=None, bmag=0.0, bcs=(), nthreads=0,
                 record_breaks=False, frozen=None, broken=None, ramp_T=1.0, nofail=None,
                 laws=None, slot_cls=None, smax=None, corrections=None, state_based=None):
        lib = _load()
        self._lib = lib
        self.x = np.ascontiguousarray(coords, dtype=np.float64)
        self.n = n = self.x.shape[0]
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.nnz = int(self.row_ptr[-1])
        v = np.asarray(vol, dtype=np.float64)
        self.vol = np.ascontiguousarray(np.full(n, float(v)) if v.ndim == 0 else v)
        self.kslot = None if kslot is None else np.ascontiguousarray(kslot, dtype=np.float64)
        self.bhat = None if bhat is None else np.ascontiguousarray(bhat, dtype=np.float64)
        self.bc_kind, self.bc_sched, self.bc_val = bc_arrays(n, bcs)
        # per-node no-failure flags (bonds touching a flagged node never break)
        self.nofail = None if nofail is None else np.ascontiguousarray(nofail, dtype=np.uint8)
        if self.nofail is not None and self.nofail.shape != (n,):
            raise ValueError("nofail needs one flag per node")
        # damage laws: a list of (stretch breakpoints, force ratios) per bond class
        MAXB = 8
        self.laws = None if not laws else list(laws)
        ncls = 0 if self.laws is None else len(self.laws)
        self.cls_nb = np.zeros(max(ncls, 1), dtype=np.int32)
        self.cls_s = np.zeros(max(ncls, 1) * MAXB)
        self.cls_r = np.zeros(max(ncls, 1) * MAXB)
        for k, (sb, rb) in enumerate(self.laws or []):
            sb, rb = np.asarray(sb, dtype=np.float64), np.asarray(rb, dtype=np.float64)
            if not (1 <= sb.shape[0] <= MAXB and sb.shape == rb.shape):
                raise ValueError("a damage law needs 1..8 breakpoints and as many ratios")
            self.cls_nb[k] = sb.shape[0]
            self.cls_s[k * MAXB: k * MAXB + sb.shape[0]] = sb
            self.cls_r[k * MAXB: k * MAXB + sb.shape[0]] = rb
        self.slot_cls = None if slot_cls is None else np.ascontiguousarray(slot_cls, dtype=np.uint8)
        self.P = _Problem(n, _ptr(self.x), _ptr(self.vol), _ptr(self.row_ptr), _ptr(self.col),
                          _ptr(self.kslot), float(c), float(s0), float(rho), float(eta), float(dt),
                          _ptr(self.bhat), float(bmag), _ptr(self.bc_kind), _ptr(self.bc_sched),
                          _ptr(self.bc_val), SCHEMES[scheme], int(nthreads), float(ramp_T),
                          _ptr(self.nofail), ncls, 0, _ptr(self.cls_nb), _ptr(self.cls_s), _ptr(self.cls_r),
                          _ptr(self.slot_cls))
        self.u = np.zeros((n, 3))
        self.v = np.zeros((n, 3))
        self.a = np.zeros((n, 3))
        self.broken = np.zeros(max(self.nnz, 1), dtype=np.uint8)
        if broken is not None:
            self.broken[: self.nnz] = np.asarray(broken, dtype=np.uint8)
        self.break_step = (np.full(max(self.nnz, 1), np.iinfo(np.int32).max, dtype=np.int32)
                           if record_breaks else None)
        self.frozen = None if frozen is None else np.ascontiguousarray(frozen, dtype=np.int32)
        # stiffness corrections: dict(micro="constant"|"conical", partial_volumes=bool,
        # surface=bool, delta=horizon of the profile / partial volumes, dx=lattice spacing)
        corr = dict(corrections or {})
        self.P.micro = 1 if corr.get("micro", "constant") == "conical" else 0
        self.P.pvol = 1 if corr.get("partial_volumes") else 0
        self.P.delta = float(corr.get("delta", 0.0))
        self.P.pv_dx = float(corr.get("dx", 0.0))
        self.P.surf = 1 if corr.get("surface") else 0
        self.famvol = np.zeros(n)
        self.P.famvol = _ptr(self.famvol)
        if self.P.surf or self.P.pvol:
            self.P.v0 = lib.pdo_family_volumes(C.byref(self.P), _ptr(self.famvol))
        # state-based linear solid: state_based = (K, G); c, kslot, laws and corrections unused
        self.m = np.zeros(n)
        self.theta = np.zeros(n)
        self.P.m = _ptr(self.m)
        self.P.theta = _ptr(self.theta)
        if state_based is not None:
            if ncls or self.kslot is not None or self.P.micro or self.P.pvol or self.P.surf:
                raise ValueError("the state-based model takes no stiffness field, damage law or correction")
            self.P.model = 1
            self.P.K, self.P.G = (float(v) for v in state_based)
            lib.pdo_weighted_volumes(C.byref(self.P), _ptr(self.m))
        self.smax = None
        if ncls:
            self.smax = np.zeros(max(self.nnz, 1))
            if smax is not None:
                self.smax[: self.nnz] = smax
        self.S = _State(_ptr(self.u), _ptr(self.v), _ptr(self.a), _ptr(self.broken),
                        _ptr(self.break_step), _ptr(self.frozen), 0, 0, 0, _ptr(self.smax))

    @property
    def step(self) -> int:
        return int(self.S.step)

    def set_state(self, u=None, v=None, a=None, step=None, a_valid=None):
        if u is not None:
            self.u[...] = u
        if v is not None:
            self.v[...] = v
        if a is not None:
            self.a[...] = a
        if step is not None:
            self.S.step = int(step)
        if a_valid is not None:
            self.S.a_valid = int(a_valid)

    def run(self, nsteps: int) -> int:
        return self._lib.pdo_run(C.byref(self.P), C.byref(self.S), int(nsteps))

    def force(self, u=None, k=None) -> np.ndarray:
        """Force density for displacement u (default: current) in pass k (updates breaks)."""
        uu = self.u if u is None else np.ascontiguousarray(u, dtype=np.float64)
        F = np.zeros((self.n, 3))
        self._lib.pdo_force(C.byref(self.P), C.byref(self.S), _ptr(uu),
                            int(self.step if k is None else k), _ptr(F))
        return F

    def damage(self) -> np.ndarray:
        phi = np.zeros(self.n)
        self._lib.pdo_damage(C.byref(self.P), _ptr(self.broken), _ptr(self.smax), _ptr(phi))
        return phi

    @property
    def broken_mask(self) -> np.ndarray:
        return self.broken[: self.nnz].astype(bool)

    def apply_jt(self, frozen, u, k, nu) -> np.ndarray:
        fr = np.ascontiguousarray(frozen, dtype=np.int32)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        nn = np.ascontiguousarray(nu, dtype=np.float64)
        out = np.zeros((self.n, 3))
        self._lib.pdo_apply_jt(C.byref(self.P), _ptr(fr), _ptr(uu), int(k), _ptr(nn), _ptr(out))
        return out

    def adjoint_ec(self, frozen, nsteps, u0, v0, step0, sensors, dLdu):
        fr = np.ascontiguousarray(frozen, dtype=np.int32)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        sens = np.ascontiguousarray(sensors, dtype=np.int64)
        g = np.ascontiguousarray(dLdu, dtype=np.float64)
        grad_k = np.zeros(max(self.nnz, 1))
        grad_A = np.zeros(1)
        rc = self._lib.pdo_adjoint_ec(C.byref(self.P), _ptr(fr), int(nsteps), _ptr(u0), _ptr(v0),
                                      int(step0), int(sens.shape[0]), _ptr(sens), _ptr(g),
                                      _ptr(grad_k), _ptr(grad_A))
        if rc != 0:
            raise MemoryError("oracle adjoint: allocation failed")
        return grad_k[: self.nnz], float(grad_A[0])


def damage(sim: OracleSim) -> np.ndarray:
    return sim.damage()


def force(sim: OracleSim, u=None, k=None) -> np.ndarray:
    return sim.force(u, k)


def apply_jt(sim: OracleSim, frozen, u, k, nu) -> np.ndarray:
    return sim.apply_jt(frozen, u, k, nu)


def adjoint_ec(sim: OracleSim, *a, **kw):
    return sim.adjoint_ec(*a, **kw)


def from_workload(w, nthreads: int = 0, record_breaks: bool = False, method: str = "cells", frozen=None):
    """Oracle simulation of a pd_inputs.Workload (family built by the oracle itself);
    ``frozen``: an optional fixed break schedule (slot b acts in pass k iff k < frozen[b])."""
    from pd_inputs import notch_mask, gaussian_node_field, slot_stiffness
    row_ptr, col = family(w.coords, w.horizon, method)
    broken = None
    if w.notch is not None:
        broken = notch_mask(w.ijk, row_ptr, col, *w.notch)
    kslot = None
    if w.stiffness_field is not None:
        sig, ell, seed = w.stiffness_field
        kslot = slot_stiffness(w.c, gaussian_node_field(w.dims, sig, ell, seed), row_ptr, col)
    bhat, bmag = (None, 0.0) if w.body_force is None else w.body_force
    slot_cls = None
    if w.laws and w.class_spec is not None:
        from pd_inputs import bond_classes
        slot_cls = bond_classes(row_ptr, col, *w.class_spec)
    nofail = None
    if w.nofail is not None:
        nofail = np.zeros(w.n, dtype=np.uint8)
        nofail[w.nofail] = 1
    return OracleSim(w.coords, row_ptr, col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=w.volume,
                     scheme=w.scheme, eta=w.eta, kslot=kslot, bhat=bhat, bmag=bmag, bcs=w.bcs,
                     nthreads=nthreads, record_breaks=record_breaks, broken=broken,
                     ramp_T=1.0 if w.ramp_T is None else w.ramp_T, nofail=nofail, frozen=frozen,
                     laws=w.laws, slot_cls=slot_cls, corrections=w.corrections,
                     state_based=w.state_based)
