"""ctypes binding of libpdmi.so: the C ABI of include/pdmi.h, argument marshalling only.

Every function here has the name of the C entry point it wraps, converts NumPy arrays
to pointers, and raises ``PdmiError`` on a non-zero status.  All computation happens
in the library's HIP kernels; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdmi.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EHIP, PD_ESTATE, PD_ENONFINITE, PD_ERANGE = 0, -1, -2, -3, -4, -5, -6
PD_FP64, PD_FP32 = 0, 1
PD_ORDER_NATURAL, PD_ORDER_MORTON, PD_ORDER_AUTO = 0, 1, 2
PD_EULER_CROMER, PD_VELOCITY_VERLET, PD_EULER_FORWARD = 0, 1, 2
PD_BC_DISP, PD_BC_VEL = 1, 2
PD_SCHED_CONST, PD_SCHED_LINEAR, PD_SCHED_RAMP5 = 0, 1, 2
PD_MAP_SLICED, PD_MAP_STAGED = 0, 1
PD_MODEL_PMB, PD_MODEL_STATE_BASED = 0, 1

SYMBOLS = [
    "pd_create", "pd_destroy", "pd_last_error", "pd_build_family", "pd_build_family_batch", "pd_set_family",
    "pd_get_u_dev", "pd_get_v_dev", "pd_get_damage_dev",
    "pd_num_instances", "pd_instance_size", "pd_get_family", "pd_set_material", "pd_set_bond_stiffness",
    "pd_set_node_stiffness",
    "pd_break_bonds", "pd_set_bcs", "pd_clear_bcs", "pd_set_bc_ramp", "pd_set_no_fail", "pd_get_force",
    "pd_get_resultant", "pd_get_mean_displacement", "pd_set_damage_law", "pd_set_bond_classes",
    "pd_clear_damage_laws", "pd_get_max_stretch", "pd_set_max_stretch", "pd_set_corrections", "pd_set_model", "pd_get_dilation",
    "pd_set_body_force", "pd_set_integrator",
    "pd_step", "pd_prepare", "pd_sync", "pd_get_step", "pd_get_u", "pd_get_v", "pd_get_a", "pd_get_damage",
    "pd_get_broken", "pd_set_state", "pd_set_step", "pd_set_mapping", "pd_set_lanes_per_node", "pd_autotune",
    "pd_get_info", "pd_last_step_ms", "pd_adj_forward", "pd_adj_backward", "pd_get_break_steps",
    "pd_get_state", "pd_load_state", "pd_stretch_exact", "pd_get_mean_displacement_noalloc",
]


class PdmiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pdmi error {code}: {msg}")
        self.code = code


class pd_material(C.Structure):
    _fields_ = [("rho", C.c_double), ("c", C.c_double), ("s0", C.c_double), ("eta", C.c_double),
                ("volume", C.c_double), ("volumes", C.c_void_p)]


class pd_state(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("a", C.c_void_p), ("broken", C.c_void_p),
                ("break_step", C.c_void_p), ("max_stretch", C.c_void_p), ("step", C.c_int64),
                ("a_valid", C.c_int32), ("pad_", C.c_int32)]


class pd_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_slots", C.c_int64), ("n_nodes_dev", C.c_int64),
                ("n_slots_dev", C.c_int64), ("n_instances", C.c_int32), ("lanes_per_node", C.c_int32),
                ("precision", C.c_int32), ("scheme", C.c_int32), ("mapping", C.c_int32), ("order", C.c_int32),
                ("model_bytes_per_step", C.c_double), ("waves_per_slice", C.c_int32), ("reserved_", C.c_int32)]


_lib = None


def load() -> C.CDLL:
    """Load the built library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2105_04150_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pd_create": [P, C.c_int, C.c_int, P],
        "pd_destroy": [P],
        "pd_build_family": [P, i64, P, d, C.c_int],
        "pd_build_family_batch": [P, i32, P, P, P, C.c_int],
        "pd_num_instances": [P, P],
        "pd_instance_size": [P, i32, P, P],
        "pd_get_family": [P, i32, P, P, P],
        "pd_set_material": [P, i32, P],
        "pd_set_bond_stiffness": [P, i32, P],
        "pd_set_node_stiffness": [P, i32, P],
        "pd_break_bonds": [P, i32, P],
        "pd_set_bcs": [P, i32, i64, P, C.c_int, C.c_int, P, C.c_int],
        "pd_clear_bcs": [P, i32],
        "pd_set_bc_ramp": [P, i32, C.c_double],
        "pd_set_no_fail": [P, i32, i64, P],
        "pd_get_force": [P, i32, P],
        "pd_get_resultant": [P, i32, i64, P, P],
        "pd_get_mean_displacement": [P, i32, i64, P, P],
        "pd_get_mean_displacement_noalloc": [P, i32, i64, P, P],
        "pd_set_damage_law": [P, i32, i32, i32, P, P],
        "pd_set_bond_classes": [P, i32, P],
        "pd_clear_damage_laws": [P, i32],
        "pd_get_max_stretch": [P, i32, P],
        "pd_set_max_stretch": [P, i32, P],
        "pd_set_corrections": [P, i32, P],
        "pd_set_model": [P, i32, C.c_int, d, d],
        "pd_get_dilation": [P, i32, P],
        "pd_set_body_force": [P, i32, P, d],
        "pd_set_integrator": [P, C.c_int, d],
        "pd_step": [P, i64],
        "pd_prepare": [P],
        "pd_sync": [P],
        "pd_get_step": [P, P],
        "pd_get_u": [P, i32, P], "pd_get_v": [P, i32, P], "pd_get_a": [P, i32, P],
        "pd_get_damage": [P, i32, P],
        "pd_set_family": [P, i64, P, P, P, C.c_int],
        "pd_get_u_dev": [P, i32, P], "pd_get_v_dev": [P, i32, P], "pd_get_damage_dev": [P, i32, P],
        "pd_get_broken": [P, i32, P],
        "pd_set_state": [P, i32, P, P, P, P],
        "pd_set_step": [P, i64],
        "pd_set_mapping": [P, C.c_int, C.c_int],
        "pd_set_lanes_per_node": [P, C.c_int],
        "pd_autotune": [P, i64, P],
        "pd_get_info": [P, P],
        "pd_last_step_ms": [P, P],
        "pd_adj_forward": [P, i64, i32, P],
        "pd_adj_backward": [P, i64, i64, P, P, P, P],
        "pd_get_break_steps": [P, i32, P],
        "pd_get_state": [P, i32, P],
        "pd_load_state": [P, i32, P],
        "pd_stretch_exact": [C.c_int, i64, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.pd_last_error.argtypes = [P]
    lib.pd_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _f64(a, shape=None):
    if a is None:
        return None
    out = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and out.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} doubles, got {out.shape}")
    return out


def _check(ctx, rc: int):
    if rc != PD_OK:
        msg = load().pd_last_error(ctx)
        raise PdmiError(rc, (msg or b"").decode())


# ------------------------------------------------------------------ one function per entry point

def pd_create(device: int = 0, precision: int = PD_FP64, stream: Optional[int] = None) -> C.c_void_p:
    lib = load()
    h = C.c_void_p()
    rc = lib.pd_create(C.byref(h), int(device), int(precision), C.c_void_p(stream) if stream else None)
    if rc != PD_OK:
        raise PdmiError(rc, (lib.pd_last_error(None) or b"").decode())
    return h


def pd_destroy(ctx) -> None:
    load().pd_destroy(ctx)


def pd_build_family(ctx, coords, horizon: float, order: int = PD_ORDER_NATURAL) -> None:
    x = _f64(coords)
    _check(ctx, load().pd_build_family(ctx, x.shape[0], _p(x), float(horizon), int(order)))


def pd_build_family_batch(ctx, coords_list, horizons, order: int = PD_ORDER_NATURAL) -> None:
    xs = [_f64(x) for x in coords_list]
    n = np.array([x.shape[0] for x in xs], dtype=np.int64)
    ptrs = (C.c_void_p * len(xs))(*[x.ctypes.data for x in xs])
    h = _f64(horizons)
    _check(ctx, load().pd_build_family_batch(ctx, len(xs), _p(n), ptrs, _p(h), int(order)))


def pd_num_instances(ctx) -> int:
    v = C.c_int32()
    _check(ctx, load().pd_num_instances(ctx, C.byref(v)))
    return v.value


def pd_instance_size(ctx, inst: int = 0):
    n, nnz = C.c_int64(), C.c_int64()
    _check(ctx, load().pd_instance_size(ctx, inst, C.byref(n), C.byref(nnz)))
    return n.value, nnz.value


def pd_get_family(ctx, inst: int = 0):
    n, nnz = pd_instance_size(ctx, inst)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    _check(ctx, load().pd_get_family(ctx, inst, _p(row_ptr), _p(col), None))
    return row_ptr, col[:nnz]


def _inst_n(ctx, inst: int) -> int:
    return pd_instance_size(ctx, inst)[0]


def pd_set_material(ctx, inst: int, rho: float, c: float, s0: float, eta: float = 0.0,
                    volume: float = 1.0, volumes=None) -> None:
    vols = _f64(volumes)
    m = pd_material(float(rho), float(c), float(s0), float(eta), float(volume),
                    None if vols is None else vols.ctypes.data)
    _check(ctx, load().pd_set_material(ctx, inst, C.byref(m)))


def pd_set_bond_stiffness(ctx, inst: int, k) -> None:
    kk = _f64(k)
    _check(ctx, load().pd_set_bond_stiffness(ctx, inst, _p(kk)))


def pd_set_node_stiffness(ctx, inst: int, k_node) -> None:
    kk = _f64(k_node)
    _check(ctx, load().pd_set_node_stiffness(ctx, inst, _p(kk)))


def pd_break_bonds(ctx, inst: int, broken) -> None:
    b = np.ascontiguousarray(broken, dtype=np.uint8)
    _check(ctx, load().pd_break_bonds(ctx, inst, _p(b)))


def pd_set_bcs(ctx, inst: int, nodes, comp_mask: int, kind: int, value, sched: int) -> None:
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    val = _f64(value, (3,))
    _check(ctx, load().pd_set_bcs(ctx, inst, nd.shape[0], _p(nd), int(comp_mask), int(kind), _p(val),
                                  int(sched)))


def pd_clear_bcs(ctx, inst: int = 0) -> None:
    _check(ctx, load().pd_clear_bcs(ctx, inst))


def pd_set_bc_ramp(ctx, inst: int, ramp_time: float) -> None:
    _check(ctx, load().pd_set_bc_ramp(ctx, inst, float(ramp_time)))


def pd_set_no_fail(ctx, inst: int, nodes) -> None:
    nd = np.ascontiguousarray(np.zeros(0) if nodes is None else nodes, dtype=np.int64)
    _check(ctx, load().pd_set_no_fail(ctx, inst, nd.shape[0], _p(nd) if nd.shape[0] else None))


def pd_get_force(ctx, inst: int = 0) -> np.ndarray:
    return _get3(load().pd_get_force, ctx, inst)


def pd_get_resultant(ctx, inst: int, nodes) -> np.ndarray:
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros(3)
    _check(ctx, load().pd_get_resultant(ctx, inst, nd.shape[0], _p(nd) if nd.shape[0] else None, _p(out)))
    return out


def pd_get_mean_displacement(ctx, inst: int, nodes) -> np.ndarray:
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros(3)
    _check(ctx, load().pd_get_mean_displacement(ctx, inst, nd.shape[0], _p(nd) if nd.shape[0] else None, _p(out)))
    return out


def pd_get_mean_displacement_noalloc(ctx, inst: int, nodes) -> np.ndarray:
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros(3)
    _check(ctx, load().pd_get_mean_displacement_noalloc(ctx, inst, nd.shape[0], _p(nd) if nd.shape[0] else None,
                                                        _p(out)))
    return out


def pd_set_damage_law(ctx, inst: int, cls: int, s_break, ratio) -> None:
    sb = np.ascontiguousarray(s_break, dtype=np.float64).ravel()
    rb = np.ascontiguousarray(ratio, dtype=np.float64).ravel()
    if sb.shape != rb.shape:
        raise ValueError("s_break and ratio need the same length")
    _check(ctx, load().pd_set_damage_law(ctx, inst, int(cls), sb.shape[0], _p(sb), _p(rb)))


def pd_set_bond_classes(ctx, inst: int, cls) -> None:
    if cls is None:
        _check(ctx, load().pd_set_bond_classes(ctx, inst, None))
        return
    nnz = pd_instance_size(ctx, inst)[1]
    c = np.ascontiguousarray(cls, dtype=np.uint8)
    if c.shape != (nnz,):
        raise ValueError(f"bond classes need shape ({nnz},)")
    _check(ctx, load().pd_set_bond_classes(ctx, inst, _p(c)))


def pd_clear_damage_laws(ctx, inst: int = 0) -> None:
    _check(ctx, load().pd_clear_damage_laws(ctx, inst))


def pd_get_max_stretch(ctx, inst: int = 0) -> np.ndarray:
    nnz = pd_instance_size(ctx, inst)[1]
    out = np.zeros(max(nnz, 1))
    _check(ctx, load().pd_get_max_stretch(ctx, inst, _p(out)))
    return out[:nnz]


def pd_set_max_stretch(ctx, inst: int, smax) -> None:
    nnz = pd_instance_size(ctx, inst)[1]
    sm = np.ascontiguousarray(smax, dtype=np.float64)
    if sm.shape != (nnz,):
        raise ValueError(f"stretch state needs shape ({nnz},)")
    _check(ctx, load().pd_set_max_stretch(ctx, inst, _p(sm)))


PD_MICRO_CONSTANT, PD_MICRO_CONICAL = 0, 1


class pd_corrections(C.Structure):
    _fields_ = [("micromodulus", C.c_int32), ("partial_volumes", C.c_int32), ("surface", C.c_int32),
                ("reserved_", C.c_int32), ("delta", C.c_double), ("dx", C.c_double)]


def pd_set_corrections(ctx, inst: int, micro: str = "constant", partial_volumes: bool = False,
                       surface: bool = False, delta: float = 0.0, dx: float = 0.0, clear: bool = False) -> None:
    if clear:
        _check(ctx, load().pd_set_corrections(ctx, inst, None))
        return
    kinds = {"constant": PD_MICRO_CONSTANT, "conical": PD_MICRO_CONICAL}
    if micro not in kinds:
        raise ValueError(f"unknown micromodulus profile {micro!r}")
    c = pd_corrections(kinds[micro], int(bool(partial_volumes)), int(bool(surface)), 0, float(delta), float(dx))
    _check(ctx, load().pd_set_corrections(ctx, inst, C.byref(c)))


def pd_set_body_force(ctx, inst: int, b_hat, magnitude: float) -> None:
    b = _f64(b_hat)
    _check(ctx, load().pd_set_body_force(ctx, inst, _p(b), float(magnitude)))


def pd_set_integrator(ctx, scheme: int, dt: float) -> None:
    _check(ctx, load().pd_set_integrator(ctx, int(scheme), float(dt)))


def pd_step(ctx, nsteps: int) -> None:
    _check(ctx, load().pd_step(ctx, int(nsteps)))


def pd_prepare(ctx) -> None:
    _check(ctx, load().pd_prepare(ctx))


def pd_sync(ctx) -> None:
    _check(ctx, load().pd_sync(ctx))


def pd_get_step(ctx) -> int:
    v = C.c_int64()
    _check(ctx, load().pd_get_step(ctx, C.byref(v)))
    return v.value


def _get3(fn, ctx, inst):
    out = np.zeros((_inst_n(ctx, inst), 3))
    _check(ctx, fn(ctx, inst, _p(out)))
    return out


def pd_get_u(ctx, inst: int = 0) -> np.ndarray:
    return _get3(load().pd_get_u, ctx, inst)


def pd_get_v(ctx, inst: int = 0) -> np.ndarray:
    return _get3(load().pd_get_v, ctx, inst)


def pd_get_a(ctx, inst: int = 0) -> np.ndarray:
    return _get3(load().pd_get_a, ctx, inst)


def pd_set_model(ctx, inst: int, model: str, K: float = 0.0, G: float = 0.0) -> None:
    code = {"pmb": PD_MODEL_PMB, "state_based": PD_MODEL_STATE_BASED}.get(model)
    if code is None:
        raise ValueError(f"unknown model {model!r}")
    _check(ctx, load().pd_set_model(ctx, inst, code, float(K), float(G)))


def pd_get_dilation(ctx, inst: int = 0) -> np.ndarray:
    out = np.zeros(_inst_n(ctx, inst))
    _check(ctx, load().pd_get_dilation(ctx, inst, _p(out)))
    return out


def pd_set_family(ctx, coords, row_ptr, col, order: int = 0) -> None:
    x = _f64(coords)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if x.ndim != 2 or x.shape[1] != 3 or rp.shape != (x.shape[0] + 1,):
        raise ValueError("coords must be n x 3 and row_ptr n + 1 long")
    if cl.shape[0] < rp[-1]:
        raise ValueError("col is shorter than row_ptr[n]")
    _check(ctx, load().pd_set_family(ctx, x.shape[0], _p(x), _p(rp), _p(cl), int(order)))


def _dev_out(out, n: int, ncomp: int) -> int:
    """Device pointer of a contiguous float64 CUDA tensor of at least n * ncomp values."""
    import torch
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64 \
            or not out.is_contiguous() or out.numel() < n * ncomp:
        raise ValueError(f"out must be a contiguous float64 CUDA tensor of >= {n * ncomp} values")
    return out.data_ptr()


def pd_get_u_dev(ctx, inst: int, out) -> None:
    _check(ctx, load().pd_get_u_dev(ctx, inst, C.c_void_p(_dev_out(out, _inst_n(ctx, inst), 3))))


def pd_get_v_dev(ctx, inst: int, out) -> None:
    _check(ctx, load().pd_get_v_dev(ctx, inst, C.c_void_p(_dev_out(out, _inst_n(ctx, inst), 3))))


def pd_get_damage_dev(ctx, inst: int, out) -> None:
    _check(ctx, load().pd_get_damage_dev(ctx, inst, C.c_void_p(_dev_out(out, _inst_n(ctx, inst), 1))))


def pd_get_damage(ctx, inst: int = 0) -> np.ndarray:
    out = np.zeros(_inst_n(ctx, inst))
    _check(ctx, load().pd_get_damage(ctx, inst, _p(out)))
    return out


def pd_get_broken(ctx, inst: int = 0) -> np.ndarray:
    nnz = pd_instance_size(ctx, inst)[1]
    out = np.zeros(max(nnz, 1), dtype=np.uint8)
    _check(ctx, load().pd_get_broken(ctx, inst, _p(out)))
    return out[:nnz]


def pd_set_state(ctx, inst: int = 0, u=None, v=None, a=None, broken=None) -> None:
    uu, vv, aa = _f64(u), _f64(v), _f64(a)
    bb = None if broken is None else np.ascontiguousarray(broken, dtype=np.uint8)
    _check(ctx, load().pd_set_state(ctx, inst, _p(uu), _p(vv), _p(aa), _p(bb)))


def pd_set_step(ctx, step: int) -> None:
    _check(ctx, load().pd_set_step(ctx, int(step)))


def pd_set_mapping(ctx, mapping: int, lanes: int = 0) -> None:
    _check(ctx, load().pd_set_mapping(ctx, int(mapping), int(lanes)))


def pd_set_lanes_per_node(ctx, lanes: int) -> None:
    _check(ctx, load().pd_set_lanes_per_node(ctx, int(lanes)))


def pd_autotune(ctx, trial_steps: int) -> int:
    v = C.c_int32()
    _check(ctx, load().pd_autotune(ctx, int(trial_steps), C.byref(v)))
    return v.value


def pd_get_info(ctx) -> dict:
    info = pd_info()
    _check(ctx, load().pd_get_info(ctx, C.byref(info)))
    return {k: getattr(info, k) for k, _ in pd_info._fields_}


def pd_last_step_ms(ctx) -> float:
    v = C.c_double()
    _check(ctx, load().pd_last_step_ms(ctx, C.byref(v)))
    return v.value


def pd_adj_forward(ctx, nsteps: int, ckpt_every: int) -> int:
    """Returns the id of the recording."""
    rec = C.c_int64()
    _check(ctx, load().pd_adj_forward(ctx, int(nsteps), int(ckpt_every), C.byref(rec)))
    return rec.value


def pd_adj_backward(ctx, sensors, dL_du, recording: int = 0):
    """Returns (grad_k[nnz], grad_A) for dL/du^T given at the sensor nodes (m x 3) of the
    recording `recording` (0: the current one)."""
    sn = np.ascontiguousarray(sensors, dtype=np.int64).reshape(-1)
    dl = _f64(dL_du, (sn.shape[0], 3))
    nnz = pd_instance_size(ctx, 0)[1]
    gk = np.zeros(max(nnz, 1))
    gA = C.c_double()
    _check(ctx, load().pd_adj_backward(ctx, int(recording), sn.shape[0], _p(sn), _p(dl), _p(gk), C.byref(gA)))
    return gk[:nnz], gA.value


def pd_get_state(ctx, inst: int = 0) -> dict:
    """The whole state of an instance: u, v, a, broken, break_step, max_stretch (arrays
    in user order), step and a_valid."""
    n, nnz = pd_instance_size(ctx, inst)
    arr = {"u": np.zeros((n, 3)), "v": np.zeros((n, 3)), "a": np.zeros((n, 3)),
           "broken": np.zeros(max(nnz, 1), dtype=np.uint8), "break_step": np.zeros(max(nnz, 1), dtype=np.int32),
           "max_stretch": np.zeros(max(nnz, 1))}
    st = pd_state(*(_p(arr[k]) for k in ("u", "v", "a", "broken", "break_step", "max_stretch")), 0, 0, 0)
    _check(ctx, load().pd_get_state(ctx, inst, C.byref(st)))
    for k in ("broken", "break_step", "max_stretch"):
        arr[k] = arr[k][:nnz]
    arr["step"], arr["a_valid"] = int(st.step), int(st.a_valid)
    return arr


def pd_load_state(ctx, inst: int, state: dict) -> None:
    """Restore a state as pd_get_state returns it (missing or None entries are kept)."""
    def get(k, dt):
        v = state.get(k)
        return None if v is None else np.ascontiguousarray(v, dtype=dt)
    u, v, a = get("u", np.float64), get("v", np.float64), get("a", np.float64)
    br, bs, sm = get("broken", np.uint8), get("break_step", np.int32), get("max_stretch", np.float64)
    st = pd_state(_p(u), _p(v), _p(a), _p(br), _p(bs), _p(sm), int(state.get("step", 0)),
                  int(state.get("a_valid", 0)), 0)
    _check(ctx, load().pd_load_state(ctx, inst, C.byref(st)))


def pd_stretch_exact(xi, y, device: int = 0) -> np.ndarray:
    """The device's exact stretch (m bonds; xi, y m x 3)."""
    xx = _f64(xi).reshape(-1, 3)
    yy = _f64(y, xx.shape)
    s = np.zeros(max(xx.shape[0], 1))
    rc = load().pd_stretch_exact(int(device), xx.shape[0], _p(xx), _p(yy), _p(s))
    if rc != PD_OK:
        raise PdmiError(rc, "pd_stretch_exact failed")
    return s[: xx.shape[0]]


def pd_get_break_steps(ctx, inst: int = 0) -> np.ndarray:
    nnz = pd_instance_size(ctx, inst)[1]
    out = np.zeros(max(nnz, 1), dtype=np.int32)
    _check(ctx, load().pd_get_break_steps(ctx, inst, _p(out)))
    return out[:nnz]
