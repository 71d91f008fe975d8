"""Seeded synthetic inputs for the peridynamics workloads.

This module is shared by the FP64 CPU oracle (``oracle/``), the HIP library's tests
and the benchmark.  It generates *inputs only*: lattice coordinates, node sets for
boundary conditions, the notch's pre-broken bond mask, random stiffness fields,
sensor sets and the per-workload parameter sets.  It performs none of the time
step's arithmetic (no stretch, force, reduction, integration or damage).

Random numbers come from one counter-based generator, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), so every
draw is a pure function of (seed, counter) and identical on every machine.

Workloads follow the paper's benchmark setting (Section 4: beams on a regular
cubic tensor grid, constant micromodulus, simple displacement / velocity control)
with sizes chosen per workload; each workload's recipe is stated in workload() below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "splitmix64", "uniform01", "normal",
    "lattice", "lattice_index", "face_nodes", "pmb_micromodulus",
    "BC_DISP", "BC_VEL", "SCHED_CONST", "SCHED_LINEAR", "SCHED_RAMP5", "BCSpec",
    "notch_mask", "gaussian_node_field", "slot_stiffness", "sample_nodes",
    "Workload", "workload", "WORKLOADS", "batch_instances",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters) -> np.ndarray:
    """SplitMix64 output for each counter: mix(seed + (counter + 1) * golden)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of SplitMix64 times 2^-53."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normal draws by the Box-Muller transform on pairs of uniforms."""
    m = (count + 1) // 2
    u1 = uniform01(seed, np.arange(0, 2 * m, 2, dtype=np.uint64))
    u2 = uniform01(seed, np.arange(1, 2 * m, 2, dtype=np.uint64))
    rad = np.sqrt(-2.0 * np.log1p(-u1))          # 1 - u1 in (0, 1]
    z = np.empty(2 * m)
    z[0::2] = rad * np.cos(2.0 * math.pi * u2)
    z[1::2] = rad * np.sin(2.0 * math.pi * u2)
    return z[:count]


# --------------------------------------------------------------------------- lattices

def lattice_index(dims: Sequence[int]) -> np.ndarray:
    """Integer lattice coordinates (n, 3) in natural order (x fastest, then y, then z)."""
    lx, ly, lz = (int(d) for d in dims)
    iz, iy, ix = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.int64)


def lattice(dims: Sequence[int], dx: float, jitter: float = 0.0, seed: int = 0,
            origin: Sequence[float] = (0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Simple-cubic lattice nodes with optional iid uniform jitter.

    Returns ``(coords, ijk)``: coords (n, 3) float64 in metres, ijk (n, 3) int64.
    Each coordinate is ``origin + i*dx + jitter*dx*(2U - 1)`` with U = uniform01(seed,
    3*node + axis), i.e. jitter is a fraction of dx.  Node volumes are dx^3 whatever
    the jitter (the tensor-grid volume of the paper's regular meshes).
    """
    ijk = lattice_index(dims)
    x = ijk.astype(np.float64) * dx + np.asarray(origin, dtype=np.float64)
    if jitter:
        n = ijk.shape[0]
        u = uniform01(seed, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
        x = x + (jitter * dx) * (2.0 * u - 1.0)
    return np.ascontiguousarray(x), ijk


def face_nodes(ijk: np.ndarray, axis: int, value: int) -> np.ndarray:
    """Indices of nodes whose lattice coordinate along ``axis`` equals ``value``."""
    return np.nonzero(ijk[:, axis] == value)[0].astype(np.int64)


def pmb_micromodulus(bulk_modulus: float, horizon: float) -> float:
    """Constant PMB micromodulus c = 18 K / (pi delta^4) (Eq. simpleBond)."""
    return 18.0 * bulk_modulus / (math.pi * horizon ** 4)


# --------------------------------------------------------------------------- boundary conditions

BC_DISP = 1      # prescribed displacement u_c = A_c g(t), velocity A_c g'(t)
BC_VEL = 2       # prescribed velocity v_c = A_c g(t), displacement advanced by dt * v_c
SCHED_CONST = 0  # g(t) = 1, g'(t) = 0
SCHED_LINEAR = 1  # g(t) = t, g'(t) = 1
SCHED_RAMP5 = 2  # fifth-order ramp from 0 to 1 over a ramp time T, then 1


@dataclass
class BCSpec:
    """One boundary-condition call: the same constraint on a set of nodes."""
    nodes: np.ndarray           # int64 node ids (user order)
    comp_mask: int              # bit d set => component d constrained
    kind: int                   # BC_DISP or BC_VEL
    value: Tuple[float, float, float]
    sched: int                  # SCHED_CONST, SCHED_LINEAR or SCHED_RAMP5


# --------------------------------------------------------------------------- notch, fields, sensors

def notch_mask(ijk: np.ndarray, row_ptr: np.ndarray, col: np.ndarray,
               plane2: int, height2: int) -> np.ndarray:
    """Per-slot mask of bonds cut by a notch, in exact integer arithmetic.

    The notch is the vertical plane x = plane2/2 (lattice units, plane2 odd so no
    node lies on it) from the bottom up to height z = height2/2.  A bond (i, j)
    is cut when its endpoints lie on opposite sides of the plane and the straight
    segment crosses it strictly below the notch top.
    """
    n = ijk.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    cols = col.astype(np.int64)
    xi, zi = ijk[rows, 0], ijk[rows, 2]
    xj, zj = ijk[cols, 0], ijk[cols, 2]
    side_i = 2 * xi - plane2
    side_j = 2 * xj - plane2
    crosses = (side_i * side_j) < 0
    d = 2 * (xj - xi)                              # != 0 where crosses
    # 2*z_c*d = 2*z_i*d + 2*(z_j - z_i)*(plane2 - 2*x_i); test z_c < height2/2
    lhs = 2 * zi * d + 2 * (zj - zi) * (plane2 - 2 * xi) - height2 * d
    below = np.where(d > 0, lhs < 0, lhs > 0)
    return (crosses & below).astype(np.uint8)


def bond_classes(row_ptr: np.ndarray, col: np.ndarray, fractions: Sequence[float], seed: int) -> np.ndarray:
    """Per-slot bond class drawn at random with the given class fractions, the same for
    both slots of a bond (a SplitMix64 uniform keyed on the unordered pair).  Returns
    uint8 in CSR order."""
    n = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr)).astype(np.uint64)
    cols = np.asarray(col, dtype=np.int64).astype(np.uint64)
    key = np.minimum(rows, cols) * np.uint64(n) + np.maximum(rows, cols)
    u = uniform01(seed, key)
    edges = np.cumsum(np.asarray(fractions, dtype=np.float64))[:-1]
    return np.searchsorted(edges, u, side="right").astype(np.uint8)


# Damage laws as (stretch breakpoints, force ratios).  The trilinear law uses the
# calibrated point estimate 1 of the trilinear parameters (Sec. 6, table of optimised
# parameters: s0 = 2.3e-4, s1 = 2.42e-4, sc = 1.45e-3) with the kink ratio 1/4; the
# fibre law of the composite variant is a bilinear law twice as strong in stretch.
LAW_TRILINEAR = ((2.3e-4, 2.42e-4, 1.45e-3), (1.0, 0.25, 0.0))
LAW_FIBRE = ((4.6e-4, 2.9e-3), (1.0, 0.0))


def _gauss_kernel(std: float) -> np.ndarray:
    r = int(math.ceil(4.0 * std))
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / std) ** 2)
    return w / w.sum()


def gaussian_node_field(dims: Sequence[int], sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """Correlated Gaussian field on the lattice, flattened in natural node order.

    White noise convolved (zero padding) with a separable Gaussian of standard
    deviation corr_len/sqrt(2) (lattice units) has covariance proportional to
    exp(-r^2 / (2 corr_len^2)); it is scaled by the interior standard deviation so
    the field has variance sigma^2 away from the faces.
    """
    lx, ly, lz = (int(d) for d in dims)
    w = normal(seed, lx * ly * lz).reshape(lz, ly, lx)
    k = _gauss_kernel(corr_len / math.sqrt(2.0))
    r = (k.shape[0] - 1) // 2

    def conv(a):  # zero-padded convolution cropped to the input length
        return np.convolve(a, k, mode="full")[r:r + a.shape[0]]

    for ax in range(3):
        w = np.apply_along_axis(conv, ax, w)
    scale = math.sqrt(float(np.sum(k * k)) ** 3)
    return (sigma / scale) * w.ravel()


def slot_stiffness(c: float, g: np.ndarray, row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Per-slot stiffness c * exp((g_i + g_j) / 2); symmetric in (i, j)."""
    n = g.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    return c * np.exp(0.5 * (g[rows] + g[col.astype(np.int64)]))


def sample_nodes(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct node ids drawn without replacement (sorted by a random key)."""
    keys = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return np.sort(np.argsort(keys, kind="stable")[:m].astype(np.int64))


# --------------------------------------------------------------------------- workloads

@dataclass
class Workload:
    """A fully specified synthetic problem (inputs only; no results)."""
    name: str
    dims: Tuple[int, int, int]
    dx: float
    horizon: float
    c: float
    rho: float
    s0: float
    dt: float
    steps: int
    scheme: str                     # "euler_cromer" | "velocity_verlet"
    coords: np.ndarray
    ijk: np.ndarray
    volume: float
    bcs: List[BCSpec]
    order: str = "natural"          # node order hint for the GPU layout
    notch: Optional[Tuple[int, int]] = None   # (plane2, height2) or None
    body_force: Optional[Tuple[np.ndarray, float]] = None   # (b_hat (n,3), magnitude)
    stiffness_field: Optional[Tuple[float, float, int]] = None  # (sigma, corr_len, seed)
    eta: float = 0.0                # dynamic-relaxation damping coefficient (kg/(m^3 s))
    ramp_T: Optional[float] = None  # duration of the SCHED_RAMP5 components
    nofail: Optional[np.ndarray] = None  # node ids of the no-failure zones
    laws: Optional[List[Tuple[Tuple[float, ...], Tuple[float, ...]]]] = None  # damage law per bond class
    class_spec: Optional[Tuple[Tuple[float, ...], int]] = None  # (class fractions, seed) for bond_classes
    corrections: Optional[Dict] = None  # stiffness corrections: micro, partial_volumes, surface, delta, dx
    state_based: Optional[Tuple[float, float]] = None  # (K, G): the state-based linear solid
    meta: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])


K_CONCRETE = 1.4e10     # bulk modulus used by every workload (Pa)
RHO = 2400.0            # density (kg/m^3)
DX = 1.0e-3             # lattice spacing (m)
JITTER = 1.0e-3         # jitter amplitude as a fraction of dx
JITTER_SEED = 1234


def _mk(name, dims, m, s0, steps, scheme, bcs_fn, order="natural", notch=None,
        body=None, fld=None, dx=DX, jitter=JITTER, seed=JITTER_SEED, dt=1.0e-7, meta=None):
    coords, ijk = lattice(dims, dx, jitter, seed)
    delta = m * dx
    w = Workload(name=name, dims=tuple(dims), dx=dx, horizon=delta,
                 c=pmb_micromodulus(K_CONCRETE, delta), rho=RHO, s0=s0, dt=dt, steps=steps,
                 scheme=scheme, coords=coords, ijk=ijk, volume=dx ** 3, bcs=[], order=order,
                 notch=notch, stiffness_field=fld, meta=dict(meta or {}))
    w.bcs = bcs_fn(ijk, dims)
    if body is not None:
        w.body_force = body(ijk, dims)
    return w


def _bcs_block(ijk, dims):
    # bottom layer clamped; top layer pulled in +z at 1e-8 m per step (0.1 m/s)
    top = dims[2] - 1
    return [BCSpec(face_nodes(ijk, 2, 0), 0b111, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(face_nodes(ijk, 2, top), 0b100, BC_DISP, (0.0, 0.0, 0.1), SCHED_LINEAR)]


def _bcs_beam3pb(ijk, dims):
    lx = dims[0]
    sup_a = np.nonzero((ijk[:, 0] == 10) & (ijk[:, 2] == 0))[0]
    sup_b = np.nonzero((ijk[:, 0] == lx - 11) & (ijk[:, 2] == 0))[0]
    mid = lx // 2
    load = np.nonzero(((ijk[:, 0] == mid - 1) | (ijk[:, 0] == mid)) & (ijk[:, 2] == dims[2] - 1))[0]
    return [BCSpec(np.concatenate([sup_a, sup_b]).astype(np.int64), 0b111, BC_DISP,
                   (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(load.astype(np.int64), 0b100, BC_VEL, (0.0, 0.0, -1.0e-3), SCHED_CONST)]


def qs_beam_sets(ijk, dims):
    """Support and load node sets of the three-point bend of Sec. 6 (span 125/175 of the
    length): 2 x 2 node cross-sections (x by z) through the thickness at the supports,
    3 x 2 at the central load."""
    mid, top = dims[0] // 2, dims[2] - 1
    half = int(round(dims[0] * 125.0 / 175.0 / 2.0))

    def box(x0, x1, z0, z1):
        return np.nonzero((ijk[:, 0] >= x0) & (ijk[:, 0] <= x1) & (ijk[:, 2] >= z0) & (ijk[:, 2] <= z1))[0]
    left = box(mid - half - 1, mid - half, 0, 1)
    right = box(mid + half, mid + half + 1, 0, 1)
    load = box(mid - 1, mid + 1, top - 1, top)
    return left.astype(np.int64), right.astype(np.int64), load.astype(np.int64)


def _bcs_qs_beam(ijk, dims, amp):
    # left support clamped, right support held in y and z, the load held in y and pushed
    # down in z by the fifth-order ramp to amplitude amp
    left, right, load = qs_beam_sets(ijk, dims)
    return [BCSpec(left, 0b111, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(right, 0b110, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(load, 0b010, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(load, 0b100, BC_DISP, (0.0, 0.0, -amp), SCHED_RAMP5)]


def _bcs_tension_x(ijk, dims):
    return [BCSpec(face_nodes(ijk, 0, 0), 0b111, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST),
            BCSpec(face_nodes(ijk, 0, dims[0] - 1), 0b001, BC_DISP, (0.1, 0.0, 0.0), SCHED_LINEAR)]


def _body_tip_down(ijk, dims):
    bhat = np.zeros((ijk.shape[0], 3))
    bhat[ijk[:, 0] == dims[0] - 1, 2] = -1.0
    return bhat, ADJOINT_LOAD


ADJOINT_LOAD = 5.0e8      # body-force density magnitude on the loaded face (N/m^3)


def shear_modulus(K: float, poisson: float) -> float:
    """Isotropic shear modulus from the bulk modulus and Poisson's ratio."""
    return 3.0 * K * (1.0 - 2.0 * poisson) / (2.0 * (1.0 + poisson))


POISSON_CONCRETE = 0.2   # Poisson's ratio of the state-based workloads (the PMB fixes 1/4)


def workload(name: str, **over) -> Workload:
    """Build one named workload.  Keyword overrides replace dims/steps for scaled-down tests;
    model="state_based" swaps the PMB bond force for the state-based linear solid with the
    same bulk modulus and Poisson's ratio ``poisson`` (default 0.2)."""
    model = over.pop("model", "pmb")
    poisson = over.pop("poisson", POISSON_CONCRETE)
    w = _workload(name, **over)
    if model == "state_based":
        w.state_based = (K_CONCRETE, shear_modulus(K_CONCRETE, poisson))
    elif model != "pmb":
        raise KeyError(model)
    return w


def _workload(name: str, **over) -> Workload:
    if name == "block10":
        dims = over.get("dims", (10, 10, 10))
        return _mk(name, dims, 3.015, 1.0e-3, over.get("steps", 1000), "euler_cromer", _bcs_block)
    if name == "beam3pb":
        dims = over.get("dims", (200, 25, 25))
        plane2 = dims[0] - 1                      # mid-span plane between the two middle layers
        return _mk(name, dims, 3.015, 5.0e-4, over.get("steps", 10000), "velocity_verlet",
                   _bcs_beam3pb, notch=(plane2, 9))
    if name in ("cube100", "cube100_wide"):
        dims = over.get("dims", (100, 100, 100))
        m = 3.015 if name == "cube100" else 5.015
        return _mk(name, dims, m, 1.0e-3, over.get("steps", 2000), "euler_cromer", _bcs_block,
                   order="morton")
    if name == "adjoint_beam":
        dims = over.get("dims", (100, 25, 20))
        return _mk(name, dims, 3.015, 1.0e-3, over.get("steps", 2000), "euler_cromer",
                   _bcs_tension_x_clamp_only, body=_body_tip_down,
                   fld=(0.2, 5.0, 2000), meta={"sensor_seed": 7, "n_sensors": 200,
                                               "target_seed": 2001, "ckpt_every": 100})
    if name == "qs_beam":
        # displacement-controlled three-point bend of a notched beam with the quasi-static
        # toolkit of Secs. 6-7: the Example 2 geometry (175 x 50 x 50 mm, notch 1/5 of the
        # depth) on a 1 mm lattice, fifth-order ramp, no-failure zones on the support and
        # load nodes, dynamic-relaxation damping, velocity Verlet
        dims = over.get("dims", (175, 50, 50))
        steps = over.get("steps", 4000)
        law = over.get("law", "brittle")
        # same bending strain at any scale; three times more with the softening laws,
        # whose bonds break at a larger stretch
        amp = over.get("amp", (1.15e-7 if law == "brittle" else 3.45e-7) * dims[0])
        ramp_T = over.get("ramp_T", 0.75 * steps * 1.0e-7)
        w = _mk(name, dims, 3.14, over.get("s0", 1.0e-4), steps, "velocity_verlet",
                lambda ijk, d: _bcs_qs_beam(ijk, d, amp), notch=(2 * (dims[0] // 2) + 1, 2 * (dims[2] // 5)))
        w.eta = over.get("eta", 2.5e6)
        w.ramp_T = ramp_T
        w.nofail = np.unique(np.concatenate(qs_beam_sets(w.ijk, dims)))
        if law == "trilinear":
            w.laws = [LAW_TRILINEAR]
        elif law == "composite":
            # matrix (70%, trilinear) and fibre (30%, bilinear) bonds mixed at random
            w.laws = [LAW_TRILINEAR, LAW_FIBRE]
            w.class_spec = ((0.7, 0.3), 4242)
        elif law != "brittle":
            raise KeyError(law)
        return w
    raise KeyError(name)


def _bcs_tension_x_clamp_only(ijk, dims):
    return [BCSpec(face_nodes(ijk, 0, 0), 0b111, BC_DISP, (0.0, 0.0, 0.0), SCHED_CONST)]


WORKLOADS = ("block10", "beam3pb", "cube100", "cube100_wide", "adjoint_beam", "qs_beam")


def adjoint_sensors(w: Workload, m: Optional[int] = None, seed: Optional[int] = None):
    """Sensor node ids and target displacements of the misfit loss.

    m distinct nodes (default: the workload's n_sensors, at most n) drawn with the
    sensor seed; targets are 1e-5 m times seeded standard normals (target seed).
    """
    m = min(w.n, m if m is not None else int(w.meta.get("n_sensors", 200)))
    sensors = sample_nodes(w.n, m, int(w.meta.get("sensor_seed", 7)) if seed is None else seed)
    target = 1.0e-5 * normal(int(w.meta.get("target_seed", 2001)), 3 * m).reshape(m, 3)
    return sensors, target


def batch_instances(count: int = 64, scale_lo: float = 1.0, scale_hi: float = 3.0,
                    base=(80, 10, 10), steps: int = 5000) -> List[Workload]:
    """Uneven-size beams for the batched uncertainty-quantification sweep.

    Instance b has dims round(base * a_b) with a_b evenly spaced in [scale_lo,
    scale_hi], a seeded log-normal stiffness field (sigma 0.2, correlation length
    5 dx, seed 1000 + b) and a critical stretch drawn from U(4e-4, 6e-4) (seed 3000).
    """
    a = np.linspace(scale_lo, scale_hi, count) if count > 1 else np.array([scale_lo])
    s0 = 4.0e-4 + 2.0e-4 * uniform01(3000, np.arange(count, dtype=np.uint64))
    out = []
    for b in range(count):
        dims = tuple(int(round(base[d] * a[b])) for d in range(3))
        w = _mk(f"beam_uq_{b}", dims, 3.015, float(s0[b]), steps, "euler_cromer", _bcs_tension_x,
                fld=(0.2, 5.0, 1000 + b), seed=JITTER_SEED + b)
        out.append(w)
    return out
