"""MI355X-native bond-based PMB peridynamics (HIP kernels behind a C ABI).

``_binding`` exposes every C entry point of ``include/pdmi.h`` under its own name;
``Simulation`` is a small owner of one context.  Importing the package does not need
a GPU; creating a context does, and fails loudly if ``libpdmi.so`` is missing.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import _binding as B
from ._binding import (PD_BC_DISP, PD_BC_VEL, PD_EULER_CROMER, PD_EULER_FORWARD, PD_FP32,  # noqa: F401
                       PD_FP64, PD_MAP_SLICED, PD_MAP_STAGED, PD_ORDER_MORTON, PD_ORDER_NATURAL,
                       PD_SCHED_CONST, PD_SCHED_LINEAR, PD_SCHED_RAMP5, PD_VELOCITY_VERLET, PdmiError)

SCHEMES = {"euler_cromer": PD_EULER_CROMER, "velocity_verlet": PD_VELOCITY_VERLET,
           "forward_euler": PD_EULER_FORWARD}
ORDERS = {"natural": PD_ORDER_NATURAL, "morton": PD_ORDER_MORTON, "auto": B.PD_ORDER_AUTO}


class Simulation:
    """Owns one library context (one HIP stream, one or more instances)."""

    def __init__(self, device: int = 0, precision: int = PD_FP64, stream: Optional[int] = None):
        self.ctx = B.pd_create(device, precision, stream)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            B.pd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # setup
    def build_family(self, coords, horizon, order="natural"):
        B.pd_build_family(self.ctx, coords, horizon, ORDERS.get(order, order))

    def set_family(self, coords, row_ptr, col, order="natural"):
        """A problem on the caller's CSR family (see pd_set_family)."""
        B.pd_set_family(self.ctx, coords, row_ptr, col, ORDERS.get(order, order))

    def u_dev(self, out, inst=0):
        """Displacement into a float64 CUDA tensor (n x 3), on the library's stream."""
        B.pd_get_u_dev(self.ctx, inst, out)

    def v_dev(self, out, inst=0):
        B.pd_get_v_dev(self.ctx, inst, out)

    def damage_dev(self, out, inst=0):
        B.pd_get_damage_dev(self.ctx, inst, out)

    def build_family_batch(self, coords_list, horizons, order="natural"):
        B.pd_build_family_batch(self.ctx, coords_list, horizons, ORDERS.get(order, order))

    def family(self, inst=0):
        return B.pd_get_family(self.ctx, inst)

    def size(self, inst=0):
        return B.pd_instance_size(self.ctx, inst)

    def set_material(self, rho, c, s0, eta=0.0, volume=1.0, volumes=None, inst=0):
        B.pd_set_material(self.ctx, inst, rho, c, s0, eta, volume, volumes)

    def set_bond_stiffness(self, k, inst=0):
        B.pd_set_bond_stiffness(self.ctx, inst, k)

    def set_node_stiffness(self, k_node, inst=0):
        """Bond stiffness sqrt(k_i k_j) from a per-node field (None removes it)."""
        B.pd_set_node_stiffness(self.ctx, inst, k_node)

    def break_bonds(self, broken, inst=0):
        B.pd_break_bonds(self.ctx, inst, broken)

    def set_bcs(self, nodes, comp_mask, kind, value, sched, inst=0):
        B.pd_set_bcs(self.ctx, inst, nodes, comp_mask, kind, value, sched)

    def clear_bcs(self, inst=0):
        B.pd_clear_bcs(self.ctx, inst)

    def set_bc_ramp(self, ramp_time, inst=0):
        """Duration of the fifth-order ramp of every PD_SCHED_RAMP5 component."""
        B.pd_set_bc_ramp(self.ctx, inst, ramp_time)

    def set_no_fail(self, nodes, inst=0):
        """No-failure zone (node ids; None or empty removes it): their bonds never break."""
        B.pd_set_no_fail(self.ctx, inst, nodes)

    def force(self, inst=0):
        """Bond force density (n x 3) at the current displacement, intact bonds only."""
        return B.pd_get_force(self.ctx, inst)

    def resultant(self, nodes, inst=0):
        """sum of V_i F_i over the given nodes (the reaction measured at a loaded set)."""
        return B.pd_get_resultant(self.ctx, inst, nodes)

    def set_damage_law(self, cls, s_break, ratio, inst=0):
        """Damage law of bond class cls: stretch breakpoints and force ratios (1 ... 0)."""
        B.pd_set_damage_law(self.ctx, inst, cls, s_break, ratio)

    def set_bond_classes(self, cls, inst=0):
        """Bond class of every slot (user CSR order, symmetric per bond); None: class 0."""
        B.pd_set_bond_classes(self.ctx, inst, cls)

    def clear_damage_laws(self, inst=0):
        B.pd_clear_damage_laws(self.ctx, inst)

    def set_corrections(self, corrections=None, inst=0):
        """Stiffness corrections: a dict with micro ("constant"/"conical"), partial_volumes,
        surface, delta, dx; None removes them."""
        if corrections is None:
            B.pd_set_corrections(self.ctx, inst, clear=True)
        else:
            B.pd_set_corrections(self.ctx, inst, **corrections)

    def set_model(self, model, K=0.0, G=0.0, inst=0):
        """Constitutive model: "pmb" or "state_based" (bulk modulus K, shear modulus G)."""
        B.pd_set_model(self.ctx, inst, model, K, G)

    def dilation(self, inst=0):
        return B.pd_get_dilation(self.ctx, inst)

    def max_stretch(self, inst=0):
        """Largest stretch of every slot beyond its law's elastic limit (0 if none)."""
        return B.pd_get_max_stretch(self.ctx, inst)

    def set_max_stretch(self, smax, inst=0):
        B.pd_set_max_stretch(self.ctx, inst, smax)

    def mean_displacement(self, nodes, inst=0):
        """Mean u over the given nodes (e.g. the mid-span deflection of a beam)."""
        return B.pd_get_mean_displacement(self.ctx, inst, nodes)

    def set_body_force(self, b_hat, magnitude, inst=0):
        B.pd_set_body_force(self.ctx, inst, b_hat, magnitude)

    def set_integrator(self, scheme, dt):
        B.pd_set_integrator(self.ctx, SCHEMES.get(scheme, scheme), dt)

    def set_lanes_per_node(self, lanes):
        B.pd_set_lanes_per_node(self.ctx, lanes)

    def set_mapping(self, mapping, lanes=0):
        """mapping: "sliced" (lanes = work-items per node) or "staged" (lanes = wavefronts
        per 64-node slice)."""
        m = {"sliced": PD_MAP_SLICED, "staged": PD_MAP_STAGED}.get(mapping, mapping)
        B.pd_set_mapping(self.ctx, m, lanes)

    def autotune(self, trial_steps=20):
        return B.pd_autotune(self.ctx, trial_steps)

    # stepping and readout
    def step(self, nsteps):
        B.pd_step(self.ctx, nsteps)

    def prepare(self):
        """Build the step graphs now rather than inside the first long pd_step."""
        B.pd_prepare(self.ctx)

    def sync(self):
        B.pd_sync(self.ctx)

    @property
    def step_count(self):
        return B.pd_get_step(self.ctx)

    def u(self, inst=0):
        return B.pd_get_u(self.ctx, inst)

    def v(self, inst=0):
        return B.pd_get_v(self.ctx, inst)

    def a(self, inst=0):
        return B.pd_get_a(self.ctx, inst)

    def damage(self, inst=0):
        return B.pd_get_damage(self.ctx, inst)

    def broken(self, inst=0):
        return B.pd_get_broken(self.ctx, inst)

    def set_state(self, u=None, v=None, a=None, broken=None, inst=0):
        B.pd_set_state(self.ctx, inst, u, v, a, broken)

    def set_step(self, step):
        B.pd_set_step(self.ctx, step)

    def get_state(self, inst=0):
        """The whole state (checkpoint): a dict of u, v, a, broken, break_step,
        max_stretch, step and a_valid."""
        return B.pd_get_state(self.ctx, inst)

    def load_state(self, state, inst=0):
        """Restore a state from get_state (this or another context on the same problem)."""
        B.pd_load_state(self.ctx, inst, state)

    # adjoint (Euler-Cromer, frozen break schedule)
    def adj_forward(self, nsteps, ckpt_every=100):
        """Records a forward run; returns the recording's id."""
        return B.pd_adj_forward(self.ctx, nsteps, ckpt_every)

    def adj_backward(self, sensors, dL_du, recording=0):
        """(grad_k[nnz], grad_A) of a loss whose gradient at the sensors is dL_du (m x 3),
        for the recording with id `recording` (0: the current one)."""
        return B.pd_adj_backward(self.ctx, sensors, dL_du, recording)

    def break_steps(self, inst=0):
        return B.pd_get_break_steps(self.ctx, inst)

    def info(self):
        return B.pd_get_info(self.ctx)

    def last_step_ms(self):
        return B.pd_last_step_ms(self.ctx)


def apply_workload(sim: Simulation, w, inst: int = 0, row_ptr=None, col=None, stiffness: str = "slot") -> None:
    """Install a synthetic workload's material, BCs, notch, stiffness field and loads.

    ``w`` is a ``pd_inputs.Workload``; its family must already be built on ``sim``.
    The notch mask and stiffness field are input data generated from the library's own
    family (pd_get_family).  ``stiffness``: "slot" passes the field as per-slot values
    c exp((g_i + g_j)/2); "node" passes the node values c exp(g_i), whose geometric
    mean over a bond is the same field.
    """
    import pd_inputs as pi
    if row_ptr is None:
        row_ptr, col = sim.family(inst)
    sim.set_material(w.rho, w.c, w.s0, w.eta, w.volume, inst=inst)
    for bc in w.bcs:
        sim.set_bcs(bc.nodes, bc.comp_mask, bc.kind, bc.value, bc.sched, inst=inst)
    if w.ramp_T is not None:
        sim.set_bc_ramp(w.ramp_T, inst=inst)
    if w.state_based is not None:
        sim.set_model("state_based", *w.state_based, inst=inst)
    if w.corrections:
        sim.set_corrections(w.corrections, inst=inst)
    if w.laws:
        for k, (sb, rb) in enumerate(w.laws):
            sim.set_damage_law(k, sb, rb, inst=inst)
        if w.class_spec is not None:
            sim.set_bond_classes(pi.bond_classes(row_ptr, col, *w.class_spec), inst=inst)
    if w.nofail is not None:
        sim.set_no_fail(w.nofail, inst=inst)
    if w.notch is not None:
        sim.break_bonds(pi.notch_mask(w.ijk, row_ptr, col, *w.notch), inst=inst)
    if w.stiffness_field is not None:
        sig, ell, seed = w.stiffness_field
        g = pi.gaussian_node_field(w.dims, sig, ell, seed)
        if stiffness == "node":
            sim.set_node_stiffness(w.c * np.exp(g), inst=inst)
        else:
            sim.set_bond_stiffness(pi.slot_stiffness(w.c, g, row_ptr, col), inst=inst)
    if w.body_force is not None:
        bhat, bmag = w.body_force
        sim.set_body_force(bhat, bmag, inst=inst)


def simulation_for(w, precision: int = PD_FP64, lanes: int = 0, device: int = 0, order=None,
                   mapping="sliced", stiffness: str = "slot") -> Simulation:
    """A single-instance Simulation set up for workload ``w`` (family built on the host)."""
    sim = Simulation(device, precision)
    if w.state_based is not None and mapping == "sliced":
        mapping = "staged"  # the state-based kernels run on the staged layout
    if lanes or mapping != "sliced":
        sim.set_mapping(mapping, lanes)
    sim.build_family(w.coords, w.horizon, order or w.order)
    sim.set_integrator(w.scheme, w.dt)
    apply_workload(sim, w, stiffness=stiffness)
    return sim
