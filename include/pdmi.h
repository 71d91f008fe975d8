/*
 * pdmi.h -- C ABI of the MI355X (gfx950) bond-based peridynamics library.
 *
 * The library advances the explicit bond-based peridynamic equation of motion
 * (paper: "PeriPy - a high performance OpenCL peridynamics package", Sec. 2):
 *
 *   rho u''_i = sum_{j in H_i} f(eta_ij, xi_ij) V_j + b_i             (Eq. discrete EOM)
 *   f = c s mu (eta + xi) / |eta + xi|,  s = (|eta + xi| - |xi|)/|xi| (Eqs. microelastic, simpleBond)
 *   mu = 0 for ever once s >= s0 (irreversible brittle breaking)       (Eq. mu)
 *   H_i = { j != i : |x_j - x_i| <= delta }                           (Eq. family)
 *
 * with an explicit time integrator (Sec. 2.4) and per-node local damage (Sec. 2.2); also
 * n-linear damage laws per bond class, stiffness corrections, quasi-static loading tools,
 * the ordinary state-based linear solid (Sec. 8.2) and a reverse-mode adjoint.
 * Every time step runs in hand-written HIP kernels on one GPU.
 *
 * Conventions (all entry points):
 *  - Return value: PD_OK (0) or a negative PD_E* code; pd_last_error() gives a
 *    message.  No C++ exception crosses this boundary.
 *  - Setters are all-or-nothing: on error the context is unchanged.
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - Node ids, slot ids and every per-node / per-slot array are in the caller's
 *    ("user") order: node ids as passed to pd_build_family, slots in the CSR order
 *    returned by pd_get_family.  Any internal renumbering is invisible.
 *  - A context serves one HIP stream; work is stream-ordered and asynchronous
 *    unless a call says it synchronises.  A context is not thread-safe.
 *  - Instances: a context holds one or more independent problems ("instances",
 *    numbered from 0) that pd_step advances together in the same kernel launches.
 *    Single-problem callers use instance 0.
 */
#ifndef PDMI_H
#define PDMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define PD_OK 0
#define PD_EINVAL (-1)      /* bad argument: NULL pointer, size or enum out of range */
#define PD_ENOMEM (-2)      /* host or device allocation failed */
#define PD_EHIP (-3)        /* a HIP runtime call failed */
#define PD_ESTATE (-4)      /* call out of order (e.g. pd_step before pd_build_family) */
#define PD_ENONFINITE (-5)  /* a displacement or velocity became non-finite */
#define PD_ERANGE (-6)      /* problem exceeds the index types (2^31-1 nodes or slots) */

/* ---------------------------------------------------------------- enumerations */
#define PD_FP64 0           /* state and arithmetic in double precision */
#define PD_FP32 1           /* state (u, v, a) and bond arithmetic in single precision */

#define PD_ORDER_NATURAL 0  /* keep the caller's node order in device memory */
#define PD_ORDER_MORTON 1   /* renumber nodes internally along a Morton (Z-order) curve */
#define PD_ORDER_AUTO 2     /* natural order until pd_autotune, which also tries Morton order */

#define PD_EULER_CROMER 0     /* v += dt (F - eta v)/rho; u += dt v_new */
#define PD_VELOCITY_VERLET 1  /* Eqs. Velocity_Verlet1-3 */
#define PD_EULER_FORWARD 2    /* u += dt v; v += dt (F - eta v)/rho (unstable; tests only) */

#define PD_BC_DISP 1        /* prescribed displacement: u_c = A_c g(t), v_c = A_c g'(t) */
#define PD_BC_VEL 2         /* prescribed velocity: v_c = A_c g(t), u_c += dt v_c */

#define PD_MAP_SLICED 0     /* slots in 64-wide rows, G lanes per node, neighbours gathered from
                               global memory through the L1 cache */
#define PD_MAP_STAGED 1     /* one lane per node; each wavefront stages runs of consecutive
                               neighbour records in LDS and reads them from there */

#define PD_SCHED_CONST 0    /* g(t) = 1 */
#define PD_SCHED_LINEAR 1   /* g(t) = t */
#define PD_SCHED_RAMP5 2    /* g(t) = 10 tau^3 - 15 tau^4 + 6 tau^5, tau = t / T, for t < T, then 1:
                               a fifth-order ramp from 0 to 1 whose velocity and acceleration
                               vanish at both ends (the smooth displacement loading of the
                               quasi-static examples, Secs. 6-7); T set by pd_set_bc_ramp */

typedef struct pd_ctx pd_ctx;

/* Material of one instance (Sec. 2.2-2.3). */
typedef struct pd_material {
    double rho;             /* mass density (kg/m^3), > 0 */
    double c;               /* micromodulus (N/m^6), e.g. 18 K / (pi delta^4); used by every
                               bond that has no per-slot stiffness (pd_set_bond_stiffness) */
    double s0;              /* critical stretch, > 0 */
    double eta;             /* dynamic-relaxation damping coefficient (Eq. damped EOM), >= 0 */
    double volume;          /* uniform node volume V (m^3) when volumes == NULL, > 0 */
    const double *volumes;  /* host array of n per-node volumes (user order), or NULL */
} pd_material;

/* Sizes of the device problem (informational; see pd_get_info). */
typedef struct pd_info {
    int64_t n_nodes;        /* user nodes, all instances */
    int64_t n_slots;        /* directed family slots, all instances (bond updates per step) */
    int64_t n_nodes_dev;    /* device node records incl. slice padding */
    int64_t n_slots_dev;    /* device slot entries incl. slice padding */
    int32_t n_instances;
    int32_t lanes_per_node; /* work-items cooperating on one node's bonds */
    int32_t precision;      /* PD_FP64 / PD_FP32 */
    int32_t scheme;         /* integrator */
    int32_t mapping;        /* PD_MAP_SLICED / PD_MAP_STAGED */
    int32_t order;          /* device node order in use: PD_ORDER_NATURAL / PD_ORDER_MORTON */
    double model_bytes_per_step; /* algorithmic HBM bytes of one step (see the design notes) */
    int32_t waves_per_slice; /* staged mapping: wavefronts sharing one 64-node slice (1 otherwise) */
    int32_t reserved_;
} pd_info;

/* ---------------------------------------------------------------- lifetime */

/* Create a context on HIP device `device` computing in `precision`.  `hip_stream` is
 * the caller's hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL,
 * in which case the library creates its own stream.  *out receives the handle. */
int pd_create(pd_ctx **out, int device, int precision, void *hip_stream);

/* Free every device and host resource of the context.  NULL is accepted. */
int pd_destroy(pd_ctx *ctx);

/* Message describing the last failure on this context ("" if none).  With ctx ==
 * NULL, the message of the last failed pd_create in this process. */
const char *pd_last_error(const pd_ctx *ctx);

/* ---------------------------------------------------------------- problem setup */

/* Build the family of a single-instance problem (Eq. family: every j != i with
 * |x_j - x_i| <= horizon, tested as ((dx^2 + dy^2) + dz^2) <= horizon^2 without
 * fused multiply-add) from `coords` (host, n x 3 row-major doubles, metres), sorted
 * ascending per row, and upload it.  `order` picks the device node order.  Resets
 * the state: u = v = a = 0, no broken bonds, no BCs, no body force, step 0.
 * Errors: PD_EINVAL (n < 1, NULL coords, non-finite coords, two nodes at the same
 * position, horizon <= 0 or not finite, bad order), PD_ERANGE (n or nnz >= 2^31, or
 * 2^24 or more device node records), PD_ENOMEM, PD_EHIP. */
int pd_build_family(pd_ctx *ctx, int64_t n, const double *coords, double horizon, int order);

/* Same for `ninst` independent instances advanced together: instance b has n[b]
 * nodes at coords[b] (host, n[b] x 3) and horizon horizon[b].  Errors as above. */
int pd_build_family_batch(pd_ctx *ctx, int32_t ninst, const int64_t *n,
                          const double *const *coords, const double *horizon, int order);

/* A single-instance problem on a family the caller supplies (reuse of a family built
 * earlier, or any other neighbourhood; Eq. family is the usual one): n nodes at coords
 * (host, n x 3), CSR row_ptr (n+1 int64, row_ptr[0] = 0) and col (int32), rows strictly
 * ascending, no self bond, every bond present in both directions (j in row i iff i in row
 * j), no two nodes at the same place.  Replaces any earlier problem like
 * pd_build_family; the family is kept as given (pd_get_family returns it).  Errors:
 * PD_EINVAL (a rule above broken), PD_ERANGE (2^31 or more slots). */
int pd_set_family(pd_ctx *ctx, int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col,
                  int order);

/* Number of instances of the current problem. */
int pd_num_instances(const pd_ctx *ctx, int32_t *ninst);

/* Node and slot counts of instance `inst` (either pointer may be NULL). */
int pd_instance_size(const pd_ctx *ctx, int32_t inst, int64_t *n, int64_t *nnz);

/* Export the family of instance `inst` in CSR form: row_ptr (n+1 int64) and col
 * (nnz int32), user order, rows ascending.  Either array may be NULL to query
 * sizes only; *nnz (if not NULL) receives the slot count.  Synchronising. */
int pd_get_family(pd_ctx *ctx, int32_t inst, int64_t *row_ptr, int32_t *col, int64_t *nnz);

/* Set the material of instance `inst` (Sec. 2.2).  Default after a family build:
 * rho = 1, c = 1, s0 = +inf (nothing breaks), eta = 0, V = 1. */
int pd_set_material(pd_ctx *ctx, int32_t inst, const pd_material *m);

/* Per-slot micromodulus k[nnz] (host, user CSR order) replacing c for instance
 * `inst` (bond classes / stiffness fields, Sec. 2.2 remark).  The two slots of a
 * bond must carry the same value for Newton's third law to hold; the library does
 * not enforce it.  k == NULL removes the field. */
int pd_set_bond_stiffness(pd_ctx *ctx, int32_t inst, const double *k);

/* Per-node stiffness k_node[n] (host, user order, finite, >= 0) for instance `inst`:
 * every bond (i, j) gets the micromodulus sqrt(k_node[i] * k_node[j]), the geometric
 * mean, which is symmetric by construction (a log-normal field k_i = c exp(g_i) gives
 * c exp((g_i + g_j)/2)).  It replaces a per-slot field of the instance (and a later
 * pd_set_bond_stiffness replaces it); k_node == NULL removes it.  The bond value is
 * formed on the device as sqrt(k_i) * sqrt(k_j) (rounding differs from the exact
 * mean by about one ulp) and costs 16 bytes per node and step instead of 8 per slot
 * when no instance carries a per-slot field. */
int pd_set_node_stiffness(pd_ctx *ctx, int32_t inst, const double *k_node);

/* Mark slots broken before or between steps (e.g. a notch pre-broken as an initial
 * condition).  broken[nnz] (host, user CSR order): nonzero = break.  Breaking is
 * irreversible; zero entries leave a slot unchanged.  Breaking one slot of a bond
 * does not break the other; pass both. */
int pd_break_bonds(pd_ctx *ctx, int32_t inst, const uint8_t *broken);

/* Boundary conditions (Sec. 3.6: directions fixed, magnitudes time-varying).  For
 * each of the m nodes (host ids, user order) and each component d with bit d of
 * comp_mask set, prescribe kind PD_BC_DISP or PD_BC_VEL with amplitude value[d] and
 * schedule `sched`.  After every step, at t = step * dt, a displacement-controlled
 * component gets u = A g(t), v = A g'(t); a velocity-controlled one gets v = A g(t)
 * and u = u_previous + dt v.  Later calls override earlier ones per component.
 * Errors: PD_EINVAL (node id out of range, empty mask, bad kind or schedule). */
int pd_set_bcs(pd_ctx *ctx, int32_t inst, int64_t m, const int64_t *nodes, int comp_mask,
               int kind, const double value[3], int sched);

/* Remove every boundary condition of instance `inst`. */
int pd_clear_bcs(pd_ctx *ctx, int32_t inst);

/* Ramp duration T > 0 (seconds) of every PD_SCHED_RAMP5 component of instance `inst`
 * (default 1).  Errors: PD_EINVAL (T not positive and finite). */
int pd_set_bc_ramp(pd_ctx *ctx, int32_t inst, double ramp_time);

/* No-failure zones (Secs. 5.1, 6, 7): the m nodes (host ids, user order) of instance
 * `inst` become the zone, replacing any earlier one; a bond with either end in the zone
 * never breaks and keeps its damage state from now on (bonds already broken stay broken,
 * softened ones keep their secant ratio, recorded break steps are kept).  m = 0 removes the zone.  Errors: PD_EINVAL (node id out of range). */
int pd_set_no_fail(pd_ctx *ctx, int32_t inst, int64_t m, const int64_t *nodes);

/* Damage law of bond class `cls` (0..7) of instance `inst` (Sec. 3.6: laws made of
 * linear splines; the trilinear law of Sec. 6, the bilinear law of Sec. 7).  nb (1..8)
 * stretch breakpoints s_break[0] < ... < s_break[nb-1], all > 0, with force ratios
 * ratio[nb] >= 0, ratio[0] = 1 and ratio[nb-1] = 0 when nb > 1.  Under a monotonic pull
 * a bond carries c s up to s_break[0], then c s_break[0] times the ratio interpolated
 * linearly between breakpoints, and breaks for good at s_break[nb-1]; nb = 1 is the
 * brittle law with s0 = s_break[0].  Damage is irreversible: a bond that has softened
 * to a largest stretch s_m carries (c s_break[0] rho(s_m) / s_m) s, the secant to the
 * origin, in tension and compression.  Once an instance has laws, they replace the s0
 * of pd_set_material.  Classes are defined in order (cls <= number defined); setting a
 * law again replaces it.  Every change of laws or classes clears the softening state
 * (broken flags and recorded break steps are kept).  Host arrays are copied.
 * Errors: PD_EINVAL (class out of range or out of order, bad breakpoints or ratios). */
int pd_set_damage_law(pd_ctx *ctx, int32_t inst, int32_t cls, int32_t nb, const double *s_break,
                      const double *ratio);

/* Bond class of every slot: cls[nnz] (host, user CSR order), each below the number of
 * laws defined; both slots of a bond must be in the same class (Sec. 2.2: bond classes
 * as a function of the two end points).  NULL puts every slot in class 0.
 * Errors: PD_EINVAL (no laws, class without a law, asymmetric classes). */
int pd_set_bond_classes(pd_ctx *ctx, int32_t inst, const uint8_t *cls);

/* Back to the brittle law with the s0 of pd_set_material (laws and classes removed). */
int pd_clear_damage_laws(pd_ctx *ctx, int32_t inst);

#define PD_MICRO_CONSTANT 0  /* c(|xi|) = c */
#define PD_MICRO_CONICAL 1   /* c(|xi|) = c max(0, 1 - |xi|/delta): c is the peak value (5 times the
                                constant micromodulus for the same bulk stiffness) */

/* Stiffness corrections of one instance (Secs. 2.2, 2.3 and 2.5), each a factor on every slot's
 * stiffness, applied in this order: the micromodulus profile; partial volumes, beta = 1
 * for |xi| <= delta - dx/2, falling linearly to 0 at delta + dx/2 (the share of a
 * neighbour's cell inside the horizon; build the family with horizon delta + dx/2 to
 * include the cut cells); the volume-method surface correction lambda_ij = 2 V0 /
 * (V_i + V_j), V_i = sum over node i's family of beta_ij V_j and V0 the largest V_i (a
 * complete family).  The staged mapping (FP64 and FP32 builds) forms the factors per slot from
 * the bond length and the two family volumes when no instance has a stiffness field or
 * per-node volumes; otherwise they are formed once on the host and the step reads the
 * corrected stiffness per slot.  Both forms give the same results up to rounding. */
typedef struct pd_corrections {
    int32_t micromodulus;      /* PD_MICRO_CONSTANT or PD_MICRO_CONICAL */
    int32_t partial_volumes;   /* nonzero: partial volumes */
    int32_t surface;           /* nonzero: volume-method surface correction */
    int32_t reserved_;
    double delta;              /* horizon of the profile and the partial volumes (> 0 when used) */
    double dx;                 /* lattice spacing of the partial volumes (> 0 when used) */
} pd_corrections;

/* Stiffness corrections of instance `inst`; NULL removes them.  They multiply whatever
 * stiffness the instance has (c, per-slot or per-node field).  The adjoint rejects
 * problems with corrections.  Errors: PD_EINVAL (unknown profile, delta or dx not
 * positive where needed). */
int pd_set_corrections(pd_ctx *ctx, int32_t inst, const pd_corrections *corr);

#define PD_MODEL_PMB 0          /* bond-based prototype microelastic brittle model (Sec. 2.2) */
#define PD_MODEL_STATE_BASED 1  /* ordinary state-based linear peridynamic solid (Sec. 8.2) */

/* Constitutive model of instance `inst`.  PD_MODEL_STATE_BASED replaces the PMB bond force
 * by the ordinary state-based linear solid of Sec. 8.2 (after Silling et al. 2007) with
 * bulk modulus K > 0 and shear modulus G >= 0 (so any Poisson ratio, where the PMB fixes
 * it at 1/4, Sec. 2.2), influence function 1:
 *   weighted volume  m_i = sum over the whole family of |xi|^2 V (reference configuration)
 *   dilation         theta_i = (3 / m_i) sum over intact bonds of |xi| e V, e = |y| - |xi|
 *   bond force       (t_ij + t_ji) y/|y| V,  t_ij = (3 K theta_i / m_i) |xi|
 *                    + (15 G / m_i) (e - theta_i |xi| / 3)
 * Bonds break at the critical stretch s0 of pd_set_material (irreversibly, on both
 * slots, not in no-failure zones), before the dilation of the same step.  Each step runs
 * two kernels (dilation, then force and integration).  The model needs the staged
 * mapping (FP64 or FP32 build; uniform or per-node volumes); it takes no stiffness field, damage
 * law or correction, the adjoint rejects it, and every instance of a context must run
 * the same model (checked here and when stepping; c of pd_set_material is unused).
 * PD_MODEL_PMB (K, G ignored) returns to the bond-based model.  Errors: PD_EINVAL. */
int pd_set_model(pd_ctx *ctx, int32_t inst, int model, double K, double G);

/* Body force density b_i = magnitude * b_hat_i (N/m^3) of instance `inst`;
 * b_hat: host n x 3, user order; NULL removes it. */
int pd_set_body_force(pd_ctx *ctx, int32_t inst, const double *b_hat, double magnitude);

/* Choose the integrator (PD_EULER_CROMER, PD_VELOCITY_VERLET, PD_EULER_FORWARD) and
 * time step dt > 0 for all instances.  Default: Euler-Cromer, dt = 1e-7 s. */
int pd_set_integrator(pd_ctx *ctx, int scheme, double dt);

/* ---------------------------------------------------------------- stepping */

/* Advance every instance by nsteps >= 0 steps.  Each step reads the current
 * displacement snapshot, gathers neighbours over the family, computes stretches,
 * breaks bonds with s >= s0 (they contribute nothing from that step on), sums the
 * PMB bond forces per node (or the state-based forces, pd_set_model), then integrates
 * and applies the BCs.  Asynchronous: a
 * non-finite state is reported by the next synchronising call (PD_ENONFINITE). */
int pd_step(pd_ctx *ctx, int64_t nsteps);

/* Capture and instantiate now the step graphs that pd_step would otherwise build on
 * first use (chunks of several steps recorded once and replayed), for the current
 * integrator, layout and loads, so that a later pd_step spends no host time on them.
 * Runs nothing on the device and changes no state.  Calls that change the layout,
 * the integrator, the loads or the no-failure zones discard the graphs again. */
int pd_prepare(pd_ctx *ctx);

/* Wait for the stream; returns PD_ENONFINITE if any step produced a non-finite
 * displacement or velocity since the state was last set. */
int pd_sync(pd_ctx *ctx);

/* Number of completed steps. */
int pd_get_step(const pd_ctx *ctx, int64_t *step);

/* ---------------------------------------------------------------- readout (synchronising) */

/* Copy the displacement / velocity / acceleration (velocity Verlet; zeros otherwise)
 * of instance `inst` into out (host, n x 3 doubles, user order). */
int pd_get_u(pd_ctx *ctx, int32_t inst, double *out);
int pd_get_v(pd_ctx *ctx, int32_t inst, double *out);
int pd_get_a(pd_ctx *ctx, int32_t inst, double *out);

/* The same readouts into device memory (for example a torch tensor on this context's
 * device): out is a device pointer to n x 3 (displacement, velocity) or n (damage)
 * doubles, written in user order.  Stream-ordered on the context's stream and not
 * synchronising: the values are there once that stream has reached this point (the
 * non-finite check is left to pd_sync).  Errors: PD_EINVAL if out is not device memory of
 * the context's device (the size cannot be checked: out must hold the values). */
int pd_get_u_dev(pd_ctx *ctx, int32_t inst, double *out);
int pd_get_v_dev(pd_ctx *ctx, int32_t inst, double *out);
int pd_get_damage_dev(pd_ctx *ctx, int32_t inst, double *out);

/* Local damage phi_i = 1 - sum_j (1 - d_ij) V_j / sum_j V_j over the initial family
 * (Sec. 2.2; d = 1 broken, d = 1 - secant ratio for a bond softened under a damage law,
 * 0 intact: with the brittle law this is 1 - sum_j mu_ij V_j / sum_j V_j), as of the
 * last completed step; 0 for a node without bonds.
 * out: host, n doubles, user order. */
int pd_get_damage(pd_ctx *ctx, int32_t inst, double *out);

/* State-based model: dilation theta_i of every node at the current displacement over
 * the bonds intact now (Sec. 8.2; breaks nothing).  out: host, n doubles, user order.
 * Errors: PD_EINVAL if the instance runs the PMB model. */
int pd_get_dilation(pd_ctx *ctx, int32_t inst, double *out);

/* Broken flags of every slot: out[nnz] (host, user CSR order), 1 = broken. */
int pd_get_broken(pd_ctx *ctx, int32_t inst, uint8_t *out);

/* Largest stretch each slot has reached beyond its damage law's elastic limit, 0 while
 * it has not (and without damage laws): out[nnz] (host, user CSR order). */
int pd_get_max_stretch(pd_ctx *ctx, int32_t inst, double *out);

/* Overwrite the stretch state (checkpoint / restart with damage laws): smax[nnz] (host,
 * user CSR order) as pd_get_max_stretch returns it; a slot with smax > 0 counts as
 * softened.  Errors: PD_ESTATE (no damage laws), PD_EINVAL (negative or non-finite). */
int pd_set_max_stretch(pd_ctx *ctx, int32_t inst, const double *smax);

/* Bond force density F_i = sum_j f_ij V_j (Eq. discrete EOM without the body force) at
 * the current displacement, over the bonds intact now, each with its damage state as it
 * stands (a softened bond with its secant ratio); no bond breaks or softens and the state
 * is not changed.  Evaluated on the device for every instance by the step kernel in a
 * force-only mode.  out: host, n x 3 doubles, user order. */
int pd_get_force(pd_ctx *ctx, int32_t inst, double *out);

/* Resultant force of a node set: out[0..2] = sum over the m nodes (host ids, user order)
 * of V_i F_i with F as pd_get_force, summed on the device in a fixed order (the load
 * measured as the resultant of the bond forces on the displacement-controlled nodes, Sec. 6).
 * Errors: PD_EINVAL (node id out of range, m < 1). */
int pd_get_resultant(pd_ctx *ctx, int32_t inst, int64_t m, const int64_t *nodes, double out[3]);

/* Mean displacement of a node set: out[0..2] = (1/m) sum over the m nodes (host ids,
 * user order) of u_i at the current level, summed on the device in a fixed order (the
 * mid-span deflection of Sec. 7: the mean deflection of the top nodes at mid-span).
 * Errors: PD_EINVAL (node id out of range, m < 1). */
int pd_get_mean_displacement(pd_ctx *ctx, int32_t inst, int64_t m, const int64_t *nodes, double out[3]);

/* pd_get_mean_displacement for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or measurement loops, harnesses that forbid hipMalloc):
 * the same readout, bit for bit, calling no hipMalloc, hipFree or other allocating
 * routine.  The node ids and the sums live in a fixed device array of this library on the
 * context's GPU (262,144 node ids and three sums, about 2 MiB per GPU, held until the
 * process ends); every call on that GPU shares it, so calls that overlap on one GPU (from
 * several threads or contexts) race.  Synchronising.  Errors: PD_EINVAL (m < 1, m >
 * 262144, node id out of range, NULL arguments), PD_ESTATE (no problem built). */
int pd_get_mean_displacement_noalloc(pd_ctx *ctx, int32_t inst, int64_t m, const int64_t *nodes, double out[3]);

/* Overwrite the state of instance `inst` (checkpoint / restart: Sec. 3.6 lets a run
 * start from an intermediate state).  Any of u, v, a (host n x 3) or broken
 * (host nnz; replaces the broken set exactly, un-breaking included) may be NULL to
 * keep the current value.  pd_set_step sets the step counter of all instances. */
int pd_set_state(pd_ctx *ctx, int32_t inst, const double *u, const double *v, const double *a,
                 const uint8_t *broken);
int pd_set_step(pd_ctx *ctx, int64_t step);

/* The whole state of one instance, for checkpoint and restart (Sec. 3.6: a run may
 * continue from a saved step).  Arrays are host memory owned by the caller, in the
 * caller's node and slot order; a NULL array is skipped. */
typedef struct pd_state {
    double *u;            /* n x 3: displacement of the current level (FP32 build: the
                             f64 master displacement the integrator advances) */
    double *v;            /* n x 3: velocity */
    double *a;            /* n x 3: acceleration (velocity Verlet; otherwise whatever the
                             problem holds, zeros for a fresh one) */
    uint8_t *broken;      /* nnz: 1 = broken */
    int32_t *break_step;  /* nnz: pass in which the slot broke, INT32_MAX intact,
                             INT32_MIN broken before recording started (pd_get_break_steps) */
    double *max_stretch;  /* nnz: damage-law stretch state (pd_get_max_stretch; zeros
                             without damage laws) */
    int64_t step;         /* step counter (shared by every instance) */
    int32_t a_valid;      /* 1 when a holds the acceleration of the current level */
    int32_t pad_;
} pd_state;

/* Export the state of instance `inst` into the caller's arrays (each NULL array is
 * skipped) and set out->step and out->a_valid.  Synchronising. */
int pd_get_state(pd_ctx *ctx, int32_t inst, pd_state *out);

/* Restore a state exported by pd_get_state, possibly into another context holding the
 * same problem (same family, material and boundary conditions): stepping on from it gives
 * bit for bit what the exporting context gives.  NULL arrays keep the current values;
 * u replaces both displacement levels; broken replaces the broken set exactly (the
 * break steps then restart from it, unless break_step is given too); a max_stretch with
 * a non-zero entry needs damage laws (PD_ESTATE otherwise; all zeros, as exported for a
 * problem without laws, is ignored); step sets the step counter of every instance;
 * a_valid is honoured only together with a.  Discards any adjoint recording.  Errors: PD_EINVAL (non-finite u, v, a or max_stretch, negative
 * max_stretch, step out of [0, 2^31 - 1)). */
int pd_load_state(pd_ctx *ctx, int32_t inst, const pd_state *in);

/* ---------------------------------------------------------------- adjoint */

/* Reverse-mode gradients of a displacement misfit after an Euler-Cromer run with the
 * bond-break schedule of that run frozen (a slot acts in pass k iff it had not broken
 * by the end of pass k; the critical-stretch rule of Sec. 2 is not differentiated).
 * FP64 build, single-instance problems, Euler-Cromer scheme; every bond's two slots
 * must carry the same stiffness and broken flag (PD_EINVAL otherwise).
 *
 * pd_adj_forward advances the problem by nsteps >= 1 steps exactly as pd_step does,
 * recording the pass in which each slot breaks and a device checkpoint of (u, v)
 * every ckpt_every >= 1 steps ((nn + 89) * 48 + nn * 24 bytes each, nn = padded node
 * count; with ckpt_every = 1 every level is kept, v is not, and the reverse pass
 * recomputes nothing).  Any later change to the problem or state (pd_step included)
 * discards the recording.  Asynchronous like pd_step.  *recording (may be NULL)
 * receives an id of this recording, unique in the process and > 0 (0 on error), which
 * pd_adj_backward takes to make sure its gradient belongs to this run. */
int pd_adj_forward(pd_ctx *ctx, int64_t nsteps, int32_t ckpt_every, int64_t *recording);

/* Gradient of a loss L(u^T) at the end of the recorded run.  The caller passes
 * dL/du^T for m >= 0 sensor nodes: sensors (host, m user node ids, repeats add up) and
 * dL_du (host, m x 3).  Outputs: grad_k (host, nnz doubles, user CSR order) = dL/dk
 * for every slot's stiffness (slots of a bond are separate parameters), and *grad_A =
 * dL/dA for the body-force magnitude of pd_set_body_force (0 without a body force).
 * Each segment between checkpoints is recomputed with the forward kernel (same
 * results bit for bit) into a trajectory buffer of min(ckpt_every, nsteps) levels,
 * then the reverse passes run last to first.  The problem state is left unchanged.
 * recording: the id pd_adj_forward returned, or 0 for whichever recording is current.
 * Synchronising; PD_ESTATE if there is no valid recording or it is not `recording`
 * (another pd_adj_forward ran since, or the problem or state changed). */
int pd_adj_backward(pd_ctx *ctx, int64_t recording, int64_t m, const int64_t *sensors, const double *dL_du,
                    double *grad_k, double *grad_A);

/* Pass index in which each slot broke (host out[nnz], user CSR order): INT32_MAX =
 * intact, INT32_MIN = already broken when the broken set was last established (problem
 * build, mapping change, pd_break_bonds, pd_set_state with a broken set, or the start
 * of pd_adj_forward).  Every step records the passes of the bonds it breaks. */
int pd_get_break_steps(pd_ctx *ctx, int32_t inst, int32_t *out);

/* ---------------------------------------------------------------- tuning and introspection */

/* Work mapping of the step kernel: PD_MAP_SLICED with `lanes` work-items cooperating on
 * one node's bonds (1, 4, 16 or 64; 0 = library default), or PD_MAP_STAGED with `lanes`
 * wavefronts sharing each 64-node slice (1, 2 or 4; 0 = 1; more than one fills the chip
 * on problems with fewer slices than SIMDs).  Rebuilds the device layout when the
 * mapping changes; the state (u, v, a, broken bonds, step) is kept. */
int pd_set_mapping(pd_ctx *ctx, int mapping, int lanes);

/* Shorthand for pd_set_mapping(ctx, PD_MAP_SLICED, lanes). */
int pd_set_lanes_per_node(pd_ctx *ctx, int lanes);

/* Time `trial_steps` steps (after as many untimed ones) of every mapping candidate on
 * the current problem (and both device node orders if the family was built with
 * PD_ORDER_AUTO) and keep the fastest; the state is restored afterwards.
 * *chosen (may be NULL) receives the lanes-per-node of the chosen sliced mapping, or
 * minus the wavefronts per slice of the chosen staged mapping. */
int pd_autotune(pd_ctx *ctx, int64_t trial_steps, int32_t *chosen);

/* Problem and layout sizes. */
int pd_get_info(const pd_ctx *ctx, pd_info *info);

/* Device time of the last pd_step call in milliseconds (HIP events recorded on the
 * context's stream around that call's kernels); synchronising. */
int pd_last_step_ms(pd_ctx *ctx, double *ms);

/* The exact stretch the FP64 step kernels decide near the break threshold (Eq. mu:
 * s = (|y| - |xi|)/|xi|, squares summed as (a^2 + b^2) + c^2, every operation rounded
 * once, no fused multiply-add, correctly rounded square roots and division), evaluated
 * on `device` for m bonds: xi and y host m x 3 (row-major), s host m doubles.  For
 * checking that the device arithmetic agrees bit for bit with an IEEE host evaluation.
 * Synchronising; allocates and frees its own device buffers.  Errors: PD_EINVAL (m < 0,
 * NULL arrays with m > 0, bad device), PD_EHIP. */
int pd_stretch_exact(int device, int64_t m, const double *xi, const double *y, double *s);

#ifdef __cplusplus
}
#endif

#endif /* PDMI_H */
