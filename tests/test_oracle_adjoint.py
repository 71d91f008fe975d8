"""Pins of the oracle's reverse-mode gradient (Euler-Cromer, frozen break schedule).

The C adjoint (`pdo_adjoint_ec`, a literal transpose-Jacobian scatter over a stored
trajectory) is checked against complex-step derivatives of an independent NumPy forward
run, against the transpose identity <J v, w> = <v, J^T w> per pass, and against
central finite differences of the C forward run.  Every check runs without damping and
with dynamic-relaxation damping (Sec. 2.3's damped equation of motion: the velocity
factor 1 - dt eta/rho enters every reverse step).
"""
import numpy as np
import pytest

import pd_inputs as pi
from oracle.cstep import ec_forward, force_cs

RHO, DT = 2400.0, 1e-7
# damping coefficients of the two cases: none, and eta with eta dt / rho = 1e-3 per step
# (4% of the velocity over the 40 steps), enough for a dropped or sign-flipped damping
# factor in the reverse step to miss the complex-step derivative by far more than 1e-9
ETAS = (0.0, 2.4e7)


def _problem(oracle_lib, seed=3, steps=40, eta=0.0):
    dims = (6, 4, 4)
    x, ijk = pi.lattice(dims, 1e-3, 2e-2, seed=seed)
    rp, col = oracle_lib.family(x, 2.0e-3)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), np.diff(rp))
    g = rng.normal(size=n) * 0.2
    c = pi.pmb_micromodulus(1.4e10, 2.0e-3)
    k = c * np.exp(0.5 * (g[rows] + g[col]))
    vol = 1e-9 * rng.uniform(0.8, 1.2, n)
    # frozen schedule: a few bonds stop acting part-way (both directions of a bond together)
    frozen = np.full(rp[-1], np.iinfo(np.int32).max, dtype=np.int32)
    for b in rng.choice(rp[-1], 6, replace=False):
        i, j = rows[b], col[b]
        rev = rp[j] + np.searchsorted(col[rp[j]:rp[j + 1]], i)
        frozen[b] = frozen[rev] = rng.integers(5, steps)
    bcs = [pi.BCSpec(pi.face_nodes(ijk, 0, 0), 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST),
           pi.BCSpec(pi.face_nodes(ijk, 2, 3)[:3], 0b010, pi.BC_VEL, (0.0, 0.02, 0.0), pi.SCHED_CONST)]
    bhat = np.zeros((n, 3))
    bhat[ijk[:, 0] == dims[0] - 1, 2] = -1.0
    bmag = 3e8
    sensors = np.array([5, 17, 40, 71, 95], dtype=np.int64)
    target = rng.normal(size=(sensors.shape[0], 3)) * 1e-7
    return dict(x=x, ijk=ijk, rp=rp, col=col, k=k, vol=vol, frozen=frozen, bcs=bcs, bhat=bhat,
                bmag=bmag, sensors=sensors, target=target, steps=steps, n=n, eta=eta)


def _sim(oracle_lib, P, k=None, bmag=None):
    return oracle_lib.OracleSim(P["x"], P["rp"], P["col"], c=0.0, s0=1.0, rho=RHO, dt=DT,
                                vol=P["vol"], kslot=P["k"] if k is None else k, bhat=P["bhat"],
                                bmag=P["bmag"] if bmag is None else bmag, bcs=P["bcs"],
                                frozen=P["frozen"], eta=P["eta"])


def _loss_cs(P, k, bmag):
    kind, sched, val = __import__("oracle").bc_arrays(P["n"], P["bcs"])
    u, _ = ec_forward(P["x"], P["rp"], P["col"], k, P["vol"], RHO, DT, P["frozen"], P["steps"],
                      bhat=P["bhat"], bmag=bmag, bc_kind=kind, bc_sched=sched, bc_val=val, eta=P["eta"])
    d = u[P["sensors"]] - P["target"]
    return (d * d).sum()


def _adjoint(oracle_lib, P):
    sim = _sim(oracle_lib, P)
    sim.run(P["steps"])
    d = 2.0 * (sim.u[P["sensors"]] - P["target"])
    z = np.zeros((P["n"], 3))
    return sim.adjoint_ec(P["frozen"], P["steps"], z, z, 0, P["sensors"], d), sim


@pytest.mark.parametrize("eta", ETAS)
def test_numpy_forward_matches_c_forward(oracle_lib, eta):
    P = _problem(oracle_lib, eta=eta)
    sim = _sim(oracle_lib, P)
    sim.run(P["steps"])
    kind, sched, val = oracle_lib.bc_arrays(P["n"], P["bcs"])
    u, v = ec_forward(P["x"], P["rp"], P["col"], P["k"], P["vol"], RHO, DT, P["frozen"], P["steps"],
                      bhat=P["bhat"], bmag=P["bmag"], bc_kind=kind, bc_sched=sched, bc_val=val, dtype=float,
                      eta=eta)
    assert np.abs(u - sim.u).max() <= 1e-13 * np.abs(sim.u).max()
    assert np.abs(sim.u).max() > 1e-9
    if eta:  # the damping visibly changes the run
        und = _sim(oracle_lib, dict(P, eta=0.0))
        und.run(P["steps"])
        assert np.abs(und.u - sim.u).max() > 1e-3 * np.abs(sim.u).max()


@pytest.mark.parametrize("eta", ETAS)
def test_adjoint_matches_complex_step(oracle_lib, eta):
    P = _problem(oracle_lib, eta=eta)
    (gk, gA), _ = _adjoint(oracle_lib, P)
    h = 1e-30
    rng = np.random.default_rng(9)
    for b in rng.choice(P["rp"][-1], 12, replace=False):
        kc = P["k"].astype(complex)
        kc[b] += 1j * h * P["k"][b]
        ref = _loss_cs(P, kc, P["bmag"]).imag / (h * P["k"][b])
        assert gk[b] == pytest.approx(ref, rel=1e-9, abs=1e-12 * abs(gk).max())
    ref_A = _loss_cs(P, P["k"].astype(complex), P["bmag"] + 1j * h * P["bmag"]).imag / (h * P["bmag"])
    assert gA == pytest.approx(ref_A, rel=1e-9)


def test_transpose_identity_per_pass(oracle_lib):
    P = _problem(oracle_lib)
    sim = _sim(oracle_lib, P)
    rng = np.random.default_rng(4)
    u = rng.normal(size=(P["n"], 3)) * 1e-6
    for k in (0, 10, 39):
        vv = rng.normal(size=(P["n"], 3))
        w = rng.normal(size=(P["n"], 3))
        h = 1e-30
        Jv = force_cs(P["x"], P["rp"], P["col"], P["k"], P["vol"], u + 1j * h * vv, P["frozen"], k).imag / h
        JTw = sim.apply_jt(P["frozen"], u, k, w)
        lhs, rhs = (Jv * w).sum(), (vv * JTw).sum()
        assert lhs == pytest.approx(rhs, rel=1e-11)


@pytest.mark.parametrize("eta", ETAS)
def test_adjoint_central_differences(oracle_lib, eta):
    P = _problem(oracle_lib, eta=eta)
    (gk, gA), _ = _adjoint(oracle_lib, P)

    def loss(k, bmag):
        sim = _sim(oracle_lib, P, k=k, bmag=bmag)
        sim.run(P["steps"])
        d = sim.u[P["sensors"]] - P["target"]
        return (d * d).sum()

    order = np.argsort(-np.abs(gk))[:4]
    for b in order:
        hb = 1e-6 * P["k"][b]
        kp, km = P["k"].copy(), P["k"].copy()
        kp[b] += hb
        km[b] -= hb
        fd = (loss(kp, P["bmag"]) - loss(km, P["bmag"])) / (2 * hb)
        assert gk[b] == pytest.approx(fd, rel=1e-5)
    hA = 1e-6 * P["bmag"]
    fdA = (loss(P["k"], P["bmag"] + hA) - loss(P["k"], P["bmag"] - hA)) / (2 * hA)
    assert gA == pytest.approx(fdA, rel=1e-6)
